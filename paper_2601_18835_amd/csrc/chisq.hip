// Ratio-filtered chi^2 signal-consistency test (Sec. VI.C).
//
// The analysis band is split into p contiguous bin ranges of equal reference
// power (u_i = w_i |h_ref,i|^2; edge b is the first bin where the sequential
// FP64 prefix sum reaches total * b / p).  Each reference slot stores its p
// band series zhat_b (the dechirp integrand restricted to band b, FP32,
// normalised by sigma_ref; they sum to zhat).  A target's band SNRs are the
// same ratio FIR on those series (Eq. 3 band by band):
//   z_b[n] = sum_k c_k zhat_b[n + k0 + k],   z = sum_b z_b,
// its shares are the fitted template's band power fractions
//   f_b = a^H M_b a / sum_b' a^H M_b' a,  M_b[l,k] = g_b[l-k],
//   g_b[m] = sum_{i in band b} u_i exp(+2 pi i i m / N),
// and chi^2 = sum_b |z_b - f_b z|^2 / f_b at each trigger.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "dev_common.h"
#include "rfd_internal.h"

namespace rfd {

constexpr int kMaxBands = 64;

// Band edges from the host copy of u (the rule in the header comment).
static int band_edges(Plan& p, const double* h_ref, int n_bands, std::vector<int64_t>& edges) {
  if (n_bands < 2 || n_bands > kMaxBands) return fail(RFD_E_INVALID, "n_bands must be in [2, 64]");
  const int64_t lo = p.i_low, hi = p.i_high, cnt = hi - lo + 1;
  std::vector<double> w(cnt);
  std::vector<double2> h(cnt);
  RFD_HIP(hipMemcpyAsync(w.data(), p.w + lo, cnt * sizeof(double), hipMemcpyDeviceToHost, p.stream));
  RFD_HIP(hipMemcpyAsync(h.data(), h_ref + 2 * lo, cnt * sizeof(double2), hipMemcpyDeviceToHost, p.stream));
  RFD_HIP(hipStreamSynchronize(p.stream));
  std::vector<double> prefix(cnt + 1, 0.0);
  for (int64_t i = 0; i < cnt; ++i) {
    const double re2 = h[i].x * h[i].x;   // separate statements: no fused multiply-add
    const double im2 = h[i].y * h[i].y;
    const double pw = re2 + im2;
    const double u = w[i] * pw;
    prefix[i + 1] = prefix[i] + u;
  }
  const double total = prefix[cnt];
  if (!(total > 0.0)) return fail(RFD_E_INVALID, "reference has no power in the analysis band");
  edges.assign(1, lo);
  for (int b = 1; b < n_bands; ++b) {
    const double thr = (total * b) / n_bands;
    const int64_t k = std::lower_bound(prefix.begin(), prefix.end(), thr) - prefix.begin();
    edges.push_back(lo + k);
  }
  edges.push_back(hi + 1);
  for (int b = 0; b < n_bands; ++b)
    if (edges[b + 1] <= edges[b]) return fail(RFD_E_INVALID, "band split produced an empty band; use fewer bands");
  return RFD_OK;
}

// num[b][j] = a_j^H M_b a_j, one workgroup per (template, band)
__global__ __launch_bounds__(256) void k_band_quad(const double2* __restrict__ a, int64_t Tp, int T,
                                                 const double2* __restrict__ g, double* __restrict__ num,
                                                 int64_t count) {
  extern __shared__ double2 sh[];
  double2* av = sh;
  double2* gv = sh + T;
  __shared__ double red[256];
  const int64_t j = blockIdx.x;
  const int b = blockIdx.y;
  const double2* aj = a + j * Tp;
  const double2* gb = g + (int64_t)b * T;
  for (int i = threadIdx.x; i < T; i += 256) {
    av[i] = aj[i];
    gv[i] = gb[i];
  }
  __syncthreads();
  double acc = 0.0;
  for (int l = threadIdx.x; l < T; l += 256) {
    double2 s = make_double2(0.0, 0.0);
    for (int k = 0; k < T; ++k) {
      const int d = l - k;
      const double2 gk = d >= 0 ? gv[d] : cconj(gv[-d]);
      s = cadd(s, cmul(gk, av[k]));
    }
    acc += av[l].x * s.x + av[l].y * s.y;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) num[(int64_t)b * count + j] = red[0];
}

// f[j][b] = num[b][j] / sum_b num[b][j]
__global__ void k_band_norm(const double* __restrict__ num, int64_t count, int p, float* __restrict__ f) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= count) return;
  double tot = 0.0;
  for (int b = 0; b < p; ++b) tot += num[(int64_t)b * count + j];
  const double inv = tot > 0.0 ? 1.0 / tot : 0.0;
  for (int b = 0; b < p; ++b) f[j * p + b] = (float)(num[(int64_t)b * count + j] * inv);
}

// Per-sub-bank metadata of the chi^2 kernel.
struct ChisqSub {
  int64_t first, count, a_base;
  int32_t T, Tp, k0, ref_id;
  const float* f;
};

// One wave per trigger: the band SNRs at the trigger sample, then chi^2.
__global__ __launch_bounds__(64) void k_chisq(const rfd_trigger* __restrict__ trig, int64_t n_trig,
                                            const ChisqSub* __restrict__ subs, int nsb,
                                            const float2* const* __restrict__ bands, int p, int64_t n,
                                            const float2* __restrict__ c32, const int32_t* __restrict__ shift,
                                            float* __restrict__ out) {
  const int64_t t = blockIdx.x;
  if (t >= n_trig) return;
  const int lane = threadIdx.x;
  const rfd_trigger tr = trig[t];
  const int sb = tr.subbank;
  bool ok = sb >= 0 && sb < nsb && tr.sample >= 0 && tr.sample < n;
  ChisqSub s{};
  if (ok) {
    s = subs[sb];
    ok = tr.tmpl >= s.first && tr.tmpl < s.first + s.count && bands[s.ref_id] != nullptr && s.f != nullptr;
  }
  if (!ok) {
    if (lane == 0) out[t] = __int_as_float(0x7fc00000);   // NaN for a trigger outside the bank
    return;
  }
  const int64_t j = tr.tmpl - s.first;
  const float2* c = c32 + s.a_base + j * s.Tp;
  const float2* zb = bands[s.ref_id];
  __shared__ float2 zs[kMaxBands];
  const int64_t base = tr.sample + s.k0 + shift[tr.tmpl];   // the template's own lag window
  for (int b = 0; b < p; ++b) {
    const float2* z = zb + (int64_t)b * n;
    float re = 0.f, im = 0.f;
    for (int k = lane; k < s.T; k += 64) {
      const float2 x = z[(base + k) & (n - 1)];
      const float2 ck = c[k];
      re += ck.x * x.x - ck.y * x.y;
      im += ck.x * x.y + ck.y * x.x;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      re += __shfl_xor(re, o);
      im += __shfl_xor(im, o);
    }
    if (lane == 0) zs[b] = make_float2(re, im);
  }
  __syncthreads();
  if (lane == 0) {
    float2 z = make_float2(0.f, 0.f);
    for (int b = 0; b < p; ++b) z = cadd(z, zs[b]);
    const float* f = s.f + j * p;
    float x = 0.f;
    for (int b = 0; b < p; ++b) {
      const float fb = f[b];
      const float dr = zs[b].x - fb * z.x, di = zs[b].y - fb * z.y;
      x += (dr * dr + di * di) / fb;
    }
    out[t] = x;
  }
}

template <typename T>
static int calloc_dev(T** p, size_t n) {
  *p = nullptr;
  if (device_malloc((void**)p, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return fail(RFD_E_NOMEM, "chi^2: hipMalloc failed");
  }
  return RFD_OK;
}

}  // namespace rfd

using namespace rfd;

extern "C" {

int rfd_dechirp_bands(rfd_plan* plan, const double* h_ref, int32_t ref_id, int32_t n_bands, int64_t* edges_out) {
  if (!plan || !h_ref) return fail(RFD_E_INVALID, "NULL argument");
  Plan& p = plan->p;
  if (ref_id < 0 || ref_id >= p.max_refs) return fail(RFD_E_INVALID, "ref_id out of range");
  if (p.seg_gen == 0) return fail(RFD_E_STATE, "no segment transformed yet");
  std::vector<int64_t> edges;
  int rc = band_edges(p, h_ref, n_bands, edges);
  if (rc) return rc;
  const int64_t need = (int64_t)n_bands * p.n;
  if (p.zband_cap[ref_id] < need) {
    RFD_HIP(hipStreamSynchronize(p.stream));
    if (p.zband[ref_id]) (void)hipFree(p.zband[ref_id]);
    p.zband[ref_id] = nullptr;
    p.zband_cap[ref_id] = 0;
    rc = calloc_dev(&p.zband[ref_id], (size_t)need);
    if (rc) return rc;
    p.zband_cap[ref_id] = need;
    ++p.res_gen;
  }
  rc = launch_dechirp_bands(p, h_ref, edges.data(), n_bands, p.zband[ref_id]);
  if (rc) return rc;
  p.zband_edges[ref_id] = edges;
  p.zband_gen[ref_id] = p.seg_gen;
  if (edges_out) memcpy(edges_out, edges.data(), edges.size() * sizeof(int64_t));
  return RFD_OK;
}

int rfd_taps_band_fractions(rfd_plan* plan, rfd_taps* taps, int32_t subbank, const double* h_ref, int32_t n_bands) {
  if (!plan || !taps || !h_ref) return fail(RFD_E_INVALID, "NULL argument");
  Plan& p = plan->p;
  Taps& t = taps->t;
  if (t.plan != &p) return fail(RFD_E_INVALID, "taps belong to another plan");
  if (subbank < 0 || subbank >= (int)t.sb.size()) return fail(RFD_E_INVALID, "subbank out of range");
  SubBankTaps& s = t.sb[subbank];
  if (s.made != s.count) return fail(RFD_E_STATE, "taps not made");
  std::vector<int64_t> edges;
  int rc = band_edges(p, h_ref, n_bands, edges);
  if (rc) return rc;
  if (s.count == 0) {
    s.band_edges = edges;
    return RFD_OK;
  }
  const int T = s.T;
  if (t.work64_cap < (size_t)p.n) {
    RFD_HIP(hipStreamSynchronize(p.stream));
    if (t.work64) (void)hipFree(t.work64);
    t.work64 = nullptr;
    t.work64_cap = 0;
    rc = calloc_dev(&t.work64, (size_t)p.n);
    if (rc) return rc;
    t.work64_cap = p.n;
  }
  double2* g = nullptr;
  double* num = nullptr;
  rc = calloc_dev(&g, (size_t)n_bands * T);
  if (!rc) rc = calloc_dev(&num, (size_t)n_bands * s.count);
  if (!rc && !s.band_f) rc = calloc_dev(&s.band_f, (size_t)s.count * kMaxBands);
  // band autocorrelations g_b at lags 0..T-1
  for (int b = 0; !rc && b < n_bands; ++b)
    rc = launch_corr64(p, t, 1, h_ref, nullptr, 1, T, 0, g + (int64_t)b * T, T, edges[b], edges[b + 1] - 1);
  if (!rc) {
    hipLaunchKernelGGL(k_band_quad, dim3((unsigned)s.count, (unsigned)n_bands), dim3(256),
                       (size_t)2 * T * sizeof(double2), p.stream, t.a64 + s.a_base, (int64_t)s.Tp, T,
                       (const double2*)g, num, s.count);
    if (hipGetLastError() != hipSuccess) rc = fail(RFD_E_DEVICE, "band quadratic form launch failed");
  }
  if (!rc) {
    hipLaunchKernelGGL(k_band_norm, dim3((unsigned)((s.count + 255) / 256)), dim3(256), 0, p.stream,
                       (const double*)num, s.count, n_bands, s.band_f);
    if (hipGetLastError() != hipSuccess) rc = fail(RFD_E_DEVICE, "band share launch failed");
  }
  (void)hipStreamSynchronize(p.stream);
  if (g) (void)hipFree(g);
  if (num) (void)hipFree(num);
  if (rc) return rc;
  s.band_edges = edges;
  return RFD_OK;
}

int rfd_taps_get_band_fractions(const rfd_taps* taps, int64_t tmpl, float* f_out, int32_t* n_bands_out) {
  if (!taps || !f_out) return fail(RFD_E_INVALID, "NULL argument");
  const Taps& t = taps->t;
  for (const SubBankTaps& s : t.sb) {
    if (tmpl < s.first || tmpl >= s.first + s.count) continue;
    if (!s.band_f || s.band_edges.empty()) return fail(RFD_E_STATE, "band shares not computed for this sub-bank");
    const int p = (int)s.band_edges.size() - 1;
    RFD_HIP(hipMemcpyAsync(f_out, s.band_f + (tmpl - s.first) * p, p * sizeof(float), hipMemcpyDeviceToHost,
                           t.plan->stream));
    RFD_HIP(hipStreamSynchronize(t.plan->stream));
    if (n_bands_out) *n_bands_out = p;
    return RFD_OK;
  }
  return fail(RFD_E_INVALID, "template index out of range");
}

int rfd_chisq(rfd_plan* plan, const rfd_taps* taps, const rfd_trigger* triggers, int64_t n, float* chisq_out) {
  if (!plan || !taps) return fail(RFD_E_INVALID, "NULL plan or taps");
  Plan& p = plan->p;
  const Taps& t = taps->t;
  if (t.plan != &p) return fail(RFD_E_INVALID, "taps belong to another plan");
  if (n < 0) return fail(RFD_E_INVALID, "n must be >= 0");
  if (n == 0) return RFD_OK;
  if (!triggers || !chisq_out) return fail(RFD_E_INVALID, "NULL triggers or output");
  int pb = -1;
  std::vector<ChisqSub> subs(t.sb.size());
  for (size_t b = 0; b < t.sb.size(); ++b) {
    const SubBankTaps& s = t.sb[b];
    subs[b] = ChisqSub{s.first, s.count, s.a_base, s.T, s.Tp, s.k0, s.ref_id, s.band_f};
    if (s.count == 0) continue;
    if (s.made != s.count) return fail(RFD_E_STATE, "taps not made");
    if (!s.band_f || s.band_edges.empty())
      return fail(RFD_E_STATE, "sub-bank " + std::to_string(b) + ": band shares not computed");
    const int ps = (int)s.band_edges.size() - 1;
    if (pb >= 0 && ps != pb) return fail(RFD_E_INVALID, "sub-banks use different numbers of bands");
    pb = ps;
    if (p.seg_gen == 0 || p.ref_gen[s.ref_id] != p.seg_gen || p.zband_gen[s.ref_id] != p.seg_gen)
      return fail(RFD_E_STATE, "sub-bank " + std::to_string(b) + ": band series not made on this segment");
    if (p.zband_edges[s.ref_id] != s.band_edges)
      return fail(RFD_E_STATE, "sub-bank " + std::to_string(b) + ": band series and shares use different bands");
  }
  if (pb < 0) return fail(RFD_E_STATE, "bank is empty");
  ChisqSub* dsubs = nullptr;
  const float2** dbands = nullptr;
  int rc = calloc_dev(&dsubs, subs.size());
  if (!rc) rc = calloc_dev(&dbands, (size_t)p.max_refs);
  std::vector<const float2*> hb(p.max_refs);
  for (int r = 0; r < p.max_refs; ++r) hb[r] = p.zband_gen[r] == p.seg_gen ? p.zband[r] : nullptr;
  if (!rc && hipMemcpyAsync(dsubs, subs.data(), subs.size() * sizeof(ChisqSub), hipMemcpyHostToDevice, p.stream) !=
                 hipSuccess)
    rc = fail(RFD_E_DEVICE, "chi^2 metadata upload failed");
  if (!rc && hipMemcpyAsync(dbands, hb.data(), hb.size() * sizeof(float2*), hipMemcpyHostToDevice, p.stream) !=
                 hipSuccess)
    rc = fail(RFD_E_DEVICE, "chi^2 metadata upload failed");
  for (int64_t t0 = 0; !rc && t0 < n; t0 += 1 << 30) {
    const int64_t cnt = std::min<int64_t>(n - t0, (int64_t)1 << 30);
    hipLaunchKernelGGL(k_chisq, dim3((unsigned)cnt), dim3(64), 0, p.stream, triggers + t0, cnt,
                       (const ChisqSub*)dsubs, (int)subs.size(), (const float2* const*)dbands, pb, p.n,
                       (const float2*)t.c32, (const int32_t*)t.d_shift, chisq_out + t0);
    if (hipGetLastError() != hipSuccess) rc = fail(RFD_E_DEVICE, "chi^2 launch failed");
  }
  (void)hipStreamSynchronize(p.stream);
  if (dsubs) (void)hipFree(dsubs);
  if (dbands) (void)hipFree(dbands);
  return rc;
}

}  // extern "C"
