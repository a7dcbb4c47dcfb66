// Low-latency streaming (Sec. VII.A): the next stretch of SNR from the newest
// data only.
//
// The data live in a ring of N samples indexed by absolute sample number mod
// N; each reference's series lives in its slot of the plan's series store
// under the same indexing.  A push of D new samples
//   1. writes them into the ring at [head, head + D) and advances head;
//   2. transforms the ring once (one N-point transform, shared by every
//      reference: the reference filters are long, so their matched filters
//      still see the whole window, as the paper's reference step does);
//   3. evaluates every reference series on the last zlen positions only,
//      [head - zlen, head): the correlation sum of Eq. 1 at zlen lags, by the
//      tap construction's lag-restricted transform (column FFTs reduced at
//      once to per-workgroup shares of the kept lags), and stores them;
//   4. runs the ratio FIR of every template over the D outputs
//      [head - D - lag, head - lag): lag >= k0 + T keeps every FIR input
//      inside the freshly evaluated stretch (the (T - 1)-sample halo plus the
//      taps' lead k0), so no template touches more than D + T - 1 reference
//      samples per push.
// Circular correlation over the ring is shift-equivariant, so positions are
// absolute: the ring is never rotated.
//
// Correlation trick of step 3: with the reference spectra as the batched
// operand and the data spectrum as the shared one, the lag-restricted sum
// yields c_b[l] = sum_i w_i h_b[i] conj(s[i]) e^{+2 pi i i (k0' + l)/N}
// = conj(z_b[-(k0' + l)]); k0' = -(n0 + zlen - 1) puts z_b[n0 + j] at
// l = zlen - 1 - j.
#include <math.h>

#include <algorithm>
#include <new>

#include "dev_common.h"
#include "rfd_internal.h"

namespace rfd {

constexpr int kStreamRefBatch = 32;    // references per lag-restricted launch

struct Stream {
  rfd_plan* handle = nullptr;
  const Taps* taps = nullptr;
  int nref = 0;
  std::vector<int32_t> slot;           // plan slot of stream reference r
  double2* href = nullptr;             // [nref][nb] stream-owned copies of the reference spectra
  double* scale = nullptr;             // [nref] 1 / (sigma_ref * data scale)
  int32_t* d_slot = nullptr;           // [nref]
  double* ring = nullptr;              // [N] data ring
  int64_t head = 0;                    // next write position (the newest sample is head - 1)
  int64_t D = 0, lag = 0, zlen = 0;
  double2* corr = nullptr;             // [nref][zlen] lag sums
  Taps work;                           // work buffer of the lag-restricted transform
  bool primed = false;
};

// sigma_ref^2 = sum_i w_i |h_i|^2 over the band, one workgroup per reference,
// fixed summation order
__global__ __launch_bounds__(1024) void k_stream_sigma(const double* __restrict__ w, const double2* __restrict__ h,
                                                     int64_t nb, int64_t i_low, int64_t i_high, double inv_alpha,
                                                     double* __restrict__ scale) {
  __shared__ double red[1024];
  const double2* hb = h + (int64_t)blockIdx.x * nb;
  double acc = 0.0;
  for (int64_t i = i_low + threadIdx.x; i <= i_high; i += 1024) acc += w[i] * (hb[i].x * hb[i].x + hb[i].y * hb[i].y);
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) scale[blockIdx.x] = red[0] > 0.0 ? inv_alpha / sqrt(red[0]) : 0.0;
}

// z_b[n0 + j] = conj(c_b[zlen - 1 - j]) into the FP32 series store (the lag
// sums already carry 1 / (sigma_b alpha)), positions mod N
__global__ __launch_bounds__(256) void k_stream_store(const double2* __restrict__ corr, int64_t zlen,
                                                    const int32_t* __restrict__ slot, float2* __restrict__ zref,
                                                    int64_t n, int64_t n0) {
  const int b = blockIdx.y;
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= zlen) return;
  const double2 c = corr[(int64_t)b * zlen + (zlen - 1 - j)];
  const int64_t m = (int64_t)slot[b] * n + ((n0 + j) & (n - 1));
  zref[m] = make_float2((float)c.x, (float)-c.y);
}

static void stream_free(Stream& s) {
  if (s.href) (void)hipFree(s.href);
  if (s.scale) (void)hipFree(s.scale);
  if (s.d_slot) (void)hipFree(s.d_slot);
  if (s.ring) (void)hipFree(s.ring);
  if (s.corr) (void)hipFree(s.corr);
  if (s.work.work64) (void)hipFree(s.work.work64);
  s.href = nullptr;
  s.scale = nullptr;
  s.d_slot = nullptr;
  s.ring = nullptr;
  s.corr = nullptr;
  s.work.work64 = nullptr;
}

template <typename T>
static int salloc(T** ptr, size_t count) {
  *ptr = nullptr;
  if (device_malloc((void**)ptr, std::max<size_t>(count, 1) * sizeof(T)) != hipSuccess) {
    *ptr = nullptr;
    (void)hipGetLastError();
    return fail(RFD_E_NOMEM, "stream: hipMalloc of " + std::to_string(count * sizeof(T)) + " bytes failed");
  }
  return RFD_OK;
}

// FIR, window peaks and compaction over the outputs [start, start + len) mod
// N (at most two contiguous pieces), one slot array and one compaction.
static int stream_filter(Plan& p, const Taps& t, int precision, float threshold, int64_t W, int64_t start,
                         int64_t len, rfd_trigger* out, int64_t capacity, int64_t* n_out) {
  Taps& tm = const_cast<Taps&>(t);
  const int64_t nwin = (p.n + W - 1) / W;
  const int64_t n_slots = t.n_templates * nwin;
  int rc = ensure_slots(p, std::max<int64_t>(n_slots, 1));
  if (rc) return rc;
  if (precision == RFD_OLS32) {
    rc = ensure_ols(p, tm);
    if (rc) return rc;
  }
  int64_t lo[2] = {start, 0}, hi[2] = {std::min(start + len, p.n), 0};
  int pieces = 1;
  if (start + len > p.n) {
    hi[1] = start + len - p.n;
    pieces = 2;
  }
  // clear and compact only the windows the outputs meet
  WinMap m;
  if (!win_map_range(nwin, W, pieces, lo, hi, &m)) m = win_map_all(nwin);
  const int64_t n_visit = t.n_templates * m.nq;
  rc = launch_slots_clear_map(p, n_visit, m);
  if (rc) return rc;
  rc = stage_begin(p, kStFir);
  if (rc) return rc;
  for (int k = 0; k < pieces && !rc; ++k) {
    if (precision == RFD_OLS32) {
      rc = launch_ols(p, t, W, nwin, threshold, lo[k], hi[k]);
    } else {
      for (size_t b = 0; !rc && b < t.sb.size(); ++b)
        rc = launch_fir(p, t, (int)b, precision, W, nwin, threshold, lo[k], hi[k] - lo[k]);
    }
  }
  if (rc) return rc;
  rc = stage_end(p);
  if (!rc) rc = stage_begin(p, kStCompact);
  if (rc) return rc;
  rc = launch_compact_bank(p, t, n_visit, nwin, W, threshold, out, capacity, &m);
  if (rc) return rc;
  rc = launch_fir_z(p, t, out, std::min<int64_t>(capacity, (int64_t)1 << 26));
  if (!rc) rc = stage_end(p);
  if (rc) return rc;
  return finish_triggers(p, capacity, n_out);
}

}  // namespace rfd

struct rfd_stream { rfd::Stream s; };

using namespace rfd;

extern "C" {

int rfd_stream_create(rfd_plan* plan, const rfd_taps* taps, int32_t n_refs, const int32_t* ref_ids,
                      const double* const* h_refs, int64_t increment, rfd_stream** out) {
  if (!plan || !taps || !ref_ids || !h_refs || !out) return fail(RFD_E_INVALID, "NULL argument");
  *out = nullptr;
  Plan& p = plan->p;
  const Taps& t = taps->t;
  if (t.plan != &p) return fail(RFD_E_INVALID, "taps belong to another plan");
  if (n_refs < 1 || n_refs > p.max_refs) return fail(RFD_E_INVALID, "n_refs must be in [1, max_refs]");
  if (increment < 256 || increment % 256 != 0 || increment > p.n / 4)
    return fail(RFD_E_INVALID, "increment must be a positive multiple of 256 and at most N/4");
  std::vector<int32_t> slot(ref_ids, ref_ids + n_refs);
  for (int r = 0; r < n_refs; ++r) {
    if (slot[r] < 0 || slot[r] >= p.max_refs) return fail(RFD_E_INVALID, "ref_id out of range");
    if (!h_refs[r]) return fail(RFD_E_INVALID, "NULL reference spectrum");
    for (int q = 0; q < r; ++q)
      if (slot[q] == slot[r]) return fail(RFD_E_INVALID, "duplicate ref_id");
  }
  // output lag and evaluated stretch from the taps: every FIR input of the D
  // outputs [head - D - lag, head - lag) lies in [head - zlen, head)
  int64_t lead = 0, back = 0;
  for (const SubBankTaps& s : t.sb) {
    if (s.count == 0) continue;
    if (std::find(slot.begin(), slot.end(), s.ref_id) == slot.end())
      return fail(RFD_E_INVALID, "a sub-bank's reference is not among the stream's references");
    lead = std::max<int64_t>(lead, (int64_t)s.k0 + s.T);
    back = std::max<int64_t>(back, -(int64_t)s.k0);
  }
  Stream st;
  st.handle = plan;
  st.taps = &t;
  st.nref = n_refs;
  st.slot = slot;
  st.D = increment;
  st.lag = round_up(lead, 256);
  st.zlen = round_up(increment + st.lag + back, 256);
  if (st.zlen > p.n / 2)
    return fail(RFD_E_INVALID, "increment plus the taps' span must stay within half the segment");
  int rc;
  const int bmax = std::min(n_refs, kStreamRefBatch);
  if ((rc = salloc(&st.href, (size_t)n_refs * p.nb)) || (rc = salloc(&st.scale, (size_t)n_refs)) ||
      (rc = salloc(&st.d_slot, (size_t)n_refs)) || (rc = salloc(&st.ring, (size_t)p.n)) ||
      (rc = salloc(&st.corr, (size_t)n_refs * st.zlen)) || (rc = salloc(&st.work.work64, (size_t)bmax * p.n))) {
    stream_free(st);
    return rc;
  }
  st.work.work64_cap = (size_t)bmax * p.n;
  for (int r = 0; r < n_refs; ++r) {
    if (hipMemcpyAsync(st.href + (int64_t)r * p.nb, h_refs[r], (size_t)p.nb * sizeof(double2),
                       hipMemcpyDeviceToDevice, p.stream) != hipSuccess) {
      stream_free(st);
      return fail(RFD_E_DEVICE, "stream: reference copy failed");
    }
  }
  if (hipMemcpyAsync(st.d_slot, slot.data(), (size_t)n_refs * sizeof(int32_t), hipMemcpyHostToDevice, p.stream) !=
      hipSuccess) {
    stream_free(st);
    return fail(RFD_E_DEVICE, "stream: slot table upload failed");
  }
  hipLaunchKernelGGL(k_stream_sigma, dim3((unsigned)n_refs), dim3(1024), 0, p.stream, (const double*)p.w,
                     (const double2*)st.href, p.nb, p.i_low, p.i_high, 1.0 / p.data_scale, st.scale);
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(p.stream) != hipSuccess) {
    stream_free(st);
    return fail(RFD_E_DEVICE, "stream: set-up kernels failed");
  }
  rfd_stream* h = new (std::nothrow) rfd_stream;
  if (!h) {
    stream_free(st);
    return fail(RFD_E_NOMEM, "stream: host allocation failed");
  }
  h->s = std::move(st);
  ++p.users;
  ++const_cast<Taps&>(t).users;
  *out = h;
  return RFD_OK;
}

int rfd_stream_info(const rfd_stream* stream, int64_t* head, int64_t* lag, int64_t* zlen) {
  if (!stream) return fail(RFD_E_INVALID, "NULL stream");
  const Stream& s = stream->s;
  if (head) *head = s.head;
  if (lag) *lag = s.lag;
  if (zlen) *zlen = s.zlen;
  return RFD_OK;
}

int rfd_stream_prime(rfd_stream* stream, const double* data) {
  if (!stream || !data) return fail(RFD_E_INVALID, "NULL argument");
  Stream& s = stream->s;
  Plan& p = s.handle->p;
  RFD_HIP(hipMemcpyAsync(s.ring, data, (size_t)p.n * sizeof(double), hipMemcpyDeviceToDevice, p.stream));
  std::vector<const double*> hp(s.nref);
  for (int r = 0; r < s.nref; ++r) hp[r] = reinterpret_cast<const double*>(s.href + (int64_t)r * p.nb);
  int rc = rfd_dechirp_refs(s.handle, s.ring, s.nref, s.slot.data(), hp.data(), nullptr);
  if (rc) return rc;
  s.head = 0;
  s.primed = true;
  return RFD_OK;
}

int rfd_stream_push(rfd_stream* stream, const double* data, int32_t precision, float threshold,
                    int64_t cluster_window, rfd_trigger* out, int64_t capacity, int64_t* n_out,
                    int64_t* out_start) {
  if (!stream || !data || !n_out) return fail(RFD_E_INVALID, "NULL argument");
  Stream& s = stream->s;
  Plan& p = s.handle->p;
  const Taps& t = *s.taps;
  if (!s.primed) return fail(RFD_E_STATE, "stream not primed with a first window");
  if (precision != RFD_FP32 && precision != RFD_BF16X3 && precision != RFD_FP16X3 && precision != RFD_OLS32)
    return fail(RFD_E_INVALID, "unknown precision");
  if (!(threshold >= 0.f) || !std::isfinite(threshold)) return fail(RFD_E_INVALID, "threshold must be finite and >= 0");
  if (cluster_window < 1 || cluster_window > p.n) return fail(RFD_E_INVALID, "cluster_window must satisfy 1 <= W <= N");
  if (capacity < 0 || (capacity > 0 && !out)) return fail(RFD_E_INVALID, "bad trigger buffer");
  for (size_t b = 0; b < t.sb.size(); ++b)
    if (t.sb[b].count > 0 && t.sb[b].made != t.sb[b].count)
      return fail(RFD_E_STATE, "sub-bank " + std::to_string(b) + ": taps not made");
  // 1. the new samples into the ring
  RFD_HIP(hipMemcpyAsync(s.ring + s.head, data, (size_t)s.D * sizeof(double), hipMemcpyDeviceToDevice, p.stream));
  s.head = (s.head + s.D) % p.n;
  // 2. one transform of the ring
  int rc = stage_begin(p, kStDataFft);
  if (!rc) rc = launch_data_fft(p, s.ring);
  if (!rc) rc = stage_end(p);
  if (rc) return rc;
  // 3. every reference series on [head - zlen, head)
  const int64_t n0 = (s.head - s.zlen + p.n) % p.n;
  const int k0c = -(int)(n0 + s.zlen - 1);
  rc = stage_begin(p, kStDechirp);
  if (rc) return rc;
  for (int r0 = 0; r0 < s.nref; r0 += kStreamRefBatch) {
    const int nb = std::min(kStreamRefBatch, s.nref - r0);
    // the stretch's column transforms in the dechirp's precision, the
    // normalisation folded into the integrand (FP32 range)
    rc = launch_corr64(p, s.work, 0, reinterpret_cast<const double*>(p.stilde64),
                       reinterpret_cast<const double*>(s.href + (int64_t)r0 * p.nb), nb, (int)s.zlen, k0c,
                       s.corr + (int64_t)r0 * s.zlen, s.zlen, -1, -1, nullptr, !p.dechirp_fp64, s.scale + r0);
    if (rc) return rc;
    hipLaunchKernelGGL(k_stream_store, dim3((unsigned)((s.zlen + 255) / 256), (unsigned)nb), dim3(256), 0, p.stream,
                       (const double2*)(s.corr + (int64_t)r0 * s.zlen), s.zlen, (const int32_t*)(s.d_slot + r0),
                       p.zref, p.n, n0);
    RFD_CHECK_LAUNCH();
  }
  rc = stage_end(p);
  if (rc) return rc;
  // the series store now holds a mix of pushes: whole-segment calls must dechirp again
  ++p.seg_gen;
  // 4. the ratio FIR over the D outputs [head - D - lag, head - lag)
  const int64_t start = (s.head - s.D - s.lag + 2 * p.n) % p.n;
  if (out_start) *out_start = start;
  return stream_filter(p, t, precision, threshold, cluster_window, start, s.D, out, capacity, n_out);
}

int rfd_stream_destroy(rfd_stream* stream) {
  if (!stream) return RFD_OK;
  Plan& p = stream->s.handle->p;
  (void)hipStreamSynchronize(p.stream);
  --p.users;
  --const_cast<Taps*>(stream->s.taps)->users;
  stream_free(stream->s);
  delete stream;
  return RFD_OK;
}

}  // extern "C"
