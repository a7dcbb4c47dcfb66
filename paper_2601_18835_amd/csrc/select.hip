// Dynamic tap count (Sec. V.A): for each template, the first T of an
// ascending ladder whose least-squares taps (lags centred on lag 0,
// k0 = -floor(T/2), or with RFD_TAPS_CENTRE on the peak of the template's
// correlation with the reference) reach a target match with the target
// template.  The match is the fitted
// template's phase-maximised overlap with the target at zero lag,
//   m = |(h_j|h_fit)(0)| / (sigma_j sigma_fit) = |a^H b| / (sigma_j sigma_fit),
// b the normal equations' right-hand side (b_k = (h_j|h_ref)(t_k)), so it
// costs O(T) per template once the taps exist.
#include <math.h>

#include <algorithm>
#include <vector>

#include "dev_common.h"
#include "rfd_internal.h"

namespace rfd {

// sigma_j^2 = sum_i w_i |h_j,i|^2, one workgroup per template
__global__ __launch_bounds__(256) void k_norm2(const double* __restrict__ w, const double2* __restrict__ h,
                                             int64_t nb, double* __restrict__ out) {
  __shared__ double red[256];
  const double2* hj = h + (int64_t)blockIdx.x * nb;
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < nb; i += 256) {
    const double2 v = hj[i];
    acc += w[i] * (v.x * v.x + v.y * v.y);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

// m_j = |a_j^H b_j| / (sigma_j sigma_fit,j), one wave per template
__global__ __launch_bounds__(64) void k_zero_lag_match(const double2* __restrict__ a, int64_t Tp,
                                                     const double2* __restrict__ b, int T,
                                                     const double* __restrict__ sig_fit,
                                                     const double* __restrict__ norm2_j, double* __restrict__ m) {
  const int64_t j = blockIdx.x;
  const double2* aj = a + j * Tp;
  const double2* bj = b + j * (int64_t)T;
  double re = 0.0, im = 0.0;
  for (int k = threadIdx.x; k < T; k += 64) {
    const double2 x = aj[k], y = bj[k];
    re += x.x * y.x + x.y * y.y;     // conj(a) b
    im += x.x * y.y - x.y * y.x;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    re += __shfl_xor(re, o);
    im += __shfl_xor(im, o);
  }
  if (threadIdx.x == 0) m[j] = sqrt(re * re + im * im) / (sqrt(norm2_j[j]) * sig_fit[j]);
}

}  // namespace rfd

using namespace rfd;

extern "C" {

int rfd_select_taps(rfd_plan* plan, const double* h_ref, const double* h_tmpl, int64_t count, double target,
                    const int32_t* ladder, int32_t n_ladder, double ridge_eps, int32_t flags, int32_t* taps_out,
                    double* match_out, int32_t* k0_out) {
  if (!plan || !h_ref || !ladder || !taps_out) return fail(RFD_E_INVALID, "NULL argument");
  if (count < 0) return fail(RFD_E_INVALID, "count must be >= 0");
  if (n_ladder < 1 || n_ladder > 64) return fail(RFD_E_INVALID, "n_ladder must be in [1, 64]");
  for (int i = 0; i < n_ladder; ++i) {
    if (ladder[i] < 1 || ladder[i] > RFD_MAX_TAPS) return fail(RFD_E_INVALID, "ladder entries must be in [1, 2048]");
    if (i && ladder[i] <= ladder[i - 1]) return fail(RFD_E_INVALID, "ladder must be strictly ascending");
  }
  if (!(target > 0.0) || !isfinite(target)) return fail(RFD_E_INVALID, "target must be finite and > 0");
  if (flags != 0 && flags != RFD_TAPS_CENTRE) return fail(RFD_E_INVALID, "flags must be 0 or RFD_TAPS_CENTRE");
  if (count == 0) return RFD_OK;
  if (!h_tmpl) return fail(RFD_E_INVALID, "h_tmpl is NULL");
  Plan& p = plan->p;
  double* norm2 = nullptr;
  double* m = nullptr;
  if (device_malloc((void**)&norm2, count * sizeof(double)) != hipSuccess ||
      device_malloc((void**)&m, count * sizeof(double)) != hipSuccess) {
    (void)hipGetLastError();
    if (norm2) (void)hipFree(norm2);
    return fail(RFD_E_NOMEM, "tap selection: hipMalloc failed");
  }
  int rc = RFD_OK;
  std::vector<double> mh(count);
  std::vector<int32_t> dh(count, 0);
  std::vector<char> done(count, 0);
  for (int64_t j0 = 0; j0 < count && !rc; j0 += 65535) {
    const int64_t c = std::min<int64_t>(count - j0, 65535);
    hipLaunchKernelGGL(k_norm2, dim3((unsigned)c), dim3(256), 0, p.stream, p.w,
                       (const double2*)h_tmpl + j0 * p.nb, p.nb, norm2 + j0);
    if (hipGetLastError() != hipSuccess) rc = fail(RFD_E_DEVICE, "norm launch failed");
  }
  for (int li = 0; li < n_ladder && !rc; ++li) {
    const int T = ladder[li];
    const int32_t k0 = -(T / 2), ref0 = 0;
    const int64_t off[2] = {0, count};
    rfd_taps* tp = nullptr;
    rc = rfd_taps_create(plan, 1, off, &ref0, &T, &k0, &tp);
    if (rc) break;
    rc = rfd_make_taps(plan, tp, 0, h_ref, h_tmpl, 0, count, RFD_TAPS_LS | flags, ridge_eps);
    if (!rc) {
      Taps& t = tp->t;
      const SubBankTaps& s = t.sb[0];
      hipLaunchKernelGGL(k_zero_lag_match, dim3((unsigned)count), dim3(64), 0, p.stream, t.a64 + s.a_base,
                         (int64_t)s.Tp, (const double2*)t.bvec, T, (const double*)t.sigma_fit,
                         (const double*)norm2, m);
      if (hipGetLastError() != hipSuccess) rc = fail(RFD_E_DEVICE, "match launch failed");
      if (!rc && hipMemcpyAsync(mh.data(), m, count * sizeof(double), hipMemcpyDeviceToHost, p.stream) != hipSuccess)
        rc = fail(RFD_E_DEVICE, "match readback failed");
      if (!rc && hipMemcpyAsync(dh.data(), t.d_shift, count * sizeof(int32_t), hipMemcpyDeviceToHost, p.stream) !=
                     hipSuccess)
        rc = fail(RFD_E_DEVICE, "lag readback failed");
      if (!rc && hipStreamSynchronize(p.stream) != hipSuccess) rc = fail(RFD_E_DEVICE, "synchronise failed");
    }
    rfd_taps_destroy(tp);
    if (rc) break;
    for (int64_t j = 0; j < count; ++j) {
      if (done[j]) continue;
      taps_out[j] = T;
      if (match_out) match_out[j] = mh[j];
      if (k0_out) k0_out[j] = k0 + dh[j];
      if (mh[j] >= target) done[j] = 1;
    }
  }
  (void)hipFree(norm2);
  (void)hipFree(m);
  return rc;
}

}  // extern "C"
