// FP64 ratio-tap construction on the device (Sec. V.A) and the fitted
// template norms (Sec. VI.B).
//
// Weighted ridge least squares: minimise sum_i u_i |R_i - A_i|^2 + lam |a|^2
// with u_i = w_i |h_ref,i|^2, R = h/h_ref, A_i = sum_k a_k exp(-2 pi i i
// (k0+k)/N).  Setting the gradient to zero gives the normal equations
//     (M + lam I) a = b,  M[l,k] = g[l-k],  g[m] = sum_i u_i exp(+2 pi i i m/N),
//     b[l] = sum_i w_i h_i conj(h_ref,i) exp(+2 pi i i (k0+l)/N),
// a Hermitian Toeplitz system shared by the whole sub-bank: g and every b
// come from FP64 FFTs (fft.hip), M + lam I is factored once per sub-bank
// (L L^H, by the Schur recursion that its Toeplitz structure allows), and each
// template costs two triangular solves.
// Norm of the fitted template h_fit = h_ref A (Parseval form of Sec. VI.B):
//     sigma_fit^2 = sum_i w_i |h_ref A|^2 = a^H M a.
// The FIR applies c = conj(a) sigma_ref / sigma_fit to zhat = z_ref/sigma_ref,
// so its output is directly the normalised SNR of h_fit.
#include <algorithm>

#include "dev_common.h"
#include "rfd_internal.h"

namespace rfd {

__device__ __forceinline__ double2 gval(const double2* g, int m) {
  return m >= 0 ? g[m] : cconj(g[-m]);
}

// Cholesky factor L (column-major, zeros above the diagonal) of the ridge
// normal matrix M + lam I, lam = eps g[0].  M[l][k] = g[l - k] is Hermitian
// Toeplitz, so its factor follows from the Schur recursion on M's
// displacement generators in O(T^2) work instead of the O(T^3) of a general
// Cholesky.  With Z the down-shift and r = (g[0] + lam, g[1], ..., g[T-1]) the
// first column, M + lam I - Z (M + lam I) Z^H = u u^H - v v^H for
// u = r / sqrt(r[0]) and v = u with v[0] = 0.  Column k of L is the current
// u; the next Schur complement has generators (Z u, v), which a hyperbolic
// rotation with rho = v[k+1] / u[k] returns to the form v[k+1] = 0:
//   v <- (v - rho Z u) / s,   u <- s Z u - conj(rho) v,   s = sqrt(1 - |rho|^2),
// the "mixed" order of the two updates, which keeps the recursion backward
// stable for positive-definite matrices.  |rho| >= 1 means M + lam I is not
// positive definite: info = step + 1.  One workgroup, T dependent steps.
constexpr int kSchurPer = (RFD_MAX_TAPS + 1023) / 1024;   // elements per thread
__global__ __launch_bounds__(1024) void k_schur_chol(const double2* __restrict__ g, int T, double eps,
                                                     double2* __restrict__ L, int* __restrict__ info) {
  __shared__ double2 u[RFD_MAX_TAPS], v[RFD_MAX_TAPS];
  const double r0 = g[0].x + eps * g[0].x;
  if (!(r0 > 0.0)) {                      // uniform
    if (threadIdx.x == 0) *info = 1;
    return;
  }
  const double inv = 1.0 / sqrt(r0);
  for (int i = threadIdx.x; i < T; i += 1024) {
    const double2 r = i == 0 ? make_double2(r0, 0.0) : g[i];
    const double2 x = make_double2(r.x * inv, r.y * inv);
    u[i] = x;
    v[i] = i == 0 ? make_double2(0.0, 0.0) : x;
    L[i] = x;                             // column 0
  }
  __syncthreads();
  for (int k = 0; k + 1 < T; ++k) {
    const double a = u[k].x;              // L[k][k]: real and positive
    const double2 b = v[k + 1];
    const double2 rho = make_double2(b.x / a, b.y / a);
    const double q = 1.0 - (rho.x * rho.x + rho.y * rho.y);
    double2 zu[kSchurPer], vi[kSchurPer];
#pragma unroll
    for (int e = 0; e < kSchurPer; ++e) {
      const int i = threadIdx.x + 1024 * e;
      if (i > k && i < T) {
        zu[e] = u[i - 1];
        vi[e] = v[i];
      }
    }
    __syncthreads();                      // every read of step k is done
    if (!(q > 0.0)) {                     // uniform: the same q in every thread
      if (threadIdx.x == 0) *info = k + 2;
      return;
    }
    const double s = sqrt(q), is = 1.0 / s;
    double2* col = L + (int64_t)(k + 1) * T;
#pragma unroll
    for (int e = 0; e < kSchurPer; ++e) {
      const int i = threadIdx.x + 1024 * e;
      if (i >= T) continue;
      if (i <= k) {
        col[i] = make_double2(0.0, 0.0);
        continue;
      }
      double2 un, vn;
      if (i == k + 1) {                   // the rotated pair: v exactly 0, u = s a
        vn = make_double2(0.0, 0.0);
        un = make_double2(s * a, 0.0);
      } else {
        vn = make_double2((vi[e].x - (rho.x * zu[e].x - rho.y * zu[e].y)) * is,
                          (vi[e].y - (rho.x * zu[e].y + rho.y * zu[e].x)) * is);
        un = make_double2(s * zu[e].x - (rho.x * vn.x + rho.y * vn.y),
                          s * zu[e].y - (rho.x * vn.y - rho.y * vn.x));
      }
      u[i] = un;
      v[i] = vn;
      col[i] = un;
    }
    __syncthreads();
  }
}

// U = L^H (column-major upper triangle)
__global__ void k_upper(const double2* __restrict__ L, int T, double2* __restrict__ U) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < (int64_t)T * T;
       e += (int64_t)gridDim.x * blockDim.x) {
    int col = (int)(e / T), row = (int)(e % T);
    U[e] = row <= col ? cconj(L[(int64_t)row * T + col]) : make_double2(0.0, 0.0);
  }
}

// (L L^H) a = b for one template per workgroup (column-oriented sweeps in LDS):
// a forward sweep with L, then a backward sweep with U = L^H.
template <int E>
struct TrsvCol {
  double2 v[E];   // column entries at rows lane + 64 q (row T - 1 past the end), unmasked
};

// Entry (j, j) of a column held as TrsvCol: lane j % 64 holds it in slot
// j / 64; read across lanes with readlane (no memory access).
template <int E>
__device__ __forceinline__ double trsv_diag(const TrsvCol<E>& c, int j) {
  // a masked sum (one nonzero term, exact) rather than a selection, which the
  // compiler would turn into an indexed access and move the ring to scratch
  double d = 0.0;
#pragma unroll
  for (int q = 0; q < E; ++q) d += (q == (j >> 6)) ? c.v[q].x : 0.0;
  const long long bits = __double_as_longlong(d);
  const int lo = __builtin_amdgcn_readlane((int)bits, j & 63);
  const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), j & 63);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

template <int E>
__device__ __forceinline__ void trsv_load(const double2* __restrict__ F, int T, int lane, TrsvCol<E>& c, int j) {
  const double2* col = F + (int64_t)min(max(j, 0), T - 1) * T;
#pragma unroll
  for (int q = 0; q < E; ++q) c.v[q] = col[min(lane + 64 * q, T - 1)];
}

// One step of a column sweep: w_j = r_j / F[j][j] (stored to out[j]), then
// r_i -= F[i][j] w_j for the rows i the step updates (forward: j < i < T,
// backward: i < j); the other rows subtract an exact zero.
template <int E, bool FWD>
__device__ __forceinline__ void trsv_step(const TrsvCol<E>& c, int j, int T, int lane, double2* r, double2* out) {
  const double inv = 1.0 / trsv_diag(c, j);
  const double2 rj = r[j];
  const double2 wj = make_double2(rj.x * inv, rj.y * inv);
  out[j] = wj;
#pragma unroll
  for (int q = 0; q < E; ++q) {
    const int i = lane + 64 * q;
    const bool active = FWD ? (i > j && i < T) : (i < j);
    const double2 v = active ? c.v[q] : make_double2(0.0, 0.0);
    r[i] = csub(r[i], cmul(v, wj));
  }
  __syncthreads();
}

// One wavefront per template; lane l owns rows l + 64 q (q < E, T <= 64 E).
// The factor is read B = 32 / E columns at a time (one batch of independent
// loads, one wait), then B steps run from registers: each workgroup meets the
// latency of a column read once per B steps (the waves of a launch read the
// same column in lockstep, so each read waits on the L2 fill).  Every step is
// branch-free (rows outside the update subtract an exact zero; x and y hold
// 64 E entries) and takes the diagonal from registers.
template <int E>
__global__ __launch_bounds__(64) void k_trsv(const double2* __restrict__ L, const double2* __restrict__ U, int T,
                                           const double2* __restrict__ b, int64_t bstride,
                                           double2* __restrict__ a, int64_t astride) {
  constexpr int B = 32 / E;
  extern __shared__ double2 sh[];
  double2* x = sh;               // [64 E]
  double2* y = sh + 64 * E;      // [64 E]
  const int lane = threadIdx.x;
  const double2* bb = b + (int64_t)blockIdx.x * bstride;
#pragma unroll
  for (int q = 0; q < E; ++q) {
    const int i = lane + 64 * q;
    x[i] = i < T ? bb[i] : make_double2(0.0, 0.0);
    y[i] = make_double2(0.0, 0.0);
  }
  __syncthreads();
  // forward: L y = b
  for (int j0 = 0; j0 < T; j0 += B) {
    TrsvCol<E> c[B];
#pragma unroll
    for (int k = 0; k < B; ++k) trsv_load<E>(L, T, lane, c[k], j0 + k);
#pragma unroll
    for (int k = 0; k < B; ++k)
      if (j0 + k < T) trsv_step<E, true>(c[k], j0 + k, T, lane, x, y);
  }
  // backward: U a = y
  for (int j0 = T - 1; j0 >= 0; j0 -= B) {
    TrsvCol<E> c[B];
#pragma unroll
    for (int k = 0; k < B; ++k) trsv_load<E>(U, T, lane, c[k], j0 - k);
#pragma unroll
    for (int k = 0; k < B; ++k)
      if (j0 - k >= 0) trsv_step<E, false>(c[k], j0 - k, T, lane, y, x);
  }
  double2* ao = a + (int64_t)blockIdx.x * astride;
  for (int i = lane; i < T; i += 64) ao[i] = x[i];
}

__device__ __forceinline__ double lane_bcast(double v, int src) {
  const long long bits = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)bits, src);
  const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), src);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Row j of a register-distributed vector (row i = lane + 64 q in slot q of
// lane i % 64), on every lane: a masked sum over the slots (one nonzero
// term, exact) and a cross-lane read.
template <int E>
__device__ __forceinline__ double row_pick(const double (&v)[E], int j) {
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < E; ++q) s += (q == (j >> 6)) ? v[q] : 0.0;
  return lane_bcast(s, j & 63);
}

// The same sweeps for T <= 64 E, E <= 8, with x, y and the inverse diagonal
// 1 / L[i][i] (= 1 / U[i][i], real) in registers: a step is a cross-lane
// read of row j and E independent updates, with no LDS and no barrier.  The
// factor columns come in batches of B = 32 / E as in k_trsv.
template <int E>
__device__ __forceinline__ void trsv_reg_step(const TrsvCol<E>& c, int j, int T, int lane, bool fwd,
                                              const double (&dinv)[E], double (&rr)[E], double (&ri)[E],
                                              double (&outr)[E], double (&outi)[E]) {
  const double inv = row_pick<E>(dinv, j);
  const double wr = row_pick<E>(rr, j) * inv, wi = row_pick<E>(ri, j) * inv;
#pragma unroll
  for (int q = 0; q < E; ++q) {
    const int i = lane + 64 * q;
    if (i == j) {
      outr[q] = wr;
      outi[q] = wi;
    }
    const bool active = fwd ? (i > j && i < T) : (i < j);
    const double2 v = active ? c.v[q] : make_double2(0.0, 0.0);
    const double2 d = csub(make_double2(rr[q], ri[q]), cmul(v, make_double2(wr, wi)));
    rr[q] = d.x;
    ri[q] = d.y;
  }
}

template <int E>
__global__ __launch_bounds__(64) void k_trsv_reg(const double2* __restrict__ L, const double2* __restrict__ U,
                                               int T, const double2* __restrict__ b, int64_t bstride,
                                               double2* __restrict__ a, int64_t astride) {
  constexpr int B = 32 / E;
  const int lane = threadIdx.x;
  const double2* bb = b + (int64_t)blockIdx.x * bstride;
  double xr[E], xi[E], yr[E], yi[E], dinv[E];
#pragma unroll
  for (int q = 0; q < E; ++q) {
    const int i = lane + 64 * q;
    const double2 v = i < T ? bb[i] : make_double2(0.0, 0.0);
    xr[q] = v.x;
    xi[q] = v.y;
    yr[q] = yi[q] = 0.0;
    dinv[q] = i < T ? 1.0 / L[(int64_t)i * T + i].x : 1.0;
  }
  // forward: y_j = x_j / L[j][j]; x_i -= L[i][j] y_j for j < i < T
  for (int j0 = 0; j0 < T; j0 += B) {
    TrsvCol<E> c[B];
#pragma unroll
    for (int k = 0; k < B; ++k) trsv_load<E>(L, T, lane, c[k], j0 + k);
#pragma unroll
    for (int k = 0; k < B; ++k)
      if (j0 + k < T) trsv_reg_step<E>(c[k], j0 + k, T, lane, true, dinv, xr, xi, yr, yi);
  }
  // backward: a_j = y_j / U[j][j] (into x); y_i -= U[i][j] a_j for i < j
  for (int j0 = T - 1; j0 >= 0; j0 -= B) {
    TrsvCol<E> c[B];
#pragma unroll
    for (int k = 0; k < B; ++k) trsv_load<E>(U, T, lane, c[k], j0 - k);
#pragma unroll
    for (int k = 0; k < B; ++k)
      if (j0 - k >= 0) trsv_reg_step<E>(c[k], j0 - k, T, lane, false, dinv, yr, yi, xr, xi);
  }
  double2* ao = a + (int64_t)blockIdx.x * astride;
#pragma unroll
  for (int q = 0; q < E; ++q) {
    const int i = lane + 64 * q;
    if (i < T) ao[i] = make_double2(xr[q], xi[q]);
  }
}

// Windowed variant: a = tukey(0.25) * (truncated inverse transform of R).
__device__ double tukey(int l, int T) {
  const double alpha = 0.25;
  if (T == 1) return 1.0;
  const double x = (double)l / (double)(T - 1);
  const double pi = 3.141592653589793238462643;
  if (x < alpha / 2) return 0.5 * (1.0 + cos(pi * (2.0 * x / alpha - 1.0)));
  if (x > 1.0 - alpha / 2) return 0.5 * (1.0 + cos(pi * (2.0 * x / alpha - 2.0 / alpha + 1.0)));
  return 1.0;
}

__global__ void k_window(const double2* __restrict__ b, int64_t bstride, int T, int64_t count,
                         double2* __restrict__ a, int64_t astride) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count * T;
       e += (int64_t)gridDim.x * blockDim.x) {
    int64_t t = e / T;
    int l = (int)(e % T);
    double2 v = b[t * bstride + l];
    double wv = tukey(l, T);
    a[t * astride + l] = make_double2(v.x * wv, v.y * wv);
  }
}

// sigma_fit^2 = a^H M a with M[l,k] = g[l-k]; one workgroup per template.
__global__ __launch_bounds__(256) void k_sigma_fit(const double2* __restrict__ a, int64_t astride, int T,
                                                 const double2* __restrict__ g, double* __restrict__ sigma) {
  extern __shared__ double2 sh[];
  double2* av = sh;
  double2* gv = sh + T;
  __shared__ double red[256];
  const double2* ab = a + (int64_t)blockIdx.x * astride;
  for (int i = threadIdx.x; i < T; i += 256) {
    av[i] = ab[i];
    gv[i] = g[i];
  }
  __syncthreads();
  double acc = 0.0;
  for (int l = threadIdx.x; l < T; l += 256) {
    double2 s = make_double2(0.0, 0.0);
    for (int k = 0; k < T; ++k) s = cadd(s, cmul(gval(gv, l - k), av[k]));
    acc += av[l].x * s.x + av[l].y * s.y;   // Re(conj(a_l) s)
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) sigma[blockIdx.x] = sqrt(red[0]);
}

// Normalised taps c = conj(a) sigma_ref / sigma_fit, and their MFMA A-operand
// packings.  Row 2t holds (Re c, -Im c) per tap, row 2t+1 holds (Im c, Re c).
//  16-bit: element e = 2 (k%4) + comp of lane (row + 16 ((k%16)/4)) in K block k/16,
//          uint4 index ((tb*KB + kb)*2 + plane)*64 + lane.
//  FP32:   K step kb2 = k/2, lane row + 16 (2 (k%2) + comp), float4 (tb*(Tp/8) + kq)*64 + lane
//          with kq = kb2/4, component kb2 % 4.
// A workgroup takes a tile of 8 templates (tb) x 16 taps (kb): the 128
// normalised taps are staged in LDS, then each wave writes one packing of the
// tile as 64 consecutive 16-byte lanes: wave 0 the BF16 hi and lo planes,
// wave 1 the FP16 planes, waves 2 and 3 the two FP32 K quads.  Lanes of
// templates outside [t_first, t_first + count) store nothing.
__device__ __forceinline__ double pack_val(double2 c, int o, int comp) {
  return o == 0 ? (comp == 0 ? c.x : -c.y) : (comp == 0 ? c.y : c.x);
}

__global__ __launch_bounds__(256) void k_pack(const double2* __restrict__ a, int64_t astride,
                                            const double* __restrict__ sigma_fit, const double2* __restrict__ g,
                                            int T, int Tp, int64_t t_first, int64_t count, float2* __restrict__ c32,
                                            uint4* __restrict__ pbf, uint4* __restrict__ pfh,
                                            float4* __restrict__ p32) {
  __shared__ double2 cs[8][16];
  const double sig_ref = sqrt(g[0].x);
  const int KB = Tp / 16;
  const int64_t tb0 = t_first / 8, tb1 = (t_first + count - 1) / 8;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int64_t tb = tb0 + blockIdx.y; tb <= tb1; tb += gridDim.y) {
    for (int kb = blockIdx.x; kb < KB; kb += gridDim.x) {
      if (threadIdx.x < 128) {
        const int trow = threadIdx.x >> 4, kk = threadIdx.x & 15;
        const int k = kb * 16 + kk;
        const int64_t t = tb * 8 + trow;
        const int64_t tl = t - t_first;
        double2 c = make_double2(0.0, 0.0);
        if (tl >= 0 && tl < count) {
          if (k < T) {
            const double2 av = a[tl * astride + k];
            const double sc = sig_ref / sigma_fit[tl];
            c = make_double2(av.x * sc, -av.y * sc);
          }
          c32[t * Tp + k] = make_float2((float)c.x, (float)c.y);
        }
        cs[trow][kk] = c;
      }
      __syncthreads();
      if (w < 2) {
        // 16-bit planes: lane = row + 16 gq, taps 4 gq .. 4 gq + 3 of the tile
        const int row = lane & 15, gq = lane >> 4, trow = row >> 1, o = row & 1;
        const int64_t tl = tb * 8 + trow - t_first;
        if (tl >= 0 && tl < count) {
          uint32_t hw[4], lw[4];
#pragma unroll
          for (int jj = 0; jj < 4; ++jj) {
            const double2 c = cs[trow][gq * 4 + jj];
            uint32_t h0, l0, h1, l1;
            if (w == 0) {
              split_bf16(pack_val(c, o, 0), h0, l0);
              split_bf16(pack_val(c, o, 1), h1, l1);
            } else {
              split_f16(pack_val(c, o, 0), h0, l0);
              split_f16(pack_val(c, o, 1), h1, l1);
            }
            hw[jj] = (h0 & 0xffffu) | (h1 << 16);
            lw[jj] = (l0 & 0xffffu) | (l1 << 16);
          }
          uint4* dst = (w == 0 ? pbf : pfh) + ((tb * KB + kb) * 2) * 64 + lane;
          dst[0] = make_uint4(hw[0], hw[1], hw[2], hw[3]);
          dst[64] = make_uint4(lw[0], lw[1], lw[2], lw[3]);
        }
      } else {
        // FP32: lane = row + 16 (2 par + comp); component sub holds tap 8 q + 2 sub + par
        const int q = w - 2;
        const int row = lane & 15, par = lane >> 5, comp = (lane >> 4) & 1, trow = row >> 1, o = row & 1;
        const int64_t tl = tb * 8 + trow - t_first;
        if (tl >= 0 && tl < count) {
          float v[4];
#pragma unroll
          for (int sub = 0; sub < 4; ++sub) v[sub] = (float)pack_val(cs[trow][8 * q + 2 * sub + par], o, comp);
          p32[(tb * (Tp / 8) + 2 * kb + q) * 64 + lane] = make_float4(v[0], v[1], v[2], v[3]);
        }
      }
      __syncthreads();
    }
  }
}

// ------------------------------------------------------------ launchers
int taps_prepare_subbank(Plan& p, Taps& tp, int b, const double* h_ref, double eps) {
  SubBankTaps& s = tp.sb[b];
  const int T = s.T;
  int rc = launch_corr64(p, tp, 1, h_ref, nullptr, 1, T, 0, s.g, T);
  if (rc) return rc;
  if (eps >= 0.0) {
    if (T > RFD_MAX_TAPS) return fail(RFD_E_INVALID, "taps out of range");
    int64_t el = (int64_t)T * T;
    int blocks = (int)((el + 255) / 256 < 4096 ? (el + 255) / 256 : 4096);
    int* info = reinterpret_cast<int*>(p.dscratch + 8);
    RFD_HIP(hipMemsetAsync(info, 0, sizeof(int), p.stream));
    hipLaunchKernelGGL(k_schur_chol, dim3(1), dim3(1024), 0, p.stream, s.g, T, eps, s.L, info);
    RFD_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_upper, dim3(blocks), dim3(256), 0, p.stream, s.L, T, s.U);
    RFD_CHECK_LAUNCH();
    int hinfo = 0;
    RFD_HIP(hipMemcpyAsync(&hinfo, info, sizeof(int), hipMemcpyDeviceToHost, p.stream));
    RFD_HIP(hipStreamSynchronize(p.stream));
    if (hinfo != 0) return fail(RFD_E_INVALID, "ridge-regularised Gram matrix is not positive definite");
    s.eps = eps;
  }
  return RFD_OK;
}

int taps_norm_and_pack(Plan& p, Taps& tp, int b, int64_t first, int64_t count);
int taps_pack(Plan& p, Taps& tp, int b, int64_t first, int64_t count);

int taps_solve_and_pack(Plan& p, Taps& tp, int b, int64_t first, int64_t count, int method) {
  SubBankTaps& s = tp.sb[b];
  const int T = s.T;
  double2* abase = tp.a64 + s.a_base + first * s.Tp;
  if (method == RFD_TAPS_LS) {
    const dim3 grid((unsigned)count);
#define RFD_TRSV(E)                                                                                              \
  hipLaunchKernelGGL(k_trsv<E>, grid, dim3(64), (size_t)2 * 64 * (E) * sizeof(double2), p.stream, s.L, s.U, T,   \
                     tp.bvec, (int64_t)T, abase, (int64_t)s.Tp)
    if (T <= 256)
      hipLaunchKernelGGL(k_trsv_reg<4>, grid, dim3(64), 0, p.stream, s.L, s.U, T, tp.bvec, (int64_t)T, abase,
                         (int64_t)s.Tp);
    else if (T <= 512)
      hipLaunchKernelGGL(k_trsv_reg<8>, grid, dim3(64), 0, p.stream, s.L, s.U, T, tp.bvec, (int64_t)T, abase,
                         (int64_t)s.Tp);
    else if (T <= 1024) RFD_TRSV(16);
    else RFD_TRSV(32);
#undef RFD_TRSV
  } else {
    int64_t el = count * T;
    int blocks = (int)((el + 255) / 256 < 4096 ? (el + 255) / 256 : 4096);
    hipLaunchKernelGGL(k_window, dim3(blocks), dim3(256), 0, p.stream, tp.bvec, (int64_t)T, T, count, abase,
                       (int64_t)s.Tp);
  }
  RFD_CHECK_LAUNCH();
  return taps_norm_and_pack(p, tp, b, first, count);
}

// sigma_fit of taps already in a64, then the normalised taps and MFMA packings.
int taps_norm_and_pack(Plan& p, Taps& tp, int b, int64_t first, int64_t count) {
  SubBankTaps& s = tp.sb[b];
  const int T = s.T;
  double2* abase = tp.a64 + s.a_base + first * s.Tp;
  double* sig = tp.sigma_fit + s.first + first;
  hipLaunchKernelGGL(k_sigma_fit, dim3((unsigned)count), dim3(256), (size_t)2 * T * sizeof(double2), p.stream,
                     abase, (int64_t)s.Tp, T, s.g, sig);
  RFD_CHECK_LAUNCH();
  return taps_pack(p, tp, b, first, count);
}

// normalised taps and MFMA packings from a64 and sigma_fit already in place
int taps_pack(Plan& p, Taps& tp, int b, int64_t first, int64_t count) {
  SubBankTaps& s = tp.sb[b];
  s.ols_valid = false;   // the overlap-save tap spectra follow the packed taps
  if (count <= 0) return RFD_OK;
  const int T = s.T;
  double2* abase = tp.a64 + s.a_base + first * s.Tp;
  double* sig = tp.sigma_fit + s.first + first;
  const int64_t ntb = (first + count - 1) / 8 - first / 8 + 1;
  const int KB = s.Tp / 16;
  dim3 grid((unsigned)std::min(KB, 8), (unsigned)std::min<int64_t>(ntb, 8192));
  hipLaunchKernelGGL(k_pack, grid, dim3(256), 0, p.stream, abase, (int64_t)s.Tp, sig, s.g, T, s.Tp, first, count,
                     tp.c32 + s.a_base, tp.pbf + s.p16_base, tp.pfh + s.p16_base, tp.p32 + s.p32_base);
  RFD_CHECK_LAUNCH();
  return RFD_OK;
}

}  // namespace rfd
