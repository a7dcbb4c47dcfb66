// Learned tap surrogate (an extension; the paper mentions ML only as a
// downstream layer): a small MLP maps template parameters to coefficients on
// an orthonormal basis of whitened ratio taps, so dense banks get taps
// without waveforms.  Everything below runs on the device:
//   alignment   a <- a e^{-i arg z}, z = ((M + lam I) a)[-k0]: the zero-lag
//               overlap of fitted template and reference made real positive
//               (|z| of the filter and every match ignore a global phase),
//   whitening   x = [Re v; Im v]/||v||, v = L^H a  (M + lam I = L L^H, so
//               ||x_hat - x||^2 is the fitted-template mismatch proxy),
//   basis       subspace iteration Q <- orth(X^T X Q) with two-pass
//               Gram-Schmidt, K orthonormal directions (B, stored K x D),
//   targets     c = X B^T... (coefficients of each training tap set),
//   MLP         4 -> H -> H -> K, SiLU; BF16 weights, FP32 accumulation,
//               hand-written forward / backward / Adam kernels,
//   inference   params -> c_hat -> x_hat = c_hat B -> a = L^-H v -> the
//               usual sigma_fit normalisation and MFMA operand packing.
// The exact taps (Sec. V.A) stay the training data, the fallback and the
// yardstick: rfd_taps_match gives the fitted templates' normalised overlap.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <random>
#include <string>
#include <vector>

#include "dev_common.h"
#include "rfd_internal.h"

namespace rfd {

int taps_norm_and_pack(Plan& p, Taps& tp, int b, int64_t first, int64_t count);
int taps_pack(Plan& p, Taps& tp, int b, int64_t first, int64_t count);

// ------------------------------------------------------------------ GEMM
// Element r of this thread in a 32 x TM (k x m) tile: consecutive threads
// run along whichever index is contiguous in memory (m for a k-major
// operand, k for an m-major one), so every load is a coalesced run.
template <int TM>
__device__ __forceinline__ void tile_pos(int r, bool k_major, int& kk, int& mm) {
  const int e = threadIdx.x + r * 256;
  if (k_major) {
    kk = e / TM;
    mm = e % TM;
  } else {
    mm = e >> 5;
    kk = e & 31;
  }
}

__device__ __forceinline__ float silu_f(float z) { return z / (1.f + __expf(-z)); }
__device__ __forceinline__ float silu_g(float z) {
  const float s = 1.f / (1.f + __expf(-z));
  return s * (1.f + z * (1.f - s));
}

// Networks trained together: every training kernel takes its per-network
// pointers from arrays indexed by the grid's network coordinate.  They are
// kernel arguments, so one captured epoch holds them, and each network's
// arithmetic is exactly that of training it alone.
constexpr int kMaxNets = 32;
template <typename T>
struct PerNet {
  T p[kMaxNets];
};
template <typename T>
static PerNet<T> one_net(T v) {
  PerNet<T> r{};
  r.p[0] = v;
  return r;
}

// What the GEMM does with each result x = op(A) op(B) [m][n]:
//   kStore   C = x (or C += x when accumulate)
//   kBiasAct z = x + bias[n]; C = z; H = silu(z)   (hidden layer, forward)
//   kBias    C = x + bias[n]                      (output layer, forward)
//   kSiluBwd C = x silu'(Z[m][n])                  (hidden layer, backward)
enum GemmEpiMode { kStore = 0, kBiasAct, kBias, kSiluBwd };
template <typename TA, typename TB>
struct GemmOps {
  PerNet<const TA*> A;
  PerNet<const TB*> B;
  PerNet<float*> C;
  PerNet<const float*> bias;   // kBiasAct, kBias
  PerNet<float*> H;            // kBiasAct
  PerNet<const float*> Z;      // kSiluBwd
};

// C[M x N] = op(A) op(B) (+ C when accumulate) for the network blockIdx.z of
// ops, op(A)[m][k] = ta ? A[k*lda + m] : A[m*lda + k],
// op(B)[k][n] = tb ? B[n*ldb + k] : B[k*ldb + n], on the matrix cores
// (v_mfma_f32_16x16x32_bf16, FP32 accumulation).  An FP32 operand enters as three BF16 parts x = x0 + x1 + x2,
// each the BF16 rounding of what the previous parts leave (so
// |x - x0 - x1 - x2| <= 2^-27 |x|); a BF16 operand (the weights) is its own
// single part.  Every part product x_i y_j with i + j <= 2 is accumulated (the
// ones left out are below 2^-27 relative), so the result keeps FP32 accuracy:
// three MFMAs per 16x16x32 block against BF16 weights, six when both operands
// are FP32.  TM x TM output tile per workgroup (TM = 64, or 32 where 64-wide
// tiles would leave most CUs idle), each of the four waves a TM/2 x TM/2
// quadrant of 16 x 16 MFMA blocks, K in steps of 32 with the next step's
// tiles loaded into registers while the current one is multiplied.  Every
// output takes the same K steps and part products in the same order at
// either width, so the results do not depend on it.
template <typename T>
struct Bf16Parts {
  static constexpr int n = 3;
};
template <>
struct Bf16Parts<uint16_t> {
  static constexpr int n = 1;
};
typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;
constexpr int kMfmaLdsRow = 40;   // 32 K values + 8 of padding (80 B rows: 16 B aligned)

template <int P>
__device__ __forceinline__ void to_parts(float x, uint16_t (&q)[3]) {
  const uint32_t p0 = bf16_bits(x);
  q[0] = (uint16_t)p0;
  if constexpr (P > 1) {
    const float r1 = x - bf16_to_float(p0);
    const uint32_t p1 = bf16_bits(r1);
    const float r2 = r1 - bf16_to_float(p1);
    q[1] = (uint16_t)p1;
    q[2] = (uint16_t)bf16_bits(r2);
  }
}
__device__ __forceinline__ float ld_f(const float* p, int64_t i) { return p[i]; }
__device__ __forceinline__ float ld_f(const uint16_t* p, int64_t i) { return bf16_to_float(p[i]); }

template <int TM, typename TA, typename TB>
__global__ __launch_bounds__(256) void k_gemm_mfma(int M, int N, int K, int lda, int ta, int ldb, int tb, int ldc,
                                                 int accumulate, int mode, GemmOps<TA, TB> ops) {
  constexpr int PA = Bf16Parts<TA>::n, PB = Bf16Parts<TB>::n;
  constexpr int R = TM * 32 / 256;       // tile elements per thread and operand
  constexpr int BW = TM / 32;            // 16 x 16 blocks per wave along each dimension
  __shared__ __align__(16) uint16_t As[PA][TM][kMfmaLdsRow];
  __shared__ __align__(16) uint16_t Bs[PB][TM][kMfmaLdsRow];
  const int z = blockIdx.z;
  const TA* __restrict__ A = ops.A.p[z];
  const TB* __restrict__ B = ops.B.p[z];
  float* __restrict__ C = ops.C.p[z];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = w >> 1, wn = w & 1;
  const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TM;
  f32x4 acc[BW][BW];
#pragma unroll
  for (int i = 0; i < BW; ++i)
#pragma unroll
    for (int j = 0; j < BW; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  float ra[R], rb[R];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      int kk, mm;
      tile_pos<TM>(r, ta != 0, kk, mm);
      int gm = m0 + mm, gk = k0 + kk;
      ra[r] = (gm < M && gk < K) ? (ta ? ld_f(A, (int64_t)gk * lda + gm) : ld_f(A, (int64_t)gm * lda + gk)) : 0.f;
      tile_pos<TM>(r, tb == 0, kk, mm);
      const int gn = n0 + mm;
      gk = k0 + kk;
      rb[r] = (gn < N && gk < K) ? (tb ? ld_f(B, (int64_t)gn * ldb + gk) : ld_f(B, (int64_t)gk * ldb + gn)) : 0.f;
    }
  };
  fetch(0);
  const int r16 = lane & 15, kq = (lane >> 4) * 8;
  for (int k0 = 0; k0 < K; k0 += 32) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      int kk, mm;
      uint16_t q[3];
      tile_pos<TM>(r, ta != 0, kk, mm);
      to_parts<PA>(ra[r], q);
#pragma unroll
      for (int p = 0; p < PA; ++p) As[p][mm][kk] = q[p];
      tile_pos<TM>(r, tb == 0, kk, mm);
      to_parts<PB>(rb[r], q);
#pragma unroll
      for (int p = 0; p < PB; ++p) Bs[p][mm][kk] = q[p];
    }
    __syncthreads();
    if (k0 + 32 < K) fetch(k0 + 32);
    uint4 a[BW][PA], b[BW][PB];
#pragma unroll
    for (int i = 0; i < BW; ++i) {
#pragma unroll
      for (int p = 0; p < PA; ++p)
        a[i][p] = *reinterpret_cast<const uint4*>(&As[p][wm * (TM / 2) + i * 16 + r16][kq]);
#pragma unroll
      for (int p = 0; p < PB; ++p)
        b[i][p] = *reinterpret_cast<const uint4*>(&Bs[p][wn * (TM / 2) + i * 16 + r16][kq]);
    }
#pragma unroll
    for (int i = 0; i < BW; ++i)
#pragma unroll
      for (int j = 0; j < BW; ++j)
#pragma unroll
        for (int p = 0; p < PA; ++p)
#pragma unroll
          for (int q = 0; q < PB; ++q)
            if (p + q <= 2)
              acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a[i][p]),
                                                                 __builtin_bit_cast(bf16x8, b[j][q]), acc[i][j], 0, 0, 0);
    __syncthreads();
  }
  // lane l holds rows 4 (l >> 4) + e, column l & 15 of each 16 x 16 block
#pragma unroll
  for (int i = 0; i < BW; ++i)
#pragma unroll
    for (int j = 0; j < BW; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int gm = m0 + wm * (TM / 2) + i * 16 + 4 * (lane >> 4) + e;
        const int gn = n0 + wn * (TM / 2) + j * 16 + r16;
        if (gm >= M || gn >= N) continue;
        const int64_t o = (int64_t)gm * ldc + gn;
        float v = acc[i][j][e];
        if (mode == kBiasAct) {
          v += ops.bias.p[z][gn];
          ops.H.p[z][o] = silu_f(v);
        } else if (mode == kBias) {
          v += ops.bias.p[z][gn];
        } else if (mode == kSiluBwd) {
          v *= silu_g(ops.Z.p[z][o]);
        } else if (accumulate) {
          v += C[o];
        }
        C[o] = v;
      }
}

// the same GEMM shape for nz networks at once
template <typename TA, typename TB>
static int gemm_n(hipStream_t st, int nz, int M, int N, int K, const GemmOps<TA, TB>& ops, int lda, int ta, int ldb,
                  int tb, int ldc, int accumulate = 0, int mode = kStore) {
  if (M <= 0 || N <= 0 || nz <= 0) return RFD_OK;
  // 32-wide tiles when 64-wide ones would leave most of the 256 CUs idle
  if ((int64_t)((N + 63) / 64) * ((M + 63) / 64) * nz < 512) {
    dim3 grid((N + 31) / 32, (M + 31) / 32, nz);
    hipLaunchKernelGGL((k_gemm_mfma<32, TA, TB>), grid, dim3(256), 0, st, M, N, K, lda, ta, ldb, tb, ldc,
                       accumulate, mode, ops);
  } else {
    dim3 grid((N + 63) / 64, (M + 63) / 64, nz);
    hipLaunchKernelGGL((k_gemm_mfma<64, TA, TB>), grid, dim3(256), 0, st, M, N, K, lda, ta, ldb, tb, ldc,
                       accumulate, mode, ops);
  }
  RFD_CHECK_LAUNCH();
  return RFD_OK;
}

// one network, plain result
template <typename TA, typename TB>
static int gemm(hipStream_t st, int M, int N, int K, const TA* A, int lda, int ta, const TB* B, int ldb, int tb,
                float* C, int ldc, int accumulate = 0) {
  GemmOps<TA, TB> ops{};
  ops.A.p[0] = A;
  ops.B.p[0] = B;
  ops.C.p[0] = C;
  return gemm_n(st, 1, M, N, K, ops, lda, ta, ldb, tb, ldc, accumulate, kStore);
}

// ------------------------------------------------------- elementwise
// Each kernel below serves the networks of a PerNet group: the network is
// blockIdx.y (grid-stride kernels) or blockIdx.x (one-thread kernels).

// dY = 2 (Y - C) / nb, and the per-block sums of squares (deterministic order)
__global__ __launch_bounds__(256) void k_loss(PerNet<const float*> Ys, PerNet<const float*> Cbs,
                                            PerNet<float*> dYs, int64_t n, float scale, PerNet<double*> parts) {
  const int z = blockIdx.y;
  const float* __restrict__ Y = Ys.p[z];
  const float* __restrict__ Cb = Cbs.p[z];
  float* __restrict__ dY = dYs.p[z];
  __shared__ double red[256];
  double acc = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
    const float r = Y[e] - Cb[e];
    dY[e] = 2.f * r * scale;
    acc += (double)r * r;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) parts.p[z][blockIdx.x] = red[0];
}

// accumulate: the flag, or when acc_from is given, whether acc_from[0] > 0
// (a training step after the epoch's first)
__global__ void k_sum_partials(PerNet<const double*> parts, int n, double scale, PerNet<double*> outs,
                               int accumulate, PerNet<const int64_t*> acc_from) {
  if (threadIdx.x != 0) return;
  const int z = blockIdx.x;
  const double* __restrict__ partial = parts.p[z];
  if (acc_from.p[z]) accumulate = acc_from.p[z][0] > 0;
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += partial[i];
  s *= scale;
  double* out = outs.p[z];
  *out = accumulate ? *out + s : s;
}

// out[j] = sum_i X[i][j]: 64 columns per workgroup, 16 row groups (rows
// g, g + 16, ...) added in LDS in a fixed order.
__global__ __launch_bounds__(1024) void k_colsum(PerNet<const float*> Xs, int64_t n, int H, PerNet<float*> outs) {
  __shared__ float red[16][64];
  const float* __restrict__ X = Xs.p[blockIdx.y];
  const int c = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int j = blockIdx.x * 64 + c;
  float s = 0.f;
  if (j < H)
    for (int64_t i = g; i < n; i += 16) s += X[i * H + j];
  red[g][c] = s;
  __syncthreads();
  if (g == 0 && j < H) {
    float t = 0.f;
#pragma unroll
    for (int q = 0; q < 16; ++q) t += red[q][c];
    outs.p[blockIdx.y][j] = t;
  }
}

// Training step state on the device, so every step of an epoch is the same
// launch sequence (and can be replayed as one captured graph):
// st[0] = batch index within the epoch, st[1] = Adam steps taken.
__global__ void k_train_state_set(PerNet<int64_t*> sts, int64_t bi, PerNet<int64_t> steps) {
  if (threadIdx.x == 0) {
    int64_t* st = sts.p[blockIdx.x];
    st[0] = bi;
    st[1] = steps.p[blockIdx.x];
  }
}
__global__ void k_train_state_advance(PerNet<int64_t*> sts) {
  if (threadIdx.x == 0) {
    int64_t* st = sts.p[blockIdx.x];
    st[0] += 1;
    st[1] += 1;
  }
}
// the mean loss of the epoch just ended, rec[z * epochs + e]
__global__ void k_loss_record(PerNet<const double*> loss, float* __restrict__ rec, int epochs, int e) {
  if (threadIdx.x == 0) rec[(int64_t)blockIdx.x * epochs + e] = (float)loss.p[blockIdx.x][0];
}

// Adam step number st[1] + 1 (bias corrections 1 - beta^t), and the BF16
// copy of each updated weight that the next step's GEMMs read
__global__ void k_adam_step(PerNet<float*> ws, PerNet<const float*> gs, PerNet<float*> ms, PerNet<float*> vs,
                            PerNet<uint16_t*> wbfs, int64_t n, float lr, float b1, float b2, float eps,
                            PerNet<const int64_t*> sts) {
  const int z = blockIdx.y;
  float* __restrict__ w = ws.p[z];
  uint16_t* __restrict__ wbf = wbfs.p[z];
  const float* __restrict__ g = gs.p[z];
  float* __restrict__ m = ms.p[z];
  float* __restrict__ v = vs.p[z];
  const float t = (float)(sts.p[z][1] + 1);
  const float bc1 = 1.f - powf(b1, t), bc2 = 1.f - powf(b2, t);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wn = w[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
    w[i] = wn;
    wbf[i] = (uint16_t)bf16_bits(wn);
  }
}

__global__ void k_to_bf16(PerNet<const float*> ws, PerNet<uint16_t*> outs, int64_t n) {
  const float* __restrict__ w = ws.p[blockIdx.y];
  uint16_t* __restrict__ out = outs.p[blockIdx.y];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (uint16_t)bf16_bits(w[i]);
}

// rows perm[st[0] nb + r], r < nb, of the parameters and targets
__global__ void k_gather(PerNet<const float*> Ps, PerNet<const float*> Cs, PerNet<const int32_t*> perms,
                         PerNet<const int64_t*> sts, int nb, int K, PerNet<float*> Pbs, PerNet<float*> Cbs) {
  const int z = blockIdx.y;
  const float* __restrict__ P = Ps.p[z];
  const float* __restrict__ C = Cs.p[z];
  float* __restrict__ Pb = Pbs.p[z];
  float* __restrict__ Cb = Cbs.p[z];
  const int32_t* idx = perms.p[z] + sts.p[z][0] * nb;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nb * (4 + K); e += gridDim.x * blockDim.x) {
    const int r = e / (4 + K), c = e % (4 + K);
    const int64_t src = idx[r];
    if (c < 4) Pb[r * 4 + c] = P[src * 4 + c];
    else Cb[(int64_t)r * K + (c - 4)] = C[src * K + (c - 4)];
  }
}

// splitmix64 (Steele, Lea, Flood 2014) of (seed, index) -> uniform in (-1, 1)
__device__ __forceinline__ float hash_uniform(uint64_t seed, uint64_t i) {
  uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return (float)((double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0);
}

__global__ void k_random(float* __restrict__ Q, int64_t n, uint64_t seed) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    Q[i] = hash_uniform(seed, (uint64_t)i);
}

// ------------------------------------------------------ whitening & basis
// Phase alignment, then whitening, one workgroup per tap set:
//   z   = ((M + lam I) a)[i0] = sum_k g[i0 - k] a_k + lam a_i0,  i0 = -k0
//         (the zero-lag tap; clamped into [0, T) when the window misses lag
//         0), lam = eps g[0]; g at negative lags is conj(g) at positive ones,
//   v   = U a e^{-i arg z}, U = L^H (column-major upper),
//   x   = [Re v; Im v] / ||v||.
__global__ __launch_bounds__(256) void k_whiten(const double2* __restrict__ a, int Tp,
                                              const double2* __restrict__ U, const double2* __restrict__ g,
                                              double eps, int i0, int T, float* __restrict__ X) {
  const double lam = eps * g[0].x;
  extern __shared__ double2 sa[];
  __shared__ double red[2][256];
  const double2* aj = a + (int64_t)blockIdx.x * Tp;
  for (int i = threadIdx.x; i < T; i += 256) sa[i] = aj[i];
  __syncthreads();
  double zr = 0.0, zi = 0.0;
  for (int k = threadIdx.x; k < T; k += 256) {
    const int d = i0 - k;
    double2 gk = d >= 0 ? g[d] : cconj(g[-d]);
    if (d == 0) gk.x += lam;
    const double2 t = cmul(gk, sa[k]);
    zr += t.x;
    zi += t.y;
  }
  red[0][threadIdx.x] = zr;
  red[1][threadIdx.x] = zi;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      red[0][threadIdx.x] += red[0][threadIdx.x + o];
      red[1][threadIdx.x] += red[1][threadIdx.x + o];
    }
    __syncthreads();
  }
  const double zabs = sqrt(red[0][0] * red[0][0] + red[1][0] * red[1][0]);
  const double2 rot = zabs > 0.0 ? make_double2(red[0][0] / zabs, -red[1][0] / zabs) : make_double2(1.0, 0.0);
  __syncthreads();
  float* xj = X + (int64_t)blockIdx.x * 2 * T;
  double nrm = 0.0;
  for (int i = threadIdx.x; i < T; i += 256) {
    double2 s = make_double2(0.0, 0.0);
    for (int k = i; k < T; ++k) s = cadd(s, cmul(U[(int64_t)k * T + i], sa[k]));
    s = cmul(s, rot);
    xj[i] = (float)s.x;
    xj[T + i] = (float)s.y;
    nrm += s.x * s.x + s.y * s.y;
  }
  red[0][threadIdx.x] = nrm;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[0][threadIdx.x] += red[0][threadIdx.x + o];
    __syncthreads();
  }
  const float inv = (float)(1.0 / sqrt(red[0][0]));
  for (int i = threadIdx.x; i < 2 * T; i += 256) xj[i] *= inv;
}

// Orthonormalise the K rows of Q (K x D) by two passes of Gram-Schmidt, one workgroup.
__global__ __launch_bounds__(1024) void k_orthonormalise(float* __restrict__ Q, int K, int D) {
  __shared__ double red[1024];
  for (int k = 0; k < K; ++k) {
    float* qk = Q + (int64_t)k * D;
    for (int pass = 0; pass < 2; ++pass) {
      for (int j = 0; j < k; ++j) {
        const float* qj = Q + (int64_t)j * D;
        double s = 0.0;
        for (int i = threadIdx.x; i < D; i += 1024) s += (double)qj[i] * qk[i];
        red[threadIdx.x] = s;
        __syncthreads();
        for (int o = 512; o > 0; o >>= 1) {
          if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
          __syncthreads();
        }
        const double r = red[0];
        __syncthreads();
        for (int i = threadIdx.x; i < D; i += 1024) qk[i] = (float)(qk[i] - r * qj[i]);
        __syncthreads();
      }
    }
    double s = 0.0;
    for (int i = threadIdx.x; i < D; i += 1024) s += (double)qk[i] * qk[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
      if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
      __syncthreads();
    }
    const double inv = red[0] > 0.0 ? 1.0 / sqrt(red[0]) : 0.0;
    __syncthreads();
    for (int i = threadIdx.x; i < D; i += 1024) qk[i] = (float)(qk[i] * inv);
    __syncthreads();
  }
}

// a_j = U^-1 v_j (back substitution, U = L^H upper), v_j = x_j[:T] + i x_j[T:].
__global__ __launch_bounds__(256) void k_unwhiten(const float* __restrict__ Xh, const double2* __restrict__ U, int T,
                                                double2* __restrict__ a, int Tp) {
  extern __shared__ double2 sh[];
  double2* y = sh;
  double2* x = sh + T;
  const float* xj = Xh + (int64_t)blockIdx.x * 2 * T;
  for (int i = threadIdx.x; i < T; i += 256) y[i] = make_double2((double)xj[i], (double)xj[T + i]);
  __syncthreads();
  for (int j = T - 1; j >= 0; --j) {
    const double2* col = U + (int64_t)j * T;
    const double inv = 1.0 / col[j].x;
    const double2 aj = make_double2(y[j].x * inv, y[j].y * inv);
    if (threadIdx.x == 0) x[j] = aj;
    for (int i = threadIdx.x; i < j; i += 256) y[i] = csub(y[i], cmul(col[i], aj));
    __syncthreads();
  }
  double2* ao = a + (int64_t)blockIdx.x * Tp;
  for (int i = threadIdx.x; i < T; i += 256) ao[i] = x[i];
}

// Coefficients -> FP64 taps and their fitted norm:
//   a_j = sum_k y_jk W_k      (W = L^-H B: row k is the back-substituted
//                              basis vector k),
//   v_j = sum_k y_jk B_k      (= L^H a_j, B_k = b_k[:T] + i b_k[T:]),
//   sigma_fit^2 = a^H M a = ||v||^2 - lam ||a||^2   (M + lam I = L L^H),
// an O(K T) form of the Sec. VI.B norm for taps given in whitened form.
// A workgroup takes kExpandRows templates and 256 taps (one per thread), so
// each tile of W and B is read from L2 once per kExpandRows templates; it
// writes its share of ||a||^2 and ||v||^2 per template, which k_expand_sigma
// adds in a fixed order (partials [template][tap block][2]).
constexpr int kExpandRows = 16;
__global__ __launch_bounds__(256) void k_expand(const float* __restrict__ Y, int n, int K,
                                              const double2* __restrict__ W, const float* __restrict__ Bt, int T,
                                              double2* __restrict__ a, int Tp, double* __restrict__ part) {
  extern __shared__ double2 yk_lds[];
  double* yk = reinterpret_cast<double*>(yk_lds);    // [kExpandRows][Kp], zero beyond K and n
  __shared__ double red[4][2 * kExpandRows];
  const int Kp = (K + 3) & ~3;
  const int j0 = blockIdx.x * kExpandRows;
  const int rows = min(kExpandRows, n - j0);
  for (int e = threadIdx.x; e < kExpandRows * Kp; e += 256) {
    const int r = e / Kp, k = e % Kp;
    yk[e] = (r < rows && k < K) ? (double)Y[(int64_t)(j0 + r) * K + k] : 0.0;
  }
  __syncthreads();
  const int t = blockIdx.y * 256 + threadIdx.x;
  const int tc = min(t, T - 1);                       // lanes past T compute a copy and store nothing
  double ar[kExpandRows], ai[kExpandRows], vr[kExpandRows], vi[kExpandRows];
#pragma unroll
  for (int r = 0; r < kExpandRows; ++r) ar[r] = ai[r] = vr[r] = vi[r] = 0.0;
  // Workgroups start the K sweep at staggered quads: those running together
  // then ask for different rows of W and B at first, and each later row is
  // already in L2 (or on its way) when the rest reach it, instead of every
  // wave of the grid waiting on the same miss at every step.
  const int nq = Kp / 4;
  const int q0 = (int)((blockIdx.x / 8) % (unsigned)nq);
  for (int qi = 0; qi < nq; ++qi) {
    const int k0 = 4 * (qi + q0 < nq ? qi + q0 : qi + q0 - nq);
    double wr[4], wi[4], br[4], bi[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int k = min(k0 + q, K - 1);                // y is zero for the clamped rows
      const double2 w = W[(int64_t)k * T + tc];
      wr[q] = w.x;
      wi[q] = w.y;
      br[q] = (double)Bt[(int64_t)k * 2 * T + tc];
      bi[q] = (double)Bt[(int64_t)k * 2 * T + T + tc];
    }
#pragma unroll
    for (int r = 0; r < kExpandRows; ++r) {
      const double2 y01 = *reinterpret_cast<const double2*>(yk + r * Kp + k0);
      const double2 y23 = *reinterpret_cast<const double2*>(yk + r * Kp + k0 + 2);
      const double y[4] = {y01.x, y01.y, y23.x, y23.y};
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        ar[r] = fma(y[q], wr[q], ar[r]);
        ai[r] = fma(y[q], wi[q], ai[r]);
        vr[r] = fma(y[q], br[q], vr[r]);
        vi[r] = fma(y[q], bi[q], vi[r]);
      }
    }
  }
  const bool live = t < T;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int r = 0; r < kExpandRows; ++r) {
    if (live && r < rows) a[(int64_t)(j0 + r) * Tp + t] = make_double2(ar[r], ai[r]);
    double aa = live ? ar[r] * ar[r] + ai[r] * ai[r] : 0.0;
    double vv = live ? vr[r] * vr[r] + vi[r] * vi[r] : 0.0;
    for (int o = 32; o > 0; o >>= 1) {
      aa += __shfl_xor(aa, o);
      vv += __shfl_xor(vv, o);
    }
    if (lane == 0) {
      red[wv][2 * r] = aa;
      red[wv][2 * r + 1] = vv;
    }
  }
  __syncthreads();
  if (threadIdx.x < 2 * rows) {
    const double v = (red[0][threadIdx.x] + red[1][threadIdx.x]) + (red[2][threadIdx.x] + red[3][threadIdx.x]);
    const int r = threadIdx.x >> 1;
    part[((int64_t)(j0 + r) * gridDim.y + blockIdx.y) * 2 + (threadIdx.x & 1)] = v;
  }
}

__global__ void k_expand_sigma(const double* __restrict__ part, int n, int nblk, double eps,
                               const double2* __restrict__ g, double* __restrict__ sigma) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double aa = 0.0, vv = 0.0;
  for (int b = 0; b < nblk; ++b) {
    aa += part[((int64_t)j * nblk + b) * 2];
    vv += part[((int64_t)j * nblk + b) * 2 + 1];
  }
  const double lam = eps * g[0].x;
  sigma[j] = sqrt(fmax(vv - lam * aa, 0.0));
}

// |a^H M b| / sqrt(a^H M a b^H M b), M[l,k] = g[l-k]; one workgroup per template.
__global__ __launch_bounds__(256) void k_match(const double2* __restrict__ A, const double2* __restrict__ Bt, int Tp,
                                             int T, const double2* __restrict__ g, double* __restrict__ out) {
  extern __shared__ double2 sh[];
  double2* av = sh;
  double2* bv = sh + T;
  double2* gv = sh + 2 * T;
  __shared__ double red[4][256];
  const double2* aj = A + (int64_t)blockIdx.x * Tp;
  const double2* bj = Bt + (int64_t)blockIdx.x * Tp;
  for (int i = threadIdx.x; i < T; i += 256) {
    av[i] = aj[i];
    bv[i] = bj[i];
    gv[i] = g[i];
  }
  __syncthreads();
  double saa = 0.0, sbb = 0.0, sabr = 0.0, sabi = 0.0;
  for (int l = threadIdx.x; l < T; l += 256) {
    double2 ma = make_double2(0.0, 0.0), mb = make_double2(0.0, 0.0);
    for (int k = 0; k < T; ++k) {
      const int d = l - k;
      const double2 gk = d >= 0 ? gv[d] : cconj(gv[-d]);
      ma = cadd(ma, cmul(gk, av[k]));
      mb = cadd(mb, cmul(gk, bv[k]));
    }
    saa += av[l].x * ma.x + av[l].y * ma.y;        // Re(conj(a_l) (M a)_l)
    sbb += bv[l].x * mb.x + bv[l].y * mb.y;
    sabr += av[l].x * mb.x + av[l].y * mb.y;       // conj(a_l) (M b)_l
    sabi += av[l].x * mb.y - av[l].y * mb.x;
  }
  red[0][threadIdx.x] = saa;
  red[1][threadIdx.x] = sbb;
  red[2][threadIdx.x] = sabr;
  red[3][threadIdx.x] = sabi;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o)
      for (int q = 0; q < 4; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = sqrt(red[2][0] * red[2][0] + red[3][0] * red[3][0]) / sqrt(red[0][0] * red[1][0]);
}

// ------------------------------------------------------------- state
constexpr int kSurMaxBatch = 1024;    // training batch and loss_grad rows
constexpr int kSurChunk = 4096;       // inference templates per forward pass and expansion
struct Surrogate {
  Plan* plan = nullptr;
  Taps* taps = nullptr;
  int sb = 0, T = 0, Tp = 0, D = 0, K = 0, H = 0;
  int64_t n = 0;                       // training tap sets
  float* X = nullptr;                  // [n x D] whitened training taps
  double2* Weff = nullptr;             // [K x T] L^-H applied to each basis vector
  float* Bt = nullptr;                 // [K x D] orthonormal basis
  float* C = nullptr;                  // [n x K] target coefficients
  float* Q2 = nullptr;                 // [n x K] scratch (X B^T during iteration)
  // parameters, flat: W1 [H x 4], b1 [H], W2 [H x H], b2 [H], W3 [K x H], b3 [K]
  int64_t np = 0, oW1 = 0, ob1 = 0, oW2 = 0, ob2 = 0, oW3 = 0, ob3 = 0;
  float *w = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
  uint16_t* wbf = nullptr;             // BF16 copy used by every GEMM
  int64_t step = 0;
  int nb = 0;                          // rows of the batch buffers (training batch, inference chunk)
  float *Pb = nullptr, *Cb = nullptr, *Z1 = nullptr, *H1 = nullptr, *Z2 = nullptr, *H2 = nullptr, *Y = nullptr,
        *dY = nullptr, *dA = nullptr, *dB = nullptr;
  int32_t* idx = nullptr;
  double* partial = nullptr;
  double* epart = nullptr;             // [nb x tap blocks x 2] expansion norm partials
  double* loss = nullptr;
  uint64_t seed = 0;
  bool basis_ready = false;            // basis, targets and Weff exist
  int64_t* tstate = nullptr;           // training step state (k_train_state_*)
  bool graphs = true;                  // training replays one captured epoch per epoch
  double* frange = nullptr;            // feature range lo[4], hi[4] (rfd_surrogate_set_feature_range)
  bool frange_set = false;
};

template <typename T>
static int salloc(T** p, size_t n) {
  *p = nullptr;
  if (device_malloc((void**)p, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return fail(RFD_E_NOMEM, "surrogate: hipMalloc failed");
  }
  return RFD_OK;
}
template <typename T>
static void sfree(T*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

static void sur_free(Surrogate& s) {
  sfree(s.X); sfree(s.Weff); sfree(s.Bt); sfree(s.C); sfree(s.Q2); sfree(s.w); sfree(s.g); sfree(s.m); sfree(s.v); sfree(s.wbf);
  sfree(s.Pb); sfree(s.Cb); sfree(s.Z1); sfree(s.H1); sfree(s.Z2); sfree(s.H2); sfree(s.Y); sfree(s.dY);
  sfree(s.dA); sfree(s.dB); sfree(s.idx); sfree(s.partial); sfree(s.epart); sfree(s.loss); sfree(s.tstate);
  sfree(s.frange);
}

// Network inputs from physical parameters (m1, m2, chi, e0): chirp mass
// M eta^(3/5), symmetric mass ratio eta = m1 m2 / M^2, chi and e0 (the same
// four degrees of freedom in the coordinates the phase depends on most),
// each mapped linearly onto [-1, 1] over the training set's range.
__device__ __forceinline__ void phys_features(const double* q, double f[4]) {
  const double m1 = q[0], m2 = q[1], mt = m1 + m2;
  const double eta = m1 * m2 / (mt * mt);
  f[0] = mt * pow(eta, 0.6);
  f[1] = eta;
  f[2] = q[2];
  f[3] = q[3];
}

// range[0..3] = min, range[4..7] = max of each feature over n rows (one workgroup)
__global__ __launch_bounds__(256) void k_feature_range(const double* __restrict__ phys, int64_t n,
                                                     double* __restrict__ range) {
  __shared__ double lo[4][256], hi[4][256];
  double l[4], h[4];
  for (int c = 0; c < 4; ++c) {
    l[c] = INFINITY;
    h[c] = -INFINITY;
  }
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    double f[4];
    phys_features(phys + 4 * i, f);
    for (int c = 0; c < 4; ++c) {
      l[c] = fmin(l[c], f[c]);
      h[c] = fmax(h[c], f[c]);
    }
  }
  for (int c = 0; c < 4; ++c) {
    lo[c][threadIdx.x] = l[c];
    hi[c][threadIdx.x] = h[c];
  }
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o)
      for (int c = 0; c < 4; ++c) {
        lo[c][threadIdx.x] = fmin(lo[c][threadIdx.x], lo[c][threadIdx.x + o]);
        hi[c][threadIdx.x] = fmax(hi[c][threadIdx.x], hi[c][threadIdx.x + o]);
      }
    __syncthreads();
  }
  if (threadIdx.x < 4) {
    range[threadIdx.x] = lo[threadIdx.x][0];
    range[4 + threadIdx.x] = hi[threadIdx.x][0];
  }
}

// scaled features 2 (f - lo) / (hi - lo) - 1 (a constant feature maps to -1)
__global__ __launch_bounds__(256) void k_features(const double* __restrict__ phys, int64_t n,
                                                const double* __restrict__ range, float* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  double f[4];
  phys_features(phys + 4 * i, f);
  for (int c = 0; c < 4; ++c) {
    const double lo = range[c], span = range[4 + c] - lo;
    out[4 * i + c] = (float)(2.0 * (f[c] - lo) / (span > 0.0 ? span : 1.0) - 1.0);
  }
}

// dynamic LDS a launch may request on the current device
static int lds_fits(size_t bytes) {
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
    return 0;
  return bytes <= (size_t)v;
}

static int grid_for(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096)); }

// Exact-tap fallback: template j takes the exact taps and fitted norm when
// its validated match is below min_match (NaN included).
__global__ __launch_bounds__(256) void k_fallback_rows(const double* __restrict__ match, double min_match, int T,
                                                     const double2* __restrict__ ea, int64_t eTp,
                                                     const double* __restrict__ esig, double2* __restrict__ ta,
                                                     int64_t tTp, double* __restrict__ tsig) {
  const int64_t j = blockIdx.x;
  if (match[j] >= min_match) return;
  for (int k = threadIdx.x; k < T; k += 256) ta[j * tTp + k] = ea[j * eTp + k];
  if (threadIdx.x == 0) tsig[j] = esig[j];
}

// Surrogates of equal shape whose training steps are launched together.
struct NetGroup {
  Surrogate* s[kMaxNets] = {};
  int n = 0;
  template <typename T, typename F>
  PerNet<T> per(F f) const {
    PerNet<T> r{};
    for (int i = 0; i < n; ++i) r.p[i] = f(*s[i]);
    return r;
  }
};
static NetGroup one_group(Surrogate& s) {
  NetGroup g;
  g.s[0] = &s;
  g.n = 1;
  return g;
}
// PerNet of one member expression of every surrogate of g
#define PER(T, expr) g.template per<T>([&](Surrogate& s) -> T { return (expr); })

static int refresh_bf16(const NetGroup& g, hipStream_t st) {
  const int64_t np = g.s[0]->np;
  hipLaunchKernelGGL(k_to_bf16, dim3(grid_for(np), g.n), dim3(256), 0, st, PER(const float*, s.w),
                     PER(uint16_t*, s.wbf), np);
  RFD_CHECK_LAUNCH();
  return RFD_OK;
}

// forward pass for n rows (n <= nb) of parameters P -> Y (and the activations)
static int forward(const NetGroup& g, hipStream_t st, const PerNet<const float*>& P, int n) {
  int rc;
  const int H = g.s[0]->H, K = g.s[0]->K;
  // biases and activations in the GEMM epilogues
  GemmOps<float, uint16_t> o{};
  o.A = P;
  o.B = PER(const uint16_t*, s.wbf + s.oW1);
  o.C = PER(float*, s.Z1);
  o.bias = PER(const float*, s.w + s.ob1);
  o.H = PER(float*, s.H1);
  if ((rc = gemm_n(st, g.n, n, H, 4, o, 4, 0, 4, 1, H, 0, kBiasAct))) return rc;
  o.A = PER(const float*, s.H1);
  o.B = PER(const uint16_t*, s.wbf + s.oW2);
  o.C = PER(float*, s.Z2);
  o.bias = PER(const float*, s.w + s.ob2);
  o.H = PER(float*, s.H2);
  if ((rc = gemm_n(st, g.n, n, H, H, o, H, 0, H, 1, H, 0, kBiasAct))) return rc;
  o.A = PER(const float*, s.H2);
  o.B = PER(const uint16_t*, s.wbf + s.oW3);
  o.C = PER(float*, s.Y);
  o.bias = PER(const float*, s.w + s.ob3);
  if ((rc = gemm_n(st, g.n, n, K, H, o, H, 0, H, 1, K, 0, kBias))) return rc;
  return RFD_OK;
}

// loss (added to *s.loss when accumulate) and gradients into s.g for n rows
// (P, Cb); with state_acc the loss accumulates after an epoch's first step
static int backward(const NetGroup& g, hipStream_t st, const PerNet<const float*>& P,
                    const PerNet<const float*>& Cb, int n, int accumulate_loss, double loss_scale,
                    bool state_acc = false) {
  int rc;
  const int H = g.s[0]->H, K = g.s[0]->K;
  const int64_t ny = (int64_t)n * K;
  const int nblk = std::min<int>(grid_for(ny), 256);
  hipLaunchKernelGGL(k_loss, dim3(nblk, g.n), dim3(256), 0, st, PER(const float*, s.Y), Cb, PER(float*, s.dY), ny,
                     1.f / n, PER(double*, s.partial));
  RFD_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_sum_partials, dim3(g.n), dim3(1), 0, st, PER(const double*, s.partial), nblk, loss_scale,
                     PER(double*, s.loss), accumulate_loss,
                     PER(const int64_t*, state_acc ? s.tstate : nullptr));
  RFD_CHECK_LAUNCH();
  // layer 3
  GemmOps<float, float> wg{};
  wg.A = PER(const float*, s.dY);
  wg.B = PER(const float*, s.H2);
  wg.C = PER(float*, s.g + s.oW3);
  if ((rc = gemm_n(st, g.n, K, H, n, wg, K, 1, H, 0, H))) return rc;
  hipLaunchKernelGGL(k_colsum, dim3((K + 63) / 64, g.n), dim3(1024), 0, st, PER(const float*, s.dY), (int64_t)n, K,
                     PER(float*, s.g + s.ob3));
  RFD_CHECK_LAUNCH();
  GemmOps<float, uint16_t> ag{};
  ag.A = PER(const float*, s.dY);
  ag.B = PER(const uint16_t*, s.wbf + s.oW3);
  ag.C = PER(float*, s.dA);
  ag.Z = PER(const float*, s.Z2);
  if ((rc = gemm_n(st, g.n, n, H, K, ag, K, 0, H, 0, H, 0, kSiluBwd))) return rc;
  // layer 2
  wg.A = PER(const float*, s.dA);
  wg.B = PER(const float*, s.H1);
  wg.C = PER(float*, s.g + s.oW2);
  if ((rc = gemm_n(st, g.n, H, H, n, wg, H, 1, H, 0, H))) return rc;
  hipLaunchKernelGGL(k_colsum, dim3((H + 63) / 64, g.n), dim3(1024), 0, st, PER(const float*, s.dA), (int64_t)n, H,
                     PER(float*, s.g + s.ob2));
  RFD_CHECK_LAUNCH();
  ag.A = PER(const float*, s.dA);
  ag.B = PER(const uint16_t*, s.wbf + s.oW2);
  ag.C = PER(float*, s.dB);
  ag.Z = PER(const float*, s.Z1);
  if ((rc = gemm_n(st, g.n, n, H, H, ag, H, 0, H, 0, H, 0, kSiluBwd))) return rc;
  // layer 1
  wg.A = PER(const float*, s.dB);
  wg.B = P;
  wg.C = PER(float*, s.g + s.oW1);
  if ((rc = gemm_n(st, g.n, H, 4, n, wg, H, 1, 4, 0, 4))) return rc;
  hipLaunchKernelGGL(k_colsum, dim3((H + 63) / 64, g.n), dim3(1024), 0, st, PER(const float*, s.dB), (int64_t)n, H,
                     PER(float*, s.g + s.ob1));
  RFD_CHECK_LAUNCH();
  return RFD_OK;
}

// Fold the inverse whitening into the basis: row k of Weff = L^-H (b_k re + i b_k im),
// so inference is a = sum_k c_k Weff_k (the map x -> a is linear).
static int update_expansion(Surrogate& s, hipStream_t st) {
  const SubBankTaps& src = s.taps->sb[s.sb];
  if (!lds_fits((size_t)2 * s.T * sizeof(double2))) return fail(RFD_E_INVALID, "T too large for the device's LDS");
  hipLaunchKernelGGL(k_unwhiten, dim3((unsigned)s.K), dim3(256), (size_t)2 * s.T * sizeof(double2), st, s.Bt,
                     (const double2*)src.U, s.T, s.Weff, s.T);
  RFD_CHECK_LAUNCH();
  return RFD_OK;
}


// Epochs of Adam on the networks of g (equal shapes, one plan), launched
// together: per step a gather, the forward and backward passes, Adam and the
// BF16 refresh, each one launch for the whole group.  Each network shuffles
// with its own generator (seed + 7) as when trained alone, so the group's
// result equals training each network by itself.  The next epoch's
// permutations are shuffled on the host while the device runs the current
// one (two pinned buffers).
static int train_group(const NetGroup& g, const PerNet<const float*>& params, int epochs, int batch, float lr,
                       float* loss_out) {
  Surrogate& s0 = *g.s[0];
  hipStream_t st = s0.plan->stream;
  const int64_t n = s0.n;
  const int K = s0.K;
  std::vector<std::mt19937_64> gens;
  std::vector<std::vector<int32_t>> perms(g.n, std::vector<int32_t>(n));
  for (int i = 0; i < g.n; ++i) {
    gens.emplace_back(g.s[i]->seed + 7);
    for (int64_t j = 0; j < n; ++j) perms[i][j] = (int32_t)j;
  }
  int32_t* dperm = nullptr;
  float* drec = nullptr;
  int32_t* hperm[2] = {nullptr, nullptr};
  hipEvent_t ev[2] = {nullptr, nullptr};
  hipGraphExec_t exec = nullptr;
  int rc = salloc(&dperm, (size_t)g.n * n);
  if (!rc) rc = salloc(&drec, (size_t)g.n * epochs);
  for (int b = 0; b < 2 && !rc; ++b) {
    if (hipHostMalloc((void**)&hperm[b], (size_t)g.n * n * sizeof(int32_t), hipHostMallocDefault) != hipSuccess ||
        hipEventCreateWithFlags(&ev[b], hipEventDisableTiming) != hipSuccess)
      rc = fail(RFD_E_NOMEM, "training buffers: allocation failed");
  }
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const int64_t nbatches = n / batch;                // whole batches only
  const double loss_scale = 1.0 / (double)(batch * nbatches);
  PerNet<const int32_t*> dp{};
  for (int i = 0; i < g.n; ++i) dp.p[i] = dperm + (int64_t)i * n;
  const PerNet<const float*> Pb = PER(const float*, s.Pb);
  const PerNet<const float*> Cb = PER(const float*, s.Cb);
  const PerNet<const int64_t*> tst = PER(const int64_t*, s.tstate);
  // one training step; its batch index and Adam step count live on the device
  auto step = [&](hipStream_t q) -> int {
    hipLaunchKernelGGL(k_gather, dim3(grid_for((int64_t)batch * (4 + K)), g.n), dim3(256), 0, q, params,
                       PER(const float*, s.C), dp, tst, batch, K, PER(float*, s.Pb), PER(float*, s.Cb));
    if (hipGetLastError() != hipSuccess) return fail(RFD_E_DEVICE, "gather launch failed");
    int r = forward(g, q, Pb, batch);
    if (!r) r = backward(g, q, Pb, Cb, batch, 0, loss_scale, true);
    if (r) return r;
    hipLaunchKernelGGL(k_adam_step, dim3(grid_for(s0.np), g.n), dim3(256), 0, q, PER(float*, s.w),
                       PER(const float*, s.g), PER(float*, s.m), PER(float*, s.v), PER(uint16_t*, s.wbf), s0.np, lr,
                       b1, b2, eps, tst);
    if (hipGetLastError() != hipSuccess) return fail(RFD_E_DEVICE, "adam launch failed");
    hipLaunchKernelGGL(k_train_state_advance, dim3(g.n), dim3(1), 0, q, PER(int64_t*, s.tstate));
    if (hipGetLastError() != hipSuccess) return fail(RFD_E_DEVICE, "step launch failed");
    return RFD_OK;
  };
  // with graphs: capture one epoch's steps once, replay it every epoch
  bool graphs = true;
  for (int i = 0; i < g.n; ++i) graphs = graphs && g.s[i]->graphs;
  if (!rc && graphs && nbatches > 1) {
    hipStream_t cs = nullptr;
    hipGraph_t gr = nullptr;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) {
      rc = fail(RFD_E_DEVICE, "capture stream creation failed");
    } else if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      rc = fail(RFD_E_DEVICE, "hipStreamBeginCapture failed");
    } else {
      for (int64_t bi = 0; bi < nbatches && !rc; ++bi) rc = step(cs);
      const hipError_t e = hipStreamEndCapture(cs, &gr);
      if (!rc && e != hipSuccess) rc = fail(RFD_E_DEVICE, "hipStreamEndCapture failed");
      if (!rc && hipGraphInstantiate(&exec, gr, nullptr, nullptr, 0) != hipSuccess)
        rc = fail(RFD_E_DEVICE, "hipGraphInstantiate failed");
    }
    if (gr) (void)hipGraphDestroy(gr);
    if (cs) (void)hipStreamDestroy(cs);
    (void)hipGetLastError();
  }
  for (int e = 0; e < epochs && !rc; ++e) {
    const int b = e & 1;
    // buffer b was last read by the copy of epoch e - 2
    if (e >= 2 && hipEventSynchronize(ev[b]) != hipSuccess) {
      rc = fail(RFD_E_DEVICE, "event wait failed");
      break;
    }
    for (int i = 0; i < g.n; ++i) {
      std::shuffle(perms[i].begin(), perms[i].end(), gens[i]);
      memcpy(hperm[b] + (int64_t)i * n, perms[i].data(), n * sizeof(int32_t));
    }
    // stream order: the copy waits for the previous epoch's steps
    if (hipMemcpyAsync(dperm, hperm[b], (size_t)g.n * n * sizeof(int32_t), hipMemcpyHostToDevice, st) != hipSuccess ||
        hipEventRecord(ev[b], st) != hipSuccess) {
      rc = fail(RFD_E_DEVICE, "permutation upload failed");
      break;
    }
    hipLaunchKernelGGL(k_train_state_set, dim3(g.n), dim3(1), 0, st, PER(int64_t*, s.tstate), (int64_t)0,
                       PER(int64_t, s.step));
    if (hipGetLastError() != hipSuccess) { rc = fail(RFD_E_DEVICE, "state launch failed"); break; }
    if (exec) {
      if (hipGraphLaunch(exec, st) != hipSuccess) rc = fail(RFD_E_DEVICE, "hipGraphLaunch failed");
    } else {
      for (int64_t bi = 0; bi < nbatches && !rc; ++bi) rc = step(st);
    }
    for (int i = 0; i < g.n; ++i) g.s[i]->step += nbatches;
    if (!rc) {
      // mean per-sample squared coefficient error over the epoch
      hipLaunchKernelGGL(k_loss_record, dim3(g.n), dim3(1), 0, st, PER(const double*, s.loss), drec, epochs, e);
      if (hipGetLastError() != hipSuccess) rc = fail(RFD_E_DEVICE, "loss record launch failed");
    }
  }
  if (!rc && loss_out &&
      hipMemcpyAsync(loss_out, drec, (size_t)g.n * epochs * sizeof(float), hipMemcpyDeviceToHost, st) != hipSuccess)
    rc = fail(RFD_E_DEVICE, "loss readback failed");
  if (hipStreamSynchronize(st) != hipSuccess && !rc) rc = fail(RFD_E_DEVICE, "training failed on the device");
  if (exec) (void)hipGraphExecDestroy(exec);
  for (int b = 0; b < 2; ++b) {
    if (ev[b]) (void)hipEventDestroy(ev[b]);
    if (hperm[b]) (void)hipHostFree(hperm[b]);
  }
  sfree(drec);
  sfree(dperm);
  return rc;
}
#undef PER

}  // namespace rfd

using namespace rfd;

struct rfd_surrogate { rfd::Surrogate s; };

extern "C" {

int rfd_surrogate_create(rfd_plan* plan, rfd_taps* taps, int32_t subbank, int32_t n_basis, int32_t hidden,
                         uint64_t seed, rfd_surrogate** out) {
  if (!out) return fail(RFD_E_INVALID, "out is NULL");
  *out = nullptr;
  if (!plan || !taps) return fail(RFD_E_INVALID, "NULL plan or taps");
  Plan& p = plan->p;
  Taps& t = taps->t;
  if (t.plan != &p) return fail(RFD_E_INVALID, "taps belong to another plan");
  if (subbank < 0 || subbank >= (int)t.sb.size()) return fail(RFD_E_INVALID, "subbank out of range");
  SubBankTaps& sb = t.sb[subbank];
  if (sb.count < 2 || sb.made != sb.count) return fail(RFD_E_STATE, "training sub-bank needs >= 2 made tap sets");
  if (!sb.U) return fail(RFD_E_STATE, "training taps must come from the least-squares route (Cholesky factor)");
  if (sb.n_centred > 0)
    return fail(RFD_E_UNSUPPORTED, "training taps must share the sub-bank's lag window (no RFD_TAPS_CENTRE)");
  if (n_basis < 1 || n_basis > 2 * sb.T || n_basis > 1024) return fail(RFD_E_INVALID, "n_basis out of range");
  if (hidden < 1 || hidden > 4096) return fail(RFD_E_INVALID, "hidden out of range");
  if (!lds_fits((size_t)kExpandRows * ((n_basis + 3) & ~3) * sizeof(double) + 8 * kExpandRows * sizeof(double)))
    return fail(RFD_E_INVALID, "n_basis too large for the device's LDS");
  rfd_surrogate* h = new (std::nothrow) rfd_surrogate();
  if (!h) return fail(RFD_E_NOMEM, "host allocation failed");
  Surrogate& s = h->s;
  s.plan = &p;
  s.taps = &t;
  s.sb = subbank;
  s.T = sb.T;
  s.Tp = sb.Tp;
  s.D = 2 * sb.T;
  s.K = n_basis;
  s.H = hidden;
  s.n = sb.count;
  s.seed = seed;
  s.nb = kSurChunk;
  const int H = s.H, K = s.K;
  s.oW1 = 0;
  s.ob1 = s.oW1 + (int64_t)H * 4;
  s.oW2 = s.ob1 + H;
  s.ob2 = s.oW2 + (int64_t)H * H;
  s.oW3 = s.ob2 + H;
  s.ob3 = s.oW3 + (int64_t)K * H;
  s.np = s.ob3 + K;
  int rc = RFD_OK;
#define TRY(x) do { rc = (x); if (rc) { sur_free(s); delete h; return rc; } } while (0)
  TRY(salloc(&s.X, (size_t)s.n * s.D));
  TRY(salloc(&s.Bt, (size_t)K * s.D));
  TRY(salloc(&s.Weff, (size_t)K * s.T));
  TRY(salloc(&s.C, (size_t)s.n * K));
  TRY(salloc(&s.Q2, (size_t)s.n * K));
  TRY(salloc(&s.w, (size_t)s.np));
  TRY(salloc(&s.g, (size_t)s.np));
  TRY(salloc(&s.m, (size_t)s.np));
  TRY(salloc(&s.v, (size_t)s.np));
  TRY(salloc(&s.wbf, (size_t)s.np));
  TRY(salloc(&s.Pb, (size_t)s.nb * 4));
  TRY(salloc(&s.Cb, (size_t)s.nb * K));
  TRY(salloc(&s.Z1, (size_t)s.nb * H));
  TRY(salloc(&s.H1, (size_t)s.nb * H));
  TRY(salloc(&s.Z2, (size_t)s.nb * H));
  TRY(salloc(&s.H2, (size_t)s.nb * H));
  TRY(salloc(&s.Y, (size_t)s.nb * K));
  TRY(salloc(&s.dY, (size_t)s.nb * K));
  TRY(salloc(&s.dA, (size_t)s.nb * H));
  TRY(salloc(&s.dB, (size_t)s.nb * H));
  TRY(salloc(&s.idx, (size_t)s.nb));
  TRY(salloc(&s.partial, 256));
  TRY(salloc(&s.epart, (size_t)s.nb * ((s.T + 255) / 256) * 2));
  TRY(salloc(&s.loss, 1));
  TRY(salloc(&s.frange, 8));
  TRY(salloc(&s.tstate, 2));
#undef TRY
  // He-uniform initial weights, zero biases (host, seeded)
  std::vector<float> w0(s.np, 0.f);
  std::mt19937_64 gen(seed);
  auto fill = [&](int64_t off, int64_t rows, int64_t cols) {
    std::uniform_real_distribution<float> u(-std::sqrt(6.f / cols), std::sqrt(6.f / cols));
    for (int64_t i = 0; i < rows * cols; ++i) w0[off + i] = u(gen);
  };
  fill(s.oW1, H, 4);
  fill(s.oW2, H, H);
  fill(s.oW3, K, H);
  hipStream_t st = p.stream;
  if (hipMemcpy(s.w, w0.data(), s.np * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemsetAsync(s.m, 0, s.np * sizeof(float), st) != hipSuccess ||
      hipMemsetAsync(s.v, 0, s.np * sizeof(float), st) != hipSuccess) {
    sur_free(s);
    delete h;
    return fail(RFD_E_DEVICE, "surrogate initialisation failed");
  }
  // whitened training taps
  hipLaunchKernelGGL(k_whiten, dim3((unsigned)s.n), dim3(256), (size_t)s.T * sizeof(double2), st,
                     t.a64 + sb.a_base, sb.Tp, (const double2*)sb.U, (const double2*)sb.g, sb.eps,
                     std::min(std::max(-sb.k0, 0), s.T - 1), s.T, s.X);
  if (hipGetLastError() != hipSuccess || refresh_bf16(one_group(s), st)) {
    sur_free(s);
    delete h;
    return fail(RFD_E_DEVICE, "surrogate whitening failed");
  }
  *out = h;
  return RFD_OK;
}

int rfd_surrogate_fit_basis(rfd_surrogate* sur, int32_t iters, double* captured_out) {
  if (!sur) return fail(RFD_E_INVALID, "NULL surrogate");
  if (iters < 1 || iters > 100) return fail(RFD_E_INVALID, "iters must be in [1, 100]");
  Surrogate& s = sur->s;
  hipStream_t st = s.plan->stream;
  const int D = s.D, K = s.K;
  const int n = (int)s.n;
  hipLaunchKernelGGL(k_random, dim3(grid_for((int64_t)K * D)), dim3(256), 0, st, s.Bt, (int64_t)K * D, s.seed ^ 0xB5ull);
  RFD_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_orthonormalise, dim3(1), dim3(1024), 0, st, s.Bt, K, D);
  RFD_CHECK_LAUNCH();
  int rc;
  for (int it = 0; it < iters; ++it) {
    // Q2 = X B^T  (n x K);  B = Q2^T X  (K x D);  orthonormalise
    if ((rc = gemm<float, float>(st, n, K, D, s.X, D, 0, s.Bt, D, 1, s.Q2, K))) return rc;
    if ((rc = gemm<float, float>(st, K, D, n, s.Q2, K, 1, s.X, D, 0, s.Bt, D))) return rc;
    hipLaunchKernelGGL(k_orthonormalise, dim3(1), dim3(1024), 0, st, s.Bt, K, D);
    RFD_CHECK_LAUNCH();
  }
  // target coefficients C = X B^T and the folded expansion matrix
  if ((rc = gemm<float, float>(st, n, K, D, s.X, D, 0, s.Bt, D, 1, s.C, K))) return rc;
  if ((rc = update_expansion(s, st))) return rc;
  s.basis_ready = true;
  if (captured_out) {
    // sum ||c_i||^2 / sum ||x_i||^2  (rows of X have unit norm)
    const int64_t ny = (int64_t)n * K;
    const int nblk = std::min<int>(grid_for(ny), 256);
    float* zeros = s.Q2;   // loss kernel of C against zero: sum of squares
    RFD_HIP(hipMemsetAsync(zeros, 0, ny * sizeof(float), st));
    float* dummy = nullptr;
    if ((rc = salloc(&dummy, (size_t)ny))) return rc;
    hipLaunchKernelGGL(k_loss, dim3(nblk), dim3(256), 0, st, one_net<const float*>(s.C), one_net<const float*>(zeros),
                       one_net(dummy), ny, 1.f, one_net(s.partial));
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(1), 0, st, one_net<const double*>(s.partial), nblk, 1.0 / n,
                       one_net(s.loss), 0, one_net<const int64_t*>(nullptr));
    double v = 0;
    RFD_HIP(hipMemcpyAsync(&v, s.loss, sizeof(double), hipMemcpyDeviceToHost, st));
    RFD_HIP(hipStreamSynchronize(st));
    sfree(dummy);
    *captured_out = v;
  }
  return RFD_OK;
}

int rfd_surrogate_train_many(rfd_surrogate* const* surs, const float* const* params, int32_t count, int32_t epochs,
                             int32_t batch, float lr, float* loss_out) {
  if (!surs || !params) return fail(RFD_E_INVALID, "NULL argument");
  if (count < 1 || count > kMaxNets) return fail(RFD_E_INVALID, "count must be in [1, 32]");
  if (epochs < 1 || batch < 1 || batch > kSurMaxBatch || !(lr > 0.f)) return fail(RFD_E_INVALID, "bad training arguments");
  NetGroup g;
  PerNet<const float*> P{};
  for (int i = 0; i < count; ++i) {
    if (!surs[i] || !params[i]) return fail(RFD_E_INVALID, "NULL surrogate or parameters");
    Surrogate& s = surs[i]->s;
    if (!s.basis_ready) return fail(RFD_E_STATE, "fit or set the basis before training");
    for (int j = 0; j < i; ++j)
      if (g.s[j] == &s) return fail(RFD_E_INVALID, "a surrogate appears twice");
    if (i > 0) {
      const Surrogate& s0 = *g.s[0];
      if (s.plan != s0.plan || s.n != s0.n || s.H != s0.H || s.K != s0.K)
        return fail(RFD_E_INVALID, "surrogates trained together need one plan and equal n, hidden and n_basis");
    }
    if (batch > s.n) return fail(RFD_E_INVALID, "batch larger than the training set");
    g.s[i] = &s;
    P.p[i] = params[i];
  }
  g.n = count;
  return train_group(g, P, epochs, batch, lr, loss_out);
}

int rfd_surrogate_train(rfd_surrogate* sur, const float* params, int32_t epochs, int32_t batch, float lr,
                        float* loss_out) {
  if (!sur || !params) return fail(RFD_E_INVALID, "NULL argument");
  return rfd_surrogate_train_many(&sur, &params, 1, epochs, batch, lr, loss_out);
}

int rfd_surrogate_set_feature_range(rfd_surrogate* sur, const double* phys, int64_t n) {
  if (!sur || !phys) return fail(RFD_E_INVALID, "NULL argument");
  if (n < 1) return fail(RFD_E_INVALID, "n must be >= 1");
  Surrogate& s = sur->s;
  hipStream_t st = s.plan->stream;
  hipLaunchKernelGGL(k_feature_range, dim3(1), dim3(256), 0, st, phys, n, s.frange);
  RFD_CHECK_LAUNCH();
  RFD_HIP(hipStreamSynchronize(st));
  s.frange_set = true;
  return RFD_OK;
}

int rfd_surrogate_features(rfd_surrogate* sur, const double* phys, int64_t n, float* out) {
  if (!sur || !phys || !out) return fail(RFD_E_INVALID, "NULL argument");
  if (n < 0) return fail(RFD_E_INVALID, "n must be >= 0");
  Surrogate& s = sur->s;
  if (!s.frange_set) return fail(RFD_E_STATE, "feature range not set (rfd_surrogate_set_feature_range)");
  if (n == 0) return RFD_OK;
  hipLaunchKernelGGL(k_features, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s.plan->stream, phys, n,
                     (const double*)s.frange, out);
  RFD_CHECK_LAUNCH();
  return RFD_OK;
}

int rfd_surrogate_set_graphs(rfd_surrogate* sur, int32_t enable) {
  if (!sur) return fail(RFD_E_INVALID, "NULL surrogate");
  sur->s.graphs = enable != 0;
  return RFD_OK;
}

int rfd_surrogate_loss_grad(rfd_surrogate* sur, const float* params, const float* targets, int32_t n, float* grads,
                            double* loss_out) {
  if (!sur || !params || !grads) return fail(RFD_E_INVALID, "NULL argument");
  Surrogate& s = sur->s;
  if (n < 1 || n > kSurMaxBatch) return fail(RFD_E_INVALID, "n out of range");
  hipStream_t st = s.plan->stream;
  const float* Cb = targets ? targets : s.C;
  const NetGroup g = one_group(s);
  int rc = forward(g, st, one_net(params), n);
  if (!rc) rc = backward(g, st, one_net(params), one_net<const float*>(Cb), n, 0, (double)1.0 / n);
  if (rc) return rc;
  RFD_HIP(hipMemcpyAsync(grads, s.g, s.np * sizeof(float), hipMemcpyDeviceToDevice, st));
  if (loss_out) {
    double v = 0;
    RFD_HIP(hipMemcpyAsync(&v, s.loss, sizeof(double), hipMemcpyDeviceToHost, st));
    RFD_HIP(hipStreamSynchronize(st));
    *loss_out = v;         // mean over rows of ||y - c||^2
  }
  return RFD_OK;
}

int rfd_surrogate_get_state(rfd_surrogate* sur, float* weights, float* basis, float* targets, int64_t* sizes) {
  if (!sur) return fail(RFD_E_INVALID, "NULL surrogate");
  Surrogate& s = sur->s;
  hipStream_t st = s.plan->stream;
  if (sizes) {
    sizes[0] = s.np;
    sizes[1] = (int64_t)s.K * s.D;
    sizes[2] = s.n * s.K;
    sizes[3] = s.D;
    sizes[4] = s.K;
    sizes[5] = s.H;
  }
  if (weights) RFD_HIP(hipMemcpyAsync(weights, s.w, s.np * sizeof(float), hipMemcpyDeviceToHost, st));
  if (basis) RFD_HIP(hipMemcpyAsync(basis, s.Bt, (size_t)s.K * s.D * sizeof(float), hipMemcpyDeviceToHost, st));
  if (targets) RFD_HIP(hipMemcpyAsync(targets, s.C, (size_t)s.n * s.K * sizeof(float), hipMemcpyDeviceToHost, st));
  RFD_HIP(hipStreamSynchronize(st));
  return RFD_OK;
}

int rfd_surrogate_set_state(rfd_surrogate* sur, const float* weights, const float* basis) {
  if (!sur || (!weights && !basis)) return fail(RFD_E_INVALID, "NULL argument");
  Surrogate& s = sur->s;
  hipStream_t st = s.plan->stream;
  if (weights) {
    // new weights restart the optimiser
    RFD_HIP(hipMemcpyAsync(s.w, weights, s.np * sizeof(float), hipMemcpyHostToDevice, st));
    RFD_HIP(hipMemsetAsync(s.m, 0, s.np * sizeof(float), st));
    RFD_HIP(hipMemsetAsync(s.v, 0, s.np * sizeof(float), st));
    s.step = 0;
  }
  if (basis) {
    RFD_HIP(hipMemcpyAsync(s.Bt, basis, (size_t)s.K * s.D * sizeof(float), hipMemcpyHostToDevice, st));
    // the training targets are the coefficients on the new basis
    int rc = gemm<float, float>(st, (int)s.n, s.K, s.D, s.X, s.D, 0, s.Bt, s.D, 1, s.C, s.K);
    if (!rc) rc = update_expansion(s, st);
    if (rc) return rc;
    s.basis_ready = true;
  }
  int rc = refresh_bf16(one_group(s), st);
  if (rc) return rc;
  RFD_HIP(hipStreamSynchronize(st));
  return RFD_OK;
}

int rfd_surrogate_make_taps(rfd_surrogate* sur, const float* params, rfd_taps* target, int32_t subbank, int64_t first,
                            int64_t count) {
  if (!sur || !params || !target) return fail(RFD_E_INVALID, "NULL argument");
  Surrogate& s = sur->s;
  Taps& t = target->t;
  if (t.plan != s.plan) return fail(RFD_E_INVALID, "target taps belong to another plan");
  if (subbank < 0 || subbank >= (int)t.sb.size()) return fail(RFD_E_INVALID, "subbank out of range");
  SubBankTaps& sb = t.sb[subbank];
  const SubBankTaps& src = s.taps->sb[s.sb];
  if (sb.T != src.T || sb.k0 != src.k0 || sb.ref_id != src.ref_id)
    return fail(RFD_E_INVALID, "target sub-bank must have the training sub-bank's reference, T and k0");
  if (count < 0 || first < 0 || first + count > sb.count) return fail(RFD_E_INVALID, "template range outside the sub-bank");
  if (count == 0) return RFD_OK;
  if (!s.basis_ready) return fail(RFD_E_STATE, "fit or set the basis before inference");
  Plan& p = *s.plan;
  hipStream_t st = p.stream;
  // the fitted-template norm of the target uses the reference autocorrelation of the training sub-bank
  RFD_HIP(hipMemcpyAsync(sb.g, src.g, sb.T * sizeof(double2), hipMemcpyDeviceToDevice, st));
  // surrogate taps use the sub-bank's lag window
  bool any_centred = false;
  for (int64_t i = first; i < first + count && !any_centred; ++i) any_centred = sb.centred_mask[i] != 0;
  if (any_centred) {
    RFD_HIP(hipMemsetAsync(t.d_shift + sb.first + first, 0, count * sizeof(int32_t), st));
    for (int64_t i = first; i < first + count; ++i)
      if (sb.centred_mask[i]) {
        sb.centred_mask[i] = 0;
        --sb.n_centred;
      }
  }
  const int64_t chunk = s.nb;
  int rc = RFD_OK;
  for (int64_t c0 = 0; c0 < count && !rc; c0 += chunk) {
    const int cn = (int)std::min<int64_t>(chunk, count - c0);
    rc = stage_begin(p, kStSurNet);
    if (!rc) rc = forward(one_group(s), st, one_net(params + 4 * c0), cn);
    if (!rc) rc = stage_end(p);
    if (!rc) rc = stage_begin(p, kStSurExpand);
    if (!rc) {
      const int tb = (s.T + 255) / 256;
      const size_t lds = (size_t)kExpandRows * ((s.K + 3) & ~3) * sizeof(double);
      hipLaunchKernelGGL(k_expand, dim3((unsigned)((cn + kExpandRows - 1) / kExpandRows), (unsigned)tb), dim3(256),
                         lds, st, s.Y, cn, s.K, (const double2*)s.Weff, s.Bt, s.T,
                         t.a64 + sb.a_base + (first + c0) * sb.Tp, sb.Tp, s.epart);
      hipLaunchKernelGGL(k_expand_sigma, dim3((unsigned)((cn + 255) / 256)), dim3(256), 0, st, s.epart, cn, tb,
                         src.eps, (const double2*)src.g, t.sigma_fit + sb.first + first + c0);
      if (hipGetLastError() != hipSuccess) rc = fail(RFD_E_DEVICE, "expansion launch failed");
    }
    if (!rc) rc = stage_end(p);
  }
  if (!rc) rc = stage_begin(p, kStSurPack);
  if (!rc) rc = taps_pack(p, t, subbank, first, count);
  if (!rc) rc = stage_end(p);
  (void)hipStreamSynchronize(st);
  if (rc) return rc;
  for (int64_t i = first; i < first + count; ++i) {
    if (!sb.made_mask[i]) {
      sb.made_mask[i] = 1;
      ++sb.made;
    }
  }
  return RFD_OK;
}

int rfd_taps_match(const rfd_taps* a, const rfd_taps* b, int32_t subbank, int64_t first, int64_t count,
                   double* match_out) {
  if (!a || !b || !match_out) return fail(RFD_E_INVALID, "NULL argument");
  const Taps& ta = a->t;
  const Taps& tb = b->t;
  if (ta.plan != tb.plan) return fail(RFD_E_INVALID, "taps belong to different plans");
  if (subbank < 0 || subbank >= (int)ta.sb.size() || subbank >= (int)tb.sb.size())
    return fail(RFD_E_INVALID, "subbank out of range");
  const SubBankTaps& sa = ta.sb[subbank];
  const SubBankTaps& sbb = tb.sb[subbank];
  if (sa.T != sbb.T || sa.count != sbb.count) return fail(RFD_E_INVALID, "sub-banks differ in T or size");
  if (count < 0 || first < 0 || first + count > sa.count) return fail(RFD_E_INVALID, "template range outside the sub-bank");
  if (count == 0) return RFD_OK;
  hipStream_t st = ta.plan->stream;
  if (!lds_fits((size_t)3 * sa.T * sizeof(double2) + 4 * 256 * sizeof(double)))
    return fail(RFD_E_INVALID, "T too large for the device's LDS");
  Plan& p = *ta.plan;
  int rc = stage_begin(p, kStMatch);
  if (rc) return rc;
  hipLaunchKernelGGL(k_match, dim3((unsigned)count), dim3(256), (size_t)3 * sa.T * sizeof(double2), st,
                     ta.a64 + sa.a_base + first * sa.Tp, tb.a64 + sbb.a_base + first * sbb.Tp, sa.Tp, sa.T,
                     (const double2*)sa.g, match_out);
  RFD_CHECK_LAUNCH();
  return stage_end(p);
}

int rfd_taps_fallback(rfd_taps* target, const rfd_taps* exact, int32_t subbank, int64_t first, int64_t count,
                      const double* match, double min_match, int64_t* n_fallback_out) {
  if (n_fallback_out) *n_fallback_out = 0;
  if (!target || !exact || (!match && count > 0)) return fail(RFD_E_INVALID, "NULL argument");
  Taps& tt = target->t;
  const Taps& te = exact->t;
  if (tt.plan != te.plan) return fail(RFD_E_INVALID, "taps belong to different plans");
  if (subbank < 0 || subbank >= (int)tt.sb.size() || subbank >= (int)te.sb.size())
    return fail(RFD_E_INVALID, "subbank out of range");
  SubBankTaps& st_ = tt.sb[subbank];
  const SubBankTaps& se = te.sb[subbank];
  if (st_.T != se.T || st_.k0 != se.k0 || st_.ref_id != se.ref_id || st_.count != se.count)
    return fail(RFD_E_INVALID, "sub-banks differ in reference, T, k0 or size");
  if (se.n_centred > 0 || st_.n_centred > 0)
    return fail(RFD_E_UNSUPPORTED, "fallback needs taps on the sub-bank's lag window (no RFD_TAPS_CENTRE)");
  if (count < 0 || first < 0 || first + count > st_.count) return fail(RFD_E_INVALID, "template range outside the sub-bank");
  if (count == 0) return RFD_OK;
  Plan& p = *tt.plan;
  hipStream_t st = p.stream;
  std::vector<double> m(count);
  RFD_HIP(hipMemcpyAsync(m.data(), match, count * sizeof(double), hipMemcpyDeviceToHost, st));
  RFD_HIP(hipStreamSynchronize(st));
  std::vector<uint8_t> fb(count, 0);
  int64_t nfb = 0;
  for (int64_t j = 0; j < count; ++j) {
    fb[j] = !(m[j] >= min_match);           // NaN falls back too
    if (fb[j]) {
      if (!se.made_mask[first + j]) return fail(RFD_E_STATE, "exact taps missing for a template that falls back");
      ++nfb;
    }
  }
  if (nfb) {
    // one launch copies every failing template's exact taps and fitted norm,
    // deciding on the device with the same comparison; one repacking of the
    // range follows (rows kept from the surrogate pack to the same values)
    RFD_HIP(hipMemcpyAsync(st_.g, se.g, st_.T * sizeof(double2), hipMemcpyDeviceToDevice, st));
    hipLaunchKernelGGL(k_fallback_rows, dim3((unsigned)count), dim3(256), 0, st, match, min_match, st_.T,
                       (const double2*)(te.a64 + se.a_base + first * se.Tp), (int64_t)se.Tp,
                       (const double*)(te.sigma_fit + se.first + first), tt.a64 + st_.a_base + first * st_.Tp,
                       (int64_t)st_.Tp, tt.sigma_fit + st_.first + first);
    RFD_CHECK_LAUNCH();
    int rc = taps_pack(p, tt, subbank, first, count);
    if (rc) return rc;
    for (int64_t j = 0; j < count; ++j) {
      if (fb[j] && !st_.made_mask[first + j]) {
        st_.made_mask[first + j] = 1;
        ++st_.made;
      }
    }
  }
  if (n_fallback_out) *n_fallback_out = nfb;
  return RFD_OK;
}

int rfd_surrogate_destroy(rfd_surrogate* sur) {
  if (!sur) return RFD_OK;
  (void)hipStreamSynchronize(sur->s.plan->stream);
  sur_free(sur->s);
  delete sur;
  return RFD_OK;
}

}  // extern "C"
