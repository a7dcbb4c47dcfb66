// K-point complex FFTs held in registers: K = 256 R (R = 4, 8, 16) by
// NTf = K/16 threads of 16 values each, index m = t + NTf r.  A radix-16
// stage over r in registers, an LDS exchange, a radix-16 stage, an LDS
// exchange, a radix-R stage; F = 256/NTf independent FFTs share a
// 256-thread workgroup.  Also the small in-register DFTs (2 to 16 points)
// these stages are built from.
#pragma once

#include "dev_common.h"

namespace rfd {

// cos / sin (2 pi k / 16), k < 16
__device__ __forceinline__ float2 w16(int k, int sign) {
  constexpr float c[16] = {1.0f, 0.92387953251128674f, 0.70710678118654752f, 0.38268343236508977f,
                           0.0f, -0.38268343236508977f, -0.70710678118654752f, -0.92387953251128674f,
                           -1.0f, -0.92387953251128674f, -0.70710678118654752f, -0.38268343236508977f,
                           0.0f, 0.38268343236508977f, 0.70710678118654752f, 0.92387953251128674f};
  return make_float2(c[k & 15], sign * c[(k + 12) & 15]);   // sin x = cos(x - pi/2)
}

// dft4 of the products a = xa ga, b = xb gb, c = xc gc, d = xd gd: the first
// sums take a's and b's products as fused multiply-adds onto c's and d's, and
// the differences follow as a - c = (a + c) - 2c: 28 operations instead of the
// 32 of four complex products and a dft4.
__device__ __forceinline__ void dft4_prod(float2& a, float2& b, float2& c, float2& d, float2 xa, float2 ga,
                                          float2 xb, float2 gb, float2 xc, float2 gc, float2 xd, float2 gd,
                                          int sign) {
  const float2 pc = cmul(xc, gc), pd = cmul(xd, gd);
  const float2 s0 = make_float2(fmaf(xa.x, ga.x, fmaf(-xa.y, ga.y, pc.x)), fmaf(xa.x, ga.y, fmaf(xa.y, ga.x, pc.y)));
  const float2 s2 = make_float2(fmaf(xb.x, gb.x, fmaf(-xb.y, gb.y, pd.x)), fmaf(xb.x, gb.y, fmaf(xb.y, gb.x, pd.y)));
  const float2 s1 = make_float2(fmaf(-2.f, pc.x, s0.x), fmaf(-2.f, pc.y, s0.y));
  const float2 s3 = cmul_si(make_float2(fmaf(-2.f, pd.x, s2.x), fmaf(-2.f, pd.y, s2.y)), sign);
  a = cadd(s0, s2);
  c = csub(s0, s2);
  b = cadd(s1, s3);
  d = csub(s1, s3);
}

// Second half of the 16-point DFT (after the first radix-4 layer over n2).
template <int SIGN>
__device__ __forceinline__ void dft16_rest(float2 (&v)[16]) {
#pragma unroll
  for (int n1 = 1; n1 < 4; ++n1)
#pragma unroll
    for (int k = 1; k < 4; ++k) {
      // a quarter turn is a swap (a product with the constant 0 would be kept)
      const int p = n1 * k;
      v[n1 + 4 * k] = p == 4 ? cmul_si(v[n1 + 4 * k], SIGN) : cmul(v[n1 + 4 * k], w16(p, SIGN));
    }
#pragma unroll
  for (int k = 0; k < 4; ++k) dft4(v[4 * k], v[4 * k + 1], v[4 * k + 2], v[4 * k + 3], SIGN);
}

// 16-point DFT in registers, V[k] = sum_n v[n] e^{sign 2 pi i n k / 16}.
// On return slot s holds V[(s >> 2) + 4 (s & 3)].
template <int SIGN>
__device__ __forceinline__ void dft16(float2 (&v)[16]) {
#pragma unroll
  for (int n1 = 0; n1 < 4; ++n1) dft4(v[n1], v[n1 + 4], v[n1 + 8], v[n1 + 12], SIGN);
  dft16_rest<SIGN>(v);
}
// The same DFT of the products x[n] g[n].
template <int SIGN>
__device__ __forceinline__ void dft16_prod(float2 (&v)[16], const float2 (&x)[16], const float2 (&g)[16]) {
#pragma unroll
  for (int n1 = 0; n1 < 4; ++n1)
    dft4_prod(v[n1], v[n1 + 4], v[n1 + 8], v[n1 + 12], x[n1], g[n1], x[n1 + 4], g[n1 + 4], x[n1 + 8], g[n1 + 8],
              x[n1 + 12], g[n1 + 12], SIGN);
  dft16_rest<SIGN>(v);
}
__device__ __forceinline__ constexpr int dft16_freq(int s) { return (s >> 2) + 4 * (s & 3); }

// R-point DFTs (R = 2, 4, 8, 16) on consecutive groups of R slots of v; slot
// g R + s holds V_g[dftR_freq(s)].
template <int R, int SIGN>
__device__ __forceinline__ void dft_r(float2 (&v)[16]) {
  if constexpr (R == 16) {
    dft16<SIGN>(v);
  } else if constexpr (R == 2) {
#pragma unroll
    for (int g = 0; g < 8; ++g) {
      const float2 a = v[2 * g], b = v[2 * g + 1];
      v[2 * g] = cadd(a, b);
      v[2 * g + 1] = csub(a, b);
    }
  } else if constexpr (R == 4) {
#pragma unroll
    for (int g = 0; g < 4; ++g) dft4(v[4 * g], v[4 * g + 1], v[4 * g + 2], v[4 * g + 3], SIGN);
  } else {   // R == 8: n = n1 + 2 n2, DFT4 over n2, twiddle, DFT2 over n1
#pragma unroll
    for (int g = 0; g < 2; ++g) {
      float2* u = v + 8 * g;
      dft4(u[0], u[2], u[4], u[6], SIGN);
      dft4(u[1], u[3], u[5], u[7], SIGN);
#pragma unroll
      for (int k = 1; k < 4; ++k) u[2 * k + 1] = cmul(u[2 * k + 1], w16(2 * k, SIGN));
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const float2 a = u[2 * k], b = u[2 * k + 1];
        u[2 * k] = cadd(a, b);
        u[2 * k + 1] = csub(a, b);
      }
    }
  }
}
template <int R>
__device__ __forceinline__ constexpr int dftr_freq(int s) {
  return R == 16 ? dft16_freq(s) : (R <= 4 ? s : (s >> 1) + 4 * (s & 1));
}

template <int K>
struct BlockFft {
  static constexpr int NTf = K / 16;       // threads per FFT
  static constexpr int R = K / 256;        // last radix
  static constexpr int G = 16 / R;         // last-stage groups per thread
  static constexpr int F = 256 / NTf;      // FFTs per workgroup
  // LDS layouts of the two exchanges, chosen so that no access of either
  // exchange meets an LDS bank twice within a pass (a 64-bit access is
  // serviced half a wave at a time):
  //  exchange 1: element (k1, t) at k1 S1 + t, S1 = NTf + R.  A stage-B reader
  //    takes elements u + R q of row k1 = t / R; the rows of one half-wave
  //    start 2R banks apart, so their R-wide column groups tile the banks.
  //  exchange 2: element (k2, k1, u) at (16 k2 + k1) R + k2 / G + u: rows of R
  //    values, each group of G rows (one stage-C reader's rows) skewed by one
  //    more element, so the readers, which take R consecutive values from
  //    rows 16 (G g + e) + k1, start in distinct banks; every offset is a
  //    compile-time constant past one per-thread base.
  // (The earlier strides S1 = NTf + 4 and S2 = R + 4 left the stage-C reads
  // 8-16-way conflicted: LDS bank-conflict cycles at 1.9x the busy cycles of
  // the 4096-point overlap-save kernel.)
  static constexpr int S1 = NTf + R;
  static constexpr int X1 = 16 * S1;                 // float2 of exchange 1
  static constexpr int X2 = 256 * R + R;             // float2 of exchange 2
  static constexpr int LDS = X1 > X2 ? X1 : X2;      // float2 per FFT
};

// Per-thread twiddles: stage A  W_K^(t k1), stage B  W_K^(16 u k2), k = 1..15.
template <int K>
struct BlockFftTw {
  float2 a[16], b[16];
};
template <int K, int SIGN>
__device__ __forceinline__ void block_fft_twiddles(BlockFftTw<K>& w, const float2* __restrict__ tw, int t) {
  using S = BlockFft<K>;
  constexpr int step = 4096 / K;
  const int u = t % S::R;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    float2 x = tw[((t * k) % K) * step];
    float2 y = tw[((16 * u * k) % K) * step];
    if (SIGN < 0) { x.y = -x.y; y.y = -y.y; }
    w.a[k] = x;
    w.b[k] = y;
  }
}

// The same twiddles with stage B's taken from a workgroup table in LDS: they
// depend on u = t % R only, so R x 16 values serve every thread, and the 32
// registers they would hold stay free (for the next operands in flight).
template <int K>
struct BlockFftTwL {
  float2 a[16];
  const float2* bl;   // LDS row of this thread's u: bl[k] = W_K^(16 u k)
};
constexpr int kTwbStride = 17;   // odd row stride: the R rows' reads meet distinct banks
template <int K>
__host__ __device__ constexpr int block_fft_twb_size() { return (K / 256) * kTwbStride; }
// Fills the table (every thread of the workgroup calls it; a barrier must
// follow before the first block_fft) and this thread's stage-A twiddles.
template <int K, int SIGN>
__device__ __forceinline__ void block_fft_twiddles_lds(BlockFftTwL<K>& w, const float2* __restrict__ tw, int t,
                                                       float2* table) {
  using S = BlockFft<K>;
  constexpr int step = 4096 / K;
  for (int e = threadIdx.x; e < S::R * 16; e += 256) {
    const int u = e / 16, k = e % 16;
    float2 y = tw[((16 * u * k) % K) * step];
    if (SIGN < 0) y.y = -y.y;
    table[u * kTwbStride + k] = y;
  }
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    float2 x = tw[((t * k) % K) * step];
    if (SIGN < 0) x.y = -x.y;
    w.a[k] = x;
  }
  w.bl = table + (t % S::R) * kTwbStride;
}
// stage-B twiddle W_K^(16 u k) of either form
template <int K>
__device__ __forceinline__ float2 twb(const BlockFftTw<K>& w, int k) { return w.b[k]; }
template <int K>
__device__ __forceinline__ float2 twb(const BlockFftTwL<K>& w, int k) { return w.bl[k]; }

// Exchange barrier: one wave per FFT (K = 1024) needs only wave-level
// ordering of its LDS traffic, so the workgroup's four FFTs run
// independently; larger FFTs span waves and synchronise the workgroup.
template <int NTf>
__device__ __forceinline__ void block_fft_sync() {
  if constexpr (NTf <= 64) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// K-point DFT of v (thread t of its FFT holds x[t + NTf r] in v[r]) with
// sign SIGN.  On return v[e * R + s] holds X[out_index(t, e, s)].  All
// threads of the workgroup call it together (it synchronises).
template <int K, int SIGN, typename TW>
__device__ __forceinline__ void block_fft_after_a(float2 (&v)[16], float2* buf, int t, const TW& w);

template <int K, int SIGN, typename TW>
__device__ __forceinline__ void block_fft(float2 (&v)[16], float2* buf, int t, const TW& w) {
  dft16<SIGN>(v);      // stage A: radix 16 over r
  block_fft_after_a<K, SIGN>(v, buf, t, w);
}
// The rest of block_fft once stage A's radix-16 DFT is in v (a caller can
// form that DFT itself, e.g. with dft16_prod).
template <int K, int SIGN, typename TW>
__device__ __forceinline__ void block_fft_after_a(float2 (&v)[16], float2* buf, int t, const TW& w) {
  using S = BlockFft<K>;
  constexpr int NTf = S::NTf, R = S::R;
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    const int k1 = dft16_freq(s);
    buf[k1 * S::S1 + t] = k1 ? cmul(v[s], w.a[k1]) : v[s];
  }
  block_fft_sync<NTf>();
  // stage B: thread (k1, u) = (t / R, t % R), radix 16 over v of t' = u + R v
  {
    const int k1 = t / R, u = t % R;
#pragma unroll
    for (int q = 0; q < 16; ++q) v[q] = buf[k1 * S::S1 + u + R * q];
  }
  block_fft_sync<NTf>();
  dft16<SIGN>(v);
  {
    const int k1 = t / R, u = t % R;
    float2* row = buf + k1 * R + u;
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      const int k2 = dft16_freq(s);
      row[k2 * 16 * R + k2 / S::G] = k2 ? cmul(v[s], twb(w, k2)) : v[s];
    }
  }
  block_fft_sync<NTf>();
  // stage C: thread (k1, g) = (t / R, t % R) takes k2 = g G + e, radix R over u
  {
    const int k1 = t / R, g = t % R;
    const float2* row = buf + (g * S::G * 16 + k1) * R + g;
#pragma unroll
    for (int e = 0; e < S::G; ++e) {
#pragma unroll
      for (int u = 0; u < R; ++u) v[e * R + u] = row[e * 16 * R + u];
    }
  }
  block_fft_sync<NTf>();
  dft_r<R, SIGN>(v);
}

// Output index of slot e * R + s of thread t after block_fft.
template <int K>
__device__ __forceinline__ int block_fft_out(int t, int e, int s) {
  using S = BlockFft<K>;
  const int k1 = t / S::R, g = t % S::R;
  const int k2 = g * (16 / S::R) + e;
  return k1 + 16 * k2 + 256 * dftr_freq<S::R>(s);
}

}  // namespace rfd
