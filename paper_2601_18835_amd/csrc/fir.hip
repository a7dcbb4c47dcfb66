// Ratio FIR (Eq. 3) as a complex GEMM on MFMA with a fused epilogue.
//
// For template j of a sub-bank with taps c_j[0..T) at lag offset k0:
//     z_j[n] = sum_k c_j[k] zhat[(n + k0 + k) mod N].
// Per workgroup tile (32 templates x 256 output samples starting at m0):
//     Y[r, m] = sum_kappa A[r, kappa] H[kappa, m],  H = Hankel window of zhat,
// in real form with kappa = 2k + comp and two rows per template:
//     row 2t   (Re z_t): ( Re c,  -Im c ) . ( Re zhat, Im zhat )
//     row 2t+1 (Im z_t): ( Im c,   Re c ) . ( Re zhat, Im zhat ).
// The window zhat[m0 + k0 + p], p < 256 + Tp, is staged once in LDS.
//
// 16-bit forms (x = hi + lo, FP32 accumulation of hi*hi + hi*lo + lo*hi) use
// v_mfma_f32_16x16x32_{bf16,f16}.  A Hankel operand depends on (column block
// + K block) only, so a wave sweeping 16 column blocks keeps a ring of 16 B
// operands in registers and loads ONE new operand (per plane) per K step.
// The A operands (taps) are pre-packed in MFMA lane order, one coalesced 16 B
// load per lane per plane per K step.
//
// Epilogue: rho^2 = Re^2 + Im^2 in registers; per (template, window) the key
// (bits(rho^2) << 32) | (0xFFFFFFFF - offset in window) is reduced across the
// wave and merged into the slot array with a 64-bit atomicMax, so the largest
// rho^2 wins and exact ties go to the lowest sample.  No series reaches HBM.
#include "dev_common.h"
#include "rfd_internal.h"

#include <algorithm>

namespace rfd {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(8))) _Float16 f16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;

struct FirArgs {
  const uint32_t* zhi;      // 16-bit planes of the reference slot ((re) | (im << 16))
  const uint32_t* zlo;
  const float2* z32;        // FP32 normalised series
  const uint4* pa16;        // packed 16-bit A operands of this sub-bank
  const float4* pa32;       // packed FP32 A operands of this sub-bank
  unsigned long long* slots;
  int64_t n;                // N (power of two)
  int64_t count;            // templates in the sub-bank
  int64_t tmpl0;            // global index of its first template
  int64_t nwin, W;
  int k0, Tp, KB;           // Tp = taps padded to 16, KB = Tp / 16
  int S;                    // 256-sample tiles swept by one workgroup
};

__device__ __forceinline__ unsigned long long peak_key(float r2, int64_t n, int64_t W, int64_t& q) {
  q = n / W;
  return ((unsigned long long)__float_as_uint(r2) << 32) |
         (unsigned long long)(0xFFFFFFFFu - (uint32_t)(n - q * W));
}

__device__ __forceinline__ unsigned long long umax64(unsigned long long a, unsigned long long b) {
  return a > b ? a : b;
}

// Reduce over the 16 lanes that share lane>>4 (the MFMA column index).
__device__ __forceinline__ unsigned long long reduce16(unsigned long long k) {
#pragma unroll
  for (int o = 1; o < 16; o <<= 1) k = umax64(k, __shfl_xor(k, o));
  return k;
}

// Window-peak bookkeeping of one wave over the tiles of its workgroup.
// acc[nb][i]: rows 4*(lane>>4)+i, column lane&15 of 16x16 block nb, i.e.
// templates 2g (rows 0,1 = Re, Im) and 2g+1 (rows 2,3), g = lane>>4.
struct PeakState {
  unsigned long long ka, kb;   // running keys when the whole range is one window
  bool one_window;
  int64_t q;                   // that window (uniform)
  int64_t qW;                  // its first sample
};

__device__ __forceinline__ unsigned long long offset_key(float r2, uint32_t off) {
  return ((unsigned long long)__float_as_uint(r2) << 32) | (unsigned long long)(0xFFFFFFFFu - off);
}

template <int NB>
__device__ __forceinline__ void fir_tile_epilogue(const f32x4 (&acc)[NB], const FirArgs& a, int64_t m0, int64_t tb,
                                                  PeakState& ps) {
  const int lane = threadIdx.x & 63;
  const int n = lane & 15, g = lane >> 4;
  const int64_t ta = tb * 8 + 2 * g;          // templates ta, ta+1 (within the sub-bank)
  const int64_t W = a.W;
  if (ps.one_window) {
    const uint32_t base = (uint32_t)(m0 - ps.qW) + (uint32_t)n;   // offset within the window
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      float r2a = acc[nb][0] * acc[nb][0] + acc[nb][1] * acc[nb][1];
      float r2b = acc[nb][2] * acc[nb][2] + acc[nb][3] * acc[nb][3];
      ps.ka = umax64(ps.ka, offset_key(r2a, base + 16u * nb));
      ps.kb = umax64(ps.kb, offset_key(r2b, base + 16u * nb));
    }
    return;
  }
  const bool va = ta < a.count, vb = ta + 1 < a.count;
  unsigned long long* sa = a.slots + (a.tmpl0 + ta) * a.nwin;
  unsigned long long* sb = sa + a.nwin;
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    const int64_t c0 = m0 + 16 * nb;
    const int64_t s = c0 + n;
    float r2a = acc[nb][0] * acc[nb][0] + acc[nb][1] * acc[nb][1];
    float r2b = acc[nb][2] * acc[nb][2] + acc[nb][3] * acc[nb][3];
    int64_t q;
    unsigned long long ka = peak_key(r2a, s, W, q);
    unsigned long long kb = peak_key(r2b, s, W, q);
    if (c0 / W == (c0 + 15) / W) {
      ka = reduce16(ka);
      kb = reduce16(kb);
      if (n == 0) {
        if (va) atomicMax(sa + q, ka);
        if (vb) atomicMax(sb + q, kb);
      }
    } else {
      if (va) atomicMax(sa + q, ka);
      if (vb) atomicMax(sb + q, kb);
    }
  }
}

__device__ __forceinline__ void fir_final_epilogue(const FirArgs& a, int64_t tb, PeakState& ps) {
  if (!ps.one_window) return;
  const int lane = threadIdx.x & 63;
  const int64_t ta = tb * 8 + 2 * (lane >> 4);
  unsigned long long ka = reduce16(ps.ka), kb = reduce16(ps.kb);
  if ((lane & 15) == 0) {
    unsigned long long* sa = a.slots + (a.tmpl0 + ta) * a.nwin + ps.q;
    if (ta < a.count) atomicMax(sa, ka);
    if (ta + 1 < a.count) atomicMax(sa + a.nwin, kb);
  }
}

__device__ __forceinline__ uint4 lds4(const uint32_t* p) {
  uint4 v;
  v.x = p[0];
  v.y = p[1];
  v.z = p[2];
  v.w = p[3];
  return v;
}

template <bool BF16>
__device__ __forceinline__ f32x4 mfma16(uint4 a, uint4 b, f32x4 c) {
  if constexpr (BF16) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                  0, 0, 0);
  } else {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x8, b), c, 0,
                                                 0, 0);
  }
}

// Stage the workgroup's window zhat[m_start + k0 + p], p < S*256 + Tp, in LDS.
template <typename V>
__device__ __forceinline__ void load_window(V* dst, const V* __restrict__ src, int64_t start, int len, int64_t nm) {
  for (int p = threadIdx.x; p < len; p += 256) dst[p] = src[(start + p) & nm];
}

template <bool BF16, int NB>
__global__ __launch_bounds__(256) void k_fir16(FirArgs a) {
  constexpr int kColsPerTile = 16 * NB;
  extern __shared__ __align__(16) uint32_t win[];
  const int Lw = a.S * kColsPerTile + a.Tp;
  uint32_t* whi = win;
  uint32_t* wlo = win + Lw;
  const int64_t mbase = (int64_t)blockIdx.x * a.S * kColsPerTile;
  const int64_t nm = a.n - 1;
  load_window(whi, a.zhi, mbase + a.k0, Lw, nm);
  load_window(wlo, a.zlo, mbase + a.k0, Lw, nm);
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t tb = (int64_t)blockIdx.y * kWavesPerBlock + wave;
  if (tb * kTmplPerWave >= a.count) return;
  const int off = (lane & 15) + 4 * (lane >> 4);
  const uint4* A = a.pa16 + tb * (int64_t)a.KB * 128 + lane;
  PeakState ps;
  ps.ka = ps.kb = 0;
  ps.q = mbase / a.W;
  ps.qW = ps.q * a.W;
  ps.one_window = ps.q == ((mbase + (int64_t)a.S * kColsPerTile - 1) / a.W);

  const int F = a.KB / NB, R = a.KB % NB;
  for (int t = 0; t < a.S; ++t) {
    const uint32_t* th = whi + t * kColsPerTile + off;
    const uint32_t* tl = wlo + t * kColsPerTile + off;
    f32x4 acc[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i) acc[i] = f32x4{0.f, 0.f, 0.f, 0.f};
    uint4 rh[NB], rl[NB];
#pragma unroll
    for (int s = 0; s < NB - 1; ++s) {
      rh[s] = lds4(th + 16 * s);
      rl[s] = lds4(tl + 16 * s);
    }
    // tap operands of steps kb (a0) and kb+1 (a1); step kb prefetches kb+2
    const int k1 = a.KB > 1 ? 1 : 0;
    uint4 a0h = A[0], a0l = A[64], a1h = A[(int64_t)k1 * 128], a1l = A[(int64_t)k1 * 128 + 64];
    auto step = [&](const int kb, const int u) __attribute__((always_inline)) {
      const int sn = kb + NB - 1;
      rh[(u + NB - 1) % NB] = lds4(th + 16 * sn);
      rl[(u + NB - 1) % NB] = lds4(tl + 16 * sn);
      const int kn = kb + 2 < a.KB ? kb + 2 : a.KB - 1;
      const uint4 nh = A[(int64_t)kn * 128];
      const uint4 nl = A[(int64_t)kn * 128 + 64];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) acc[nb] = mfma16<BF16>(a0h, rh[(u + nb) % NB], acc[nb]);
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) acc[nb] = mfma16<BF16>(a0h, rl[(u + nb) % NB], acc[nb]);
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) acc[nb] = mfma16<BF16>(a0l, rh[(u + nb) % NB], acc[nb]);
      a0h = a1h;
      a0l = a1l;
      a1h = nh;
      a1l = nl;
    };
    // full chunks of NB steps: straight-line code, static ring slots
    for (int f = 0; f < F; ++f) {
#pragma unroll
      for (int u = 0; u < NB; ++u) step(f * NB + u, u);
    }
    // remaining KB mod NB steps
#pragma unroll
    for (int u = 0; u < NB - 1; ++u)
      if (u < R) step(F * NB + u, u);
    fir_tile_epilogue<NB>(acc, a, mbase + (int64_t)t * kColsPerTile, tb, ps);
  }
  fir_final_epilogue(a, tb, ps);
}

// FP32: v_mfma_f32_16x16x4f32, K step = 2 complex taps; B read from LDS.
template <int NB>
__global__ __launch_bounds__(256) void k_fir32(FirArgs a) {
  constexpr int kColsPerTile = 16 * NB;
  extern __shared__ __align__(16) float2 wz[];
  const int Lw = a.S * kColsPerTile + a.Tp;
  const int64_t mbase = (int64_t)blockIdx.x * a.S * kColsPerTile;
  load_window(wz, a.z32, mbase + a.k0, Lw, a.n - 1);
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t tb = (int64_t)blockIdx.y * kWavesPerBlock + wave;
  if (tb * kTmplPerWave >= a.count) return;
  const float4* A = a.pa32 + tb * (int64_t)(a.Tp / 8) * 64 + lane;
  const int KQ = a.Tp / 8;
  PeakState ps;
  ps.ka = ps.kb = 0;
  ps.q = mbase / a.W;
  ps.qW = ps.q * a.W;
  ps.one_window = ps.q == ((mbase + (int64_t)a.S * kColsPerTile - 1) / a.W);
  for (int t = 0; t < a.S; ++t) {
    const float* wf = reinterpret_cast<const float*>(wz + t * kColsPerTile) + 2 * (lane & 15) + (lane >> 4);
    f32x4 acc[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i) acc[i] = f32x4{0.f, 0.f, 0.f, 0.f};
    float4 av = A[0];
    for (int kq = 0; kq < KQ; ++kq) {
      const float4 an = A[(int64_t)(kq + 1 < KQ ? kq + 1 : kq) * 64];
      const float avs[4] = {av.x, av.y, av.z, av.w};
#pragma unroll
      for (int sub = 0; sub < 4; ++sub) {
        const int kb2 = 4 * kq + sub;
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          const float bv = wf[32 * nb + 4 * kb2];
          acc[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(avs[sub], bv, acc[nb], 0, 0, 0);
        }
      }
      av = an;
    }
    fir_tile_epilogue<NB>(acc, a, mbase + (int64_t)t * kColsPerTile, tb, ps);
  }
  fir_final_epilogue(a, tb, ps);
}

// Tiles per workgroup: one workgroup covers a whole cluster window when W is
// a multiple of 256 (so each (template, window) peak gets one update), capped
// at 8 tiles; otherwise 4 tiles.
static int tiles_per_block(int64_t n, int64_t W, int cols) {
  const int smax = 2048 / cols;
  int S = (W % cols == 0) ? (int)std::min<int64_t>(W / cols, smax) : std::max(1, smax / 2);
  while (S > 1 && (n % ((int64_t)S * cols)) != 0) S >>= 1;
  return S < 1 ? 1 : S;
}

int launch_fir(Plan& p, const Taps& tp, int b, int precision, int64_t W, int64_t nwin) {
  const SubBankTaps& s = tp.sb[b];
  if (s.count == 0) return RFD_OK;
  FirArgs a;
  int64_t o = (int64_t)s.ref_id * p.n;
  a.zhi = (precision == RFD_FP16X3 ? p.zh_hi : p.zbf_hi) + o;
  a.zlo = (precision == RFD_FP16X3 ? p.zh_lo : p.zbf_lo) + o;
  a.z32 = p.zref + o;
  a.pa16 = (precision == RFD_FP16X3 ? tp.pfh : tp.pbf) + s.p16_base;
  a.pa32 = tp.p32 + s.p32_base;
  a.slots = p.slots;
  a.n = p.n;
  a.count = s.count;
  a.tmpl0 = s.first;
  a.nwin = nwin;
  a.W = W;
  a.k0 = s.k0;
  a.Tp = s.Tp;
  a.KB = s.Tp / 16;
  // column blocks per wave: FP32 16; 16-bit forms 8 (tile config knob)
  const int nb = precision == RFD_FP32 ? 16 : p.fir_nb16;
  const int cols = 16 * nb;
  a.S = tiles_per_block(p.n, W, cols);
  dim3 grid((unsigned)(p.n / ((int64_t)a.S * cols)), (unsigned)((s.count + kTmplTile - 1) / kTmplTile));
  const int Lw = a.S * cols + s.Tp;
  if (precision == RFD_FP32) {
    hipLaunchKernelGGL(k_fir32<16>, grid, dim3(256), (size_t)Lw * sizeof(float2), p.stream, a);
  } else {
    size_t sh = (size_t)2 * Lw * sizeof(uint32_t);
    const bool bf = precision == RFD_BF16X3;
    if (nb == 16) {
      if (bf) hipLaunchKernelGGL((k_fir16<true, 16>), grid, dim3(256), sh, p.stream, a);
      else hipLaunchKernelGGL((k_fir16<false, 16>), grid, dim3(256), sh, p.stream, a);
    } else {
      if (bf) hipLaunchKernelGGL((k_fir16<true, 8>), grid, dim3(256), sh, p.stream, a);
      else hipLaunchKernelGGL((k_fir16<false, 8>), grid, dim3(256), sh, p.stream, a);
    }
  }
  RFD_CHECK_LAUNCH();
  return RFD_OK;
}

}  // namespace rfd
