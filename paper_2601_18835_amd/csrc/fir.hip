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

// Epilogue over NB 16x16 accumulator blocks of one wave.
// acc[nb][i]: rows 4*(lane>>4)+i, column lane&15 of block nb.
template <int NB>
__device__ __forceinline__ void fir_epilogue(const f32x4 (&acc)[NB], const FirArgs& a, int64_t m0, int64_t tb) {
  const int lane = threadIdx.x & 63;
  const int n = lane & 15, g = lane >> 4;
  const int64_t ta = tb * 8 + 2 * g;          // templates ta, ta+1 (within the sub-bank)
  const bool va = ta < a.count, vb = ta + 1 < a.count;
  unsigned long long* sa = a.slots + (a.tmpl0 + ta) * a.nwin;
  unsigned long long* sb = sa + a.nwin;
  const int64_t W = a.W;
  if (m0 / W == (m0 + 16 * NB - 1) / W) {
    // whole tile inside one window
    unsigned long long ka = 0, kb = 0;
    int64_t q = 0;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int64_t s = m0 + 16 * nb + n;
      float r2a = acc[nb][0] * acc[nb][0] + acc[nb][1] * acc[nb][1];
      float r2b = acc[nb][2] * acc[nb][2] + acc[nb][3] * acc[nb][3];
      ka = umax64(ka, peak_key(r2a, s, W, q));
      kb = umax64(kb, peak_key(r2b, s, W, q));
    }
    ka = reduce16(ka);
    kb = reduce16(kb);
    if (n == 0) {
      if (va) atomicMax(sa + q, ka);
      if (vb) atomicMax(sb + q, kb);
    }
    return;
  }
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

template <bool BF16>
__global__ __launch_bounds__(256) void k_fir16(FirArgs a) {
  constexpr int NB = kColBlocks;
  extern __shared__ __align__(16) uint32_t win[];
  const int Lw = kColsPerTile + a.Tp;
  uint32_t* whi = win;
  uint32_t* wlo = win + Lw;
  const int64_t m0 = (int64_t)blockIdx.x * kColsPerTile;
  const int64_t nm = a.n - 1;
  for (int p = threadIdx.x; p < Lw; p += 256) {
    int64_t s = (m0 + a.k0 + p) & nm;
    whi[p] = a.zhi[s];
    wlo[p] = a.zlo[s];
  }
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t tb = (int64_t)blockIdx.y * kWavesPerBlock + wave;
  if (tb * kTmplPerWave >= a.count) return;
  const int off = (lane & 15) + 4 * (lane >> 4);

  f32x4 acc[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) acc[i] = f32x4{0.f, 0.f, 0.f, 0.f};
  uint4 rh[NB], rl[NB];
#pragma unroll
  for (int s = 0; s < NB - 1; ++s) {
    rh[s] = lds4(whi + 16 * s + off);
    rl[s] = lds4(wlo + 16 * s + off);
  }
  const uint4* A = a.pa16 + tb * (int64_t)a.KB * 128 + lane;
  for (int kb0 = 0; kb0 < a.KB; kb0 += NB) {
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int kb = kb0 + u;
      if (kb < a.KB) {
        const int sn = kb + NB - 1;
        rh[(u + NB - 1) % NB] = lds4(whi + 16 * sn + off);
        rl[(u + NB - 1) % NB] = lds4(wlo + 16 * sn + off);
        const uint4 ah = A[(int64_t)kb * 128];
        const uint4 al = A[(int64_t)kb * 128 + 64];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          const int sl = (u + nb) % NB;
          acc[nb] = mfma16<BF16>(ah, rh[sl], acc[nb]);
          acc[nb] = mfma16<BF16>(ah, rl[sl], acc[nb]);
          acc[nb] = mfma16<BF16>(al, rh[sl], acc[nb]);
        }
      }
    }
  }
  fir_epilogue<NB>(acc, a, m0, tb);
}

// FP32: v_mfma_f32_16x16x4f32, K step = 2 complex taps; B read from LDS.
__global__ __launch_bounds__(256) void k_fir32(FirArgs a) {
  constexpr int NB = kColBlocks;
  extern __shared__ __align__(16) float2 wz[];
  const int Lw = kColsPerTile + a.Tp;
  const int64_t m0 = (int64_t)blockIdx.x * kColsPerTile;
  const int64_t nm = a.n - 1;
  for (int p = threadIdx.x; p < Lw; p += 256) wz[p] = a.z32[(m0 + a.k0 + p) & nm];
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t tb = (int64_t)blockIdx.y * kWavesPerBlock + wave;
  if (tb * kTmplPerWave >= a.count) return;
  const float* wf = reinterpret_cast<const float*>(wz) + 2 * (lane & 15) + (lane >> 4);
  f32x4 acc[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) acc[i] = f32x4{0.f, 0.f, 0.f, 0.f};
  const float4* A = a.pa32 + tb * (int64_t)(a.Tp / 8) * 64 + lane;
  const int KQ = a.Tp / 8;
  for (int kq = 0; kq < KQ; ++kq) {
    const float4 av = A[(int64_t)kq * 64];
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
  }
  fir_epilogue<NB>(acc, a, m0, tb);
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
  dim3 grid((unsigned)(p.n / kColsPerTile), (unsigned)((s.count + kTmplTile - 1) / kTmplTile));
  if (precision == RFD_FP32) {
    size_t sh = (size_t)(kColsPerTile + s.Tp) * sizeof(float2);
    hipLaunchKernelGGL(k_fir32, grid, dim3(256), sh, p.stream, a);
  } else {
    size_t sh = (size_t)2 * (kColsPerTile + s.Tp) * sizeof(uint32_t);
    if (precision == RFD_BF16X3)
      hipLaunchKernelGGL(k_fir16<true>, grid, dim3(256), sh, p.stream, a);
    else
      hipLaunchKernelGGL(k_fir16<false>, grid, dim3(256), sh, p.stream, a);
  }
  RFD_CHECK_LAUNCH();
  return RFD_OK;
}

}  // namespace rfd
