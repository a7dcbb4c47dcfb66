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
// rho^2 wins and exact ties go to the lowest sample.  A key whose rho^2 does
// not exceed threshold^2 cannot be a reported peak and is not written (its
// window's slot stays 0 unless a sample above the threshold arrives).  No
// series reaches HBM.
#include "dev_common.h"
#include "rfd_internal.h"

#include <algorithm>
#include <bitset>
#include <cstring>

namespace rfd {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(8))) _Float16 f16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;

// tap groups (8 complex taps, 64 real products) per FP32 MFMA accumulation chunk
constexpr int kFir32Chunk = 4;
// column blocks per wave of the FP32 form: its running sums and chunk partials
// are two accumulator sets, and 8 blocks keep both within three waves per SIMD
// (16 blocks needed 276 registers: one wave per SIMD, 37% slower)
constexpr int kFir32Nb = 8;

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
  int64_t m_off = 0;        // first output sample of the launch (range filtering)
  uint32_t thr2_bits = 0;   // bits of threshold^2: keys at or below it never fire, so are not written
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
        if (va && (uint32_t)(ka >> 32) > a.thr2_bits) atomicMax(sa + q, ka);
        if (vb && (uint32_t)(kb >> 32) > a.thr2_bits) atomicMax(sb + q, kb);
      }
    } else {
      if (va && (uint32_t)(ka >> 32) > a.thr2_bits) atomicMax(sa + q, ka);
      if (vb && (uint32_t)(kb >> 32) > a.thr2_bits) atomicMax(sb + q, kb);
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
    if (ta < a.count && (uint32_t)(ka >> 32) > a.thr2_bits) atomicMax(sa, ka);
    if (ta + 1 < a.count && (uint32_t)(kb >> 32) > a.thr2_bits) atomicMax(sa + a.nwin, kb);
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

// One workgroup's work: S tiles of 16*NB samples from mbase, for the 4 template
// blocks tb0..tb0+3 (8 templates per wave).  All threads must call it.
template <bool BF16, int NB>
__device__ __forceinline__ void fir16_block(const FirArgs& a, int64_t mbase, int64_t tb0, uint32_t* win) {
  constexpr int kColsPerTile = 16 * NB;
  const int Lw = a.S * kColsPerTile + a.Tp;
  uint32_t* whi = win;
  uint32_t* wlo = win + Lw;
  const int64_t nm = a.n - 1;
  load_window(whi, a.zhi, mbase + a.k0, Lw, nm);
  load_window(wlo, a.zlo, mbase + a.k0, Lw, nm);
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t tb = tb0 + wave;
  if (tb * kTmplPerWave >= a.count) return;   // wave-uniform; no barrier follows
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

// three waves per SIMD at 8 column blocks: 158 registers, none spilled (180
// and two waves without the bound); 16 blocks need more than a third of the
// register file and keep the compiler's own allocation
template <bool BF16, int NB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(NB <= 8 ? 3 : 1))) void k_fir16(FirArgs a) {
  extern __shared__ __align__(16) uint32_t win[];
  fir16_block<BF16, NB>(a, a.m_off + (int64_t)blockIdx.x * a.S * 16 * NB, (int64_t)blockIdx.y * kWavesPerBlock, win);
}

// FP32: v_mfma_f32_16x16x4f32, K step = 2 complex taps; B read from LDS.
template <int NB>
__device__ __forceinline__ void fir32_block(const FirArgs& a, int64_t mbase, int64_t tb0, float2* wz) {
  constexpr int kColsPerTile = 16 * NB;
  const int Lw = a.S * kColsPerTile + a.Tp;
  load_window(wz, a.z32, mbase + a.k0, Lw, a.n - 1);
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t tb = tb0 + wave;
  if (tb * kTmplPerWave >= a.count) return;   // wave-uniform; no barrier follows
  const float4* A = a.pa32 + tb * (int64_t)(a.Tp / 8) * 64 + lane;
  const int KQ = a.Tp / 8;
  PeakState ps;
  ps.ka = ps.kb = 0;
  ps.q = mbase / a.W;
  ps.qW = ps.q * a.W;
  ps.one_window = ps.q == ((mbase + (int64_t)a.S * kColsPerTile - 1) / a.W);
  for (int t = 0; t < a.S; ++t) {
    const float* wf = reinterpret_cast<const float*>(wz + t * kColsPerTile) + 2 * (lane & 15) + (lane >> 4);
    // The K sweep runs in chunks of kFir32Chunk tap groups (8 complex taps,
    // 16 real products each): every chunk accumulates from zero in the MFMA
    // and is then added to the running sum with a rounded FP32 add.  One
    // accumulator over all 2T products lets its rounding error grow with the
    // sweep length (measured 2.2e-5 in rho at T = 1024); chunks bound the
    // MFMA's share to 64 products.
    f32x4 acc[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i) acc[i] = f32x4{0.f, 0.f, 0.f, 0.f};
    float4 av = A[0];
    for (int c0 = 0; c0 < KQ; c0 += kFir32Chunk) {
      const int c1 = c0 + kFir32Chunk < KQ ? c0 + kFir32Chunk : KQ;
      f32x4 part[NB];
#pragma unroll
      for (int i = 0; i < NB; ++i) part[i] = f32x4{0.f, 0.f, 0.f, 0.f};
      for (int kq = c0; kq < c1; ++kq) {
        const float4 an = A[(int64_t)(kq + 1 < KQ ? kq + 1 : kq) * 64];
        const float avs[4] = {av.x, av.y, av.z, av.w};
#pragma unroll
        for (int sub = 0; sub < 4; ++sub) {
          const int kb2 = 4 * kq + sub;
#pragma unroll
          for (int nb = 0; nb < NB; ++nb) {
            const float bv = wf[32 * nb + 4 * kb2];
            part[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(avs[sub], bv, part[nb], 0, 0, 0);
          }
        }
        av = an;
      }
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) acc[nb] += part[nb];
    }
    fir_tile_epilogue<NB>(acc, a, mbase + (int64_t)t * kColsPerTile, tb, ps);
  }
  fir_final_epilogue(a, tb, ps);
}

template <int NB>
__global__ __launch_bounds__(256) void k_fir32(FirArgs a) {
  extern __shared__ __align__(16) float2 wz[];
  fir32_block<NB>(a, a.m_off + (int64_t)blockIdx.x * a.S * 16 * NB, (int64_t)blockIdx.y * kWavesPerBlock, wz);
}

// ------------------------------------------------------------ persistent
// One launch for every sub-bank: a fixed grid of workgroups pulls work items
// (sub-bank, template tile of 32, group of S tiles) from a global counter.
// Items are ordered heaviest sub-bank first (n_b * T_b), and within a
// sub-bank sample groups fastest, so concurrent workgroups share the same
// template tile's taps in L2 and the short items fill the tail.
struct PersistArgs {
  FirArgs base;                 // n, nwin, W, slots
  const int64_t* it_off;        // [nsb+1] first item of each (sorted) sub-bank
  const int32_t* it_sb;         // sorted position -> sub-bank
  const int32_t* it_S;          // tiles per item
  const int64_t* it_nsg;        // sample groups per template tile
  const int64_t* sb_first;      // global index of the first template
  const int32_t* sb_meta;       // ref_id, T, Tp, k0
  const int64_t* sb_p16;        // packed 16-bit operand base (uint4)
  const int64_t* sb_p32;        // packed FP32 operand base (float4)
  const int64_t* sb_count;
  const uint32_t* zhi_all;      // slot-major planes
  const uint32_t* zlo_all;
  const float2* z32_all;
  const uint4* pa16_all;
  const float4* pa32_all;
  unsigned long long* counter;
  int64_t total;
  int nsb;
  int cols;
};

__device__ __forceinline__ bool next_item(const PersistArgs& pa, FirArgs& a, int64_t& mbase, int64_t& tb0) {
  __shared__ long long s_item;
  __syncthreads();                                  // previous item's LDS reads are done
  if (threadIdx.x == 0) s_item = (long long)atomicAdd(pa.counter, 1ull);
  __syncthreads();
  const int64_t w = s_item;
  if (w >= pa.total) return false;
  int lo = 0, hi = pa.nsb - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (pa.it_off[mid] <= w) lo = mid; else hi = mid - 1;
  }
  const int b = pa.it_sb[lo];
  const int64_t rem = w - pa.it_off[lo];
  const int64_t nsg = pa.it_nsg[lo];
  const int64_t tt = rem / nsg, sg = rem - tt * nsg;
  a = pa.base;
  const int ref = pa.sb_meta[4 * b + 0];
  a.Tp = pa.sb_meta[4 * b + 2];
  a.k0 = pa.sb_meta[4 * b + 3];
  a.KB = a.Tp / 16;
  a.S = pa.it_S[lo];
  a.count = pa.sb_count[b];
  a.tmpl0 = pa.sb_first[b];
  a.zhi = pa.zhi_all + (int64_t)ref * a.n;
  a.zlo = pa.zlo_all + (int64_t)ref * a.n;
  a.z32 = pa.z32_all + (int64_t)ref * a.n;
  a.pa16 = pa.pa16_all + pa.sb_p16[b];
  a.pa32 = pa.pa32_all + pa.sb_p32[b];
  mbase = sg * a.S * pa.cols;
  tb0 = tt * kWavesPerBlock;
  return true;
}

// (bounded to three waves per SIMD like k_fir16 it spills per-item values to
// scratch and measured no faster at ecc512s: left at two)
template <bool BF16, int NB>
__global__ __launch_bounds__(256) void k_fir16_persistent(PersistArgs pa) {
  extern __shared__ __align__(16) uint32_t win[];
  FirArgs a;
  int64_t mbase, tb0;
  while (next_item(pa, a, mbase, tb0)) fir16_block<BF16, NB>(a, mbase, tb0, win);
}

template <int NB>
__global__ __launch_bounds__(256) void k_fir32_persistent(PersistArgs pa) {
  extern __shared__ __align__(16) float2 wz[];
  FirArgs a;
  int64_t mbase, tb0;
  while (next_item(pa, a, mbase, tb0)) fir32_block<NB>(a, mbase, tb0, wz);
}

__global__ void k_zero_counter(unsigned long long* c) { *c = 0ull; }

// 16-bit hi/lo planes (x = hi + lo, each part rounded to the format) of the
// FP32 reference series of one slot over samples [start, start + len) mod N:
// word (re) | (im << 16) per sample, as the Hankel windows read them.
template <bool BF16>
__global__ __launch_bounds__(256) void k_ref_planes(const float2* __restrict__ z, int64_t n, int64_t start,
                                                    int64_t len, uint32_t* __restrict__ hi,
                                                    uint32_t* __restrict__ lo) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < len; i += (int64_t)gridDim.x * 256) {
    const int64_t m = (start + i) & (n - 1);
    const float2 v = z[m];
    uint32_t rh, rl, ih, il;
    if (BF16) {
      split_bf16(v.x, rh, rl);
      split_bf16(v.y, ih, il);
    } else {
      split_f16(v.x, rh, rl);
      split_f16(v.y, ih, il);
    }
    hi[m] = (rh & 0xffffu) | (ih << 16);
    lo[m] = (rl & 0xffffu) | (il << 16);
  }
}

// Planes of reference slot `ref` for the 16-bit form `precision`, over the
// samples a FIR launch reads: [start, start + len) mod N (len >= N: all).
static int launch_ref_planes(Plan& p, int precision, int ref, int64_t start, int64_t len) {
  const bool bf = precision == RFD_BF16X3;
  const int64_t o = (int64_t)ref * p.n;
  uint32_t* hi = (bf ? p.zbf_hi : p.zh_hi) + o;
  uint32_t* lo = (bf ? p.zbf_lo : p.zh_lo) + o;
  if (len >= p.n) {
    start = 0;
    len = p.n;
  }
  start &= p.n - 1;
  const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((len + 255) / 256, 4096));
  if (bf) hipLaunchKernelGGL(k_ref_planes<true>, dim3((unsigned)blocks), dim3(256), 0, p.stream, p.zref + o, p.n, start, len, hi, lo);
  else hipLaunchKernelGGL(k_ref_planes<false>, dim3((unsigned)blocks), dim3(256), 0, p.stream, p.zref + o, p.n, start, len, hi, lo);
  RFD_CHECK_LAUNCH();
  return RFD_OK;
}

// Tiles per workgroup: one workgroup covers a whole cluster window when W is
// a multiple of 256 (so each (template, window) peak gets one update), capped
// at 8 tiles; otherwise 4 tiles.
static int tiles_per_block(int64_t n, int64_t W, int cols, int smax_cfg) {
  const int smax = std::max(1, std::min(2048 / cols, smax_cfg));
  int S = (W % cols == 0) ? (int)std::min<int64_t>(W / cols, smax) : std::max(1, smax / 2);
  while (S > 1 && (n % ((int64_t)S * cols)) != 0) S >>= 1;
  return S < 1 ? 1 : S;
}

static uint32_t thr2_bits(float threshold) {
  const float t2 = threshold * threshold;     // as the compaction compares
  uint32_t b;
  std::memcpy(&b, &t2, sizeof(b));
  return b;
}

int launch_fir(Plan& p, const Taps& tp, int b, int precision, int64_t W, int64_t nwin, float threshold,
               int64_t n_start, int64_t n_len) {
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
  a.thr2_bits = thr2_bits(threshold);
  a.k0 = s.k0;
  a.Tp = s.Tp;
  a.KB = s.Tp / 16;
  // column blocks per wave: FP32 kFir32Nb; 16-bit forms the tile config knob (8 by default)
  const int nb = precision == RFD_FP32 ? kFir32Nb : p.fir_nb16;
  const int cols = 16 * nb;
  if (n_len < 0) {             // the whole segment
    n_start = 0;
    n_len = p.n;
  }
  a.S = tiles_per_block(n_len, W, cols, p.fir_smax);
  while (a.S > 1 && n_start % ((int64_t)a.S * cols) != 0) a.S >>= 1;
  a.m_off = n_start;
  dim3 grid((unsigned)(n_len / ((int64_t)a.S * cols)), (unsigned)((s.count + kTmplTile - 1) / kTmplTile));
  const int Lw = a.S * cols + s.Tp;
  int rc = stage_begin(p, kStFirKernel);
  if (rc) return rc;
  if (precision != RFD_FP32) {
    // the windows read samples [n_start + k0, n_start + n_len + k0 + Tp)
    rc = launch_ref_planes(p, precision, s.ref_id, n_start + s.k0 + p.n, n_len + s.Tp);
    if (rc) return rc;
  }
  if (precision == RFD_FP32) {
    hipLaunchKernelGGL(k_fir32<kFir32Nb>, grid, dim3(256), (size_t)Lw * sizeof(float2), p.stream, a);
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
  return stage_end(p);
}

}  // namespace rfd

namespace rfd {

static int fir_cols(const Plan& p, int precision) { return 16 * (precision == RFD_FP32 ? kFir32Nb : p.fir_nb16); }

template <typename K>
static int persistent_grid(Plan& p, K kernel, size_t lds, int64_t total) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 256, lds) != hipSuccess || per_cu < 1) per_cu = 1;
  if (p.fir_wg_per_cu > 0) per_cu = std::min(per_cu, p.fir_wg_per_cu);
  int64_t g = (int64_t)per_cu * std::max(p.n_cu, 1);
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, total));
}

int prepare_fir_items(Plan& p, Taps& tp, int precision, int64_t W) {
  const int cols = fir_cols(p, precision);
  if (tp.it_key_W == W && tp.it_key_cols == cols && tp.it_key_smax == p.fir_smax && tp.it_key_prec == precision &&
      tp.it_key_wg == p.fir_wg_per_cu)
    return RFD_OK;
  ++tp.res_gen;   // the tables below are reallocated
  const int nsb = (int)tp.sb.size();
  std::vector<int> order;
  for (int b = 0; b < nsb; ++b)
    if (tp.sb[b].count > 0) order.push_back(b);
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
    return tp.sb[x].count * tp.sb[x].Tp > tp.sb[y].count * tp.sb[y].Tp;
  });
  const int m = (int)order.size();
  std::vector<int64_t> off(m + 1, 0), nsg(std::max(m, 1), 0);
  std::vector<int32_t> S(std::max(m, 1), 1), sbv(std::max(m, 1), 0);
  size_t lds = 0;
  for (int j = 0; j < m; ++j) {
    const SubBankTaps& s = tp.sb[order[j]];
    S[j] = tiles_per_block(p.n, W, cols, p.fir_smax);
    nsg[j] = p.n / ((int64_t)S[j] * cols);
    sbv[j] = order[j];
    off[j + 1] = off[j] + nsg[j] * ((s.count + kTmplTile - 1) / kTmplTile);
    const size_t win = (size_t)(S[j] * cols + s.Tp) * (precision == RFD_FP32 ? sizeof(float2) : 2 * sizeof(uint32_t));
    lds = std::max(lds, win);
  }
  auto up = [&](auto*& dst, const auto& src, size_t n) -> int {
    if (dst) { (void)hipFree(dst); dst = nullptr; }
    if (device_malloc((void**)&dst, std::max<size_t>(n, 1) * sizeof(src[0])) != hipSuccess)
      return fail(RFD_E_NOMEM, "work-item table allocation failed");
    if (n && hipMemcpy(dst, src.data(), n * sizeof(src[0]), hipMemcpyHostToDevice) != hipSuccess)
      return fail(RFD_E_DEVICE, "work-item table upload failed");
    return RFD_OK;
  };
  int rc;
  if ((rc = up(tp.d_it_off, off, m + 1))) return rc;
  if ((rc = up(tp.d_it_sb, sbv, m))) return rc;
  if ((rc = up(tp.d_it_S, S, m))) return rc;
  if ((rc = up(tp.d_it_nsg, nsg, m))) return rc;
  tp.it_total = off[m];
  tp.it_nsb = m;
  tp.it_lds = lds;
  const bool f16 = precision == RFD_FP16X3;
  if (precision == RFD_FP32)
    tp.it_grid = persistent_grid(p, k_fir32_persistent<kFir32Nb>, lds, tp.it_total);
  else if (p.fir_nb16 == 16)
    tp.it_grid = persistent_grid(p, f16 ? k_fir16_persistent<false, 16> : k_fir16_persistent<true, 16>, lds, tp.it_total);
  else
    tp.it_grid = persistent_grid(p, f16 ? k_fir16_persistent<false, 8> : k_fir16_persistent<true, 8>, lds, tp.it_total);
  tp.it_key_W = W;
  tp.it_key_cols = cols;
  tp.it_key_smax = p.fir_smax;
  tp.it_key_prec = precision;
  tp.it_key_wg = p.fir_wg_per_cu;
  return RFD_OK;
}

int launch_fir_persistent(Plan& p, const Taps& tp, int precision, int64_t W, int64_t nwin, float threshold) {
  if (tp.it_total == 0) return RFD_OK;
  PersistArgs pa;
  FirArgs& a = pa.base;
  a.zhi = a.zlo = nullptr;
  a.z32 = nullptr;
  a.pa16 = nullptr;
  a.pa32 = nullptr;
  a.slots = p.slots;
  a.n = p.n;
  a.count = 0;
  a.tmpl0 = 0;
  a.nwin = nwin;
  a.W = W;
  a.thr2_bits = thr2_bits(threshold);
  a.k0 = a.Tp = a.KB = 0;
  a.S = 1;
  pa.it_off = tp.d_it_off;
  pa.it_sb = tp.d_it_sb;
  pa.it_S = tp.d_it_S;
  pa.it_nsg = tp.d_it_nsg;
  pa.sb_first = tp.d_first;
  pa.sb_meta = tp.d_meta;
  pa.sb_p16 = tp.d_p16;
  pa.sb_p32 = tp.d_p32;
  pa.sb_count = tp.d_count;
  const bool f16 = precision == RFD_FP16X3;
  pa.zhi_all = f16 ? p.zh_hi : p.zbf_hi;
  pa.zlo_all = f16 ? p.zh_lo : p.zbf_lo;
  pa.z32_all = p.zref;
  pa.pa16_all = f16 ? tp.pfh : tp.pbf;
  pa.pa32_all = tp.p32;
  pa.counter = p.counter;
  pa.total = tp.it_total;
  pa.nsb = tp.it_nsb;
  pa.cols = fir_cols(p, precision);
  hipLaunchKernelGGL(k_zero_counter, dim3(1), dim3(1), 0, p.stream, p.counter);
  RFD_CHECK_LAUNCH();
  if (tp.it_key_prec != precision || tp.it_key_W != W || tp.it_key_cols != pa.cols)
    return fail(RFD_E_STATE, "persistent FIR work items were prepared for another configuration");
  const size_t lds = tp.it_lds;
  const dim3 grid(tp.it_grid);
  int rc = stage_begin(p, kStFirKernel);
  if (rc) return rc;
  if (precision != RFD_FP32) {
    std::bitset<kMaxRefSlots> done;     // reference slots already split
    for (const SubBankTaps& s : tp.sb) {
      if (s.count == 0 || done[s.ref_id]) continue;
      done[s.ref_id] = true;
      if ((rc = launch_ref_planes(p, precision, s.ref_id, 0, p.n))) return rc;
    }
  }
  if (precision == RFD_FP32) {
    hipLaunchKernelGGL(k_fir32_persistent<kFir32Nb>, grid, dim3(256), lds, p.stream, pa);
  } else if (p.fir_nb16 == 16) {
    if (f16) hipLaunchKernelGGL((k_fir16_persistent<false, 16>), grid, dim3(256), lds, p.stream, pa);
    else hipLaunchKernelGGL((k_fir16_persistent<true, 16>), grid, dim3(256), lds, p.stream, pa);
  } else {
    if (f16) hipLaunchKernelGGL((k_fir16_persistent<false, 8>), grid, dim3(256), lds, p.stream, pa);
    else hipLaunchKernelGGL((k_fir16_persistent<true, 8>), grid, dim3(256), lds, p.stream, pa);
  }
  RFD_CHECK_LAUNCH();
  return stage_end(p);
}

}  // namespace rfd
