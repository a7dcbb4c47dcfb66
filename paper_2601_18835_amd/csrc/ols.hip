// Ratio FIR of Eq. 3 by overlap-save block convolution in the frequency
// domain: the paper's own realisation of the short filter (blocks of K
// samples, K a small power of two, FFT-based), here on one workgroup per
// group of blocks.
//
// With L = K - T + 1 valid outputs per block, block b's input is
//   x_b[m] = zhat[(b L + k0 + m) mod N],  m < K,
// and its outputs z_j[b L + i], i < L, are the first L samples of the
// circular correlation of x_b with the taps (a launch over the outputs
// [n_lo, n_hi) places its blocks from n_lo, b L -> n_lo + b L, so a short
// range needs ceil((n_hi - n_lo) / L) blocks wherever it starts):
//   z_j[b L + i] = sum_k c_k x_b[i + k] = (1/K) sum_f X_b[f] G_j[f] e^{+2 pi i f i / K},
//   X_b[f] = sum_m x_b[m] e^{-2 pi i f m / K},   G_j[f] = sum_k c_k e^{+2 pi i f k / K}.
// X_b is computed once per reference series and segment (all blocks), G_j
// once per tap set (FP64 sum, stored with the 1/K in FP32).  The main kernel
// multiplies, runs one K-point inverse FFT per (template, block) in registers
// and LDS, and feeds the same window-peak keys as the MFMA forms.
//
// FFT: the register-resident K-point transform of block_fft.h (K = 1024,
// 2048, 4096), 4096/K blocks per workgroup.
#include <math.h>

#include <algorithm>

#include "block_fft.h"
#include "dev_common.h"
#include "rfd_internal.h"

namespace rfd {

// Window-peak key of one output sample: bits(rho^2) above the complement of
// its offset in the window (largest rho^2 wins, then the earliest sample).
__device__ __forceinline__ unsigned long long offset_key_ols(float r2, uint32_t off) {
  return ((unsigned long long)__float_as_uint(r2) << 32) | (unsigned long long)(0xFFFFFFFFu - off);
}
// windows one block may touch before the epilogue switches to per-sample atomics
constexpr int kOlsMaxWin = 8;
__device__ __forceinline__ unsigned long long umax64_ols(unsigned long long a, unsigned long long b) {
  return a > b ? a : b;
}

// ------------------------------------------------------------ block spectra
// X[b][f] for every block b of the reference series (forward FFT).
template <int K>
__device__ __forceinline__ void ols_x_body(const float2* __restrict__ z, int64_t n, int k0, int L, int64_t nB,
                                           int64_t org, const float2* __restrict__ tw, float2* __restrict__ X,
                                           uint32_t bx, float2* lds) {
  using S = BlockFft<K>;
  const int f = threadIdx.x / S::NTf, t = threadIdx.x % S::NTf;
  const int64_t b = (int64_t)bx * S::F + f;     // row of X: the block whose outputs start at org + b L
  BlockFftTw<K> w;
  block_fft_twiddles<K, -1>(w, tw, t);
  float2 v[16];
  const int64_t start = org + b * L + k0;
#pragma unroll
  for (int r = 0; r < 16; ++r) v[r] = b < nB ? z[(start + t + S::NTf * r) & (n - 1)] : make_float2(0.f, 0.f);
  block_fft<K, -1>(v, lds + f * S::LDS, t, w);
  if (b >= nB) return;
  float2* xb = X + b * K;
#pragma unroll
  for (int e = 0; e < 16 / S::R; ++e)
#pragma unroll
    for (int s = 0; s < S::R; ++s) xb[block_fft_out<K>(t, e, s)] = v[e * S::R + s];
}

template <int K>
__global__ __launch_bounds__(256) void k_ols_x(const float2* __restrict__ z, int64_t n, int k0, int L, int64_t nB,
                                            int64_t org, const float2* __restrict__ tw, float2* __restrict__ X) {
  __shared__ float2 lds[BlockFft<K>::F * BlockFft<K>::LDS];
  ols_x_body<K>(z, n, k0, L, nB, org, tw, X, blockIdx.x, lds);
}

// --------------------------------------------------------- tap spectra (FP64)
// G_j[f] = (1/K) sum_k c_k e^{+2 pi i f k / K}, c = the normalised FP32 taps:
// one K-point FP64 transform of the zero-padded taps per template, in LDS
// (radix-4 Stockham), rounded once to FP32.  O(K log K) per template instead
// of the O(K T) of the defining sum (4.2 ms -> a few hundred us for 512
// templates at T = 1024, which matters where taps are regenerated per
// segment, as the learned surrogate does).
template <int K>
__global__ __launch_bounds__(256) void k_ols_g(const float2* __restrict__ c32, int Tp, int T,
                                            const double2* __restrict__ tw64, float2* __restrict__ G) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int LP = lds_col<K>();
  double2* buf = reinterpret_cast<double2*>(smem);
  double2* twl = buf + LP;
  for (int k = threadIdx.x; k < K; k += 256) twl[lpad(k)] = tw64[k * (4096 / K)];
  const float2* cj = c32 + (int64_t)blockIdx.x * Tp;
  for (int k = threadIdx.x; k < K; k += 256)
    buf[lpad(k)] = k < T ? make_double2((double)cj[k].x, (double)cj[k].y) : make_double2(0.0, 0.0);
  __syncthreads();
  lds_fft<double2, K, 1, 256>(buf, twl, +1);
  const double inv = 1.0 / K;
  float2* gj = G + (int64_t)blockIdx.x * K;
  for (int f = threadIdx.x; f < K; f += 256) {
    const double2 v = buf[lpad(f)];
    gj[f] = make_float2((float)(v.x * inv), (float)(v.y * inv));
  }
}

// -------------------------------------------------------------- main kernel
struct OlsArgs {
  const float2* X;           // [nB][K] block spectra of this sub-bank's series
  const float2* G;           // [count][K] tap spectra
  const float2* tw;          // exp(+2 pi i m / 4096), m < 4096
  unsigned long long* slots;
  int64_t n, count, tmpl0, nwin, W, nB;   // nB: blocks of this launch (rows of X)
  int64_t org;               // first output sample of X's row 0 (block b: [org + b L, org + b L + L))
  int64_t n_lo, n_hi;        // output samples kept: [n_lo, n_hi)
  int L, J;                  // valid outputs per block, templates per workgroup
  float thr2;                // threshold^2 of the compaction (a key <= it never fires)
};

template <int K>
__device__ __forceinline__ unsigned long long ols_reduce(unsigned long long k) {
  constexpr int NTf = BlockFft<K>::NTf;
  constexpr int span = NTf < 64 ? NTf : 64;
#pragma unroll
  for (int o = 1; o < span; o <<= 1) k = umax64_ols(k, __shfl_xor(k, o));
  return k;
}

// Slot (e, s) of a thread after block_fft is kept when NF == 0 (any L), or
// when its output group dftr_freq(s) < NF: with L = 256 NF every output of
// the block at index < L lies in groups 0..NF-1 (index = k1 + 16 k2 + 256
// group, k1 + 16 k2 < 256), so the discarded groups are never read and the
// compiler drops the last DFT stage's work for them.
template <int K, int NF>
__device__ __forceinline__ constexpr bool ols_slot_kept(int s) {
  return NF == 0 || dftr_freq<BlockFft<K>::R>(s) < NF;
}

// Tile of the (block group, template group) grid a workgroup takes.  The
// dispatcher hands consecutive workgroups to the 8 XCDs in turn, and each XCD
// has its own L2.  So the hardware order h is renumbered: XCD c = h mod 8
// takes a contiguous run of a logical order in which the block groups are cut
// into 8 column tiles of near-equal width (tile c: [c gx / 8, (c+1) gx / 8)),
// each swept template row by template row.  The workgroups an XCD runs
// together then share one row's tap spectra and one tile's block spectra in
// its L2, and a tap spectrum leaves HBM about once per XCD instead of once
// per L2 pass.  Any bijection is correct; this one only decides where the
// re-reads land.
struct OlsTile {
  uint32_t bx, by;
};
__device__ __forceinline__ OlsTile ols_tile() {
  constexpr uint32_t kXcd = 8;
  const uint32_t gx = gridDim.x, gy = gridDim.y;
  const uint32_t lg = xcd_contiguous(blockIdx.x + gx * blockIdx.y, gx * gy);
  uint32_t x0 = 0, x1 = gx;
  for (uint32_t k = 1; k <= kXcd; ++k) {                     // the tile holding lg (empty ones skipped)
    x1 = k * gx / kXcd;
    if (lg < x1 * gy) break;
    x0 = x1;
  }
  const uint32_t w = x1 - x0, r = lg - x0 * gy;
  return OlsTile{x0 + r % w, r / w};
}

// One workgroup's (block group bx, template group by) of a sub-bank.
template <int K, int NF>
__device__ __forceinline__ void ols_body(const OlsArgs& a, uint32_t bx, uint32_t by, float2* lds,
                                         float2* twb_table) {
  using S = BlockFft<K>;
  const int f = threadIdx.x / S::NTf, t = threadIdx.x % S::NTf;
  const int64_t b = (int64_t)bx * S::F + f;
  const bool bvalid = b < a.nB;
  BlockFftTwL<K> w;
  block_fft_twiddles_lds<K, 1>(w, a.tw, t, twb_table);
  float2 xb[16];
  const float2* Xb = a.X + (bvalid ? b : 0) * K;
#pragma unroll
  for (int r = 0; r < 16; ++r) xb[r] = Xb[t + S::NTf * r];
  __syncthreads();     // the twiddle table is complete
  // this block's output samples and their windows (uniform per FFT)
  const int64_t n0 = a.org + b * a.L;
  const int64_t nbeg = std::max<int64_t>(n0, a.n_lo);
  const int64_t nend = std::min<int64_t>(std::min<int64_t>(n0 + a.L, a.n), a.n_hi);
  const bool has_out = bvalid && nend > nbeg;
  // every kept slot is an output of the launch: no per-sample range test
  const bool whole = NF > 0 && has_out && nbeg == n0 && nend == n0 + a.L;
  const int64_t q0 = has_out ? nbeg / a.W : 0, q1 = has_out ? (nend - 1) / a.W : 0;
  const int64_t j0 = (int64_t)by * a.J;
  const int64_t j1 = std::min<int64_t>(j0 + a.J, a.count);
  const bool lead = (threadIdx.x & 63) == 0;
  // the next template's tap spectrum is fetched while the current one is
  // transformed (its loads would otherwise stall all waves of the FFT)
  float2 gn[16];
  auto fetch_g = [&](int64_t j) {
    const float2* gj = a.G + (j < j1 ? j : j0) * K;
#pragma unroll
    for (int r = 0; r < 16; ++r) gn[r] = gj[t + S::NTf * r];
  };
  fetch_g(j0);
  for (int64_t j = j0; j < j1; ++j) {
    float2 v[16];
    dft16_prod<1>(v, xb, gn);     // stage A of the transform of X_b G_j, the product fused in
    fetch_g(j + 1);     // unconditional (the last one rereads j0's): no merge of old and new registers
    block_fft_after_a<K, 1>(v, lds + f * S::LDS, t, w);
    if (!has_out) continue;
    unsigned long long* slot = a.slots + (a.tmpl0 + j) * a.nwin;
    float r2[16];
    // maximum of the kept samples' rho^2 as bit patterns (non-negative floats
    // order as their bits).  The discarded outputs stay out: where the block's
    // correlation wraps, taps that cancel only against the series' own
    // correlations lose that cancellation and would cross the threshold.
    uint32_t r2max = 0u;
    // rho^2 of every kept slot, then its maximum with or without the range
    // test.  Where the FFT spans waves, rho^2 is formed once ahead of the two
    // branches (the compiler otherwise keeps a copy per branch: 0.928 -> 0.887
    // ms at K = 4096); the one-wave K = 1024 transform runs as fast or a little
    // faster with it formed inside each branch (2.53 against 2.54 ms on one GPU).
    constexpr bool kAhead = S::NTf > 64;
    auto rho2 = [&](int i) {
      if constexpr (kAhead) return r2[i];
      const float2 y = v[i];
      return r2[i] = y.x * y.x + y.y * y.y;
    };
    if constexpr (kAhead) {
#pragma unroll
      for (int e = 0; e < 16 / S::R; ++e)
#pragma unroll
        for (int s = 0; s < S::R; ++s) {
          if (!ols_slot_kept<K, NF>(s)) continue;
          const float2 y = v[e * S::R + s];
          r2[e * S::R + s] = y.x * y.x + y.y * y.y;
        }
    }
    if (whole) {
#pragma unroll
      for (int e = 0; e < 16 / S::R; ++e)
#pragma unroll
        for (int s = 0; s < S::R; ++s) {
          if (!ols_slot_kept<K, NF>(s)) continue;
          r2max = max(r2max, __float_as_uint(rho2(e * S::R + s)));
        }
    } else {
#pragma unroll
      for (int e = 0; e < 16 / S::R; ++e)
#pragma unroll
        for (int s = 0; s < S::R; ++s) {
          if (!ols_slot_kept<K, NF>(s)) continue;
          const float x = rho2(e * S::R + s);
          const int64_t nn = n0 + block_fft_out<K>(t, e, s);
          if (nn >= nbeg && nn < nend) r2max = max(r2max, __float_as_uint(x));
        }
    }
    // the compaction reports a window only if its peak exceeds thr2: a wave
    // with no sample above it cannot contribute a reported peak
    if (!__any(r2max > __float_as_uint(a.thr2))) continue;
    if (q1 - q0 < kOlsMaxWin) {
      // one reduction and one atomic per window the block touches
      for (int64_t qw = q0; qw <= q1; ++qw) {
        const int64_t wq = qw * a.W;
        const int64_t ws = std::max<int64_t>(wq, nbeg), we = std::min<int64_t>(wq + a.W, nend);
        unsigned long long k = 0;
#pragma unroll
        for (int e = 0; e < 16 / S::R; ++e)
#pragma unroll
          for (int s = 0; s < S::R; ++s) {
            if (!ols_slot_kept<K, NF>(s)) continue;
            const int64_t nn = n0 + block_fft_out<K>(t, e, s);
            if (nn >= ws && nn < we) k = umax64_ols(k, offset_key_ols(r2[e * S::R + s], (uint32_t)(nn - wq)));
          }
        k = ols_reduce<K>(k);
        if (lead) atomicMax(slot + qw, k);
      }
    } else {
      // windows shorter than a block / kOlsMaxWin: one atomic per sample
#pragma unroll
      for (int e = 0; e < 16 / S::R; ++e)
#pragma unroll
        for (int s = 0; s < S::R; ++s) {
          if (!ols_slot_kept<K, NF>(s)) continue;
          const int64_t nn = n0 + block_fft_out<K>(t, e, s);
          if (nn >= nbeg && nn < nend) {
            const int64_t q = nn / a.W;
            atomicMax(slot + q, offset_key_ols(r2[e * S::R + s], (uint32_t)(nn - q * a.W)));
          }
        }
    }
  }
}

template <int K, int NF>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_ols(OlsArgs a) {
  __shared__ float2 lds[BlockFft<K>::F * BlockFft<K>::LDS];
  __shared__ float2 twb_table[block_fft_twb_size<K>()];
  const OlsTile wg = ols_tile();
  ols_body<K, NF>(a, wg.bx, wg.by, lds, twb_table);
}

// ------------------------------------------------- several sub-banks at once
// A short output range gives each sub-bank a few blocks only: one launch then
// covers up to kOlsMulti sub-banks of one block size, their workgroups laid
// end to end (sub-bank s owns workgroups [wg0, wg0 + gx gy) of k_ols_multi and
// [wgx0, wgx0 + gx) of k_ols_x_multi).  The descriptors travel by value in the
// kernel arguments (nothing to upload, and a captured graph keeps them).
// 32 per launch rather than 16: 32 sub-banks of one block size (ecc512s) take
// one launch pair instead of two (stream FIR 0.18 -> 0.15 ms per push).
constexpr int kOlsMulti = 32;
struct OlsSb {
  const float2* z;           // the sub-bank's reference series
  float2* X;                 // its block spectra [nB][K]
  const float2* G;           // its tap spectra [count][K]
  int64_t count, tmpl0, nB;
  int k0, L, J;
  uint32_t gx, wg0, wgx0;
};
struct OlsMultiArgs {
  OlsSb sb[kOlsMulti];
  const float2* tw;
  unsigned long long* slots;
  int64_t n, nwin, W, n_lo, n_hi;
  float thr2;
  int nsb;
};
static_assert(sizeof(OlsMultiArgs) <= 4096, "the descriptors must fit the kernel argument segment");

// sub-bank of workgroup g (by the first-workgroup fields), with constant
// indices only, so the descriptors stay in the argument segment
template <bool X>
__device__ __forceinline__ int ols_multi_find(const OlsMultiArgs& m, uint32_t g) {
  int s = 0;
#pragma unroll
  for (int i = 1; i < kOlsMulti; ++i)
    if (i < m.nsb && g >= (X ? m.sb[i].wgx0 : m.sb[i].wg0)) s = i;
  return s;
}

template <int K>
__global__ __launch_bounds__(256) void k_ols_x_multi(OlsMultiArgs m) {
  __shared__ float2 lds[BlockFft<K>::F * BlockFft<K>::LDS];
  const int s = ols_multi_find<true>(m, blockIdx.x);
  const float2* z = nullptr;
  float2* X = nullptr;
  int64_t nB = 0;
  int k0 = 0, L = 1;
  uint32_t wgx0 = 0;
#pragma unroll
  for (int i = 0; i < kOlsMulti; ++i)
    if (i == s) {
      z = m.sb[i].z;
      X = m.sb[i].X;
      nB = m.sb[i].nB;
      k0 = m.sb[i].k0;
      L = m.sb[i].L;
      wgx0 = m.sb[i].wgx0;
    }
  ols_x_body<K>(z, m.n, k0, L, nB, m.n_lo, m.tw, X, blockIdx.x - wgx0, lds);
}

template <int K, int NF>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_ols_multi(OlsMultiArgs m) {
  __shared__ float2 lds[BlockFft<K>::F * BlockFft<K>::LDS];
  __shared__ float2 twb_table[block_fft_twb_size<K>()];
  const int s = ols_multi_find<false>(m, blockIdx.x);
  OlsArgs a;
  a.tw = m.tw;
  a.slots = m.slots;
  a.n = m.n;
  a.nwin = m.nwin;
  a.W = m.W;
  a.n_lo = m.n_lo;
  a.n_hi = m.n_hi;
  a.org = m.n_lo;
  a.thr2 = m.thr2;
  uint32_t gx = 1, wg0 = 0;
#pragma unroll
  for (int i = 0; i < kOlsMulti; ++i)
    if (i == s) {
      a.X = m.sb[i].X;
      a.G = m.sb[i].G;
      a.count = m.sb[i].count;
      a.tmpl0 = m.sb[i].tmpl0;
      a.nB = m.sb[i].nB;
      a.L = m.sb[i].L;
      a.J = m.sb[i].J;
      gx = m.sb[i].gx;
      wg0 = m.sb[i].wg0;
    }
  const uint32_t l = blockIdx.x - wg0;
  ols_body<K, NF>(a, l % gx, l / gx, lds, twb_table);
}

// ------------------------------------------------------------------ host
// Measured throughput of each block size per unit of FFT work, relative to
// K = 2048 (MI355X: one-wave FFTs without workgroup barriers at 1024, a
// whole-workgroup FFT at 4096).
// (FFT flops per second of the whole-segment launches at T = 256 and 1024: 59.5,
// 50.9 and 50.4-51.1 TFLOP/s).
static double ols_efficiency(int K) { return K == 1024 ? 1.17 : (K == 2048 ? 1.0 : 0.99); }
// ... and the gain of an aligned output length (L = 256 NF: the discarded
// outputs are never computed, interior blocks skip per-sample range tests)
// (measured 1.01 at K = 4096 and 1.036 at K = 1024 on equal block counts)
constexpr double kOlsAlignedGain = 1.03;

// aligned output groups the kernels are built for, per block size
static bool ols_nf_built(int K, int nf) {
  switch (K) {
    case 1024: return nf == 3;
    case 2048: return nf == 6 || nf == 7;
    case 4096: return nf >= 12 && nf <= 15;
    default: return false;
  }
}

OlsShape ols_shape(const Plan& p, int T) {
  OlsShape best{4096, 4096 - T + 1, 0};
  double best_cost = 1e30;
  for (int K = 1024; K <= 4096; K *= 2) {
    if (K <= T) continue;
    if (p.ols_block > T && K != p.ols_block) continue;
    const int L0 = K - T + 1;
    const double flops = 5.0 * std::log2((double)K) + 6.0;
    // the general form keeps every valid output, the aligned form whole groups of 256
    const double cost0 = flops * K / (double)L0 / ols_efficiency(K);
    if (cost0 < best_cost - 1e-9) {
      best_cost = cost0;
      best = OlsShape{K, L0, 0};
    }
    const int nf = L0 / 256;
    if (p.ols_aligned && nf > 0 && ols_nf_built(K, nf)) {
      const double cost1 = flops * K / (double)(256 * nf) / (ols_efficiency(K) * kOlsAlignedGain);
      if (cost1 < best_cost - 1e-9) {
        best_cost = cost1;
        best = OlsShape{K, 256 * nf, nf};
      }
    }
  }
  return best;
}

int ols_block_size(const Plan& p, int T) { return ols_shape(p, T).K; }

static int ols_templates_per_wg(int64_t nB, int F, int64_t count, int n_cu) {
  // enough workgroups to fill the chip several times, at least 4 templates each
  const int64_t gx = (nB + F - 1) / F;
  int J = 32;
  while (J > 4 && gx * ((count + J - 1) / J) < (int64_t)8 * n_cu) J /= 2;
  return J;
}

int ensure_ols(Plan& p, Taps& t, bool allow_alloc, bool need_block_spectra) {
  for (size_t bi = 0; bi < t.sb.size(); ++bi) {
    SubBankTaps& s = t.sb[bi];
    if (s.count == 0) continue;
    const OlsShape sh = ols_shape(p, s.T);
    const int K = sh.K, L = sh.L;
    const int64_t nB = (p.n + L - 1) / L;
    const bool need_x = need_block_spectra && (s.ols_x == nullptr || s.ols_x_cap < nB * K);
    const bool need_g = s.ols_g == nullptr || s.ols_K != K;
    if ((need_x || need_g) && !allow_alloc)
      return fail(RFD_E_STATE, "overlap-save buffers changed since capture; create the graph again");
    if (need_x || need_g) ++t.res_gen;
    if (need_x) {
      RFD_HIP(hipStreamSynchronize(p.stream));
      if (s.ols_x) (void)hipFree(s.ols_x);
      s.ols_x = nullptr;
      if (device_malloc((void**)&s.ols_x, (size_t)nB * K * sizeof(float2)) != hipSuccess) {
        s.ols_x = nullptr;
        (void)hipGetLastError();
        return fail(RFD_E_NOMEM, "overlap-save block spectra: hipMalloc failed");
      }
      s.ols_x_cap = nB * K;
    }
    if (need_g) {
      RFD_HIP(hipStreamSynchronize(p.stream));
      if (s.ols_g) (void)hipFree(s.ols_g);
      s.ols_g = nullptr;
      if (device_malloc((void**)&s.ols_g, (size_t)s.count * K * sizeof(float2)) != hipSuccess) {
        s.ols_g = nullptr;
        (void)hipGetLastError();
        return fail(RFD_E_NOMEM, "overlap-save tap spectra: hipMalloc failed");
      }
      s.ols_valid = false;
    }
    s.ols_K = K;
    s.ols_L = L;
    s.ols_nf = sh.nf;
    s.ols_nB = nB;
    if (!s.ols_valid) {
      switch (K) {
        case 1024:
          hipLaunchKernelGGL(k_ols_g<1024>, dim3((unsigned)s.count), dim3(256),
                             (size_t)(lds_col<1024>() + 1024 + 64) * sizeof(double2), p.stream, t.c32 + s.a_base,
                             s.Tp, s.T, (const double2*)p.ols_tw64, s.ols_g);
          break;
        case 2048:
          hipLaunchKernelGGL(k_ols_g<2048>, dim3((unsigned)s.count), dim3(256),
                             (size_t)(lds_col<2048>() + 2048 + 128) * sizeof(double2), p.stream, t.c32 + s.a_base,
                             s.Tp, s.T, (const double2*)p.ols_tw64, s.ols_g);
          break;
        default:
          hipLaunchKernelGGL(k_ols_g<4096>, dim3((unsigned)s.count), dim3(256),
                             (size_t)(lds_col<4096>() + 4096 + 256) * sizeof(double2), p.stream, t.c32 + s.a_base,
                             s.Tp, s.T, (const double2*)p.ols_tw64, s.ols_g);
      }
      RFD_CHECK_LAUNCH();
      s.ols_valid = true;
    }
  }
  return RFD_OK;
}

template <int K, int NF>
static int launch_ols_k(Plan& p, const Taps& t, const SubBankTaps& s, int64_t W, int64_t nwin, float threshold,
                        int64_t n_lo, int64_t n_hi, float2* X) {
  using S = BlockFft<K>;
  const float2* z = p.zref + (int64_t)s.ref_id * p.n;
  const int64_t nB = (n_hi - n_lo + s.ols_L - 1) / s.ols_L;      // <= s.ols_nB
  const unsigned gx = (unsigned)((nB + S::F - 1) / S::F);
  hipLaunchKernelGGL(k_ols_x<K>, dim3(gx), dim3(256), 0, p.stream, z, p.n, s.k0, s.ols_L, nB, n_lo,
                     (const float2*)p.ols_tw32, X);
  RFD_CHECK_LAUNCH();
  OlsArgs a;
  a.X = X;
  a.G = s.ols_g;
  a.tw = p.ols_tw32;
  a.slots = p.slots;
  a.n = p.n;
  a.count = s.count;
  a.tmpl0 = s.first;
  a.nwin = nwin;
  a.W = W;
  a.nB = nB;
  a.org = n_lo;
  a.n_lo = n_lo;
  a.n_hi = n_hi;
  a.L = s.ols_L;
  a.J = ols_templates_per_wg(nB, S::F, s.count, p.n_cu);
  a.thr2 = threshold * threshold;
  const unsigned gy = (unsigned)((s.count + a.J - 1) / a.J);
  int rc = stage_begin(p, kStFirKernel);
  if (rc) return rc;
  hipLaunchKernelGGL((k_ols<K, NF>), dim3(gx, gy), dim3(256), 0, p.stream, a);
  RFD_CHECK_LAUNCH();
  return stage_end(p);
}

// Up to kOlsMulti sub-banks of one block size (K, NF) over the output range
// [n_lo, n_hi) in one k_ols_x_multi and one k_ols_multi launch.
template <int K, int NF>
static int launch_ols_multi(Plan& p, const Taps& t, const int* sbs, int nsb, int64_t W, int64_t nwin,
                            float threshold, int64_t n_lo, int64_t n_hi) {
  using S = BlockFft<K>;
  OlsMultiArgs m{};
  m.tw = p.ols_tw32;
  m.slots = p.slots;
  m.n = p.n;
  m.nwin = nwin;
  m.W = W;
  m.n_lo = n_lo;
  m.n_hi = n_hi;
  m.thr2 = threshold * threshold;
  m.nsb = nsb;
  for (int i = 0; i < nsb; ++i) {
    const SubBankTaps& s = t.sb[sbs[i]];
    OlsSb& d = m.sb[i];
    d.z = p.zref + (int64_t)s.ref_id * p.n;
    d.X = s.ols_x;
    d.G = s.ols_g;
    d.count = s.count;
    d.tmpl0 = s.first;
    d.nB = (n_hi - n_lo + s.ols_L - 1) / s.ols_L;
    d.k0 = s.k0;
    d.L = s.ols_L;
    d.gx = (uint32_t)((d.nB + S::F - 1) / S::F);
  }
  // templates per workgroup: enough workgroups over the whole launch to fill
  // the chip several times, at least 4 templates each
  int J = 32;
  auto total = [&](int j) {
    int64_t w = 0;
    for (int i = 0; i < nsb; ++i) w += (int64_t)m.sb[i].gx * ((m.sb[i].count + j - 1) / j);
    return w;
  };
  while (J > 4 && total(J) < (int64_t)8 * p.n_cu) J /= 2;
  uint32_t wg = 0, wgx = 0;
  for (int i = 0; i < nsb; ++i) {
    OlsSb& d = m.sb[i];
    d.J = J;
    d.wg0 = wg;
    d.wgx0 = wgx;
    wg += d.gx * (uint32_t)((d.count + J - 1) / J);
    wgx += d.gx;
  }
  hipLaunchKernelGGL(k_ols_x_multi<K>, dim3(wgx), dim3(256), 0, p.stream, m);
  RFD_CHECK_LAUNCH();
  int rc = stage_begin(p, kStFirKernel);
  if (rc) return rc;
  hipLaunchKernelGGL((k_ols_multi<K, NF>), dim3(wg), dim3(256), 0, p.stream, m);
  RFD_CHECK_LAUNCH();
  return stage_end(p);
}

int launch_ols(Plan& p, const Taps& t, int64_t W, int64_t nwin, float threshold, int64_t n_lo, int64_t n_hi,
               float2* x_scratch) {
  if (n_hi < 0) n_hi = p.n;
  if (n_lo < 0 || n_hi > p.n || n_lo >= n_hi) return fail(RFD_E_INVALID, "overlap-save: empty output range");
  int active = 0;
  for (const SubBankTaps& s : t.sb) {
    if (s.count == 0) continue;
    if (!s.ols_valid || !(x_scratch ? x_scratch : s.ols_x)) return fail(RFD_E_STATE, "overlap-save spectra not prepared");
    ++active;
  }
  // A short output range leaves each sub-bank's launch a small part of the
  // chip: the sub-banks of one block size then share launches (their window
  // keys are disjoint slots, their block spectra separate buffers).  Whole
  // segments keep one launch per sub-bank, each filling the chip, so that a
  // sub-bank's block spectra are used while still in the last-level cache.  A
  // shared block-spectrum scratch keeps one launch per sub-bank as well.
  if (!x_scratch && active > 1 && (n_hi - n_lo) * 8 <= p.n) {
    std::vector<char> done(t.sb.size(), 0);
    for (size_t b0 = 0; b0 < t.sb.size(); ++b0) {
      const SubBankTaps& s0 = t.sb[b0];
      if (s0.count == 0 || done[b0]) continue;
      int sbs[kOlsMulti], nsb = 0;
      for (size_t b = b0; b < t.sb.size() && nsb < kOlsMulti; ++b) {
        const SubBankTaps& s = t.sb[b];
        if (s.count == 0 || done[b] || s.ols_K != s0.ols_K || s.ols_nf != s0.ols_nf) continue;
        done[b] = 1;
        sbs[nsb++] = (int)b;
      }
      int rc;
      switch (s0.ols_K * 16 + s0.ols_nf) {
#define OLS_CASE(KK, NN) \
        case KK * 16 + NN: rc = launch_ols_multi<KK, NN>(p, t, sbs, nsb, W, nwin, threshold, n_lo, n_hi); break;
        OLS_CASE(1024, 0) OLS_CASE(1024, 3)
        OLS_CASE(2048, 0) OLS_CASE(2048, 6) OLS_CASE(2048, 7)
        OLS_CASE(4096, 0) OLS_CASE(4096, 12) OLS_CASE(4096, 13) OLS_CASE(4096, 14) OLS_CASE(4096, 15)
#undef OLS_CASE
        default: rc = fail(RFD_E_INVALID, "overlap-save block size must be 1024, 2048 or 4096");
      }
      if (rc) return rc;     // sub-banks past kOlsMulti of this block size start the next chunk
    }
    return RFD_OK;
  }
  for (const SubBankTaps& s : t.sb) {
    if (s.count == 0) continue;
    float2* X = x_scratch ? x_scratch : s.ols_x;
    int rc;
    switch (s.ols_K * 16 + s.ols_nf) {
#define OLS_CASE(KK, NN) \
      case KK * 16 + NN: rc = launch_ols_k<KK, NN>(p, t, s, W, nwin, threshold, n_lo, n_hi, X); break;
      OLS_CASE(1024, 0) OLS_CASE(1024, 3)
      OLS_CASE(2048, 0) OLS_CASE(2048, 6) OLS_CASE(2048, 7)
      OLS_CASE(4096, 0) OLS_CASE(4096, 12) OLS_CASE(4096, 13) OLS_CASE(4096, 14) OLS_CASE(4096, 15)
#undef OLS_CASE
      default: rc = fail(RFD_E_INVALID, "overlap-save block size must be 1024, 2048 or 4096");
    }
    if (rc) return rc;
  }
  return RFD_OK;
}

}  // namespace rfd
