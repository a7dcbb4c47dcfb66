// Two-pass Stockham FFTs with fused loads and stores.
//
// N = N1 * N2.  For z[n] = sum_i Q[i] exp(s 2 pi i i n / N) with
// i = i1 + N1 i2 and n = n2 + N2 n1:
//   pass A (per column i1): X[i1][n2] = sum_i2 Q[i1 + N1 i2] exp(s 2 pi i i2 n2 / N2),
//           times exp(s 2 pi i i1 n2 / N), stored at Y[n2 N1 + i1];
//   pass B (per row n2):    z[n2 + N2 n1] = sum_i1 Y[n2 N1 + i1] exp(s 2 pi i i1 n1 / N1).
// Each workgroup transforms C adjacent columns (pass A) or rows (pass B) in
// LDS, so every global access is a run of C contiguous elements.  The first
// pass fuses the pointwise product of Eq. 1 (data x conj(template) x weight);
// the second fuses the consumer: spectrum store, reference-series store with
// its 16-bit hi/lo planes.  Tap construction evaluates only the T
// correlation lags it keeps: each pass-A workgroup reduces its columns at
// once to its share of every kept lag (k_corr_part, k_corr_reduce), or, where
// those shares would not fit the work buffer, pass A stores the rows the lags
// read and k_lags_direct sums them.  FINDCHIRP's own transforms live with its
// kernels.
#include <algorithm>
#include <type_traits>

#include "dev_common.h"
#include "rfd_internal.h"

namespace rfd {

constexpr int kNT = 256;

template <typename V> struct Cols;
template <> struct Cols<float2> { static constexpr int value(int L) { return L >= 2048 ? 4 : 8; } };   // 8 columns of 2048 spill registers
template <> struct Cols<double2> { static constexpr int value(int L) { return L >= 2048 ? 2 : 4; } };

template <typename V, int L, int C>
constexpr size_t lds_bytes() { return (size_t)C * lds_col<L>() * sizeof(V) + (size_t)(L + L / 16) * sizeof(V); }

// ---------------------------------------------------------------- loaders
struct LoadData64 {        // real FP64 series, scaled, FP64 complex
  const double* x; double scale;
  __device__ double2 operator()(int, int64_t i) const { return make_double2(x[i] * scale, 0.0); }
};
struct LoadDechirp64 {     // s_i * F_ref,i over the band, FP64 (Eq. 1 integrand)
  const double2* s; const double2* f; int64_t i_low, i_high;
  __device__ double2 operator()(int, int64_t i) const {
    if (i < i_low || i > i_high) return make_double2(0.0, 0.0);
    return cmul(s[i], f[i]);
  }
};
// References of one batched dechirp, carried by value in the kernel arguments
// (so eager launches and captured graphs need no pointer table in memory).
struct DechirpRefs {
  const double2* h[kDechirpBatch];   // reference templates, complex128 [nb]
  int32_t slot[kDechirpBatch];       // reference-series slots they fill
};
// Loaders with a Raw type split an element into fetch (the loads only, no
// branch: an out-of-band lane reads bin i_low and gets a zero weight) and make
// (the arithmetic), so that a thread can have the loads of several elements
// in flight before it combines any (see gather_columns).
struct LoadDechirpRefs {   // s_i w_i conj(h_b,i) / (sigma_b alpha) over the band, FP64
  const double2* s; const double* w; DechirpRefs r; const double* scale; int64_t i_low, i_high;
  struct Raw { double2 h, s; double w; };
  __device__ Raw fetch(int b, int64_t i) const {
    const bool in = i >= i_low && i <= i_high;
    const int64_t k = in ? i : i_low;
    Raw x;
    x.h = r.h[b][k];
    x.s = s[k];
    x.w = w[k];
    if (!in) x.w = 0.0;
    return x;
  }
  __device__ double2 make(int b, int64_t, const Raw& x) const {
    const double f = x.w * scale[b];
    return cmul(x.s, make_double2(f * x.h.x, -f * x.h.y));
  }
  __device__ double2 operator()(int b, int64_t i) const { return make(b, i, fetch(b, i)); }
};
struct LoadDechirpRefs32 { // the same integrand, formed in FP64 and rounded once to FP32
  LoadDechirpRefs d;
  using Raw = LoadDechirpRefs::Raw;
  __device__ Raw fetch(int b, int64_t i) const { return d.fetch(b, i); }
  __device__ float2 make(int b, int64_t i, const Raw& x) const {
    const double2 v = d.make(b, i, x);
    return make_float2((float)v.x, (float)v.y);
  }
  __device__ float2 operator()(int b, int64_t i) const { return make(b, i, fetch(b, i)); }
};
struct LoadFindchirp {     // s_i * F_j,i with F_j stored over band bins
  const float2* s; const float2* f; int64_t i_low, i_high, n_band;
  __device__ float2 operator()(int b, int64_t i) const {
    if (i < i_low || i > i_high) return make_float2(0.f, 0.f);
    return cmul(s[i], f[(int64_t)b * n_band + (i - i_low)]);
  }
};
struct LoadCorr64 {        // FP64 correlation integrands (tap construction, streaming series)
  const double* w; const double2* hr; const double2* ht; int64_t nb, i_low, i_high; int mode;
  const double* bscale;    // mode 0: per-member factor folded into the integrand (nullptr: none)
  struct Raw { double2 r, t; double w; };
  __device__ Raw fetch(int b, int64_t i) const {
    const bool in = i >= i_low && i <= i_high;
    const int64_t k = in ? i : i_low;
    Raw x;
    x.r = hr[k];
    x.t = ht[(int64_t)b * nb + k];     // (mode 1: ht is hr, unused)
    x.w = w[k];
    if (!in) x.w = 0.0;
    return x;
  }
  __device__ double2 make(int b, int64_t, const Raw& x) const {
    const double2 r = x.r, t = x.t;
    double wi = x.w;
    if (mode == 1) return make_double2(wi * (r.x * r.x + r.y * r.y), 0.0);
    if (bscale) wi *= bscale[b];
    if (mode == 0) return make_double2(wi * (t.x * r.x + t.y * r.y), wi * (t.y * r.x - t.x * r.y));
    // mode 2: ratio R = t / r where the chi^2 weight w |r|^2 is non-zero
    const double rr = r.x * r.x + r.y * r.y;
    if (!(wi * rr > 0.0)) return make_double2(0.0, 0.0);
    return make_double2((t.x * r.x + t.y * r.y) / rr, (t.y * r.x - t.x * r.y) / rr);
  }
  __device__ double2 operator()(int b, int64_t i) const { return make(b, i, fetch(b, i)); }
};

// The same integrands rounded once to FP32.  w_i alone is of order 1 / S_n
// (about 1e46 for a strain PSD), so an unnormalised integrand overflows FP32:
// FP32 callers fold the normalisation of the result in through bscale (the
// streaming series use 1 / (sigma_ref alpha), as the FP32 dechirp passes do).
struct LoadCorr32 {
  LoadCorr64 d;
  using Raw = LoadCorr64::Raw;
  __device__ Raw fetch(int b, int64_t i) const { return d.fetch(b, i); }
  __device__ float2 make(int b, int64_t i, const Raw& x) const {
    const double2 v = d.make(b, i, x);
    return make_float2((float)v.x, (float)v.y);
  }
  __device__ float2 operator()(int b, int64_t i) const { return make(b, i, fetch(b, i)); }
};

// ---------------------------------------------------------------- storers
struct StoreSpectrum64 {   // FP64 spectrum and its FP32 copy (FINDCHIRP operand)
  double2* s64; float2* s32; int64_t half;
  __device__ void operator()(int, int64_t n, double2 v) const {
    if (n <= half) {
      s64[n] = v;
      s32[n] = make_float2((float)v.x, (float)v.y);
    }
  }
};
// Reference series are stored as FP32 only; the 16-bit hi/lo planes the MFMA
// forms read are split from them by the FIR launch, over the window it reads.
struct StoreRefSlots {     // FP64 series -> FP32, into the slot of batch entry b
  float2* z; int64_t n; DechirpRefs r;
  __device__ void operator()(int b, int64_t m, double2 v) const {
    z[(int64_t)r.slot[b] * n + m] = make_float2((float)v.x, (float)v.y);
  }
};
struct StoreRefSlots32 {   // FP32 series into the slot of batch entry b
  float2* z; int64_t n; DechirpRefs r;
  __device__ void operator()(int b, int64_t m, float2 v) const { z[(int64_t)r.slot[b] * n + m] = v; }
};
struct StoreBand {         // FP64 series -> FP32 band series
  float2* z;
  __device__ void operator()(int, int64_t n, double2 v) const { z[n] = make_float2((float)v.x, (float)v.y); }
};

// ------------------------------------------------------------------ passes
template <typename V, int L>
__device__ void load_twl(V* twl, const V* __restrict__ tab, int stride = 1) {
  for (int k = threadIdx.x; k < L; k += kNT) twl[lpad(k)] = tab[k * stride];
}

// The C columns c0 + c (stride n1 through the input) into LDS, [C][LP]
// padded.  Each thread issues U elements' loads before storing any, so U
// memory round trips overlap (one at a time, the loop waited for every load).
template <class LD, class = void> struct HasRaw : std::false_type {};
template <class LD> struct HasRaw<LD, std::void_t<typename LD::Raw>> : std::true_type {};

// elements per thread in flight: at most U, and no more than a thread has
// (C L and kNT are powers of two, so U * kNT divides C L when C L >= kNT)
template <int E, int U>
__host__ __device__ constexpr int gather_batch() { return E / kNT >= U ? U : (E / kNT >= 1 ? E / kNT : 1); }

template <typename V, int L, int C, int U0, class LD>
__device__ __forceinline__ void gather_columns(V* buf, const LD& ld, int b, int c0, int n1) {
  constexpr int LP = lds_col<L>();
  constexpr int E = C * L;
  constexpr int U = gather_batch<E, U0>();
  for (int e0 = 0; e0 < E; e0 += U * kNT) {
    if constexpr (HasRaw<LD>::value) {
      typename LD::Raw x[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = e0 + u * kNT + (int)threadIdx.x;
        if (E % (U * kNT) == 0 || e < E) x[u] = ld.fetch(b, (int64_t)(c0 + e % C) + (int64_t)n1 * (e / C));
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = e0 + u * kNT + (int)threadIdx.x;
        if (E % (U * kNT) == 0 || e < E)
          buf[(e % C) * LP + lpad(e / C)] = ld.make(b, (int64_t)(c0 + e % C) + (int64_t)n1 * (e / C), x[u]);
      }
    } else {
      V v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = e0 + u * kNT + (int)threadIdx.x;
        if (E % (U * kNT) == 0 || e < E) v[u] = ld(b, (int64_t)(c0 + e % C) + (int64_t)n1 * (e / C));
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = e0 + u * kNT + (int)threadIdx.x;
        if (E % (U * kNT) == 0 || e < E) buf[(e % C) * LP + lpad(e / C)] = v[u];
      }
    }
  }
}
constexpr int kGatherU = 8;

// pass A: L = N2-point transforms of C columns; writes Y with the inter-pass
// twiddle.  tabL[k * tab_stride] = exp(+2 pi i k / L).  Only the rows n2 in
// [row_lo, row_lo + row_cnt) mod L are written (all rows: 0, L): a consumer
// that evaluates a few outputs of the second pass reads no others.
template <typename V, int L, class LD>
__global__ __launch_bounds__(kNT) void k_pass_a(LD ld, V* __restrict__ Y, const V* __restrict__ coarse,
                                              const V* __restrict__ fine, const V* __restrict__ tabL,
                                              int n1, int sign, int tab_stride, int row_lo, int row_cnt) {
  constexpr int C = Cols<V>::value(L);
  constexpr int LP = lds_col<L>();
  extern __shared__ __align__(16) unsigned char smem[];
  V* buf = reinterpret_cast<V*>(smem);
  V* twl = buf + C * LP;
  const int b = blockIdx.y;
  const int c0 = blockIdx.x * C;
  const int64_t n = (int64_t)n1 * L;
  load_twl<V, L>(twl, tabL, tab_stride);
  gather_columns<V, L, C, kGatherU>(buf, ld, b, c0, n1);
  __syncthreads();
  lds_fft<V, L, C, kNT>(buf, twl, sign);
  V* Yb = Y + (int64_t)b * n;
  for (int e = threadIdx.x; e < C * L; e += kNT) {
    int c = e % C, n2 = e / C;
    if (((n2 - row_lo) & (L - 1)) >= row_cnt) continue;
    int i1 = c0 + c;
    V v = buf[c * LP + lpad(n2)];
    uint32_t p = (uint32_t)i1 * (uint32_t)n2;   // < N
    if (p) v = cmul(v, twiddle_n(coarse, fine, p, sign));
    Yb[(int64_t)n2 * n1 + i1] = v;
  }
}

template <typename V, int L>
__device__ void pass_b_load(const V* __restrict__ Yb, V* buf, V* twl, const V* __restrict__ tabL, int r0) {
  constexpr int C = Cols<V>::value(L);
  constexpr int LP = lds_col<L>();
  load_twl<V, L>(twl, tabL);
  constexpr int E = C * L;
  constexpr int U = gather_batch<E, kGatherU>();
  for (int e0 = 0; e0 < E; e0 += U * kNT) {      // U loads in flight per thread
    V v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = e0 + u * kNT + (int)threadIdx.x;
      if (E % (U * kNT) == 0 || e < E) v[u] = Yb[(int64_t)(r0 + e / L) * L + e % L];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = e0 + u * kNT + (int)threadIdx.x;
      if (E % (U * kNT) == 0 || e < E) buf[(e / L) * LP + lpad(e % L)] = v[u];
    }
  }
  __syncthreads();
}

// pass B: L = N1-point transforms of C rows, generic storer
template <typename V, int L, class ST>
__global__ __launch_bounds__(kNT) void k_pass_b(const V* __restrict__ Y, ST st, const V* __restrict__ tabL,
                                              int n2, int sign) {
  constexpr int C = Cols<V>::value(L);
  constexpr int LP = lds_col<L>();
  extern __shared__ __align__(16) unsigned char smem[];
  V* buf = reinterpret_cast<V*>(smem);
  V* twl = buf + C * LP;
  const int b = blockIdx.y;
  const int r0 = blockIdx.x * C;
  const V* Yb = Y + (int64_t)b * L * n2;
  pass_b_load<V, L>(Yb, buf, twl, tabL, r0);
  lds_fft<V, L, C, kNT>(buf, twl, sign);
  for (int e = threadIdx.x; e < C * L; e += kNT) {
    int c = e % C, n1 = e / C;
    st(b, (int64_t)(r0 + c) + (int64_t)n2 * n1, buf[c * LP + lpad(n1)]);
  }
}

// -------------------------------------------------------------- dispatch
template <typename V, class LD>
static int run_pass_a(Plan& p, LD ld, V* Y, const V* coarse, const V* fine, const V* tab2, int batch, int sign,
                      int row_lo = 0, int row_cnt = 1 << 30) {
  dim3 blk(kNT);
  switch (p.n2) {
#define CASE_A(LL)                                                                         \
  case LL: {                                                                               \
    constexpr int C = Cols<V>::value(LL);                                                  \
    size_t sh = lds_bytes<V, LL, C>();                                                     \
    hipLaunchKernelGGL((k_pass_a<V, LL, LD>), dim3(p.n1 / C, batch), blk, sh, p.stream, ld, Y, coarse, \
                       fine, tab2, p.n1, sign, 1, row_lo & (LL - 1), std::min(row_cnt, LL));  \
    break;                                                                                 \
  }
    CASE_A(32) CASE_A(64) CASE_A(128) CASE_A(256) CASE_A(512) CASE_A(1024) CASE_A(2048)
#undef CASE_A
    default: return fail(RFD_E_UNSUPPORTED, "fft: unsupported N2");
  }
  RFD_CHECK_LAUNCH();
  return RFD_OK;
}

template <typename V, class ST>
static int run_pass_b(Plan& p, const V* Y, ST st, const V* tab1, int batch, int sign) {
  dim3 blk(kNT);
  switch (p.n1) {
#define CASE_B(LL)                                                                          \
  case LL: {                                                                                \
    constexpr int C = Cols<V>::value(LL);                                                   \
    size_t sh = lds_bytes<V, LL, C>();                                                      \
    hipLaunchKernelGGL((k_pass_b<V, LL, ST>), dim3(p.n2 / C, batch), blk, sh, p.stream, Y, st, tab1, \
                       p.n2, sign);                                                         \
    break;                                                                                  \
  }
    CASE_B(32) CASE_B(64) CASE_B(128) CASE_B(256) CASE_B(512) CASE_B(1024) CASE_B(2048)
#undef CASE_B
    default: return fail(RFD_E_UNSUPPORTED, "fft: unsupported N1");
  }
  RFD_CHECK_LAUNCH();
  return RFD_OK;
}

// Only the T lags m = (k0 + l) mod N, l < T, of pass B's output, each as a
// direct sum over its row, z[m] = sum_i1 Y[n2 N1 + i1] exp(+2 pi i i1 n1 / N1)
// with n2 = m mod N2 and n1 = m div N2: tap construction keeps T of N
// outputs, and T N1 terms cost far less than the whole pass.  One wave per
// lag, FP64.
__global__ __launch_bounds__(256) void k_lags_direct(const double2* __restrict__ Y, int64_t n, int n1, int n2,
                                                   const double2* __restrict__ tab1, int k0,
                                                   const int32_t* __restrict__ k0s, int T, double scale,
                                                   double2* __restrict__ out, int64_t stride) {
  const int l = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (l >= T) return;                      // uniform per wave
  if (k0s) k0 = k0s[blockIdx.y];           // per-template lag window
  const int64_t m = ((int64_t)k0 + l) & (n - 1);
  const int64_t r = m % n2, c = m / n2;
  const double2* row = Y + (int64_t)blockIdx.y * n + r * n1;
  double re = 0.0, im = 0.0;
  for (int i1 = lane; i1 < n1; i1 += 64) {
    const double2 y = row[i1];
    const double2 w = tab1[(int)((i1 * c) & (n1 - 1))];
    re += y.x * w.x - y.y * w.y;
    im += y.x * w.y + y.y * w.x;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    re += __shfl_xor(re, o);
    im += __shfl_xor(im, o);
  }
  if (lane == 0) out[(int64_t)blockIdx.y * stride + l] = make_double2(re * scale, im * scale);
}

// Correlation lags without the pass-A intermediate: the workgroup's C
// column transforms (as k_pass_a, inter-pass twiddle included) are reduced at
// once to their share of every kept lag m = k0 + l,
//   part[b][g][l] = sum_{i1 in group g} Y[m mod N2][i1] exp(+2 pi i i1 (m div N2) / N1),
// and k_corr_reduce adds the N1 / C shares of each lag in a fixed order.
// V = double2: FP64 column transforms and shares (tap construction); V =
// float2: FP32 column transforms of the integrand rounded once from FP64, each
// share summed in FP64 and stored in FP32 (half the share traffic), the shares
// then added in FP64 (the streaming reference series, like the FP32 dechirp
// passes).
template <typename V, int L, class LD>
__global__ __launch_bounds__(kNT) void k_corr_part(LD ld, V* __restrict__ part, const double2* __restrict__ coarse,
                                                 const double2* __restrict__ fine, const V* __restrict__ tabL,
                                                 int n1, int k0, const int32_t* __restrict__ k0s, int T) {
  constexpr int C = Cols<V>::value(L);
  constexpr int LP = lds_col<L>();
  extern __shared__ __align__(16) unsigned char smem[];
  V* buf = reinterpret_cast<V*>(smem);
  V* twl = buf + C * LP;
  const int b = blockIdx.y;
  if (k0s) k0 = k0s[b];                    // per-template lag window
  // column group of this workgroup: consecutive workgroups go to different
  // XCDs (round robin over 8), so groups g and g + 1, which read the two
  // halves of the same cache lines, are given to workgroups of one XCD
  const int G = gridDim.x;
  const int g = (G % 8 == 0) ? (int)(blockIdx.x % 8) * (G / 8) + (int)(blockIdx.x / 8) : (int)blockIdx.x;
  const int c0 = g * C;
  const int64_t n = (int64_t)n1 * L;
  load_twl<V, L>(twl, tabL, 1);
  gather_columns<V, L, C, kGatherU>(buf, ld, b, c0, n1);
  __syncthreads();
  lds_fft<V, L, C, kNT>(buf, twl, +1);
  __syncthreads();
  // share of lag m = k0 + l: sum_c Y_c[m mod L] e^{+2 pi i (c0 + c) m / N}
  // (the inter-pass twiddle and the N1-point DFT at m div L in one factor).
  // The factor is e^{+2 pi i c0 m / N} (e^{+2 pi i m / N})^c, in FP64: the
  // first part turns by e^{+2 pi i c0 kNT / N} from one of the thread's lags
  // to its next, the second is read at m (consecutive over a wave's lanes), so
  // no table read depends on the column.
  V* pb = part + ((int64_t)b * G + g) * T;
  const uint64_t nmask = (uint64_t)n - 1;
  const uint64_t m_first = (uint64_t)((int64_t)k0 + (int64_t)threadIdx.x) & nmask;
  const double2 adv = twiddle_n(coarse, fine, (uint32_t)(((uint64_t)c0 * kNT) & nmask), +1);
  double2 base = twiddle_n(coarse, fine, (uint32_t)(((uint64_t)c0 * m_first) & nmask), +1);
  for (int l = threadIdx.x; l < T; l += kNT) {
    const uint32_t m = (uint32_t)((uint64_t)((int64_t)k0 + l) & nmask);
    const int r = (int)(m % L);
    const double2 step = twiddle_n(coarse, fine, m, +1);
    double2 f = base;
    double re = 0.0, im = 0.0;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const V v = buf[c * LP + lpad(r)];
      re += (double)v.x * f.x - (double)v.y * f.y;
      im += (double)v.x * f.y + (double)v.y * f.x;
      if (c + 1 < C) f = cmul(f, step);
    }
    if constexpr (std::is_same<V, float2>::value)
      pb[l] = make_float2((float)re, (float)im);
    else
      pb[l] = make_double2(re, im);
    base = cmul(base, adv);
  }
}

// 32 lags per workgroup; 8 slices of the groups per lag (slice s adds groups
// s, s + 8, ...), then the slices in order: a fixed summation order.
template <typename V>
__global__ __launch_bounds__(256) void k_corr_reduce(const V* __restrict__ part, int groups, int T,
                                                   double scale, double2* __restrict__ out, int64_t stride) {
  __shared__ double2 red[8][32];
  const int ll = threadIdx.x & 31, sl = threadIdx.x >> 5;
  const int l = blockIdx.x * 32 + ll;
  double re = 0.0, im = 0.0;
  if (l < T) {
    const V* pb = part + (int64_t)blockIdx.y * groups * T + l;
    for (int g = sl; g < groups; g += 8) {
      const V v = pb[(int64_t)g * T];
      re += v.x;
      im += v.y;
    }
  }
  red[sl][ll] = make_double2(re, im);
  __syncthreads();
  if (sl == 0 && l < T) {
#pragma unroll
    for (int k = 1; k < 8; ++k) {
      re += red[k][ll].x;
      im += red[k][ll].y;
    }
    out[(int64_t)blockIdx.y * stride + l] = make_double2(re * scale, im * scale);
  }
}

// ------------------------------------------------------- small kernels
// sigma^2 = sum_i w_i |h_i|^2 in FP64 by one workgroup (fixed order).
__global__ __launch_bounds__(1024) void k_sigma_sq(const double* __restrict__ w, const double2* __restrict__ h,
                                                  int64_t nb, int64_t stride, double* __restrict__ out) {
  __shared__ double red[1024];
  const double2* hb = h + (int64_t)blockIdx.x * stride;
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < nb; i += 1024) {
    double2 v = hb[i];
    acc += w[i] * (v.x * v.x + v.y * v.y);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 512; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

// sigma^2 of each reference of a batch in two steps of fixed order:
// kSigParts workgroups per reference reduce contiguous bin ranges to
// partial sums, then one thread per reference adds its partials in order and
// stores sigma^2 by slot and the filter scale 1 / (sigma alpha).
__global__ __launch_bounds__(256) void k_sigma_part(const double* __restrict__ w, DechirpRefs r, int64_t nb,
                                                   double* __restrict__ part) {
  __shared__ double red[256];
  const double2* hb = r.h[blockIdx.y];
  const int64_t chunk = (nb + kSigParts - 1) / kSigParts;
  const int64_t i0 = (int64_t)blockIdx.x * chunk, i1 = std::min<int64_t>(i0 + chunk, nb);
  double acc = 0.0;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += 256) {
    const double2 v = hb[i];
    acc += w[i] * (v.x * v.x + v.y * v.y);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.y * kSigParts + blockIdx.x] = red[0];
}
__global__ void k_sigma_final(DechirpRefs r, int nr, const double* __restrict__ part,
                              double* __restrict__ sig2_by_slot, double* __restrict__ scale, double inv_alpha) {
  const int b = threadIdx.x;
  if (b >= nr) return;
  double s2 = 0.0;
  for (int k = 0; k < kSigParts; ++k) s2 += part[b * kSigParts + k];
  sig2_by_slot[r.slot[b]] = s2;
  scale[b] = inv_alpha / sqrt(s2);
}

// F[i] = w_i conj(h_i) / (sigma * alpha), FP64 then rounded to FP32.
__global__ void k_build_filter(const double* __restrict__ w, const double2* __restrict__ h, int64_t nb,
                               int64_t hstride, const double* __restrict__ sigma_sq, double inv_alpha,
                               int64_t i_low, int64_t n_band, float2* __restrict__ out, int64_t ostride,
                               int band_only) {
  const int b = blockIdx.y;
  const double s = inv_alpha / sqrt(sigma_sq[b]);
  int64_t cnt = band_only ? n_band : nb;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < cnt; k += (int64_t)gridDim.x * blockDim.x) {
    int64_t i = band_only ? k + i_low : k;
    double2 v = h[(int64_t)b * hstride + i];
    double f = w[i] * s;
    out[(int64_t)b * ostride + k] = make_float2((float)(f * v.x), (float)(-f * v.y));
  }
}

// F[i] = w_i conj(h_i) / (sigma * alpha) kept in FP64 (reference filter).
__global__ void k_build_filter64(const double* __restrict__ w, const double2* __restrict__ h, int64_t nb,
                                 const double* __restrict__ sigma_sq, double inv_alpha, double2* __restrict__ out) {
  const double s = inv_alpha / sqrt(sigma_sq[0]);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nb; i += (int64_t)gridDim.x * blockDim.x) {
    double2 v = h[i];
    double f = w[i] * s;
    out[i] = make_double2(f * v.x, -f * v.y);
  }
}

__global__ void k_sqrt_to(const double* __restrict__ in, double* __restrict__ out, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = sqrt(in[i]);
}

// ------------------------------------------------------------ launchers
// The segment transform and the reference filters run in FP64: they are
// cheap (once per segment / per reference) and the ratio FIR amplifies any
// white rounding noise in the reference series by its out-of-band gain.
int launch_data_fft(Plan& p, const double* data) {
  LoadData64 ld{data, p.data_scale / p.fs};
  int rc = run_pass_a<double2>(p, ld, p.work64, p.tw64c, p.tw64f, p.tw64_n2, 1, -1);
  if (rc) return rc;
  StoreSpectrum64 st{p.stilde64, p.stilde, p.n / 2};
  return run_pass_b<double2>(p, p.work64, st, p.tw64_n1, 1, -1);
}

int dechirp_batch_size(const Plan& p) {
  // intermediates of a batch (FP32 or FP64 complex): at most 64 MiB and
  // kDechirpBatch references.  A batch's pass-A output then stays small
  // beside the 256 MB last-level cache when pass B reads it back (0.61 ->
  // 0.56 ms for 32 references at N = 2^20 against 256 MiB batches)
  const int64_t elem = p.dechirp_fp64 ? (int64_t)sizeof(double2) : (int64_t)sizeof(float2);
  int64_t b = ((int64_t)64 << 20) / (p.n * elem);
  return (int)std::max<int64_t>(1, std::min<int64_t>(b, kDechirpBatch));
}

size_t dechirp_work_double2(const Plan& p) {
  const int64_t elem = p.dechirp_fp64 ? (int64_t)sizeof(double2) : (int64_t)sizeof(float2);
  return (size_t)((dechirp_batch_size(p) * p.n * elem + (int64_t)sizeof(double2) - 1) / (int64_t)sizeof(double2));
}

// Every reference through the same launches, in batches: sigma^2 (by slot,
// into p.dref_sig2, from kSigParts partial sums each), then pass A with the filter formed on the fly, then
// pass B into each reference's slot of the series store.
int launch_dechirp_refs(Plan& p, int n_refs, const int32_t* ref_ids, const double* const* h_refs) {
  const int bs = dechirp_batch_size(p);
  double2* work = bs > 1 ? p.work64b : p.work64;
  if (bs > 1 && p.work64b_cap < dechirp_work_double2(p)) return fail(RFD_E_STATE, "dechirp: batch buffer too small");
  for (int r0 = 0; r0 < n_refs; r0 += bs) {
    const int nr = std::min(bs, n_refs - r0);
    DechirpRefs refs{};
    for (int b = 0; b < nr; ++b) {
      refs.h[b] = reinterpret_cast<const double2*>(h_refs[r0 + b]);
      refs.slot[b] = ref_ids[r0 + b];
    }
    hipLaunchKernelGGL(k_sigma_part, dim3(kSigParts, (unsigned)nr), dim3(256), 0, p.stream, p.w, refs, p.nb,
                       p.dref_part);
    RFD_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_sigma_final, dim3(1), dim3(kDechirpBatch), 0, p.stream, refs, nr,
                       (const double*)p.dref_part, p.dref_sig2, p.dref_scale, 1.0 / p.data_scale);
    RFD_CHECK_LAUNCH();
    LoadDechirpRefs ld{p.stilde64, p.w, refs, p.dref_scale, p.i_low, p.i_high};
    int rc;
    if (p.dechirp_fp64) {
      rc = run_pass_a<double2>(p, ld, work, p.tw64c, p.tw64f, p.tw64_n2, nr, +1);
      if (rc) return rc;
      StoreRefSlots st{p.zref, p.n, refs};
      rc = run_pass_b<double2>(p, work, st, p.tw64_n1, nr, +1);
    } else {
      // the integrand (and the reference norm) in FP64, both transform passes in
      // FP32 with twiddles rounded once from FP64
      float2* w32 = reinterpret_cast<float2*>(work);
      rc = run_pass_a<float2>(p, LoadDechirpRefs32{ld}, w32, p.tw32c, p.tw32f, p.tw32_n2, nr, +1);
      if (rc) return rc;
      StoreRefSlots32 st{p.zref, p.n, refs};
      rc = run_pass_b<float2>(p, w32, st, p.tw32_n1, nr, +1);
    }
    if (rc) return rc;
  }
  return RFD_OK;
}

// Band series of one reference: the dechirp integrand restricted to bins
// [edges[b], edges[b+1]) and transformed, for every band (FP32 out, [p][N]).
int launch_dechirp_bands(Plan& p, const double* h_ref, const int64_t* edges, int n_bands, float2* out) {
  double* sig = p.dscratch + 16;
  hipLaunchKernelGGL(k_sigma_sq, dim3(1), dim3(1024), 0, p.stream, p.w, (const double2*)h_ref, p.nb, p.nb, sig);
  RFD_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_build_filter64, dim3(256), dim3(256), 0, p.stream, p.w, (const double2*)h_ref, p.nb,
                     (const double*)sig, 1.0 / p.data_scale, p.fref64);
  RFD_CHECK_LAUNCH();
  for (int b = 0; b < n_bands; ++b) {
    LoadDechirp64 ld{p.stilde64, p.fref64, edges[b], edges[b + 1] - 1};
    int rc = run_pass_a<double2>(p, ld, p.work64, p.tw64c, p.tw64f, p.tw64_n2, 1, +1);
    if (rc) return rc;
    StoreBand st{out + (int64_t)b * p.n};
    rc = run_pass_b<double2>(p, p.work64, st, p.tw64_n1, 1, +1);
    if (rc) return rc;
  }
  return RFD_OK;
}

int launch_findchirp_prepare(Plan& p, const double* h, int64_t count, float2* filt, double* sigma) {
  // sigma^2 into the output buffer (or scratch), then the filters
  double* s2 = sigma;
  for (int64_t b0 = 0; b0 < count; b0 += 65535) {
    int64_t nbat = count - b0 < 65535 ? count - b0 : 65535;
    hipLaunchKernelGGL(k_sigma_sq, dim3((unsigned)nbat), dim3(1024), 0, p.stream, p.w,
                       (const double2*)h + b0 * p.nb, p.nb, p.nb, s2 + b0);
    RFD_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_build_filter, dim3(64, (unsigned)nbat), dim3(256), 0, p.stream, p.w,
                       (const double2*)h + b0 * p.nb, p.nb, p.nb, (const double*)(s2 + b0), 1.0 / p.data_scale,
                       p.i_low, p.n_band, filt + b0 * p.n_band, p.n_band, 1);
    RFD_CHECK_LAUNCH();
  }
  hipLaunchKernelGGL(k_sqrt_to, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, p.stream, s2, s2, count);
  RFD_CHECK_LAUNCH();
  return RFD_OK;
}

// FINDCHIRP pass A for N2 = N / 4096 > 256 (segments of 2^21 and 2^22
// samples): the LDS Stockham column transform into the [N2][4096] layout of
// the register-FFT row pass, twiddles from the 4096-entry table.
int launch_fc_cols_lds(Plan& p, const float2* filt, int nb, float2* Y, int n1, int n2) {
  LoadFindchirp ld{p.stilde, filt, p.i_low, p.i_high, p.n_band};
  dim3 blk(kNT);
  switch (n2) {
#define CASE_L(LL)                                                                             \
  case LL: {                                                                                   \
    constexpr int C = Cols<float2>::value(LL);                                                 \
    size_t sh = lds_bytes<float2, LL, C>();                                                    \
    hipLaunchKernelGGL((k_pass_a<float2, LL, LoadFindchirp>), dim3(n1 / C, nb), blk, sh, p.stream, \
                       ld, Y, p.tw32c, p.tw32f, p.ols_tw32, n1, +1, 4096 / LL, 0, LL);         \
    break;                                                                                     \
  }
    CASE_L(512) CASE_L(1024)
#undef CASE_L
    default: return fail(RFD_E_UNSUPPORTED, "findchirp: unsupported column length");
  }
  RFD_CHECK_LAUNCH();
  return RFD_OK;
}

int launch_corr64(Plan& p, Taps& tp, int mode, const double* h_r, const double* h_t, int64_t batch, int T,
                  int k0, double2* out, int64_t out_stride, int64_t lo, int64_t hi, const int32_t* k0s, bool fp32,
                  const double* bscale) {
  size_t need = (size_t)batch * p.n;
  if (tp.work64_cap < need) return fail(RFD_E_INVALID, "corr64: work buffer too small");
  if (fp32 && mode == 0 && !bscale) return fail(RFD_E_INVALID, "corr64: FP32 integrands need their normalisation");
  // (a single-spectrum mode reads its spectrum as the second one too: the
  // loads need no branch on the mode)
  LoadCorr64 ld{p.w, (const double2*)h_r, (const double2*)(h_t ? h_t : h_r), h_t ? p.nb : 0,
                lo >= 0 ? lo : p.i_low, hi >= 0 ? hi : p.i_high, mode, mode == 0 ? bscale : nullptr};
  const double scale = mode == 2 ? 1.0 / (double)p.n : 1.0;
  // fused form: per-workgroup lag shares in the work buffer, then their sums
  const int C = fp32 ? Cols<float2>::value(p.n2) : Cols<double2>::value(p.n2);
  const int groups = p.n1 / C;
  if ((int64_t)groups * T <= p.n) {
    dim3 blk(kNT);
    switch (p.n2) {
#define CASE_C(LL)                                                                                       \
  case LL: {                                                                                             \
    if (fp32) {                                                                                          \
      const size_t sh = lds_bytes<float2, LL, Cols<float2>::value(LL)>();                                \
      hipLaunchKernelGGL((k_corr_part<float2, LL, LoadCorr32>), dim3(groups, (unsigned)batch), blk, sh,  \
                         p.stream, LoadCorr32{ld}, (float2*)tp.work64, (const double2*)p.tw64c,             \
                         (const double2*)p.tw64f, p.tw32_n2, p.n1, k0, k0s, T);                            \
    } else {                                                                                             \
      const size_t sh = lds_bytes<double2, LL, Cols<double2>::value(LL)>();                              \
      hipLaunchKernelGGL((k_corr_part<double2, LL, LoadCorr64>), dim3(groups, (unsigned)batch), blk, sh, \
                         p.stream, ld, tp.work64, (const double2*)p.tw64c, (const double2*)p.tw64f,          \
                         p.tw64_n2, p.n1, k0, k0s, T);                                                     \
    }                                                                                                    \
    break;                                                                                               \
  }
      CASE_C(32) CASE_C(64) CASE_C(128) CASE_C(256) CASE_C(512) CASE_C(1024) CASE_C(2048)
#undef CASE_C
      default: return fail(RFD_E_UNSUPPORTED, "fft: unsupported N2");
    }
    RFD_CHECK_LAUNCH();
    if (fp32)
      hipLaunchKernelGGL(k_corr_reduce<float2>, dim3((unsigned)((T + 31) / 32), (unsigned)batch), dim3(256), 0,
                         p.stream, (const float2*)tp.work64, groups, T, scale, out, out_stride);
    else
      hipLaunchKernelGGL(k_corr_reduce<double2>, dim3((unsigned)((T + 31) / 32), (unsigned)batch), dim3(256), 0,
                         p.stream, (const double2*)tp.work64, groups, T, scale, out, out_stride);
    RFD_CHECK_LAUNCH();
    return RFD_OK;
  }
  // k_lags_direct reads the pass-A rows (k0 + l) mod N2, l < T (every row
  // when the lag window differs per template)
  const int row_lo = k0s ? 0 : (int)(((int64_t)k0 % p.n2 + p.n2) % p.n2);
  int rc = run_pass_a<double2>(p, ld, tp.work64, p.tw64c, p.tw64f, p.tw64_n2, (int)batch, +1, row_lo,
                               k0s ? p.n2 : T);
  if (rc) return rc;
  hipLaunchKernelGGL(k_lags_direct, dim3((unsigned)((T + 3) / 4), (unsigned)batch), dim3(256), 0, p.stream,
                     (const double2*)tp.work64, p.n, p.n1, p.n2, (const double2*)p.tw64_n1, k0, k0s, T, scale, out,
                     out_stride);
  RFD_CHECK_LAUNCH();
  return RFD_OK;
}


// ------------------------------------------------- lag of the correlation peak
// |b|^2 of pass B's output (natural order) for the peak search
struct StorePow {
  double* pw;
  int64_t n;
  __device__ void operator()(int b, int64_t idx, double2 v) const { pw[(int64_t)b * n + idx] = v.x * v.x + v.y * v.y; }
};

// Per template: the lag of the largest |b[l]|^2 over all N lags (lowest
// index 0..N-1 on exact ties), mapped into (-N/2, N/2]; the lag window
// k0_j = peak - floor(T/2) and its offset from the sub-bank's k0.  Two
// stages: kPeakParts workgroups per template each reduce one contiguous
// chunk to (value, index), then one thread per template takes the chunks
// in index order (a strict > keeps the lowest index).
__global__ __launch_bounds__(256) void k_peak_part(const double* __restrict__ pw, int64_t n,
                                                 double* __restrict__ pv, int64_t* __restrict__ pi) {
  __shared__ double bv[256];
  __shared__ int64_t bi[256];
  const int64_t chunk = n / kPeakParts;              // n is a power of two >= 1024
  const double* row = pw + (int64_t)blockIdx.y * n + (int64_t)blockIdx.x * chunk;
  double best = -1.0;
  int64_t idx = 0;
  for (int64_t i = threadIdx.x; i < chunk; i += 256) {
    const double v = row[i];
    if (v > best) {          // increasing i: the first maximum stays
      best = v;
      idx = i;
    }
  }
  bv[threadIdx.x] = best;
  bi[threadIdx.x] = idx;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      const double v = bv[threadIdx.x + o];
      const int64_t j = bi[threadIdx.x + o];
      if (v > bv[threadIdx.x] || (v == bv[threadIdx.x] && j < bi[threadIdx.x])) {
        bv[threadIdx.x] = v;
        bi[threadIdx.x] = j;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    pv[(int64_t)blockIdx.y * kPeakParts + blockIdx.x] = bv[0];
    pi[(int64_t)blockIdx.y * kPeakParts + blockIdx.x] = (int64_t)blockIdx.x * chunk + bi[0];
  }
}
__global__ void k_peak_lag(const double* __restrict__ pv, const int64_t* __restrict__ pi, int64_t batch, int64_t n,
                           int T, int k0_sb, int32_t* __restrict__ k0_out, int32_t* __restrict__ d_out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= batch) return;
  double best = -1.0;
  int64_t i = 0;
  for (int c = 0; c < kPeakParts; ++c) {
    const double v = pv[t * kPeakParts + c];
    if (v > best) {
      best = v;
      i = pi[t * kPeakParts + c];
    }
  }
  const int lag = (int)(i <= n / 2 ? i : i - n);
  const int k0 = lag - T / 2;
  k0_out[t] = k0;
  if (d_out) d_out[t] = k0 - k0_sb;
}

int launch_corr_peak(Plan& p, Taps& tp, const double* h_r, const double* h_t, int64_t batch, int T, int k0_sb,
                     double* pw, int32_t* k0_out, int32_t* d_out) {
  if (tp.work64_cap < (size_t)batch * p.n) return fail(RFD_E_INVALID, "corr peak: work buffer too small");
  if (tp.peak_cap < (size_t)batch * p.n || tp.peak_parts_cap < (size_t)batch * kPeakParts || p.n < 1024)
    return fail(RFD_E_INVALID, "corr peak: scratch too small");
  LoadCorr64 ld{p.w, (const double2*)h_r, (const double2*)h_t, p.nb, p.i_low, p.i_high, 0, nullptr};
  int rc = run_pass_a<double2>(p, ld, tp.work64, p.tw64c, p.tw64f, p.tw64_n2, (int)batch, +1);
  if (rc) return rc;
  rc = run_pass_b<double2>(p, (const double2*)tp.work64, StorePow{pw, p.n}, p.tw64_n1, (int)batch, +1);
  if (rc) return rc;
  hipLaunchKernelGGL(k_peak_part, dim3(kPeakParts, (unsigned)batch), dim3(256), 0, p.stream, (const double*)pw,
                     p.n, tp.peak_part, tp.peak_idx);
  RFD_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_peak_lag, dim3((unsigned)((batch + 63) / 64)), dim3(64), 0, p.stream,
                     (const double*)tp.peak_part, (const int64_t*)tp.peak_idx, batch, p.n, T, k0_sb, k0_out, d_out);
  RFD_CHECK_LAUNCH();
  return RFD_OK;
}

}  // namespace rfd
