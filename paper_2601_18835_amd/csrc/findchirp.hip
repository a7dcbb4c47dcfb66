// FINDCHIRP baseline: the matched filter of Eq. 1 evaluated the classic way,
// one full-length inverse FFT per template,
//   z_j[n] = sum_i Q_i e^{+2 pi i i n / N},  Q_i = s_i F_j,i  (band bins only),
// with the |z|^2 threshold and window-peak keys fused into the last pass.
//
// Four-step split N = N1 N2 (N1 = 4096 or all of N when N <= 4096),
// i = i1 + N1 i2 and
// n = n2 + N2 n1, so that with w_M = e^{+2 pi i / M}
//   pass A (column i1):  Y[n2][i1] = w_N^(i1 n2) sum_i2 Q[i1 + N1 i2] w_N2^(i2 n2)
//   pass B (row n2):     z[n2 + N2 n1] = sum_i1 Y[n2][i1] w_N1^(i1 n1).
// Pass B is the register-resident N1-point FFT of block_fft.h.  Pass A
// keeps each column's N2 values in registers: up to 16 points one thread
// per column; 32 to 256 points as a radix-16 stage over
// 16 values per thread, an LDS exchange and a radix-N2/16 stage across the
// column's N2/16 threads.  Adjacent lanes take adjacent columns, so every
// load of Q and every store of Y is a run of 16 or more contiguous values.
// The inter-pass twiddles w_N^(i1 n2) of a thread's 16 outputs come from
// three FP64 table values by FP64 recurrence (at most 16 products, so the
// error stays near FP64 rounding), rounded once to FP32: table gathers
// whose addresses stride by n2 across lanes would otherwise dominate.
// Each workgroup of either pass takes several templates (pass A) or rows
// (pass B) in turn and fetches the next one's operands during the current
// transform.
// Segments of 2^21 and 2^22 samples (N2 = 512, 1024) take pass A from the
// LDS Stockham transform instead.  When N <= 4096 there is no pass A: pass B
// loads Q directly.
#include <algorithm>

#include "block_fft.h"
#include "dev_common.h"
#include "rfd_internal.h"

namespace rfd {

constexpr int kFcN1 = 4096;    // row length when N > 4096

// Small in-register DFTs on v[0..N) (N = 1, 2, 4, 8, 16), sign SIGN; slot s
// then holds X[small_freq<N>(s)].
template <int N, int SIGN>
__device__ __forceinline__ void dft_small(float2 (&v)[16]) {
  if constexpr (N == 16) {
    dft16<SIGN>(v);
  } else if constexpr (N == 8) {
    dft4(v[0], v[2], v[4], v[6], SIGN);
    dft4(v[1], v[3], v[5], v[7], SIGN);
#pragma unroll
    for (int k = 1; k < 4; ++k) v[2 * k + 1] = cmul(v[2 * k + 1], w16(2 * k, SIGN));
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const float2 a = v[2 * k], b = v[2 * k + 1];
      v[2 * k] = cadd(a, b);
      v[2 * k + 1] = csub(a, b);
    }
  } else if constexpr (N == 4) {
    dft4(v[0], v[1], v[2], v[3], SIGN);
  } else if constexpr (N == 2) {
    const float2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
}
template <int N>
__device__ __forceinline__ constexpr int small_freq(int s) {
  return N == 16 ? dft16_freq(s) : (N == 8 ? (s >> 1) + 4 * (s & 1) : s);
}

// Pass A geometry: M2 threads per column, CW columns per workgroup.
template <int N2>
struct FcCols {
  static constexpr int M2 = N2 >= 16 ? N2 / 16 : 1;
  static constexpr int CW = 256 / M2;
  static constexpr int V = N2 >= 16 ? 16 : N2;   // values per thread
};

struct FcColArgs {
  const float2* s;           // data spectrum, FP32 [N/2 + 1]
  const float2* filt;        // filters of this batch [count][n_band]
  const float2* tw;          // e^{+2 pi i m / 4096}, m < 4096
  const double2* coarse;     // e^{+2 pi i 1024 k / N} (FP64)
  const double2* fine;       // e^{+2 pi i k / N}, k < 1024 (FP64)
  float2* Y;                 // [count][N2][N1]
  int64_t i_low, i_high, n_band, count;
  uint32_t nmask;            // N - 1
  int JT;                    // templates per workgroup
};

// Pass A: workgroup (x, y) transforms columns [x CW, (x + 1) CW) of templates
// [y JT, (y + 1) JT).  The data values, band offsets and all twiddles of a
// thread are loaded once; the next template's filter values are fetched
// while the current one is transformed.
template <int N1, int N2>
__global__ __launch_bounds__(256) void k_fc_cols(FcColArgs a) {
  using G = FcCols<N2>;
  constexpr int M2 = G::M2, CW = G::CW, V = G::V;
  const int c = threadIdx.x % CW, m = threadIdx.x / CW;
  const uint32_t i1 = blockIdx.x * CW + c;
  const int64_t b0 = (int64_t)blockIdx.y * a.JT;
  const int64_t b1 = std::min<int64_t>(b0 + a.JT, a.count);
  // thread (c, m) holds x[m + M2 r] = Q[i1 + N1 (m + M2 r)], r < V
  float2 sv[V];
  int32_t off[V];                      // filter offset i - i_low, -1 outside the band
#pragma unroll
  for (int r = 0; r < V; ++r) {
    const int64_t i = (int64_t)i1 + (int64_t)N1 * (m + M2 * r);
    const bool in = i >= a.i_low && i <= a.i_high;
    sv[r] = in ? a.s[i] : make_float2(0.f, 0.f);
    off[r] = in ? (int32_t)(i - a.i_low) : -1;
  }
  // inter-pass twiddles w_N^(i1 n2) of the thread's output slots (FP64, rounded once)
  float2 ti[V];
  const double2 w1 = twiddle_n(a.coarse, a.fine, i1 & a.nmask, 1);   // w_N^(i1)
  [[maybe_unused]] float2 ts[16];      // stage twiddles w_N2^(m k1)
  if constexpr (M2 == 1) {
    double2 wt = make_double2(1.0, 0.0);
    double2 wn[V];                     // w_N^(i1 n2), n2 < V
#pragma unroll
    for (int k = 0; k < V; ++k) {
      wn[k] = wt;
      wt = cmul(wt, w1);
    }
#pragma unroll
    for (int s = 0; s < V; ++s) {
      const double2 x = wn[small_freq<V>(s)];
      ti[s] = make_float2((float)x.x, (float)x.y);
    }
  } else {
    // n2 = k1 + 16 k2 with k1 = m (16 / M2) + e:  w_N^(i1 k1) w_N^(16 i1 k2)
    const int k1_0 = m * (16 / M2);
    double2 wk = twiddle_n(a.coarse, a.fine, (i1 * (uint32_t)k1_0) & a.nmask, 1);
    const double2 w16i = twiddle_n(a.coarse, a.fine, (16u * i1) & a.nmask, 1);
    double2 wp[M2];
    wp[0] = make_double2(1.0, 0.0);
#pragma unroll
    for (int k = 1; k < M2; ++k) wp[k] = cmul(wp[k - 1], w16i);
#pragma unroll
    for (int e = 0; e < 16 / M2; ++e) {
#pragma unroll
      for (int s = 0; s < M2; ++s) {
        const double2 x = cmul(wk, wp[dftr_freq<M2>(s)]);
        ti[e * M2 + s] = make_float2((float)x.x, (float)x.y);
      }
      wk = cmul(wk, w1);
    }
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      const int pw = (m * dft16_freq(s)) % N2;
      ts[s] = pw ? a.tw[pw * (4096 / N2)] : make_float2(1.f, 0.f);
    }
  }
  float2 fv[V];
  if (b0 < b1) {
    const float2* fb = a.filt + b0 * a.n_band;
#pragma unroll
    for (int r = 0; r < V; ++r) fv[r] = off[r] >= 0 ? fb[off[r]] : make_float2(0.f, 0.f);
  }
  [[maybe_unused]] __shared__ float2 lds[M2 > 1 ? 16 * M2 * CW : 1];
  for (int64_t b = b0; b < b1; ++b) {
    float2 v[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = r < V ? cmul(sv[r], fv[r]) : make_float2(0.f, 0.f);
    if (b + 1 < b1) {
      const float2* fb = a.filt + (b + 1) * a.n_band;
#pragma unroll
      for (int r = 0; r < V; ++r) fv[r] = off[r] >= 0 ? fb[off[r]] : make_float2(0.f, 0.f);
    }
    float2* Yb = a.Y + b * N2 * N1;
    if constexpr (M2 == 1) {
      dft_small<V, 1>(v);
#pragma unroll
      for (int s = 0; s < V; ++s) Yb[(int64_t)small_freq<V>(s) * N1 + i1] = cmul(v[s], ti[s]);
    } else {
      // radix 16 over r, twiddle, exchange, radix M2 over m
      dft16<1>(v);
#pragma unroll
      for (int s = 0; s < 16; ++s) lds[(dft16_freq(s) * M2 + m) * CW + c] = cmul(v[s], ts[s]);
      __syncthreads();
#pragma unroll
      for (int e = 0; e < 16 / M2; ++e)
#pragma unroll
        for (int u = 0; u < M2; ++u) v[e * M2 + u] = lds[((m * (16 / M2) + e) * M2 + u) * CW + c];
      __syncthreads();                 // the next template rewrites the exchange buffer
      dft_r<M2, 1>(v);
#pragma unroll
      for (int e = 0; e < 16 / M2; ++e)
#pragma unroll
        for (int s = 0; s < M2; ++s) {
          const int n2 = m * (16 / M2) + e + 16 * dftr_freq<M2>(s);
          Yb[(int64_t)n2 * N1 + i1] = cmul(v[e * M2 + s], ti[e * M2 + s]);
        }
    }
  }
}

struct FcRowArgs {
  const float2* Y;           // [count][N2][N1] (pass A output), or
  const float2* s;           // with no pass A: data spectrum and filters
  const float2* filt;
  const float2* tw;          // e^{+2 pi i m / 4096}
  unsigned long long* slots;
  int64_t i_low, i_high, n_band;
  int64_t N2, count, tmpl0, nwin, W;
  float thr2;                // threshold^2 of the compaction
  int JR;                    // (template, row) pairs per FFT slot of a workgroup
};

// Window-peak key: bits(rho^2) over the complement of the offset in the window.
__device__ __forceinline__ unsigned long long fc_key(float r2, uint32_t off) {
  return ((unsigned long long)__float_as_uint(r2) << 32) | (unsigned long long)(0xFFFFFFFFu - off);
}

// Pass B: FFT slot f of workgroup x takes (template, row) pairs
// (x JR + j) F + f, j < JR, fetching the next pair's values while the
// current one is transformed.
template <int N1, bool DIRECT>
__global__ __launch_bounds__(256) void k_fc_rows(FcRowArgs a) {
  using S = BlockFft<N1>;
  __shared__ float2 lds[S::F * S::LDS];
  const int f = threadIdx.x / S::NTf, t = threadIdx.x % S::NTf;
  const int64_t npairs = a.count * a.N2;
  BlockFftTw<N1> w;
  block_fft_twiddles<N1, 1>(w, a.tw, t);
  [[maybe_unused]] float2 sv[16];      // data values (one-pass form: the same for every template)
  [[maybe_unused]] int32_t off[16];
  if constexpr (DIRECT) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int64_t i = t + S::NTf * r;
      const bool in = i >= a.i_low && i <= a.i_high;
      sv[r] = in ? a.s[i] : make_float2(0.f, 0.f);
      off[r] = in ? (int32_t)(i - a.i_low) : -1;
    }
  }
  auto fetch = [&](int64_t pair, float2 (&x)[16]) {
    if (pair >= npairs) return;
    if constexpr (DIRECT) {
      const float2* fb = a.filt + pair * a.n_band;
#pragma unroll
      for (int r = 0; r < 16; ++r) x[r] = off[r] >= 0 ? fb[off[r]] : make_float2(0.f, 0.f);
    } else {
      const float2* yr = a.Y + pair * N1;
#pragma unroll
      for (int r = 0; r < 16; ++r) x[r] = yr[t + S::NTf * r];
    }
  };
  const int64_t base = (int64_t)blockIdx.x * a.JR * S::F + f;
  float2 nx[16];
  fetch(base, nx);
  for (int j = 0; j < a.JR; ++j) {
    const int64_t pair = base + (int64_t)j * S::F;
    const bool valid = pair < npairs;
    float2 v[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      if constexpr (DIRECT) v[r] = valid ? cmul(sv[r], nx[r]) : make_float2(0.f, 0.f);
      else v[r] = valid ? nx[r] : make_float2(0.f, 0.f);
    }
    fetch(pair + S::F, nx);
    block_fft<N1, 1>(v, lds + f * S::LDS, t, w);
    float r2[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) r2[q] = v[q].x * v[q].x + v[q].y * v[q].y;
    float r2max = r2[0];
#pragma unroll
    for (int q = 1; q < 15; q += 2) r2max = fmaxf(fmaxf(r2max, r2[q]), r2[q + 1]);
    r2max = fmaxf(r2max, r2[15]);
    // only samples above the threshold can be a reported window peak
    if (!valid || !__any(r2max > a.thr2)) continue;
    const int64_t b = pair / a.N2, row = pair % a.N2;
    unsigned long long* slot = a.slots + (a.tmpl0 + b) * a.nwin;
#pragma unroll
    for (int e = 0; e < 16 / S::R; ++e)
#pragma unroll
      for (int s = 0; s < S::R; ++s) {
        const float x = r2[e * S::R + s];
        if (x > a.thr2) {
          const int64_t n = row + a.N2 * block_fft_out<N1>(t, e, s);
          const int64_t q = n / a.W;
          atomicMax(slot + q, fc_key(x, (uint32_t)(n - q * a.W)));
        }
      }
  }
}

// Items per workgroup so that a launch holds about kFcWgPerCu workgroups per
// compute unit (at least one item each, at most 16).  Measured on MI355X at
// N = 2^19: two workgroups per CU with up to 16 items beat one per item by
// 1.5x (the prefetch hides the loads) and beat one per CU by 1.2x.
constexpr int kFcWgPerCu = 2;
static int fc_items_per_wg(int64_t wgs_at_one, int n_cu) {
  int64_t j = wgs_at_one / ((int64_t)kFcWgPerCu * n_cu);
  return (int)std::max<int64_t>(1, std::min<int64_t>(16, j));
}

template <int N2>
static void launch_cols(Plan& p, FcColArgs a) {
  const int64_t gx = kFcN1 / FcCols<N2>::CW;
  a.JT = fc_items_per_wg(gx * a.count, p.n_cu);
  const unsigned gy = (unsigned)((a.count + a.JT - 1) / a.JT);
  hipLaunchKernelGGL((k_fc_cols<kFcN1, N2>), dim3((unsigned)gx, gy), dim3(256), 0, p.stream, a);
}

template <int N1, bool DIRECT>
static void launch_rows(Plan& p, FcRowArgs a) {
  const int64_t F = BlockFft<N1>::F;
  const int64_t slots = (a.count * a.N2 + F - 1) / F;
  a.JR = fc_items_per_wg(slots, p.n_cu);
  const unsigned gx = (unsigned)((slots + a.JR - 1) / a.JR);
  hipLaunchKernelGGL((k_fc_rows<N1, DIRECT>), dim3(gx), dim3(256), 0, p.stream, a);
}

int findchirp_batch_size(const Plan& p) {
  // pass-A output of a batch: up to 256 MiB (64 templates at N = 2^19)
  int64_t b = ((int64_t)256 << 20) / (p.n * (int64_t)sizeof(float2));
  if (b < 1) b = 1;
  if (b > 64) b = 64;
  return (int)b;
}

size_t findchirp_work_size(const Plan& p) {
  // the [N2][N1] intermediate of a batch; none when one pass covers N
  return p.n > kFcN1 ? (size_t)findchirp_batch_size(p) * (size_t)p.n : 0;
}

int launch_findchirp(Plan& p, const float2* filt, int64_t n_templates, int64_t W, int64_t nwin, float threshold) {
  const int64_t N1 = std::min<int64_t>(p.n, kFcN1);
  const int64_t N2 = p.n / N1;
  if (p.fc_work_cap < findchirp_work_size(p)) return fail(RFD_E_STATE, "findchirp: work buffer too small");
  const int bs = findchirp_batch_size(p);
  for (int64_t t0 = 0; t0 < n_templates; t0 += bs) {
    const int nb = (int)std::min<int64_t>(n_templates - t0, bs);
    const float2* fb = filt + t0 * p.n_band;
    if (N2 > 1) {
      FcColArgs ca{p.stilde, fb, p.ols_tw32, p.tw64c, p.tw64f, p.fc_work, p.i_low, p.i_high, p.n_band, nb,
                   (uint32_t)(p.n - 1), 1};
      switch (N2) {
        case 2: launch_cols<2>(p, ca); break;
        case 4: launch_cols<4>(p, ca); break;
        case 8: launch_cols<8>(p, ca); break;
        case 16: launch_cols<16>(p, ca); break;
        case 32: launch_cols<32>(p, ca); break;
        case 64: launch_cols<64>(p, ca); break;
        case 128: launch_cols<128>(p, ca); break;
        case 256: launch_cols<256>(p, ca); break;
        default: {
          int rc = launch_fc_cols_lds(p, fb, nb, p.fc_work, (int)N1, (int)N2);
          if (rc) return rc;
        }
      }
      RFD_CHECK_LAUNCH();
    }
    FcRowArgs ra{p.fc_work, p.stilde, fb, p.ols_tw32, p.slots, p.i_low, p.i_high, p.n_band,
                 N2, nb, t0, nwin, W, threshold * threshold, 1};
    if (N2 > 1) {
      launch_rows<kFcN1, false>(p, ra);
    } else {
      switch (N1) {
        case 1024: launch_rows<1024, true>(p, ra); break;
        case 2048: launch_rows<2048, true>(p, ra); break;
        case 4096: launch_rows<4096, true>(p, ra); break;
        default: return fail(RFD_E_UNSUPPORTED, "findchirp: unsupported segment length");
      }
    }
    RFD_CHECK_LAUNCH();
  }
  return RFD_OK;
}

}  // namespace rfd
