// Trigger accumulation (Table II's last stage): slot clearing, deterministic
// compaction of the per-(template, window) peak keys by prefix sum, and the
// FP32 re-evaluation of the complex SNR at each trigger.
#include <algorithm>

#include "dev_common.h"
#include "rfd_internal.h"

namespace rfd {

constexpr int kSegThreads = 256;
constexpr int kSegPer = 16;
constexpr int kSeg = kSegThreads * kSegPer;   // slots per compaction block
// Each wave of a compaction block takes kSegPer rounds of 64 consecutive
// slots (1024 in all, coalesced 512-byte reads); the waves of a block and the
// blocks follow each other in slot order, so the triggers come out in
// ascending slot order.

__device__ __forceinline__ int64_t map_slot(const WinMap& m, int64_t v) {
  const int64_t t = v / m.nq, qi = v - t * m.nq;
  const int64_t q = qi < m.cnt0 ? m.lo0 + qi : m.lo1 + (qi - m.cnt0);
  return t * m.nwin + q;
}
// every window of every template, in order: slot index = visit index
__device__ __forceinline__ bool map_identity(const WinMap& m) {
  return m.nq == m.nwin && m.cnt0 == m.nq && m.lo0 == 0;
}

__global__ void k_fill_u64(unsigned long long* __restrict__ p, int64_t n, WinMap m) {
  const bool ident = map_identity(m);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[ident ? i : map_slot(m, i)] = 0ull;
}

__device__ __forceinline__ bool slot_fires(unsigned long long k, float thr2) {
  return k != 0ull && __uint_as_float((uint32_t)(k >> 32)) > thr2;
}

// lanes below this one whose bit is set in a wave-wide mask
__device__ __forceinline__ int lanes_below(unsigned long long mask) {
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// The wave's keys and firing masks over its kSegPer rounds.
struct WaveSlots {
  unsigned long long key[kSegPer];
  unsigned long long fire[kSegPer];
  int count;
};
__device__ __forceinline__ void wave_slots(WaveSlots& w, const unsigned long long* __restrict__ slots, int64_t n,
                                           float thr2, const WinMap& m, int64_t base) {
  const int lane = threadIdx.x & 63;
  const bool ident = map_identity(m);
  w.count = 0;
#pragma unroll
  for (int r = 0; r < kSegPer; ++r) {
    const int64_t v = base + 64 * r + lane;
    w.key[r] = v < n ? slots[ident ? v : map_slot(m, v)] : 0ull;
    w.fire[r] = __ballot(slot_fires(w.key[r], thr2));
    w.count += __popcll(w.fire[r]);
  }
}

__global__ __launch_bounds__(kSegThreads) void k_count(const unsigned long long* __restrict__ slots, int64_t n,
                                                     float thr2, long long* __restrict__ counts, WinMap m) {
  __shared__ int wc[kSegThreads / 64];
  const int wave = threadIdx.x >> 6;
  WaveSlots w;
  wave_slots(w, slots, n, thr2, m, (int64_t)blockIdx.x * kSeg + (int64_t)wave * 64 * kSegPer);
  if ((threadIdx.x & 63) == 0) wc[wave] = w.count;
  __syncthreads();
  if (threadIdx.x == 0) {
    long long c = 0;
    for (int i = 0; i < kSegThreads / 64; ++i) c += wc[i];
    counts[blockIdx.x] = c;
  }
}

// single-workgroup exclusive scan of the block counts; total at counts[nblk]
__global__ __launch_bounds__(1024) void k_scan(long long* __restrict__ counts, int64_t nblk,
                                             long long* __restrict__ total) {
  __shared__ long long sh[1024];
  __shared__ long long carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int64_t b0 = 0; b0 < nblk; b0 += 1024) {
    int64_t i = b0 + threadIdx.x;
    long long v = i < nblk ? counts[i] : 0;
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
      long long x = threadIdx.x >= (unsigned)o ? sh[threadIdx.x - o] : 0;
      __syncthreads();
      sh[threadIdx.x] += x;
      __syncthreads();
    }
    if (i < nblk) counts[i] = carry + sh[threadIdx.x] - v;
    long long add = sh[1023];
    __syncthreads();
    if (threadIdx.x == 0) carry += add;
    __syncthreads();
  }
  if (threadIdx.x == 0) *total = carry;
}

__device__ __forceinline__ int find_subbank(const int64_t* first, int nsb, int64_t t) {
  int lo = 0, hi = nsb - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (first[mid] <= t) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__global__ __launch_bounds__(kSegThreads) void k_write(const unsigned long long* __restrict__ slots, int64_t n,
                                                     float thr2, const long long* __restrict__ offs, int64_t nwin,
                                                     int64_t W, rfd_trigger* __restrict__ out, int64_t capacity,
                                                     const int64_t* __restrict__ sb_first, int nsb, WinMap m,
                                                     const int32_t* __restrict__ shift, int64_t nseg) {
  __shared__ int wc[kSegThreads / 64];
  const int wave = threadIdx.x >> 6;
  const int64_t base = (int64_t)blockIdx.x * kSeg + (int64_t)wave * 64 * kSegPer;
  WaveSlots w;
  wave_slots(w, slots, n, thr2, m, base);
  if ((threadIdx.x & 63) == 0) wc[wave] = w.count;
  __syncthreads();
  if (w.count == 0) return;     // wave-uniform; no barrier follows
  int64_t pos = offs[blockIdx.x];
  for (int i = 0; i < wave; ++i) pos += wc[i];
  const bool ident = map_identity(m);
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int r = 0; r < kSegPer; ++r) {
    const unsigned long long k = w.key[r];
    const int64_t at = pos + lanes_below(w.fire[r]);
    pos += __popcll(w.fire[r]);
    if (!((w.fire[r] >> lane) & 1ull) || at >= capacity) continue;
    const int64_t v = base + 64 * r + lane;
    const int64_t si = ident ? v : map_slot(m, v);
    const int64_t tmpl = si / nwin, q = si - tmpl * nwin;
    rfd_trigger t;
    // filter index m of the peak; sample n = m - d (mod N) under lag centring
    t.sample = q * W + (int64_t)(0xFFFFFFFFu - (uint32_t)(k & 0xFFFFFFFFull));
    if (shift) t.sample = (t.sample - shift[tmpl]) & (nseg - 1);
    t.tmpl = (int32_t)tmpl;
    t.subbank = sb_first ? find_subbank(sb_first, nsb, tmpl) : 0;
    t.rho = sqrtf(__uint_as_float((uint32_t)(k >> 32)));
    t.z_re = 0.f;
    t.z_im = 0.f;
    t.flags = 1u;       // complex SNR not yet evaluated
    out[at] = t;
  }
}

// z_j[n] = sum_k c_j[k] zhat[(n + k0 + d_j + k) mod N]: one wave per
// trigger, grid-stride over the triggers (the count is known only on the
// device).
__global__ __launch_bounds__(256) void k_fir_z(rfd_trigger* __restrict__ out, const long long* __restrict__ total,
                                             int64_t capacity, const float2* __restrict__ c32,
                                             const float2* __restrict__ zref, int64_t n,
                                             const int64_t* __restrict__ sb_first, const int32_t* __restrict__ meta,
                                             const int64_t* __restrict__ abase, const int32_t* __restrict__ shift) {
  const int64_t lim = *total < capacity ? *total : capacity;
  const int lane = threadIdx.x & 63;
  for (int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); i < lim; i += (int64_t)gridDim.x * 4) {
    const rfd_trigger t = out[i];
    const int b = t.subbank;
    const int ref = meta[4 * b + 0], T = meta[4 * b + 1], Tp = meta[4 * b + 2];
    const int k0 = meta[4 * b + 3] + shift[t.tmpl];
    const float2* c = c32 + abase[b] + (int64_t)(t.tmpl - sb_first[b]) * Tp;
    const float2* z = zref + (int64_t)ref * n;
    float re = 0.f, im = 0.f;
    for (int k = lane; k < T; k += 64) {
      const float2 v = cmul(c[k], z[(t.sample + k0 + k) & (n - 1)]);
      re += v.x;
      im += v.y;
    }
    for (int o = 32; o > 0; o >>= 1) {
      re += __shfl_xor(re, o);
      im += __shfl_xor(im, o);
    }
    if (lane == 0) {
      out[i].z_re = re;
      out[i].z_im = im;
      out[i].flags = 0u;
    }
  }
}

// FINDCHIRP: z_j[n] = sum_band s_i F_j,i exp(+2 pi i i n / N) at each trigger.
// One block per trigger (segments of at most 4096 samples: a few bins per
// thread) ...
__global__ __launch_bounds__(256) void k_fc_z(rfd_trigger* __restrict__ out, const long long* __restrict__ total,
                                            int64_t capacity, const float2* __restrict__ s,
                                            const float2* __restrict__ filt, int64_t i_low, int64_t n_band,
                                            int64_t n, const float2* __restrict__ coarse,
                                            const float2* __restrict__ fine) {
  __shared__ float red[2][256];
  int64_t lim = *total < capacity ? *total : capacity;
  int64_t i = blockIdx.x;
  if (i >= lim) return;
  rfd_trigger t = out[i];
  const float2* f = filt + (int64_t)t.tmpl * n_band;
  float re = 0.f, im = 0.f;
  for (int64_t k = threadIdx.x; k < n_band; k += 256) {
    int64_t bin = k + i_low;
    uint32_t p = (uint32_t)((bin * t.sample) & (n - 1));
    float2 v = cmul(cmul(s[bin], f[k]), twiddle_n(coarse, fine, p, +1));
    re += v.x;
    im += v.y;
  }
  red[0][threadIdx.x] = re;
  red[1][threadIdx.x] = im;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      red[0][threadIdx.x] += red[0][threadIdx.x + o];
      red[1][threadIdx.x] += red[1][threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[i].z_re = red[0][0];
    out[i].z_im = red[1][0];
    out[i].flags = 0u;
  }
}

// ... or, for long segments, kZParts blocks per trigger over contiguous bin
// ranges (grid-stride over the triggers), their partial sums then added in
// a fixed order by one thread per trigger.
__global__ __launch_bounds__(256) void k_fc_z_part(const rfd_trigger* __restrict__ out,
                                                 const long long* __restrict__ total, int64_t capacity,
                                                 const float2* __restrict__ s, const float2* __restrict__ filt,
                                                 int64_t i_low, int64_t n_band, int64_t n,
                                                 const float2* __restrict__ coarse, const float2* __restrict__ fine,
                                                 float2* __restrict__ part) {
  __shared__ float red[2][256];
  const int64_t lim = *total < capacity ? *total : capacity;
  const int64_t chunk = (n_band + kZParts - 1) / kZParts;
  const int64_t k0 = (int64_t)blockIdx.x * chunk, k1 = std::min<int64_t>(k0 + chunk, n_band);
  for (int64_t i = blockIdx.y; i < lim; i += gridDim.y) {
    const rfd_trigger t = out[i];
    const float2* f = filt + (int64_t)t.tmpl * n_band;
    float re = 0.f, im = 0.f;
    for (int64_t k = k0 + threadIdx.x; k < k1; k += 256) {
      const int64_t bin = k + i_low;
      const uint32_t p = (uint32_t)((bin * t.sample) & (n - 1));
      const float2 v = cmul(cmul(s[bin], f[k]), twiddle_n(coarse, fine, p, +1));
      re += v.x;
      im += v.y;
    }
    red[0][threadIdx.x] = re;
    red[1][threadIdx.x] = im;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (threadIdx.x < o) {
        red[0][threadIdx.x] += red[0][threadIdx.x + o];
        red[1][threadIdx.x] += red[1][threadIdx.x + o];
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) part[i * kZParts + blockIdx.x] = make_float2(red[0][0], red[1][0]);
    __syncthreads();
  }
}
__global__ __launch_bounds__(256) void k_fc_z_final(rfd_trigger* __restrict__ out, const long long* __restrict__ total,
                                                  int64_t capacity, const float2* __restrict__ part) {
  const int64_t lim = *total < capacity ? *total : capacity;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= lim) return;
  float re = 0.f, im = 0.f;
  for (int k = 0; k < kZParts; ++k) {
    const float2 v = part[i * kZParts + k];
    re += v.x;
    im += v.y;
  }
  out[i].z_re = re;
  out[i].z_im = im;
  out[i].flags = 0u;
}

// ------------------------------------------------------------ launchers
WinMap win_map_all(int64_t nwin) { return WinMap{nwin, nwin, nwin, 0, 0}; }

bool win_map_range(int64_t nwin, int64_t W, int pieces, const int64_t* lo, const int64_t* hi, WinMap* m) {
  int64_t a[2], b[2];       // inclusive window runs
  for (int k = 0; k < pieces; ++k) {
    a[k] = lo[k] / W;
    b[k] = (hi[k] - 1) / W;
  }
  if (pieces == 2) {
    if (a[1] < a[0]) {      // increasing q
      std::swap(a[0], a[1]);
      std::swap(b[0], b[1]);
    }
    if (a[1] <= b[0] + 1) { // overlapping or adjacent runs merge
      b[0] = std::max(b[0], b[1]);
      pieces = 1;
    }
  }
  if (pieces == 1) {
    *m = WinMap{nwin, b[0] - a[0] + 1, b[0] - a[0] + 1, a[0], 0};
    return true;
  }
  if (pieces != 2) return false;
  *m = WinMap{nwin, (b[0] - a[0] + 1) + (b[1] - a[1] + 1), b[0] - a[0] + 1, a[0], a[1]};
  return true;
}

int launch_slots_clear(Plan& p, int64_t n_slots) {
  // every slot: templates x windows, identity order
  return launch_slots_clear_map(p, n_slots, win_map_all(std::max<int64_t>(n_slots, 1)));
}

int launch_slots_clear_map(Plan& p, int64_t n_visit, const WinMap& m) {
  int64_t blocks = (n_visit + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)blocks), dim3(256), 0, p.stream, p.slots, n_visit, m);
  RFD_CHECK_LAUNCH();
  return RFD_OK;
}

int launch_compact_impl(Plan& p, int64_t n_slots, int64_t nwin, int64_t W, float threshold, rfd_trigger* out,
                        int64_t capacity, const int64_t* sb_first, int nsb, const WinMap& m,
                        const int32_t* shift = nullptr) {
  int64_t nblk = (n_slots + kSeg - 1) / kSeg;
  if ((size_t)nblk > p.counts_cap) return fail(RFD_E_INVALID, "compaction scratch too small");
  float thr2 = threshold * threshold;
  hipLaunchKernelGGL(k_count, dim3((unsigned)nblk), dim3(kSegThreads), 0, p.stream, p.slots, n_slots, thr2,
                     p.counts, m);
  RFD_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, p.stream, p.counts, nblk, p.total);
  RFD_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_write, dim3((unsigned)nblk), dim3(kSegThreads), 0, p.stream, p.slots, n_slots, thr2,
                     p.counts, nwin, W, out, capacity, sb_first, nsb, m, shift, p.n);
  RFD_CHECK_LAUNCH();
  return RFD_OK;
}

int launch_compact(Plan& p, int64_t n_slots, int64_t nwin, int64_t W, float threshold, rfd_trigger* out,
                   int64_t capacity) {
  return launch_compact_impl(p, n_slots, nwin, W, threshold, out, capacity, nullptr, 1, win_map_all(nwin));
}

int compaction_blocks(int64_t n_slots) { return (int)((n_slots + kSeg - 1) / kSeg); }

int launch_compact_bank(Plan& p, const Taps& tp, int64_t n_slots, int64_t nwin, int64_t W, float threshold,
                        rfd_trigger* out, int64_t capacity, const WinMap* m) {
  // the lag offsets are always read (zero where a template is not centred), so
  // a captured graph stays right when taps are later re-made with or without
  // centring
  return launch_compact_impl(p, n_slots, nwin, W, threshold, out, capacity, tp.d_first, (int)tp.sb.size(),
                             m ? *m : win_map_all(nwin), tp.d_shift);
}

int launch_fir_z(Plan& p, const Taps& tp, rfd_trigger* out, int64_t capacity) {
  if (capacity <= 0) return RFD_OK;
  const int64_t blocks = std::min<int64_t>((capacity + 3) / 4, 1024);
  hipLaunchKernelGGL(k_fir_z, dim3((unsigned)blocks), dim3(256), 0, p.stream, out, (const long long*)p.total,
                     capacity, tp.c32, p.zref, p.n, tp.d_first, tp.d_meta, tp.d_abase, (const int32_t*)tp.d_shift);
  RFD_CHECK_LAUNCH();
  return RFD_OK;
}

int launch_findchirp_z(Plan& p, const float2* filt, rfd_trigger* out, int64_t capacity) {
  if (capacity <= 0) return RFD_OK;
  if (p.fc_work && p.fc_work_cap >= (size_t)capacity * kZParts) {
    // partial sums in FINDCHIRP's (now idle) intermediate buffer
    const unsigned gy = (unsigned)std::min<int64_t>(capacity, 256);
    hipLaunchKernelGGL(k_fc_z_part, dim3(kZParts, gy), dim3(256), 0, p.stream, (const rfd_trigger*)out,
                       (const long long*)p.total, capacity, p.stilde, filt, p.i_low, p.n_band, p.n, p.tw32c, p.tw32f,
                       p.fc_work);
    RFD_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_fc_z_final, dim3((unsigned)((capacity + 255) / 256)), dim3(256), 0, p.stream, out,
                       (const long long*)p.total, capacity, (const float2*)p.fc_work);
    RFD_CHECK_LAUNCH();
    return RFD_OK;
  }
  hipLaunchKernelGGL(k_fc_z, dim3((unsigned)capacity), dim3(256), 0, p.stream, out, (const long long*)p.total,
                     capacity, p.stilde, filt, p.i_low, p.n_band, p.n, p.tw32c, p.tw32f);
  RFD_CHECK_LAUNCH();
  return RFD_OK;
}

}  // namespace rfd
