// Device helpers: complex arithmetic, 16-bit splits, twiddles, LDS FFT.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rfd {

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
// multiply by s*i (s = +-1)
__device__ __forceinline__ float2 cmul_si(float2 a, int s) {
  return s > 0 ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}
__device__ __forceinline__ double2 cmul_si(double2 a, int s) {
  return s > 0 ? make_double2(-a.y, a.x) : make_double2(a.y, -a.x);
}

// ------------------------------------------------------------ 16-bit splits
// bfloat16 round-to-nearest-even from float (finite inputs).
__device__ __forceinline__ uint32_t bf16_bits(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return u >> 16;
}
__device__ __forceinline__ float bf16_to_float(uint32_t b) { return __uint_as_float(b << 16); }
__device__ __forceinline__ uint32_t f16_bits(float x) {
  _Float16 h = (_Float16)x;
  return (uint32_t)__builtin_bit_cast(uint16_t, h);
}
__device__ __forceinline__ float f16_to_float(uint32_t b) {
  return (float)__builtin_bit_cast(_Float16, (uint16_t)b);
}
// x = hi + lo, each in bfloat16; lo carries the FP32 residual.
__device__ __forceinline__ void split_bf16(float x, uint32_t& hi, uint32_t& lo) {
  hi = bf16_bits(x);
  lo = bf16_bits(x - bf16_to_float(hi));
}
__device__ __forceinline__ void split_f16(float x, uint32_t& hi, uint32_t& lo) {
  hi = f16_bits(x);
  lo = f16_bits(x - f16_to_float(hi));
}
// Splits of an FP64 value (taps): hi from the nearest float, lo of the rest.
__device__ __forceinline__ void split_bf16(double x, uint32_t& hi, uint32_t& lo) {
  hi = bf16_bits((float)x);
  lo = bf16_bits((float)(x - (double)bf16_to_float(hi)));
}
__device__ __forceinline__ void split_f16(double x, uint32_t& hi, uint32_t& lo) {
  hi = f16_bits((float)x);
  lo = f16_bits((float)(x - (double)f16_to_float(hi)));
}

// ------------------------------------------------------- workgroup order
// The dispatcher deals consecutive workgroups (linear index h over the whole
// grid) to the 8 XCDs in turn, and each XCD has its own L2.  This bijection
// of [0, total) gives XCD c = h mod 8 a contiguous run of logical indices, so
// logical neighbours, which touch neighbouring memory, share an L2: their
// reads of common lines hit, and their writes to the two halves of a line
// merge there instead of leaving two XCDs as partial lines.
__device__ __forceinline__ uint32_t xcd_contiguous(uint32_t h, uint32_t total) {
  constexpr uint32_t kXcd = 8;
  const uint32_t c = h % kXcd, base = total / kXcd, rem = total % kXcd;
  return c * base + min(c, rem) + h / kXcd;
}

// ------------------------------------------------------------------ twiddles
// exp(sign * 2 pi i p / N) for 0 <= p < N from the factored table.
template <typename V>
__device__ __forceinline__ V twiddle_n(const V* __restrict__ coarse, const V* __restrict__ fine,
                                       uint32_t p, int sign) {
  V t = cmul(coarse[p >> 10], fine[p & 1023u]);
  if (sign < 0) t.y = -t.y;
  return t;
}

// ------------------------------------------------------------------ LDS FFT
// C independent L-point DFTs, X[k] = sum_n x[n] exp(sign 2 pi i n k / L), on
// LDS data laid out [C][LP] (LP = lds_col<L>(), elements at lpad(i)), Stockham autosort, radix 4
// stages then one radix-2 stage when log2 L is odd.  `twl` holds
// exp(+2 pi i k / L), k < L, in LDS.  All NT threads of the block must call.
template <typename V>
__device__ __forceinline__ void dft4(V& a, V& b, V& c, V& d, int sign) {
  V s0 = cadd(a, c), s1 = csub(a, c), s2 = cadd(b, d), s3 = cmul_si(csub(b, d), sign);
  a = cadd(s0, s2);
  c = csub(s0, s2);
  b = cadd(s1, s3);
  d = csub(s1, s3);
}

// LDS position of element x of a column (or of the twiddle table): one
// complex value of padding after every 16, so the strided butterfly writes
// of the early radix-4 stages spread over the banks.
__device__ __forceinline__ constexpr int lpad(int x) { return x + (x >> 4); }
// column stride of an L-point column in LDS (odd: column loads stay conflict free)
template <int L>
__host__ __device__ constexpr int lds_col() { return L + L / 16 + 1; }

template <typename V>
__device__ __forceinline__ V tw_lds(const V* twl, int idx, int sign) {
  V t = twl[lpad(idx)];
  if (sign < 0) t.y = -t.y;
  return t;
}

template <typename V, int L, int C, int NT>
__device__ void lds_fft(V* buf, const V* twl, int sign) {
  constexpr int LP = lds_col<L>();
  constexpr int LOG = __builtin_ctz(L);
  constexpr int NBF4 = C * (L / 4);
  constexpr int PER4 = (NBF4 + NT - 1) / NT;
  const int tid = threadIdx.x;
  int Ns = 1;
#pragma unroll 1
  for (int st = 0; st < LOG / 2; ++st) {
    V v[PER4][4];
#pragma unroll
    for (int t = 0; t < PER4; ++t) {
      int idx = tid + t * NT;
      if ((NBF4 % NT) == 0 || idx < NBF4) {
        int c = idx / (L / 4), j = idx % (L / 4);
        const V* col = buf + c * LP;
#pragma unroll
        for (int r = 0; r < 4; ++r) v[t][r] = col[lpad(j + r * (L / 4))];
        int k = j & (Ns - 1);
        if (Ns > 1) {
          int step = L / (4 * Ns);
#pragma unroll
          for (int r = 1; r < 4; ++r) v[t][r] = cmul(v[t][r], tw_lds(twl, k * r * step, sign));
        }
        dft4(v[t][0], v[t][1], v[t][2], v[t][3], sign);
      }
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < PER4; ++t) {
      int idx = tid + t * NT;
      if ((NBF4 % NT) == 0 || idx < NBF4) {
        int c = idx / (L / 4), j = idx % (L / 4);
        int k = j & (Ns - 1);
        V* col = buf + c * LP;
        int d = (j / Ns) * Ns * 4 + k;
#pragma unroll
        for (int r = 0; r < 4; ++r) col[lpad(d + r * Ns)] = v[t][r];
      }
    }
    __syncthreads();
    Ns *= 4;
  }
  if (LOG & 1) {
    constexpr int NBF2 = C * (L / 2);
    constexpr int PER2 = (NBF2 + NT - 1) / NT;
    V v[PER2][2];
#pragma unroll
    for (int t = 0; t < PER2; ++t) {
      int idx = tid + t * NT;
      if ((NBF2 % NT) == 0 || idx < NBF2) {
        int c = idx / (L / 2), j = idx % (L / 2);
        const V* col = buf + c * LP;
        v[t][0] = col[lpad(j)];
        v[t][1] = col[lpad(j + L / 2)];
        int k = j & (Ns - 1);
        if (Ns > 1) v[t][1] = cmul(v[t][1], tw_lds(twl, k * (L / (2 * Ns)), sign));
        V a = cadd(v[t][0], v[t][1]), b = csub(v[t][0], v[t][1]);
        v[t][0] = a;
        v[t][1] = b;
      }
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < PER2; ++t) {
      int idx = tid + t * NT;
      if ((NBF2 % NT) == 0 || idx < NBF2) {
        int c = idx / (L / 2), j = idx % (L / 2);
        int k = j & (Ns - 1);
        V* col = buf + c * LP;
        int d = (j / Ns) * Ns * 2 + k;
        col[lpad(d)] = v[t][0];
        col[lpad(d + Ns)] = v[t][1];
      }
    }
    __syncthreads();
  }
}

}  // namespace rfd
