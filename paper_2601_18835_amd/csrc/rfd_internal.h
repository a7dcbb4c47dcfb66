// Internal declarations shared by the HIP translation units of librfd.
// Method: ratio-filter dechirping, arXiv:2601.18835 (see include/rfd.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "rfd.h"

namespace rfd {

// ---------------------------------------------------------------- errors
void set_error(const std::string& msg);
int fail(int code, const std::string& msg);
#define RFD_HIP(call)                                                                   \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess)                                                             \
      return ::rfd::fail(RFD_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)
#define RFD_CHECK_LAUNCH() RFD_HIP(hipGetLastError())
// every device allocation of the library goes through here (hipMalloc, or an
// injected failure requested with rfd_debug_fail_allocation)
hipError_t device_malloc(void** ptr, size_t bytes);

constexpr int kFineBits = 10;                 // twiddle factorisation p = (c << 10) | f
constexpr int kFine = 1 << kFineBits;
constexpr int kDechirpBatch = 32;               // references per batched dechirp launch
constexpr int kMaxRefSlots = 4096;              // reference-series slots of a plan, at most
constexpr int kSigParts = 64;                   // partial sums per reference norm
constexpr int kZParts = 32;                     // partial sums per FINDCHIRP trigger z

// ------------------------------------------------------------- plan state
struct Plan {
  int64_t n = 0, nb = 0, i_low = 0, i_high = 0, n_band = 0;
  int log2n = 0, n1 = 0, n2 = 0;
  double fs = 0, f_low = 0, df = 0, data_scale = 0;
  int max_refs = 0;
  hipStream_t stream = nullptr;

  // FP64 PSD weights w_i = 4 df / S_n(f_i) in band, 0 elsewhere  [nb]
  double* w = nullptr;
  // twiddles exp(+2 pi i p / N) = coarse[p >> 10] * fine[p & 1023]
  float2* tw32c = nullptr;  float2* tw32f = nullptr;
  double2* tw64c = nullptr; double2* tw64f = nullptr;
  // exp(+2 pi i k / L) for the two sub-transform lengths
  float2* tw32_n1 = nullptr; float2* tw32_n2 = nullptr;
  double2* tw64_n1 = nullptr; double2* tw64_n2 = nullptr;

  double2* stilde64 = nullptr; // current segment transform (scaled, FP64), [nb]
  float2* stilde = nullptr;   // its FP32 copy (FINDCHIRP operand), [nb]
  double2* work64 = nullptr;  // one N-point FP64 intermediate
  double2* work64b = nullptr; size_t work64b_cap = 0;   // batched dechirp intermediates (grown)
  double* dref_sig2 = nullptr;    // sigma_ref^2 by reference slot [max_refs]
  double* dref_scale = nullptr;   // 1 / (sigma alpha) of a dechirp batch [kDechirpBatch]
  double* dref_part = nullptr;    // partial sums of their norms [kDechirpBatch][kSigParts]
  double2* fref64 = nullptr;  // reference filter scratch [nb]
  double* dscratch = nullptr; // small FP64 scratch (sigma etc.)  [64]
  // reference series store, slot-major [max_refs][n]
  float2* zref = nullptr;
  uint32_t* zbf_hi = nullptr; uint32_t* zbf_lo = nullptr;
  uint32_t* zh_hi = nullptr;  uint32_t* zh_lo = nullptr;
  int64_t seg_gen = 0;
  std::vector<int64_t> ref_gen;   // generation each slot was dechirped at (0: never)

  // epilogue and compaction scratch (grown on demand)
  unsigned long long* slots = nullptr; size_t slots_cap = 0;
  long long* counts = nullptr; size_t counts_cap = 0;
  long long* total = nullptr;

  // FINDCHIRP batch intermediates (grown on demand)
  float2* fc_work = nullptr; size_t fc_work_cap = 0;
  // slots, counts and fc_work point into caller-owned workspace (never grown or freed)
  bool ws_external = false;

  // FIR tile configuration of the 16-bit forms: MFMA column blocks per wave (8 or 16)
  int fir_nb16 = 8;
  // FIR launch mode: 0 auto (persistent when more than one sub-bank), 1 one launch
  // per sub-bank, 2 persistent work queue always
  int fir_mode = 0;
  // largest number of tiles one work item sweeps (1, 2, 4, ..., 16)
  int fir_smax = 16;
  // persistent grid: workgroups per CU (0: as many as fit)
  int fir_wg_per_cu = 0;
  int n_cu = 0;
  // bumped whenever a buffer a captured graph may point at is reallocated
  int64_t res_gen = 0;
  unsigned long long* counter = nullptr;   // persistent work-queue counter
  // overlap-save FIR: block size (0: per sub-bank by cost model) and
  // exp(+2 pi i m / 4096), m < 4096, in FP32 and FP64
  int ols_block = 0;
  bool ols_aligned = true;     // allow aligned output lengths (L = 256 nf)
  bool dechirp_fp64 = false;   // reference transforms in FP64 (default: FP32 passes, FP64 integrand)
  float2* ols_tw32 = nullptr;
  double2* ols_tw64 = nullptr;
  // chi^2 band series per reference slot: [n_bands][n] FP32, the band edges
  // they were made with and the segment generation
  std::vector<float2*> zband;
  std::vector<int64_t> zband_cap;
  std::vector<std::vector<int64_t>> zband_edges;
  std::vector<int64_t> zband_gen;

  // objects that keep a pointer to this plan (graphs, streams): destroy refuses while > 0
  int users = 0;
  // optional stage timing (hipEvent pairs on `stream`)
  bool timing = false;
  struct Mark { int stage; hipEvent_t a, b; bool open; };
  std::vector<Mark> marks;
  std::vector<hipEvent_t> event_pool;   // events of read-out marks, reused by later stages
};

enum Stage {
  kStDataFft = 0, kStDechirp, kStFir, kStCompact, kStFindchirp, kStTaps, kStSurNet, kStSurExpand, kStSurPack,
  kStMatch, kStFirKernel,
  kNumStages
};
// Record the start / stop of a stage when timing is enabled.  Stages nest:
// stage_end closes the innermost open one (kStFirKernel marks each main FIR
// kernel launch inside kStFir).
int stage_begin(Plan& p, int stage);
int stage_end(Plan& p);

struct SubBankTaps {
  int64_t first = 0, count = 0;     // global template range
  int32_t ref_id = 0, T = 0, Tp = 0, k0 = 0;
  int64_t npad = 0;                 // count rounded up to the FIR template tile
  int64_t a_base = 0;               // offset (elements) into a64 / c32
  int64_t p16_base = 0;             // offset (uint4) into packed 16-bit arrays
  int64_t p32_base = 0;             // offset (float4) into packed fp32 array
  double2* L = nullptr;             // Cholesky factor, column-major T x T
  double2* U = nullptr;             // L^H, column-major
  double2* g = nullptr;             // autocorrelation g[0..T-1]
  double eps = -1.0;                // ridge of the cached factor
  int64_t made = 0;                 // templates whose taps exist
  std::vector<uint8_t> made_mask;
  int64_t n_centred = 0;            // templates whose lag window is their own (d != 0 possible)
  std::vector<uint8_t> centred_mask;
  // overlap-save FIR state: block spectra of the series (rebuilt every
  // filter call), tap spectra (rebuilt after the taps change)
  int ols_K = 0, ols_L = 0, ols_nf = 0;   // ols_nf > 0: L = 256 ols_nf (aligned output groups)
  int64_t ols_nB = 0, ols_x_cap = 0;
  float2* ols_x = nullptr;
  float2* ols_g = nullptr;
  bool ols_valid = false;
  // chi^2 band shares f_b per template [count][n_bands] and their band edges
  float* band_f = nullptr;
  std::vector<int64_t> band_edges;
};

struct Taps {
  Plan* plan = nullptr;
  std::vector<SubBankTaps> sb;
  int64_t n_templates = 0;
  double2* a64 = nullptr;           // FP64 taps a (Sec. V.A), [sum count*Tp]
  double* sigma_fit = nullptr;      // [n_templates]
  float2* c32 = nullptr;            // normalised FIR taps c = conj(a) sigma_ref/sigma_fit
  uint4* pbf = nullptr;             // packed bf16 hi/lo MFMA A operands
  uint4* pfh = nullptr;             // packed fp16 hi/lo MFMA A operands
  float4* p32 = nullptr;            // packed fp32 MFMA A operands
  // per-template lag centring: template j's taps sit at lags k0 + d[j] + k of
  // its sub-bank's k0 (d = 0 unless made with RFD_TAPS_CENTRE); the FIR
  // kernels work on the filter index m = n + d, compaction and trigger
  // evaluation convert
  int32_t* d_shift = nullptr;       // [n_templates]
  // device copy of per-sub-bank metadata for trigger kernels
  int64_t* d_first = nullptr; int32_t* d_meta = nullptr;  // meta: ref_id, T, Tp, k0 per sub-bank
  int64_t* d_abase = nullptr;
  // static per-sub-bank tables for the persistent FIR
  int64_t* d_p16 = nullptr; int64_t* d_p32 = nullptr; int64_t* d_count = nullptr;
  // work-item tables for the persistent FIR (rebuilt when the key changes)
  int64_t* d_it_off = nullptr; int32_t* d_it_sb = nullptr; int32_t* d_it_S = nullptr; int64_t* d_it_nsg = nullptr;
  int64_t it_key_W = -1; int it_key_cols = -1; int it_key_smax = -1; int it_key_prec = -1; int it_key_wg = -1;
  int64_t it_total = 0; int it_nsb = 0; size_t it_lds = 0; int it_grid = 1;
  // bumped whenever a buffer a captured graph may point at is reallocated
  int64_t res_gen = 0;
  // objects that keep a pointer to these taps (graphs, streams): destroy refuses while > 0
  int users = 0;
  // scratch for tap construction
  double2* work64 = nullptr; size_t work64_cap = 0;
  double2* bvec = nullptr; size_t bvec_cap = 0;
  double* peak_pw = nullptr; size_t peak_cap = 0;      // |b|^2 of the full correlations (centring)
  double* peak_part = nullptr; int64_t* peak_idx = nullptr; size_t peak_parts_cap = 0;   // chunk maxima
  int32_t* k0buf = nullptr; size_t k0buf_cap = 0;      // per-template k0 of one make_taps call
};

// FIR tiling shared by packing and kernels
constexpr int kTmplPerWave = 8;                 // 16 real MFMA rows
constexpr int kWavesPerBlock = 4;
constexpr int kTmplTile = kTmplPerWave * kWavesPerBlock;   // 32 templates per workgroup

inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// ----------------------------------------------------- launchers (fft.hip)
int launch_data_fft(Plan& p, const double* data);
int dechirp_batch_size(const Plan& p);
size_t dechirp_work_double2(const Plan& p);   // batch buffer size in double2 units
int launch_dechirp_refs(Plan& p, int n_refs, const int32_t* ref_ids, const double* const* h_refs);
int launch_findchirp_prepare(Plan& p, const double* h, int64_t count, float2* filt, double* sigma);
int launch_findchirp(Plan& p, const float2* filt, int64_t n_templates, int64_t W, int64_t nwin, float threshold);
int launch_fc_cols_lds(Plan& p, const float2* filt, int nb, float2* Y, int n1, int n2);
// FP64 correlation: out[t][l] = sum_i P_t[i] exp(+2 pi i i (k0+l)/N), l < T
// mode 0: P = w h_t conj(h_r); mode 1: P = w |h_r|^2 (batch 1); mode 2: P = h_t/h_r
// where w |h_r|^2 > 0, scaled by 1/N.
// lo / hi (inclusive bins, -1: the analysis band) restrict the sum to a band.
// k0s (device, per batch entry, may be NULL) replaces k0 template by template.
// fp32: FP32 column transforms of the integrand rounded once (shares and
// sums in FP64); applies to the fused form, the row form stays FP64.
int launch_corr64(Plan& p, Taps& tp, int mode, const double* h_r, const double* h_t, int64_t batch,
                  int T, int k0, double2* out, int64_t out_stride, int64_t lo = -1, int64_t hi = -1,
                  const int32_t* k0s = nullptr, bool fp32 = false, const double* bscale = nullptr);
constexpr int kPeakParts = 64;   // chunks per template in the peak-lag reduction
// Per-template lag centring: the full weighted cross-correlation b (mode 0)
// of each batch entry, |b|^2 into pw [batch][N], and its peak lag l in
// (-N/2, N/2]: k0_out[t] = l - floor(T/2), d_out[t] = k0_out[t] - k0_sb.
int launch_corr_peak(Plan& p, Taps& tp, const double* h_r, const double* h_t, int64_t batch, int T, int k0_sb,
                     double* pw, int32_t* k0_out, int32_t* d_out);
// band series [n_bands][N] (FP32, normalised by sigma_ref) of one reference
int launch_dechirp_bands(Plan& p, const double* h_ref, const int64_t* edges, int n_bands, float2* out);

// ---------------------------------------------------- launchers (taps.hip)
int taps_prepare_subbank(Plan& p, Taps& tp, int b, const double* h_ref, double eps);
int taps_solve_and_pack(Plan& p, Taps& tp, int b, int64_t first, int64_t count, int method);
// sigma_fit of the taps in a64 (with the sub-bank's g), then the normalised packings
int taps_norm_and_pack(Plan& p, Taps& tp, int b, int64_t first, int64_t count);

// ----------------------------------------------------- launchers (fir.hip)
// n_len < 0: the whole segment; else output samples [n_start, n_start + n_len),
// both multiples of 256
int launch_fir(Plan& p, const Taps& tp, int b, int precision, int64_t W, int64_t nwin, float threshold,
               int64_t n_start = 0, int64_t n_len = -1);
// all sub-banks in one persistent launch (builds the work-item tables if needed;
// must not be called for the first time with a given key inside graph capture)
int prepare_fir_items(Plan& p, Taps& tp, int precision, int64_t W);
int launch_fir_persistent(Plan& p, const Taps& tp, int precision, int64_t W, int64_t nwin, float threshold);

// ----------------------------------------------------- launchers (ols.hip)
// overlap-save block shape for T taps: block size K, outputs kept per block
// L (K - T + 1, or 256 nf when the aligned form is cheaper), nf (0: general)
struct OlsShape { int K, L, nf; };
OlsShape ols_shape(const Plan& p, int T);
int ols_block_size(const Plan& p, int T);
// allocate block / tap spectra (only if allow_alloc; else RFD_E_STATE when one
// is missing) and rebuild stale tap spectra in place (not inside capture);
// need_block_spectra false: the caller brings the block-spectra buffer itself
int ensure_ols(Plan& p, Taps& t, bool allow_alloc = true, bool need_block_spectra = true);
// block spectra + overlap-save FIR of every sub-bank
// outputs [n_lo, n_hi) only (default: the whole segment); blocks whose samples
// all have rho <= threshold skip the window keys (they can never fire)
// x_scratch (optional): block-spectra buffer of at least ceil(N/L) K complex
// values, used for every sub-bank in turn instead of the sub-bank's own
int launch_ols(Plan& p, const Taps& t, int64_t W, int64_t nwin, float threshold, int64_t n_lo = 0,
               int64_t n_hi = -1, float2* x_scratch = nullptr);

// ------------------------------------------------------ helpers (api.hip)
// window-peak slots and compaction counts for n_slots slots (grown on demand,
// or checked against caller-owned workspace)
int ensure_slots(Plan& p, int64_t n_slots);
// reads the trigger total back (synchronises) into *n_out; RFD_E_OVERFLOW
// when it exceeds capacity
int finish_triggers(Plan& p, int64_t capacity, int64_t* n_out);

// ------------------------------------------------ launchers (triggers.hip)
// Slots a clear or compaction visits, template-major: the windows
// [lo0, lo0 + cnt0) then [lo1, lo1 + nq - cnt0) (increasing q) of every
// template; n_visit = n_templates * nq.  win_map_all: every window.
struct WinMap { int64_t nwin, nq, cnt0, lo0, lo1; };
WinMap win_map_all(int64_t nwin);
// the windows met by output pieces [lo[k], hi[k]) (k < pieces <= 2) as at most two
// runs in increasing order; false when they do not form such runs
bool win_map_range(int64_t nwin, int64_t W, int pieces, const int64_t* lo, const int64_t* hi, WinMap* m);
int launch_slots_clear(Plan& p, int64_t n_slots);
int launch_slots_clear_map(Plan& p, int64_t n_visit, const WinMap& m);
int launch_compact(Plan& p, int64_t n_slots, int64_t nwin, int64_t W, float threshold,
                   rfd_trigger* out, int64_t capacity);
// n_slots = slots visited (n_templates * m->nq with a map, else all)
int launch_compact_bank(Plan& p, const Taps& tp, int64_t n_slots, int64_t nwin, int64_t W, float threshold,
                        rfd_trigger* out, int64_t capacity, const WinMap* m = nullptr);
int compaction_blocks(int64_t n_slots);
int findchirp_batch_size(const Plan& p);
size_t findchirp_work_size(const Plan& p);
int launch_fir_z(Plan& p, const Taps& tp, rfd_trigger* out, int64_t capacity);
int launch_findchirp_z(Plan& p, const float2* filt, rfd_trigger* out, int64_t capacity);

}  // namespace rfd

struct rfd_plan { rfd::Plan p; };
struct rfd_taps { rfd::Taps t; };
