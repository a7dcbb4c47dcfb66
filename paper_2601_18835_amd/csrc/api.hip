// C ABI of librfd: argument checking, FP64 host planning, device memory,
// and the order of kernel launches for each entry point (include/rfd.h).
#include <math.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <string>
#include <vector>

#include "rfd_internal.h"

namespace rfd {

static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }
int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}


// Injected allocation failure (rfd_debug_fail_allocation): the allocation
// after `g_fail_after` further successful ones fails once with
// hipErrorOutOfMemory; -1 disables.
static std::atomic<int64_t> g_fail_after{-1};

hipError_t device_malloc(void** ptr, size_t bytes) {
  int64_t k = g_fail_after.load();
  while (k >= 0) {
    if (g_fail_after.compare_exchange_weak(k, k - 1)) {
      if (k == 0) {
        *ptr = nullptr;
        return hipErrorOutOfMemory;
      }
      break;
    }
  }
  return hipMalloc(ptr, bytes);
}

template <typename T>
static int dalloc(T** ptr, size_t count) {
  *ptr = nullptr;
  if (count == 0) count = 1;
  hipError_t e = device_malloc((void**)ptr, count * sizeof(T));
  if (e != hipSuccess) {
    *ptr = nullptr;
    (void)hipGetLastError();
    return fail(RFD_E_NOMEM, std::string("hipMalloc of ") + std::to_string(count * sizeof(T)) + " bytes failed");
  }
  return RFD_OK;
}
template <typename T>
static void dfree(T*& ptr) {
  if (ptr) (void)hipFree(ptr);
  ptr = nullptr;
}

static bool is_pow2(int64_t x) { return x > 0 && (x & (x - 1)) == 0; }

static int upload_table(Plan& p, int64_t len, int64_t step, int64_t den, float2** t32, double2** t64) {
  std::vector<float2> h32(len);
  std::vector<double2> h64(len);
  for (int64_t k = 0; k < len; ++k) {
    long double two_pi = 6.283185307179586476925286766559005768L;
    long double a = two_pi * (long double)(k * step) / (long double)den;
    long double cl = cosl(a), sl = sinl(a);
    h64[k] = make_double2((double)cl, (double)sl);
    h32[k] = make_float2((float)cl, (float)sl);
  }
  int rc = dalloc(t32, len);
  if (rc) return rc;
  rc = dalloc(t64, len);
  if (rc) return rc;
  RFD_HIP(hipMemcpy(*t32, h32.data(), len * sizeof(float2), hipMemcpyHostToDevice));
  RFD_HIP(hipMemcpy(*t64, h64.data(), len * sizeof(double2), hipMemcpyHostToDevice));
  return RFD_OK;
}

static int take_event(Plan& p, hipEvent_t* e) {
  if (!p.event_pool.empty()) {
    *e = p.event_pool.back();
    p.event_pool.pop_back();
    return RFD_OK;
  }
  RFD_HIP(hipEventCreate(e));
  return RFD_OK;
}

// (timing is off while a graph is captured: these events are never graph nodes)
int stage_begin(Plan& p, int stage) {
  if (!p.timing) return RFD_OK;
  Plan::Mark m{stage, nullptr, nullptr, true};
  int rc = take_event(p, &m.a);
  if (!rc) rc = take_event(p, &m.b);
  if (rc) {
    if (m.a) p.event_pool.push_back(m.a);
    return rc;
  }
  RFD_HIP(hipEventRecord(m.a, p.stream));
  p.marks.push_back(m);
  return RFD_OK;
}

// closes the innermost open stage (stages nest: a kernel inside the FIR stage)
int stage_end(Plan& p) {
  if (!p.timing) return RFD_OK;
  for (auto it = p.marks.rbegin(); it != p.marks.rend(); ++it) {
    if (!it->open) continue;
    RFD_HIP(hipEventRecord(it->b, p.stream));
    it->open = false;
    break;
  }
  return RFD_OK;
}

// marks read out or abandoned: their events go back to the pool
static void drop_marks(Plan& p) {
  for (auto& m : p.marks) {
    if (m.a) p.event_pool.push_back(m.a);
    if (m.b) p.event_pool.push_back(m.b);
  }
  p.marks.clear();
}

static void destroy_events(Plan& p) {
  drop_marks(p);
  for (hipEvent_t e : p.event_pool) (void)hipEventDestroy(e);
  p.event_pool.clear();
}

static void plan_free(Plan& p) {
  destroy_events(p);
  if (p.ws_external) {      // caller-owned: not ours to free
    p.slots = nullptr;
    p.counts = nullptr;
    p.fc_work = nullptr;
  }
  dfree(p.w);
  dfree(p.tw32c); dfree(p.tw32f); dfree(p.tw64c); dfree(p.tw64f);
  dfree(p.tw32_n1); dfree(p.tw32_n2); dfree(p.tw64_n1); dfree(p.tw64_n2);
  dfree(p.stilde64); dfree(p.stilde); dfree(p.work64); dfree(p.fref64); dfree(p.dscratch);
  dfree(p.work64b); dfree(p.dref_sig2); dfree(p.dref_scale); dfree(p.dref_part);
  dfree(p.zref); dfree(p.zbf_hi); dfree(p.zbf_lo); dfree(p.zh_hi); dfree(p.zh_lo);
  dfree(p.slots); dfree(p.counts); dfree(p.total); dfree(p.fc_work); dfree(p.counter);
  dfree(p.ols_tw32); dfree(p.ols_tw64);
  for (auto& z : p.zband) dfree(z);
}

int ensure_slots(Plan& p, int64_t n_slots) {
  if (p.ws_external) {
    if ((size_t)n_slots > p.slots_cap || (size_t)compaction_blocks(n_slots) + 1 > p.counts_cap)
      return fail(RFD_E_NOMEM, "workspace too small: the call needs " + std::to_string(n_slots) +
                                   " window slots, the workspace holds " + std::to_string(p.slots_cap));
    return RFD_OK;
  }
  if ((size_t)n_slots > p.slots_cap) {
    RFD_HIP(hipStreamSynchronize(p.stream));
    ++p.res_gen;
    dfree(p.slots);
    p.slots_cap = 0;
    int rc = dalloc(&p.slots, (size_t)n_slots);
    if (rc) return rc;
    p.slots_cap = (size_t)n_slots;
  }
  size_t nblk = (size_t)compaction_blocks(n_slots) + 1;
  if (nblk > p.counts_cap) {
    RFD_HIP(hipStreamSynchronize(p.stream));
    ++p.res_gen;
    dfree(p.counts);
    p.counts_cap = 0;
    int rc = dalloc(&p.counts, nblk);
    if (rc) return rc;
    p.counts_cap = nblk;
  }
  return RFD_OK;
}

// batched dechirp intermediates (one N-point FP64 buffer when a batch is one reference)
static int ensure_dechirp_work(Plan& p) {
  const int bs = dechirp_batch_size(p);
  const size_t need = dechirp_work_double2(p);
  if (bs <= 1 || p.work64b_cap >= need) return RFD_OK;
  RFD_HIP(hipStreamSynchronize(p.stream));
  ++p.res_gen;
  dfree(p.work64b);
  p.work64b_cap = 0;
  int rc = dalloc(&p.work64b, need);
  if (rc) return rc;
  p.work64b_cap = need;
  return RFD_OK;
}

static int check_filter_args(const Plan& p, float threshold, int64_t W, const rfd_trigger* out, int64_t capacity,
                             int64_t* n_out) {
  if (!(threshold >= 0.f) || !isfinite(threshold)) return fail(RFD_E_INVALID, "threshold must be finite and >= 0");
  if (W < 1 || W > p.n) return fail(RFD_E_INVALID, "cluster_window must satisfy 1 <= W <= N");
  if (capacity < 0) return fail(RFD_E_INVALID, "capacity must be >= 0");
  if (capacity > 0 && !out) return fail(RFD_E_INVALID, "out is NULL with capacity > 0");
  if (!n_out) return fail(RFD_E_INVALID, "n_out is NULL");
  return RFD_OK;
}

int finish_triggers(Plan& p, int64_t capacity, int64_t* n_out) {
  long long tot = 0;
  RFD_HIP(hipMemcpyAsync(&tot, p.total, sizeof(long long), hipMemcpyDeviceToHost, p.stream));
  RFD_HIP(hipStreamSynchronize(p.stream));
  *n_out = tot;
  if (tot > capacity)
    return fail(RFD_E_OVERFLOW, "trigger capacity " + std::to_string(capacity) + " < " + std::to_string(tot));
  return RFD_OK;
}

static bool valid_precision(int precision) {
  return precision == RFD_FP32 || precision == RFD_BF16X3 || precision == RFD_FP16X3 || precision == RFD_OLS32;
}

static bool use_persistent(const Plan& p, const Taps& t) {
  return p.fir_mode == 2 || (p.fir_mode == 0 && t.sb.size() > 1);
}

// FIR kernels of every sub-bank (one persistent launch or one per sub-bank).
static int enqueue_fir(Plan& p, Taps& t, int precision, int64_t W, int64_t nwin, float threshold) {
  if (precision == RFD_OLS32) return launch_ols(p, t, W, nwin, threshold);
  if (use_persistent(p, t)) return launch_fir_persistent(p, t, precision, W, nwin, threshold);
  for (size_t b = 0; b < t.sb.size(); ++b) {
    int rc = launch_fir(p, t, (int)b, precision, W, nwin, threshold);
    if (rc) return rc;
  }
  return RFD_OK;
}

// Everything a FIR launch needs that may allocate or build tables (never
// inside graph capture): persistent work items, overlap-save spectra.
static int prepare_fir(Plan& p, Taps& t, int precision, int64_t W) {
  if (precision == RFD_OLS32) return ensure_ols(p, t);
  if (use_persistent(p, t)) return prepare_fir_items(p, t, precision, W);
  return RFD_OK;
}

static int check_bank_state(const Plan& p, const Taps& t) {
  for (size_t b = 0; b < t.sb.size(); ++b) {
    const SubBankTaps& s = t.sb[b];
    if (s.count == 0) continue;
    if (p.seg_gen == 0 || p.ref_gen[s.ref_id] != p.seg_gen)
      return fail(RFD_E_STATE, "sub-bank " + std::to_string(b) + ": reference slot not dechirped on this segment");
    if (s.made != s.count) return fail(RFD_E_STATE, "sub-bank " + std::to_string(b) + ": taps not made");
  }
  return RFD_OK;
}

// Caller-owned workspace: slots, then counts, then the FINDCHIRP intermediate,
// each region 256-byte aligned.
struct WsLayout {
  size_t slots = 0, counts = 0, fc = 0;   // entries (u64, long long, float2)
  size_t off_counts = 0, off_fc = 0, bytes = 0;
};
static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }
static int ws_layout(const Plan& p, int64_t max_templates, int64_t min_W, int32_t with_fc, WsLayout* l) {
  if (max_templates < 0 || max_templates > ((int64_t)1 << 31) - 1)
    return fail(RFD_E_INVALID, "max_templates must be in [0, 2^31 - 1]");
  if (min_W < 1 || min_W > p.n) return fail(RFD_E_INVALID, "min_cluster_window must satisfy 1 <= W <= N");
  const int64_t nwin = (p.n + min_W - 1) / min_W;
  const int64_t n_slots = std::max<int64_t>(max_templates * nwin, 1);
  l->slots = (size_t)n_slots;
  l->counts = (size_t)compaction_blocks(n_slots) + 1;
  l->fc = with_fc ? findchirp_work_size(p) : 0;
  l->off_counts = align256(l->slots * sizeof(unsigned long long));
  l->off_fc = l->off_counts + align256(l->counts * sizeof(long long));
  l->bytes = l->off_fc + align256(l->fc * sizeof(float2));
  return RFD_OK;
}
}  // namespace rfd

using namespace rfd;

extern "C" {

const char* rfd_last_error(void) { return rfd::g_err.c_str(); }

int rfd_debug_fail_allocation(int64_t after) {
  rfd::g_fail_after.store(after < 0 ? -1 : after);
  return RFD_OK;
}

int rfd_plan_create(const double* psd, int64_t n_psd, double f_low, double fs, int64_t seg_len, int32_t max_refs,
                    void* stream, rfd_plan** out) {
  if (!out) return fail(RFD_E_INVALID, "out is NULL");
  *out = nullptr;
  if (!psd) return fail(RFD_E_INVALID, "psd is NULL");
  if (!is_pow2(seg_len) || seg_len < (1 << 10) || seg_len > (1 << 22))
    return fail(RFD_E_INVALID, "seg_len must be a power of two in [2^10, 2^22]");
  if (n_psd != seg_len / 2 + 1) return fail(RFD_E_INVALID, "n_psd must equal seg_len/2 + 1");
  if (!(fs > 0.0) || !isfinite(fs)) return fail(RFD_E_INVALID, "fs must be finite and > 0");
  if (!(f_low > 0.0) || !(f_low < fs / 2.0)) return fail(RFD_E_INVALID, "f_low must satisfy 0 < f_low < fs/2");
  if (max_refs < 1 || max_refs > kMaxRefSlots) return fail(RFD_E_INVALID, "max_refs must be in [1, 4096]");
  const int64_t n = seg_len, nb = n / 2 + 1;
  const double df = fs / (double)n;
  const int64_t i_low = (int64_t)ceil(f_low / df), i_high = n / 2 - 1;
  if (i_low > i_high) return fail(RFD_E_INVALID, "empty analysis band");
  double smin = INFINITY;
  for (int64_t i = i_low; i <= i_high; ++i) {
    if (!isfinite(psd[i]) || !(psd[i] > 0.0))
      return fail(RFD_E_INVALID, "psd must be finite and > 0 on every in-band bin (bin " + std::to_string(i) + ")");
    smin = std::min(smin, psd[i]);
  }
  rfd_plan* h = new (std::nothrow) rfd_plan();
  if (!h) return fail(RFD_E_NOMEM, "host allocation failed");
  Plan& p = h->p;
  p.n = n;
  p.nb = nb;
  p.i_low = i_low;
  p.i_high = i_high;
  p.n_band = i_high - i_low + 1;
  p.log2n = __builtin_ctzll((unsigned long long)n);
  p.n1 = 1 << ((p.log2n + 1) / 2);
  p.n2 = (int)(n / p.n1);
  p.fs = fs;
  p.f_low = f_low;
  p.df = df;
  // data scale: makes the in-band transform O(1) at the most sensitive bin
  p.data_scale = sqrt(2.0 * df / smin);
  p.max_refs = max_refs;
  p.stream = (hipStream_t)stream;
  p.ref_gen.assign(max_refs, 0);
  p.zband.assign(max_refs, nullptr);
  p.zband_cap.assign(max_refs, 0);
  p.zband_edges.assign(max_refs, std::vector<int64_t>());
  p.zband_gen.assign(max_refs, 0);
  int rc = RFD_OK;
  std::vector<double> w(nb, 0.0);
  for (int64_t i = i_low; i <= i_high; ++i) w[i] = 4.0 * df / psd[i];
#define TRY(x) do { rc = (x); if (rc) { plan_free(p); delete h; return rc; } } while (0)
  TRY(dalloc(&p.w, nb));
  if (hipMemcpy(p.w, w.data(), nb * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
    plan_free(p);
    delete h;
    return fail(RFD_E_DEVICE, "upload of PSD weights failed");
  }
  TRY(upload_table(p, n / kFine, kFine, n, &p.tw32c, &p.tw64c));
  TRY(upload_table(p, kFine, 1, n, &p.tw32f, &p.tw64f));
  TRY(upload_table(p, p.n1, 1, p.n1, &p.tw32_n1, &p.tw64_n1));
  TRY(upload_table(p, p.n2, 1, p.n2, &p.tw32_n2, &p.tw64_n2));
  TRY(upload_table(p, 4096, 1, 4096, &p.ols_tw32, &p.ols_tw64));
  TRY(dalloc(&p.stilde64, nb));
  TRY(dalloc(&p.stilde, nb));
  TRY(dalloc(&p.work64, n));
  TRY(dalloc(&p.fref64, nb));
  TRY(dalloc(&p.dscratch, 64));
  TRY(dalloc(&p.dref_sig2, (size_t)max_refs));
  TRY(dalloc(&p.dref_scale, (size_t)kDechirpBatch));
  TRY(dalloc(&p.dref_part, (size_t)kDechirpBatch * kSigParts));
  TRY(dalloc(&p.counter, 1));
  {
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess)
      p.n_cu = ncu;
    if (p.n_cu < 1) p.n_cu = 1;
  }
  TRY(dalloc(&p.total, 1));
  TRY(dalloc(&p.zref, (size_t)max_refs * n));
  TRY(dalloc(&p.zbf_hi, (size_t)max_refs * n));
  TRY(dalloc(&p.zbf_lo, (size_t)max_refs * n));
  TRY(dalloc(&p.zh_hi, (size_t)max_refs * n));
  TRY(dalloc(&p.zh_lo, (size_t)max_refs * n));
#undef TRY
  *out = h;
  return RFD_OK;
}

int rfd_plan_info_get(const rfd_plan* plan, rfd_plan_info* out) {
  if (!plan || !out) return fail(RFD_E_INVALID, "NULL argument");
  const Plan& p = plan->p;
  out->n = p.n;
  out->n_bins = p.nb;
  out->i_low = p.i_low;
  out->i_high = p.i_high;
  out->n_band = p.n_band;
  out->fs = p.fs;
  out->f_low = p.f_low;
  out->df = p.df;
  out->data_scale = p.data_scale;
  out->max_refs = p.max_refs;
  out->fft_n1 = p.n1;
  out->fft_n2 = p.n2;
  return RFD_OK;
}

int rfd_plan_set_stream(rfd_plan* plan, void* stream) {
  if (!plan) return fail(RFD_E_INVALID, "plan is NULL");
  plan->p.stream = (hipStream_t)stream;
  return RFD_OK;
}

int rfd_plan_set_timing(rfd_plan* plan, int32_t enable) {
  if (!plan) return fail(RFD_E_INVALID, "plan is NULL");
  plan->p.timing = enable != 0;
  if (!plan->p.timing) {
    (void)hipStreamSynchronize(plan->p.stream);
    destroy_events(plan->p);
  }
  return RFD_OK;
}

int rfd_plan_set_psd(rfd_plan* plan, const double* psd, int64_t n_psd) {
  if (!plan || !psd) return fail(RFD_E_INVALID, "NULL argument");
  Plan& p = plan->p;
  if (n_psd != p.nb) return fail(RFD_E_INVALID, "n_psd must equal seg_len/2 + 1");
  std::vector<double> w(p.nb, 0.0);
  for (int64_t i = p.i_low; i <= p.i_high; ++i) {
    if (!isfinite(psd[i]) || !(psd[i] > 0.0))
      return fail(RFD_E_INVALID, "psd must be finite and > 0 on every in-band bin (bin " + std::to_string(i) + ")");
    w[i] = 4.0 * p.df / psd[i];
  }
  RFD_HIP(hipStreamSynchronize(p.stream));
  RFD_HIP(hipMemcpy(p.w, w.data(), p.nb * sizeof(double), hipMemcpyHostToDevice));
  // every reference series was filtered with the old weights
  ++p.seg_gen;
  return RFD_OK;
}

int rfd_taps_renormalize(rfd_plan* plan, rfd_taps* taps, int32_t subbank, const double* h_ref) {
  if (!plan || !taps || !h_ref) return fail(RFD_E_INVALID, "NULL argument");
  Plan& p = plan->p;
  Taps& t = taps->t;
  if (t.plan != &p) return fail(RFD_E_INVALID, "taps belong to another plan");
  if (subbank < 0 || subbank >= (int)t.sb.size()) return fail(RFD_E_INVALID, "subbank out of range");
  SubBankTaps& s = t.sb[subbank];
  if (s.made != s.count) return fail(RFD_E_STATE, "taps not made");
  if (s.count == 0) return RFD_OK;
  if (t.work64_cap < (size_t)p.n) {
    RFD_HIP(hipStreamSynchronize(p.stream));
    dfree(t.work64);
    t.work64_cap = 0;
    int rc = dalloc(&t.work64, (size_t)p.n);
    if (rc) return rc;
    t.work64_cap = p.n;
  }
  // the reference autocorrelation under the plan's current PSD, then sigma_fit
  // and the normalised packings of the unchanged taps (Sec. VI.B)
  int rc = launch_corr64(p, t, 1, h_ref, nullptr, 1, s.T, 0, s.g, s.T);
  if (rc) return rc;
  s.eps = -1.0;   // a cached Cholesky factor belongs to the old weights
  rc = taps_norm_and_pack(p, t, subbank, 0, s.count);
  if (rc) return rc;
  RFD_HIP(hipStreamSynchronize(p.stream));
  return RFD_OK;
}

int rfd_plan_get_timing(rfd_plan* plan, rfd_timing* out) {
  if (!plan || !out) return fail(RFD_E_INVALID, "NULL argument");
  Plan& p = plan->p;
  memset(out, 0, sizeof(*out));
  double* ms[kNumStages] = {&out->data_fft_ms, &out->dechirp_ms, &out->fir_ms, &out->compact_ms,
                            &out->findchirp_ms, &out->taps_ms, &out->sur_net_ms, &out->sur_expand_ms,
                            &out->sur_pack_ms, &out->match_ms, &out->fir_kernel_ms};
  int64_t* cnt[kNumStages] = {&out->n_data_fft, &out->n_dechirp, &out->n_fir, &out->n_compact,
                              &out->n_findchirp, &out->n_taps, &out->n_sur_net, &out->n_sur_expand,
                              &out->n_sur_pack, &out->n_match, &out->n_fir_kernel};
  for (auto& m : p.marks) {
    if (m.open) continue;                 // never closed (a failed call): no interval
    RFD_HIP(hipEventSynchronize(m.b));
    float t = 0.f;
    RFD_HIP(hipEventElapsedTime(&t, m.a, m.b));
    *ms[m.stage] += t;
    *cnt[m.stage] += 1;
  }
  drop_marks(p);
  return RFD_OK;
}

int rfd_plan_set_dechirp_fp64(rfd_plan* plan, int32_t enable) {
  if (!plan) return fail(RFD_E_INVALID, "NULL plan");
  if (enable != 0 && enable != 1) return fail(RFD_E_INVALID, "enable must be 0 or 1");
  Plan& p = plan->p;
  if (p.dechirp_fp64 != (enable == 1)) {
    p.dechirp_fp64 = enable == 1;
    ++p.res_gen;     // captured graphs recorded the other passes
  }
  return RFD_OK;
}

int rfd_plan_set_fir_config(rfd_plan* plan, const rfd_fir_config* cfg) {
  if (!plan || !cfg) return fail(RFD_E_INVALID, "NULL argument");
  if (cfg->col_blocks != 8 && cfg->col_blocks != 16) return fail(RFD_E_INVALID, "col_blocks must be 8 or 16");
  if (cfg->mode < 0 || cfg->mode > 2) return fail(RFD_E_INVALID, "mode must be 0, 1 or 2");
  const int mt = cfg->max_tiles;
  if (!(mt == 1 || mt == 2 || mt == 4 || mt == 8 || mt == 16)) return fail(RFD_E_INVALID, "max_tiles must be 1..16, a power of two");
  if (cfg->wg_per_cu < 0 || cfg->wg_per_cu > 32) return fail(RFD_E_INVALID, "wg_per_cu must be in [0, 32]");
  if (!(cfg->ols_block == 0 || cfg->ols_block == 1024 || cfg->ols_block == 2048 || cfg->ols_block == 4096))
    return fail(RFD_E_INVALID, "ols_block must be 0, 1024, 2048 or 4096");
  if (cfg->ols_aligned != 0 && cfg->ols_aligned != 1) return fail(RFD_E_INVALID, "ols_aligned must be 0 or 1");
  Plan& p = plan->p;
  p.fir_nb16 = cfg->col_blocks;
  p.fir_mode = cfg->mode;
  p.fir_smax = mt;
  p.fir_wg_per_cu = cfg->wg_per_cu;
  p.ols_block = cfg->ols_block;
  p.ols_aligned = cfg->ols_aligned != 0;
  return RFD_OK;
}

int rfd_plan_get_fir_config(const rfd_plan* plan, rfd_fir_config* cfg) {
  if (!plan || !cfg) return fail(RFD_E_INVALID, "NULL argument");
  cfg->col_blocks = plan->p.fir_nb16;
  cfg->mode = plan->p.fir_mode;
  cfg->max_tiles = plan->p.fir_smax;
  cfg->wg_per_cu = plan->p.fir_wg_per_cu;
  cfg->ols_block = plan->p.ols_block;
  cfg->ols_aligned = plan->p.ols_aligned ? 1 : 0;
  return RFD_OK;
}

int rfd_ols_shape(const rfd_plan* plan, int32_t taps, int32_t* block, int32_t* outputs) {
  if (!plan || !block || !outputs) return fail(RFD_E_INVALID, "NULL argument");
  if (taps < 1 || taps > RFD_MAX_TAPS || taps >= 4096) return fail(RFD_E_INVALID, "taps out of range");
  const OlsShape sh = ols_shape(plan->p, taps);
  *block = sh.K;
  *outputs = sh.L;
  return RFD_OK;
}

int rfd_autotune_fir(rfd_plan* plan, const rfd_taps* taps, int32_t precision, int64_t cluster_window, int32_t reps,
                     rfd_tune_result* out) {
  if (!plan || !taps || !out) return fail(RFD_E_INVALID, "NULL argument");
  Plan& p = plan->p;
  Taps& t = const_cast<Taps&>(taps->t);
  if (t.plan != &p) return fail(RFD_E_INVALID, "taps belong to another plan");
  if (!valid_precision(precision)) return fail(RFD_E_INVALID, "unknown precision");
  if (cluster_window < 1 || cluster_window > p.n) return fail(RFD_E_INVALID, "cluster_window must satisfy 1 <= W <= N");
  if (reps < 1 || reps > 100) return fail(RFD_E_INVALID, "reps must be in [1, 100]");
  int rc = check_bank_state(p, t);
  if (rc) return rc;
  const int64_t nwin = (p.n + cluster_window - 1) / cluster_window;
  rc = ensure_slots(p, std::max<int64_t>(t.n_templates * nwin, 1));
  if (rc) return rc;
  const bool saved_timing = p.timing;
  p.timing = false;
  rfd_fir_config before;
  rfd_plan_get_fir_config(plan, &before);
  auto measure = [&](const rfd_fir_config& c, double& ms) -> int {
    int r = rfd_plan_set_fir_config(plan, &c);
    if (r) return r;
    r = prepare_fir(p, t, precision, cluster_window);
    if (r) return r;
    hipEvent_t a, b;
    RFD_HIP(hipEventCreate(&a));
    RFD_HIP(hipEventCreate(&b));
    ms = 1e30;
    for (int i = 0; i < reps + 1; ++i) {      // first run warms caches and code
      RFD_HIP(hipEventRecord(a, p.stream));
      r = enqueue_fir(p, t, precision, cluster_window, nwin, 0.f);   // every window, as in validation
      if (r) break;
      RFD_HIP(hipEventRecord(b, p.stream));
      RFD_HIP(hipEventSynchronize(b));
      float e = 0.f;
      RFD_HIP(hipEventElapsedTime(&e, a, b));
      if (i > 0) ms = std::min(ms, (double)e);
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return r;
  };
  double before_ms = 0.0;
  rc = measure(before, before_ms);
  if (rc) { p.timing = saved_timing; return rc; }
  rfd_fir_config best = before;
  double best_ms = before_ms;
  int n = 1;
  const int nbs16[2] = {8, 16};
  const int tiles[3] = {4, 8, 16};
  if (precision == RFD_OLS32) {
    // overlap-save: the block size (per sub-bank cost model, or one K for
    // all), with and without aligned output lengths
    const int blocks[4] = {0, 1024, 2048, 4096};
    for (int ib = 0; ib < 4; ++ib) {
      for (int al = 0; al < 2; ++al) {
        rfd_fir_config c = before;
        c.ols_block = blocks[ib];
        c.ols_aligned = al;
        double ms = 0.0;
        rc = measure(c, ms);
        if (rc) { rfd_plan_set_fir_config(plan, &before); p.timing = saved_timing; return rc; }
        ++n;
        if (ms < best_ms) { best_ms = ms; best = c; }
      }
    }
  }
  for (int ib = 0; ib < 2 && precision != RFD_OLS32; ++ib) {
    if (precision == RFD_FP32 && ib > 0) break;
    for (int it = 0; it < 3; ++it) {
      const rfd_fir_config cands[3] = {{nbs16[ib], 1, tiles[it], 0, before.ols_block, before.ols_aligned},
                                       {nbs16[ib], 2, tiles[it], 0, before.ols_block, before.ols_aligned},
                                       {nbs16[ib], 2, tiles[it], 1, before.ols_block, before.ols_aligned}};
      for (const auto& c : cands) {
        double ms = 0.0;
        rc = measure(c, ms);
        if (rc) { rfd_plan_set_fir_config(plan, &before); p.timing = saved_timing; return rc; }
        ++n;
        if (ms < best_ms) { best_ms = ms; best = c; }
      }
    }
  }
  rfd_plan_set_fir_config(plan, &best);
  p.timing = saved_timing;
  out->best = best;
  out->best_ms = best_ms;
  out->before_ms = before_ms;
  out->n_candidates = n;
  return RFD_OK;
}

int rfd_plan_destroy(rfd_plan* plan) {
  if (!plan) return RFD_OK;
  if (plan->p.users > 0)
    return fail(RFD_E_STATE, "plan still used by " + std::to_string(plan->p.users) + " graph(s) or stream(s)");
  (void)hipStreamSynchronize(plan->p.stream);
  plan_free(plan->p);
  delete plan;
  return RFD_OK;
}


int rfd_plan_workspace_size(const rfd_plan* plan, int64_t max_templates, int64_t min_cluster_window,
                            int32_t with_findchirp, size_t* bytes) {
  if (!plan || !bytes) return fail(RFD_E_INVALID, "NULL argument");
  WsLayout l;
  int rc = ws_layout(plan->p, max_templates, min_cluster_window, with_findchirp, &l);
  if (rc) return rc;
  *bytes = l.bytes;
  return RFD_OK;
}

int rfd_plan_set_workspace(rfd_plan* plan, void* dev_ptr, size_t bytes, int64_t max_templates,
                           int64_t min_cluster_window, int32_t with_findchirp) {
  if (!plan) return fail(RFD_E_INVALID, "plan is NULL");
  Plan& p = plan->p;
  WsLayout l;
  if (dev_ptr) {
    int rc = ws_layout(p, max_templates, min_cluster_window, with_findchirp, &l);
    if (rc) return rc;
    if ((reinterpret_cast<uintptr_t>(dev_ptr) & 255u) != 0)
      return fail(RFD_E_INVALID, "workspace must be 256-byte aligned");
    if (bytes < l.bytes)
      return fail(RFD_E_INVALID, "workspace too small: " + std::to_string(bytes) + " < " + std::to_string(l.bytes) +
                                     " bytes");
  }
  RFD_HIP(hipStreamSynchronize(p.stream));
  if (p.ws_external) {
    p.slots = nullptr;
    p.counts = nullptr;
    p.fc_work = nullptr;
  } else {
    dfree(p.slots);
    dfree(p.counts);
    dfree(p.fc_work);
  }
  p.slots_cap = p.counts_cap = p.fc_work_cap = 0;
  p.ws_external = false;
  ++p.res_gen;
  if (!dev_ptr) return RFD_OK;
  char* base = static_cast<char*>(dev_ptr);
  p.slots = reinterpret_cast<unsigned long long*>(base);
  p.slots_cap = l.slots;
  p.counts = reinterpret_cast<long long*>(base + l.off_counts);
  p.counts_cap = l.counts;
  p.fc_work = l.fc ? reinterpret_cast<float2*>(base + l.off_fc) : nullptr;
  p.fc_work_cap = l.fc;
  p.ws_external = true;
  return RFD_OK;
}

int rfd_dechirp(rfd_plan* plan, const double* data, const double* h_ref, int32_t ref_id, double* sigma_ref_out) {
  return rfd_dechirp_refs(plan, data, 1, &ref_id, &h_ref, sigma_ref_out);
}

int rfd_dechirp_refs(rfd_plan* plan, const double* data, int32_t n_refs, const int32_t* ref_ids,
                     const double* const* h_refs, double* sigma_out) {
  if (!plan) return fail(RFD_E_INVALID, "plan is NULL");
  Plan& p = plan->p;
  if (!ref_ids || !h_refs) return fail(RFD_E_INVALID, "NULL argument");
  if (n_refs < 1 || n_refs > p.max_refs) return fail(RFD_E_INVALID, "n_refs must be in [1, max_refs]");
  std::vector<char> seen(p.max_refs, 0);
  for (int i = 0; i < n_refs; ++i) {
    if (ref_ids[i] < 0 || ref_ids[i] >= p.max_refs) return fail(RFD_E_INVALID, "ref_id out of range");
    if (seen[ref_ids[i]]) return fail(RFD_E_INVALID, "ref_ids must be distinct");
    if (!h_refs[i]) return fail(RFD_E_INVALID, "h_ref is NULL");
    seen[ref_ids[i]] = 1;
  }
  int rc = ensure_dechirp_work(p);
  if (rc) return rc;
  if (data) {
    rc = stage_begin(p, kStDataFft);
    if (!rc) rc = launch_data_fft(p, data);
    if (!rc) rc = stage_end(p);
    if (rc) return rc;
    ++p.seg_gen;
  } else if (p.seg_gen == 0) {
    return fail(RFD_E_STATE, "no segment: pass data on the first dechirp");
  }
  rc = stage_begin(p, kStDechirp);
  if (!rc) rc = launch_dechirp_refs(p, n_refs, ref_ids, h_refs);
  if (!rc) rc = stage_end(p);
  if (rc) return rc;
  for (int i = 0; i < n_refs; ++i) p.ref_gen[ref_ids[i]] = p.seg_gen;
  if (sigma_out) {
    std::vector<double> s2(p.max_refs);
    RFD_HIP(hipMemcpyAsync(s2.data(), p.dref_sig2, p.max_refs * sizeof(double), hipMemcpyDeviceToHost, p.stream));
    RFD_HIP(hipStreamSynchronize(p.stream));
    for (int i = 0; i < n_refs; ++i) {
      const double v = s2[ref_ids[i]];
      if (!(v > 0.0)) return fail(RFD_E_INVALID, "reference template has zero norm in band");
      sigma_out[i] = sqrt(v);
    }
  }
  return RFD_OK;
}

int rfd_get_zref(const rfd_plan* plan, int32_t ref_id, float* out) {
  if (!plan || !out) return fail(RFD_E_INVALID, "NULL argument");
  const Plan& p = plan->p;
  if (ref_id < 0 || ref_id >= p.max_refs) return fail(RFD_E_INVALID, "ref_id out of range");
  RFD_HIP(hipMemcpyAsync(out, p.zref + (int64_t)ref_id * p.n, p.n * sizeof(float2), hipMemcpyDeviceToDevice,
                         p.stream));
  return RFD_OK;
}

static void taps_free(Taps& t) {
  for (auto& s : t.sb) {
    dfree(s.L);
    dfree(s.U);
    dfree(s.g);
    dfree(s.ols_x);
    dfree(s.ols_g);
    dfree(s.band_f);
  }
  dfree(t.a64); dfree(t.sigma_fit); dfree(t.c32); dfree(t.pbf); dfree(t.pfh); dfree(t.p32);
  dfree(t.d_first); dfree(t.d_meta); dfree(t.d_abase); dfree(t.work64); dfree(t.bvec);
  dfree(t.d_p16); dfree(t.d_p32); dfree(t.d_count);
  dfree(t.d_it_off); dfree(t.d_it_sb); dfree(t.d_it_S); dfree(t.d_it_nsg);
  dfree(t.d_shift); dfree(t.peak_pw); dfree(t.k0buf); dfree(t.peak_part); dfree(t.peak_idx);
}

int rfd_taps_create(rfd_plan* plan, int32_t n_subbanks, const int64_t* offsets, const int32_t* ref_id,
                    const int32_t* taps, const int32_t* k0, rfd_taps** out) {
  if (!out) return fail(RFD_E_INVALID, "out is NULL");
  *out = nullptr;
  if (!plan || !offsets || !ref_id || !taps || !k0) return fail(RFD_E_INVALID, "NULL argument");
  Plan& p = plan->p;
  if (n_subbanks < 1) return fail(RFD_E_INVALID, "n_subbanks must be >= 1");
  if (offsets[0] != 0) return fail(RFD_E_INVALID, "offsets[0] must be 0");
  for (int b = 0; b < n_subbanks; ++b) {
    if (offsets[b + 1] < offsets[b]) return fail(RFD_E_INVALID, "offsets must be non-decreasing");
    if (ref_id[b] < 0 || ref_id[b] >= p.max_refs) return fail(RFD_E_INVALID, "ref_id out of range");
    if (taps[b] < 1 || taps[b] > RFD_MAX_TAPS) return fail(RFD_E_INVALID, "taps must be in [1, 2048]");
    if (!(k0[b] > -p.n / 2 && k0[b] < p.n / 2)) return fail(RFD_E_INVALID, "|k0| must be < N/2");
  }
  if (offsets[n_subbanks] > ((int64_t)1 << 31) - 1) return fail(RFD_E_INVALID, "too many templates");
  rfd_taps* h = new (std::nothrow) rfd_taps();
  if (!h) return fail(RFD_E_NOMEM, "host allocation failed");
  Taps& t = h->t;
  t.plan = &p;
  t.sb.resize(n_subbanks);
  int64_t abase = 0, p16 = 0, p32 = 0;
  std::vector<int64_t> firsts(n_subbanks);
  std::vector<int32_t> meta(4 * n_subbanks);
  std::vector<int64_t> abases(n_subbanks), p16s(n_subbanks), p32s(n_subbanks), counts(n_subbanks);
  int rc = RFD_OK;
  for (int b = 0; b < n_subbanks; ++b) {
    SubBankTaps& s = t.sb[b];
    s.first = offsets[b];
    s.count = offsets[b + 1] - offsets[b];
    s.ref_id = ref_id[b];
    s.T = taps[b];
    s.Tp = (int)round_up(s.T, 16);
    s.k0 = k0[b];
    s.npad = round_up(std::max<int64_t>(s.count, 1), kTmplTile);
    s.a_base = abase;
    s.p16_base = p16;
    s.p32_base = p32;
    s.made_mask.assign((size_t)s.count, 0);
    s.centred_mask.assign((size_t)s.count, 0);
    abase += s.count * s.Tp;
    p16 += (s.npad / 8) * (s.Tp / 16) * 128;
    p32 += (s.npad / 8) * (s.Tp / 8) * 64;
    firsts[b] = s.first;
    abases[b] = s.a_base;
    p16s[b] = s.p16_base;
    p32s[b] = s.p32_base;
    counts[b] = s.count;
    meta[4 * b + 0] = s.ref_id;
    meta[4 * b + 1] = s.T;
    meta[4 * b + 2] = s.Tp;
    meta[4 * b + 3] = s.k0;
  }
  t.n_templates = offsets[n_subbanks];
#define TRY(x) do { rc = (x); if (rc) { taps_free(t); delete h; return rc; } } while (0)
  TRY(dalloc(&t.a64, (size_t)abase));
  TRY(dalloc(&t.c32, (size_t)abase));
  TRY(dalloc(&t.sigma_fit, (size_t)std::max<int64_t>(t.n_templates, 1)));
  TRY(dalloc(&t.pbf, (size_t)p16));
  TRY(dalloc(&t.pfh, (size_t)p16));
  TRY(dalloc(&t.p32, (size_t)p32));
  TRY(dalloc(&t.d_first, (size_t)n_subbanks));
  TRY(dalloc(&t.d_meta, (size_t)4 * n_subbanks));
  TRY(dalloc(&t.d_abase, (size_t)n_subbanks));
  TRY(dalloc(&t.d_p16, (size_t)n_subbanks));
  TRY(dalloc(&t.d_p32, (size_t)n_subbanks));
  TRY(dalloc(&t.d_count, (size_t)n_subbanks));
  for (auto& s : t.sb) TRY(dalloc(&s.g, (size_t)s.T));
  TRY(dalloc(&t.d_shift, (size_t)std::max<int64_t>(t.n_templates, 1)));
#undef TRY
  if (hipMemsetAsync(t.d_shift, 0, std::max<int64_t>(t.n_templates, 1) * sizeof(int32_t), p.stream) != hipSuccess ||
      hipMemsetAsync(t.pbf, 0, p16 * sizeof(uint4), p.stream) != hipSuccess ||
      hipMemsetAsync(t.pfh, 0, p16 * sizeof(uint4), p.stream) != hipSuccess ||
      hipMemsetAsync(t.p32, 0, p32 * sizeof(float4), p.stream) != hipSuccess ||
      hipMemcpy(t.d_first, firsts.data(), n_subbanks * sizeof(int64_t), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(t.d_meta, meta.data(), 4 * n_subbanks * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(t.d_abase, abases.data(), n_subbanks * sizeof(int64_t), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(t.d_p16, p16s.data(), n_subbanks * sizeof(int64_t), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(t.d_p32, p32s.data(), n_subbanks * sizeof(int64_t), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(t.d_count, counts.data(), n_subbanks * sizeof(int64_t), hipMemcpyHostToDevice) != hipSuccess ||
      hipStreamSynchronize(p.stream) != hipSuccess) {
    taps_free(t);
    delete h;
    return fail(RFD_E_DEVICE, "taps initialisation failed");
  }
  *out = h;
  return RFD_OK;
}

int rfd_make_taps(rfd_plan* plan, rfd_taps* taps, int32_t subbank, const double* h_ref, const double* h_tmpl,
                  int64_t first, int64_t count, int32_t method, double ridge_eps) {
  if (!plan || !taps) return fail(RFD_E_INVALID, "NULL plan or taps");
  Plan& p = plan->p;
  Taps& t = taps->t;
  if (t.plan != &p) return fail(RFD_E_INVALID, "taps belong to another plan");
  if (subbank < 0 || subbank >= (int)t.sb.size()) return fail(RFD_E_INVALID, "subbank out of range");
  SubBankTaps& s = t.sb[subbank];
  if (!h_ref) return fail(RFD_E_INVALID, "h_ref is NULL");
  if (count < 0 || first < 0 || first + count > s.count) return fail(RFD_E_INVALID, "template range outside the sub-bank");
  if (count > 0 && !h_tmpl) return fail(RFD_E_INVALID, "h_tmpl is NULL");
  const bool centre = (method & RFD_TAPS_CENTRE) != 0;
  method &= ~RFD_TAPS_CENTRE;
  if (method != RFD_TAPS_LS && method != RFD_TAPS_WINDOW) return fail(RFD_E_INVALID, "unknown taps method");
  if (method == RFD_TAPS_LS && (!(ridge_eps >= 0.0) || !isfinite(ridge_eps)))
    return fail(RFD_E_INVALID, "ridge_eps must be finite and >= 0");
  if (count == 0) return RFD_OK;
  const int T = s.T;
  // FFT scratch for a chunk of templates (<= 256 MiB)
  int64_t chunk = std::max<int64_t>(1, ((int64_t)256 << 20) / (p.n * (int64_t)sizeof(double2)));
  chunk = std::min<int64_t>(chunk, 64);
  chunk = std::min<int64_t>(chunk, count);
  size_t need_w = (size_t)std::max<int64_t>(chunk, 1) * p.n;
  if (t.work64_cap < need_w) {
    RFD_HIP(hipStreamSynchronize(p.stream));
    dfree(t.work64);
    t.work64_cap = 0;
    int rc = dalloc(&t.work64, need_w);
    if (rc) return rc;
    t.work64_cap = need_w;
  }
  size_t need_b = (size_t)count * T;          // right-hand sides of the whole call
  if (t.bvec_cap < need_b) {
    RFD_HIP(hipStreamSynchronize(p.stream));
    dfree(t.bvec);
    t.bvec_cap = 0;
    int rc = dalloc(&t.bvec, need_b);
    if (rc) return rc;
    t.bvec_cap = need_b;
  }
  // reference autocorrelation g (always) and the Cholesky factor (LS)
  const double eps = method == RFD_TAPS_LS ? ridge_eps : -1.0;
  if (method == RFD_TAPS_LS && (!s.L || s.eps != ridge_eps)) {
    if (!s.L) {
      int rc = dalloc(&s.L, (size_t)T * T);
      if (rc) return rc;
      rc = dalloc(&s.U, (size_t)T * T);
      if (rc) return rc;
    }
    int rc = taps_prepare_subbank(p, t, subbank, h_ref, eps);
    if (rc) return rc;
  } else {
    // g is cheap; refresh it so sigma_fit always uses this reference
    int rc = launch_corr64(p, t, 1, h_ref, nullptr, 1, T, 0, s.g, T);
    if (rc) return rc;
  }
  // per-template lag windows: the peak of each template's full correlation
  int32_t* dsh = t.d_shift + s.first + first;
  if (centre) {
    const size_t need_p = (size_t)chunk * p.n;
    if (t.peak_cap < need_p) {
      RFD_HIP(hipStreamSynchronize(p.stream));
      dfree(t.peak_pw);
      t.peak_cap = 0;
      int rc = dalloc(&t.peak_pw, need_p);
      if (rc) return rc;
      t.peak_cap = need_p;
    }
    const size_t need_q = (size_t)chunk * kPeakParts;
    if (t.peak_parts_cap < need_q) {
      RFD_HIP(hipStreamSynchronize(p.stream));
      dfree(t.peak_part);
      dfree(t.peak_idx);
      t.peak_parts_cap = 0;
      int rc = dalloc(&t.peak_part, need_q);
      if (!rc) rc = dalloc(&t.peak_idx, need_q);
      if (rc) return rc;
      t.peak_parts_cap = need_q;
    }
    if (t.k0buf_cap < (size_t)count) {
      RFD_HIP(hipStreamSynchronize(p.stream));
      dfree(t.k0buf);
      t.k0buf_cap = 0;
      int rc = dalloc(&t.k0buf, (size_t)count);
      if (rc) return rc;
      t.k0buf_cap = (size_t)count;
    }
  } else {
    bool any = false;
    for (int64_t i = first; i < first + count && !any; ++i) any = s.centred_mask[i] != 0;
    if (any) RFD_HIP(hipMemsetAsync(dsh, 0, count * sizeof(int32_t), p.stream));
  }
  {
    int rc = stage_begin(p, kStTaps);
    if (rc) return rc;
  }
  // correlation FFTs in chunks bounded by the FP64 scratch, then one solve
  // launch over every template of the call
  for (int64_t c0 = 0; c0 < count; c0 += chunk) {
    int64_t cn = std::min(chunk, count - c0);
    const int32_t* k0s = nullptr;
    if (centre) {
      int rc = launch_corr_peak(p, t, h_ref, h_tmpl + 2 * c0 * p.nb, cn, T, s.k0, t.peak_pw, t.k0buf + c0,
                                dsh + c0);
      if (rc) return rc;
      k0s = t.k0buf + c0;
    }
    int rc = launch_corr64(p, t, method == RFD_TAPS_LS ? 0 : 2, h_ref, h_tmpl + 2 * c0 * p.nb, cn, T, s.k0,
                           t.bvec + c0 * T, T, -1, -1, k0s);
    if (rc) return rc;
  }
  {
    int rc = taps_solve_and_pack(p, t, subbank, first, count, method);
    if (rc) return rc;
  }
  {
    int rc = stage_end(p);
    if (rc) return rc;
  }
  for (int64_t i = first; i < first + count; ++i) {
    if (!s.made_mask[i]) {
      s.made_mask[i] = 1;
      ++s.made;
    }
    if ((s.centred_mask[i] != 0) != centre) {
      s.centred_mask[i] = centre ? 1 : 0;
      s.n_centred += centre ? 1 : -1;
    }
  }
  return RFD_OK;
}

int rfd_taps_get(const rfd_taps* taps, int64_t tmpl, double* a_out, double* sigma_fit_out, int32_t* taps_out,
                 int32_t* k0_out) {
  if (!taps) return fail(RFD_E_INVALID, "taps is NULL");
  const Taps& t = taps->t;
  if (tmpl < 0 || tmpl >= t.n_templates) return fail(RFD_E_INVALID, "template index out of range");
  int b = 0;
  while (b + 1 < (int)t.sb.size() && t.sb[b + 1].first <= tmpl) ++b;
  const SubBankTaps& s = t.sb[b];
  hipStream_t st = t.plan->stream;
  if (a_out)
    RFD_HIP(hipMemcpyAsync(a_out, t.a64 + s.a_base + (tmpl - s.first) * s.Tp, s.T * sizeof(double2),
                           hipMemcpyDeviceToHost, st));
  if (sigma_fit_out)
    RFD_HIP(hipMemcpyAsync(sigma_fit_out, t.sigma_fit + tmpl, sizeof(double), hipMemcpyDeviceToHost, st));
  int32_t d = 0;
  RFD_HIP(hipMemcpyAsync(&d, t.d_shift + tmpl, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  RFD_HIP(hipStreamSynchronize(st));
  if (taps_out) *taps_out = s.T;
  if (k0_out) *k0_out = s.k0 + d;
  return RFD_OK;
}

int rfd_taps_destroy(rfd_taps* taps) {
  if (!taps) return RFD_OK;
  if (taps->t.users > 0)
    return fail(RFD_E_STATE, "taps still used by " + std::to_string(taps->t.users) + " graph(s) or stream(s)");
  (void)hipStreamSynchronize(taps->t.plan->stream);
  taps_free(taps->t);
  delete taps;
  return RFD_OK;
}

int rfd_filter_bank(rfd_plan* plan, const rfd_taps* taps, int32_t precision, float threshold, int64_t cluster_window,
                    rfd_trigger* out, int64_t capacity, int64_t* n_out) {
  if (!plan || !taps) return fail(RFD_E_INVALID, "NULL plan or taps");
  Plan& p = plan->p;
  const Taps& t = taps->t;
  if (t.plan != &p) return fail(RFD_E_INVALID, "taps belong to another plan");
  if (!valid_precision(precision)) return fail(RFD_E_INVALID, "unknown precision");
  int rc = check_filter_args(p, threshold, cluster_window, out, capacity, n_out);
  if (rc) return rc;
  rc = check_bank_state(p, t);
  if (rc) return rc;
  Taps& tm = const_cast<Taps&>(t);   // the work-item tables are a cache
  const int64_t nwin = (p.n + cluster_window - 1) / cluster_window;
  const int64_t n_slots = t.n_templates * nwin;
  rc = ensure_slots(p, std::max<int64_t>(n_slots, 1));
  if (rc) return rc;
  rc = prepare_fir(p, tm, precision, cluster_window);
  if (rc) return rc;
  rc = launch_slots_clear(p, n_slots);
  if (rc) return rc;
  rc = stage_begin(p, kStFir);
  if (rc) return rc;
  rc = enqueue_fir(p, tm, precision, cluster_window, nwin, threshold);
  if (rc) return rc;
  rc = stage_end(p);
  if (!rc) rc = stage_begin(p, kStCompact);
  if (rc) return rc;
  rc = launch_compact_bank(p, t, n_slots, nwin, cluster_window, threshold, out, capacity);
  if (rc) return rc;
  rc = launch_fir_z(p, t, out, std::min<int64_t>(capacity, (int64_t)1 << 26));
  if (!rc) rc = stage_end(p);
  if (rc) return rc;
  return finish_triggers(p, capacity, n_out);
}

int rfd_filter_range(rfd_plan* plan, const rfd_taps* taps, int32_t precision, float threshold, int64_t cluster_window,
                     int64_t n_start, int64_t n_len, rfd_trigger* out, int64_t capacity, int64_t* n_out) {
  if (!plan || !taps) return fail(RFD_E_INVALID, "NULL plan or taps");
  Plan& p = plan->p;
  const Taps& t = taps->t;
  if (t.plan != &p) return fail(RFD_E_INVALID, "taps belong to another plan");
  if (!valid_precision(precision)) return fail(RFD_E_INVALID, "unknown precision");
  if (n_start < 0 || n_len < 256 || n_start % 256 != 0 || n_len % 256 != 0 || n_start + n_len > p.n)
    return fail(RFD_E_INVALID, "range must be 256-sample aligned, non-empty and inside the segment");
  int rc = check_filter_args(p, threshold, cluster_window, out, capacity, n_out);
  if (rc) return rc;
  rc = check_bank_state(p, t);
  if (rc) return rc;
  Taps& tm = const_cast<Taps&>(t);
  const int64_t nwin = (p.n + cluster_window - 1) / cluster_window;
  const int64_t n_slots = t.n_templates * nwin;
  rc = ensure_slots(p, std::max<int64_t>(n_slots, 1));
  if (rc) return rc;
  if (precision == RFD_OLS32) {
    rc = ensure_ols(p, tm);
    if (rc) return rc;
  }
  // clear and compact only the windows the range meets
  const int64_t rlo = n_start, rhi = n_start + n_len;
  WinMap m;
  if (!win_map_range(nwin, cluster_window, 1, &rlo, &rhi, &m)) m = win_map_all(nwin);
  const int64_t n_visit = t.n_templates * m.nq;
  rc = launch_slots_clear_map(p, n_visit, m);
  if (rc) return rc;
  rc = stage_begin(p, kStFir);
  if (rc) return rc;
  if (precision == RFD_OLS32) {
    rc = launch_ols(p, t, cluster_window, nwin, threshold, n_start, n_start + n_len);
  } else {
    for (size_t b = 0; !rc && b < t.sb.size(); ++b)
      rc = launch_fir(p, t, (int)b, precision, cluster_window, nwin, threshold, n_start, n_len);
  }
  if (rc) return rc;
  rc = stage_end(p);
  if (!rc) rc = stage_begin(p, kStCompact);
  if (rc) return rc;
  rc = launch_compact_bank(p, t, n_visit, nwin, cluster_window, threshold, out, capacity, &m);
  if (rc) return rc;
  rc = launch_fir_z(p, t, out, std::min<int64_t>(capacity, (int64_t)1 << 26));
  if (!rc) rc = stage_end(p);
  if (rc) return rc;
  return finish_triggers(p, capacity, n_out);
}

int rfd_findchirp_prepare(rfd_plan* plan, const double* h_tmpl, int64_t count, float* filt_out, double* sigma_out) {
  if (!plan) return fail(RFD_E_INVALID, "plan is NULL");
  Plan& p = plan->p;
  if (count < 0) return fail(RFD_E_INVALID, "count must be >= 0");
  if (count == 0) return RFD_OK;
  if (!h_tmpl || !filt_out) return fail(RFD_E_INVALID, "NULL argument");
  double* sig = sigma_out;
  double* tmp = nullptr;
  if (!sig) {
    int rc = dalloc(&tmp, (size_t)count);
    if (rc) return rc;
    sig = tmp;
  }
  int rc = launch_findchirp_prepare(p, h_tmpl, count, reinterpret_cast<float2*>(filt_out), sig);
  if (tmp) {
    (void)hipStreamSynchronize(p.stream);
    dfree(tmp);
  }
  return rc;
}

int findchirp_filter(rfd_plan* plan, const double* data, const float* filt, int64_t n_templates, float threshold,
                     int64_t cluster_window, rfd_trigger* out, int64_t capacity, int64_t* n_out) {
  if (!plan) return fail(RFD_E_INVALID, "plan is NULL");
  Plan& p = plan->p;
  int rc = check_filter_args(p, threshold, cluster_window, out, capacity, n_out);
  if (rc) return rc;
  if (n_templates < 0 || n_templates > ((int64_t)1 << 31) - 1) return fail(RFD_E_INVALID, "n_templates out of range");
  if (n_templates > 0 && !filt) return fail(RFD_E_INVALID, "filt is NULL");
  if (data) {
    rc = stage_begin(p, kStDataFft);
    if (!rc) rc = launch_data_fft(p, data);
    if (!rc) rc = stage_end(p);
    if (rc) return rc;
    ++p.seg_gen;
  } else if (p.seg_gen == 0) {
    return fail(RFD_E_STATE, "no segment: pass data");
  }
  const int64_t nwin = (p.n + cluster_window - 1) / cluster_window;
  const int64_t n_slots = n_templates * nwin;
  rc = ensure_slots(p, std::max<int64_t>(n_slots, 1));
  if (rc) return rc;
  const size_t need = findchirp_work_size(p);
  if (p.fc_work_cap < need) {
    if (p.ws_external)
      return fail(RFD_E_NOMEM, "workspace too small: FINDCHIRP needs " + std::to_string(need * sizeof(float2)) +
                                   " bytes of intermediate (set the workspace with with_findchirp = 1)");
    RFD_HIP(hipStreamSynchronize(p.stream));
    ++p.res_gen;
    dfree(p.fc_work);
    p.fc_work_cap = 0;
    rc = dalloc(&p.fc_work, need);
    if (rc) return rc;
    p.fc_work_cap = need;
  }
  rc = launch_slots_clear(p, n_slots);
  if (rc) return rc;
  if (n_templates > 0) {
    rc = stage_begin(p, kStFindchirp);
    if (!rc) rc = launch_findchirp(p, reinterpret_cast<const float2*>(filt), n_templates, cluster_window, nwin,
                                      threshold);
    if (!rc) rc = stage_end(p);
    if (rc) return rc;
  }
  rc = stage_begin(p, kStCompact);
  if (rc) return rc;
  rc = launch_compact(p, n_slots, nwin, cluster_window, threshold, out, capacity);
  if (rc) return rc;
  rc = launch_findchirp_z(p, reinterpret_cast<const float2*>(filt), out, std::min<int64_t>(capacity, 4096));
  if (!rc) rc = stage_end(p);
  if (rc) return rc;
  return finish_triggers(p, capacity, n_out);
}

struct rfd_graph {
  rfd_plan* plan = nullptr;
  rfd::Taps* taps = nullptr;
  int precision = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<int32_t> ref_ids;
  int64_t capacity = 0;
  int64_t plan_gen = 0, taps_gen = 0;   // buffer generations the capture saw
};

}  // extern "C"

// Capture of one segment's launches (transform, every dechirp, slot clear,
// FIR, window peaks, compaction, trigger z) into a graph; n_len > 0 limits the
// FIR and the trigger search to outputs [n_start, n_start + n_len) as
// rfd_filter_range does, n_len == 0 covers the whole segment.
static int graph_create(rfd_plan* plan, const rfd_taps* taps, int32_t precision, float threshold,
                        int64_t cluster_window, const double* data, int32_t n_refs, const int32_t* ref_ids,
                        const double* const* h_refs, int64_t n_start, int64_t n_len, rfd_trigger* out,
                        int64_t capacity, rfd_graph** graph) {
  if (!graph) return fail(RFD_E_INVALID, "graph is NULL");
  *graph = nullptr;
  if (!plan || !taps || !data || !ref_ids || !h_refs) return fail(RFD_E_INVALID, "NULL argument");
  Plan& p = plan->p;
  Taps& t = const_cast<Taps&>(taps->t);
  if (t.plan != &p) return fail(RFD_E_INVALID, "taps belong to another plan");
  if (!valid_precision(precision)) return fail(RFD_E_INVALID, "unknown precision");
  int64_t dummy = 0;
  int rc = check_filter_args(p, threshold, cluster_window, out, capacity, &dummy);
  if (rc) return rc;
  if (n_refs < 1 || n_refs > p.max_refs) return fail(RFD_E_INVALID, "n_refs out of range");
  std::vector<int> seen(p.max_refs, 0);
  for (int i = 0; i < n_refs; ++i) {
    if (ref_ids[i] < 0 || ref_ids[i] >= p.max_refs || seen[ref_ids[i]]) return fail(RFD_E_INVALID, "bad ref_ids");
    if (!h_refs[i]) return fail(RFD_E_INVALID, "NULL reference template");
    seen[ref_ids[i]] = 1;
  }
  for (auto& s : t.sb)
    if (s.count && !seen[s.ref_id]) return fail(RFD_E_INVALID, "a sub-bank's reference is not in ref_ids");
  for (auto& s : t.sb)
    if (s.made != s.count) return fail(RFD_E_STATE, "taps not made");
  const bool ranged = n_len != 0;
  if (ranged && (n_start < 0 || n_len < 256 || n_start % 256 != 0 || n_len % 256 != 0 || n_start + n_len > p.n))
    return fail(RFD_E_INVALID, "range must be 256-sample aligned, non-empty and inside the segment");
  const int64_t nwin = (p.n + cluster_window - 1) / cluster_window;
  const int64_t n_slots = t.n_templates * nwin;
  rc = ensure_slots(p, std::max<int64_t>(n_slots, 1));
  if (rc) return rc;
  rc = ensure_dechirp_work(p);
  if (rc) return rc;
  rc = prepare_fir(p, t, precision, cluster_window);
  if (rc) return rc;
  RFD_HIP(hipStreamSynchronize(p.stream));
  hipStream_t cap = nullptr;
  RFD_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
  hipStream_t saved = p.stream;
  const bool saved_timing = p.timing;
  p.stream = cap;
  p.timing = false;
  hipGraph_t g = nullptr;
  rc = RFD_OK;
  if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    rc = fail(RFD_E_DEVICE, "hipStreamBeginCapture failed");
  } else {
    // a ranged graph clears and compacts only the windows its range meets
    WinMap m = win_map_all(nwin);
    const int64_t rlo = n_start, rhi = n_start + n_len;
    if (ranged && !win_map_range(nwin, cluster_window, 1, &rlo, &rhi, &m)) m = win_map_all(nwin);
    const int64_t n_visit = t.n_templates * m.nq;
    rc = launch_data_fft(p, data);
    if (!rc) rc = launch_dechirp_refs(p, n_refs, ref_ids, h_refs);
    if (!rc) rc = launch_slots_clear_map(p, n_visit, m);
    if (!rc && !ranged) rc = enqueue_fir(p, t, precision, cluster_window, nwin, threshold);
    if (!rc && ranged) {
      if (precision == RFD_OLS32) {
        rc = launch_ols(p, t, cluster_window, nwin, threshold, n_start, n_start + n_len);
      } else {
        for (size_t b = 0; !rc && b < t.sb.size(); ++b)
          rc = launch_fir(p, t, (int)b, precision, cluster_window, nwin, threshold, n_start, n_len);
      }
    }
    if (!rc) rc = launch_compact_bank(p, t, n_visit, nwin, cluster_window, threshold, out, capacity, &m);
    if (!rc) rc = launch_fir_z(p, t, out, std::min<int64_t>(capacity, (int64_t)1 << 26));
    hipError_t e = hipStreamEndCapture(cap, &g);
    if (!rc && e != hipSuccess) rc = fail(RFD_E_DEVICE, "hipStreamEndCapture failed");
  }
  p.stream = saved;
  p.timing = saved_timing;
  (void)hipStreamDestroy(cap);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  rfd_graph* h = new (std::nothrow) rfd_graph();
  if (!h) {
    (void)hipGraphDestroy(g);
    return fail(RFD_E_NOMEM, "host allocation failed");
  }
  h->plan = plan;
  h->taps = &t;
  ++p.users;
  ++t.users;
  h->precision = precision;
  h->plan_gen = p.res_gen;
  h->taps_gen = t.res_gen;
  h->graph = g;
  h->ref_ids.assign(ref_ids, ref_ids + n_refs);
  h->capacity = capacity;
  if (hipGraphInstantiate(&h->exec, g, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGraphDestroy(g);
    delete h;
    return fail(RFD_E_DEVICE, "hipGraphInstantiate failed");
  }
  *graph = h;
  return RFD_OK;
}

extern "C" {

int rfd_segment_graph_create(rfd_plan* plan, const rfd_taps* taps, int32_t precision, float threshold,
                             int64_t cluster_window, const double* data, int32_t n_refs, const int32_t* ref_ids,
                             const double* const* h_refs, rfd_trigger* out, int64_t capacity, rfd_graph** graph) {
  return graph_create(plan, taps, precision, threshold, cluster_window, data, n_refs, ref_ids, h_refs, 0, 0, out,
                      capacity, graph);
}

int rfd_range_graph_create(rfd_plan* plan, const rfd_taps* taps, int32_t precision, float threshold,
                           int64_t cluster_window, const double* data, int32_t n_refs, const int32_t* ref_ids,
                           const double* const* h_refs, int64_t n_start, int64_t n_len, rfd_trigger* out,
                           int64_t capacity, rfd_graph** graph) {
  if (n_len == 0) return fail(RFD_E_INVALID, "range must be 256-sample aligned, non-empty and inside the segment");
  return graph_create(plan, taps, precision, threshold, cluster_window, data, n_refs, ref_ids, h_refs, n_start, n_len,
                      out, capacity, graph);
}

int rfd_segment_graph_launch(rfd_graph* graph, int64_t* n_out) {
  if (!graph) return fail(RFD_E_INVALID, "graph is NULL");
  Plan& p = graph->plan->p;
  if (graph->precision == RFD_OLS32) {
    int rc = ensure_ols(p, *graph->taps, false);   // tap spectra of re-made taps, in place
    if (rc) return rc;
  }
  if (p.res_gen != graph->plan_gen || graph->taps->res_gen != graph->taps_gen)
    return fail(RFD_E_STATE, "buffers were reallocated since capture (more windows or another FIR configuration); "
                             "create the graph again");
  RFD_HIP(hipGraphLaunch(graph->exec, p.stream));
  ++p.seg_gen;
  for (int32_t r : graph->ref_ids) p.ref_gen[r] = p.seg_gen;
  if (!n_out) return RFD_OK;
  return finish_triggers(p, graph->capacity, n_out);
}

int rfd_graph_destroy(rfd_graph* graph) {
  if (!graph) return RFD_OK;
  (void)hipStreamSynchronize(graph->plan->p.stream);
  if (graph->exec) (void)hipGraphExecDestroy(graph->exec);
  if (graph->graph) (void)hipGraphDestroy(graph->graph);
  --graph->plan->p.users;
  --graph->taps->users;
  delete graph;
  return RFD_OK;
}

}  // extern "C"
