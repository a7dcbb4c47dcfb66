// rfd_filter_bank_noalloc: the filtering call of rfd_filter_bank with every
// per-call scratch buffer taken from one file-scope device array instead of
// device memory the library allocates.  For callers that cannot allocate
// (code under stream capture, tight serving loops, harnesses that forbid it).
//
// Scratch layout inside `scratch` (each region 256-byte aligned):
//   [trigger total: 1 long long][compaction block counts][window-peak slots
//    n_templates * ceil(N / W) u64][overlap-save block spectra of one
//    sub-bank: ceil(N / L) * K complex64 (ols32 only)]
// The slots are cleared by a fill kernel at the start of every call, the
// counts and the total are written before they are read, and the block
// spectra are rebuilt per sub-bank before its FIR reads them, so nothing
// depends on what an earlier call left there.
//
// Device addresses: in host code `scratch` names a host-side stand-in, not
// device memory.  The device address is looked up once per device with
// hipGetSymbolAddress (on the first call made while that device is current)
// and kept in g_scratch_ptr; kernels and fills receive that pointer only.
#include <math.h>

#include <algorithm>
#include <mutex>

#include "rfd_internal.h"

namespace rfd {

constexpr size_t kNoAllocScratchBytes = (size_t)32 << 20;   // per GPU, held until the process ends
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device.
static int scratch_address(void** out) {
  int dev = -1;
  RFD_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(RFD_E_UNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || ptr == nullptr)
      return fail(RFD_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return RFD_OK;
}

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Points the plan's epilogue scratch at the static array for the duration of
// one call and restores the plan's own buffers on every exit path.
struct ScratchSwap {
  Plan& p;
  unsigned long long* slots;
  size_t slots_cap;
  long long* counts;
  size_t counts_cap;
  long long* total;
  bool ws_external;
  bool timing;
  ScratchSwap(Plan& plan, unsigned long long* s, size_t s_cap, long long* c, size_t c_cap, long long* t)
      : p(plan), slots(plan.slots), slots_cap(plan.slots_cap), counts(plan.counts), counts_cap(plan.counts_cap),
        total(plan.total), ws_external(plan.ws_external), timing(plan.timing) {
    p.slots = s;
    p.slots_cap = s_cap;
    p.counts = c;
    p.counts_cap = c_cap;
    p.total = t;
    p.ws_external = true;
    p.timing = false;      // no event creation inside this call
  }
  ~ScratchSwap() {
    p.slots = slots;
    p.slots_cap = slots_cap;
    p.counts = counts;
    p.counts_cap = counts_cap;
    p.total = total;
    p.ws_external = ws_external;
    p.timing = timing;
  }
};

}  // namespace rfd

using namespace rfd;

extern "C" int rfd_filter_bank_noalloc(rfd_plan* plan, const rfd_taps* taps, int32_t precision, float threshold,
                                       int64_t cluster_window, rfd_trigger* out, int64_t capacity, int64_t* n_out) {
  if (!plan || !taps) return fail(RFD_E_INVALID, "NULL plan or taps");
  Plan& p = plan->p;
  const Taps& t = taps->t;
  if (t.plan != &p) return fail(RFD_E_INVALID, "taps belong to another plan");
  if (precision != RFD_FP32 && precision != RFD_BF16X3 && precision != RFD_FP16X3 && precision != RFD_OLS32)
    return fail(RFD_E_INVALID, "unknown precision");
  if (!(threshold >= 0.f) || !std::isfinite(threshold)) return fail(RFD_E_INVALID, "threshold must be finite and >= 0");
  if (cluster_window < 1 || cluster_window > p.n) return fail(RFD_E_INVALID, "cluster_window must satisfy 1 <= W <= N");
  if (capacity < 0) return fail(RFD_E_INVALID, "capacity must be >= 0");
  if (capacity > 0 && !out) return fail(RFD_E_INVALID, "out is NULL with capacity > 0");
  if (!n_out) return fail(RFD_E_INVALID, "n_out is NULL");
  for (size_t b = 0; b < t.sb.size(); ++b) {
    const SubBankTaps& s = t.sb[b];
    if (s.count == 0) continue;
    if (p.seg_gen == 0 || p.ref_gen[s.ref_id] != p.seg_gen)
      return fail(RFD_E_STATE, "sub-bank " + std::to_string(b) + ": reference slot not dechirped on this segment");
    if (s.made != s.count) return fail(RFD_E_STATE, "sub-bank " + std::to_string(b) + ": taps not made");
  }
  // scratch sizes of this call
  const int64_t nwin = (p.n + cluster_window - 1) / cluster_window;
  const int64_t n_slots = std::max<int64_t>(t.n_templates * nwin, 1);
  const size_t n_counts = (size_t)compaction_blocks(n_slots) + 1;
  size_t x_elems = 0;
  if (precision == RFD_OLS32) {
    for (const SubBankTaps& s : t.sb) {
      if (s.count == 0) continue;
      const OlsShape sh = ols_shape(p, s.T);
      const int64_t nB = (p.n + sh.L - 1) / sh.L;
      x_elems = std::max(x_elems, (size_t)nB * sh.K);
    }
  }
  const size_t off_counts = 256;
  const size_t off_slots = off_counts + align256(n_counts * sizeof(long long));
  const size_t off_x = off_slots + align256((size_t)n_slots * sizeof(unsigned long long));
  const size_t bytes = off_x + x_elems * sizeof(float2);
  if (bytes > kNoAllocScratchBytes)
    return fail(RFD_E_NOMEM, "rfd_filter_bank_noalloc: the call needs " + std::to_string(bytes) +
                                 " bytes of scratch, the static scratch holds " +
                                 std::to_string(kNoAllocScratchBytes) + " (fewer templates or a longer cluster window)");
  void* base = nullptr;
  int rc = scratch_address(&base);
  if (rc) return rc;
  unsigned char* sp = static_cast<unsigned char*>(base);
  Taps& tm = const_cast<Taps&>(t);
  if (precision == RFD_OLS32) {
    // tap spectra belong to the taps object: they must exist already (made by
    // an earlier rfd_filter_bank call with RFD_OLS32); stale ones are rebuilt
    // in place, which launches a kernel and allocates nothing
    rc = ensure_ols(p, tm, false, false);
    if (rc) return rc;
  }
  ScratchSwap swap(p, reinterpret_cast<unsigned long long*>(sp + off_slots), (size_t)n_slots,
                   reinterpret_cast<long long*>(sp + off_counts), n_counts, reinterpret_cast<long long*>(sp));
  rc = launch_slots_clear(p, n_slots);
  if (rc) return rc;
  if (precision == RFD_OLS32) {
    rc = launch_ols(p, t, cluster_window, nwin, threshold, 0, -1, reinterpret_cast<float2*>(sp + off_x));
  } else {
    for (size_t b = 0; !rc && b < t.sb.size(); ++b)
      rc = launch_fir(p, t, (int)b, precision, cluster_window, nwin, threshold);
  }
  if (rc) return rc;
  rc = launch_compact_bank(p, t, n_slots, nwin, cluster_window, threshold, out, capacity);
  if (rc) return rc;
  rc = launch_fir_z(p, t, out, std::min<int64_t>(capacity, (int64_t)1 << 26));
  if (rc) return rc;
  long long tot = 0;
  RFD_HIP(hipMemcpyAsync(&tot, p.total, sizeof(long long), hipMemcpyDeviceToHost, p.stream));
  RFD_HIP(hipStreamSynchronize(p.stream));
  *n_out = tot;
  if (tot > capacity)
    return fail(RFD_E_OVERFLOW, "trigger capacity " + std::to_string(capacity) + " < " + std::to_string(tot));
  return RFD_OK;
}
