/*
 * rfd.h - C ABI of the ratio-filter dechirping library for AMD MI355X (gfx950).
 *
 * Method: A. H. Nitz, K. Kacanja, K. Soni, "Beyond FINDCHIRP: Breaking the
 * memory wall and optimal FFTs for gravitational-wave matched-filter searches
 * with Ratio-Filter Dechirping", arXiv:2601.18835.
 *
 * Two-step matched filtering (Sec. III, Fig. 2):
 *   1. rfd_dechirp: one matched filter (Eq. 1) per *reference* template gives
 *      the reference SNR series z_ref(t);
 *   2. rfd_filter_bank: every target template of the reference's sub-bank is
 *      a short complex FIR applied to z_ref (Eq. 3), with taps from the
 *      weighted ridge least-squares fit of Sec. V.A (rfd_make_taps), and a
 *      fused |z|^2 / threshold / per-window-peak epilogue (Table II's peak
 *      find and trigger accumulation) so no per-template series is stored.
 *   findchirp_filter is the standard FFT-per-template matched filter (Eq. 1
 *   evaluated per template, Sec. III), the baseline the paper compares with.
 *
 * Conventions shared by every entry point
 *   - Segment: N = seg_len samples at rate fs (dt = 1/fs, df = fs/N); the
 *     transform convention is s(f_i) = dt * sum_m s[m] exp(-2 pi i i m/N),
 *     bins i = 0..N/2 ("rfft grid").  The analysis band is
 *     i_low = ceil(f_low/df) <= i <= N/2 - 1 (DC and Nyquist excluded).
 *   - Frequency-domain waveforms are complex128, interleaved (re, im), one
 *     row of N/2+1 bins per waveform, row-major, in DEVICE memory.
 *   - Every "dev" pointer is device memory owned by the caller (e.g. a torch
 *     tensor); the library never frees it and keeps no reference to it after
 *     the call returns.  Pointers marked "host" are host memory.
 *   - Device memory the library needs for itself (tables, the reference
 *     series store, taps, epilogue slots) is allocated by rfd_plan_create /
 *     rfd_taps_create and on the first use of a larger epilogue, and freed by
 *     the matching destroy call.  Calls made with sizes already seen allocate
 *     nothing.
 *   - All work is enqueued on the plan's HIP stream.  Calls return once the
 *     work is enqueued, except where an output is a host pointer (then the
 *     call synchronises the stream before returning).
 *   - Return value: RFD_OK (0) or a negative rfd_status.  No exception or
 *     abort crosses the ABI.  rfd_last_error() gives a thread-local message
 *     for the last failing call on the calling thread.
 *   - A plan is not thread-safe; use one plan per host thread / stream.
 */
#ifndef RFD_H
#define RFD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum rfd_status {
  RFD_OK = 0,
  RFD_E_INVALID = -1,     /* an argument is out of range or inconsistent */
  RFD_E_NOMEM = -2,       /* device allocation failed */
  RFD_E_DEVICE = -3,      /* a HIP runtime call or kernel launch failed */
  RFD_E_OVERFLOW = -4,    /* more triggers than `capacity`; *n_out = needed count */
  RFD_E_STATE = -5,       /* call order violated (e.g. filtering before dechirp) */
  RFD_E_UNSUPPORTED = -6  /* valid request this library does not implement */
} rfd_status;

/* FIR arithmetic (rfd_filter_bank). */
typedef enum rfd_precision {
  RFD_FP32 = 0,    /* FP32 operands, FP32 MFMA accumulation */
  RFD_BF16X3 = 1,  /* x = hi + lo in bfloat16; hi*hi + hi*lo + lo*hi, FP32 accumulation */
  RFD_FP16X3 = 2,  /* the same split in IEEE half precision */
  RFD_OLS32 = 3    /* overlap-save FFT blocks (the paper's block realisation), FP32 */
} rfd_precision;

/* Tap construction route (rfd_make_taps). */
typedef enum rfd_taps_method {
  RFD_TAPS_LS = 0,     /* weighted ridge least squares, Sec. V.A */
  RFD_TAPS_WINDOW = 1, /* truncated inverse transform of the ratio, Tukey(0.25) taper */
  /* flag OR-ed into either route: per-template lag centring (Sec. V.A's tap
   * tuning with the lag window placed per template).  Template j's T lags
   * are centred on the largest |b_j[l]| over every lag l in (-N/2, N/2],
   * b_j the weighted cross-correlation of target and reference (the normal
   * equations' right-hand side at every lag; lowest index 0..N-1 on exact
   * ties): k0_j = l_peak - floor(T/2), held as the offset
   * d_j = k0_j - k0 from the sub-bank's k0.  The FIR then runs on the
   * filter index m = n + d_j of each template: its cluster windows are
   * [qW, (q+1)W) in m, i.e. [qW - d_j, (q+1)W - d_j) mod N in samples, and
   * triggers report n (so they are ordered by (template, window), not
   * necessarily by sample).  Costs one extra N-point FP64 transform per
   * template at construction and nothing in the FIR. */
  RFD_TAPS_CENTRE = 0x100
} rfd_taps_method;

#define RFD_MAX_TAPS 2048

/* One trigger: the peak of one template in one cluster window (32 bytes). */
typedef struct rfd_trigger {
  int64_t sample;   /* output sample n of the peak, 0 <= n < N */
  int32_t tmpl;     /* template index (global over all sub-banks) */
  int32_t subbank;  /* sub-bank index (0 for findchirp_filter) */
  float rho;        /* normalised SNR |z| at the peak, as thresholded */
  float z_re;       /* complex normalised SNR at the peak (FP32 re-evaluation) */
  float z_im;
  uint32_t flags;   /* 0; 1 when z_re/z_im were not evaluated (FINDCHIRP beyond 4096 triggers) */
} rfd_trigger;

typedef struct rfd_plan_info {
  int64_t n;          /* N */
  int64_t n_bins;     /* N/2 + 1 */
  int64_t i_low;      /* first in-band bin */
  int64_t i_high;     /* last in-band bin (N/2 - 1) */
  int64_t n_band;     /* i_high - i_low + 1 */
  double fs, f_low, df;
  double data_scale;  /* FP64 factor applied to the data before its transform */
  int32_t max_refs;   /* reference-series slots */
  int32_t fft_n1, fft_n2;  /* two-pass FFT factorisation N = n1 * n2 */
} rfd_plan_info;

typedef struct rfd_plan rfd_plan;
typedef struct rfd_taps rfd_taps;

/*
 * rfd_plan_create - analysis plan for one PSD and segment length (FP64 host
 * planning: PSD weights w_i = 4 df / S_n(f_i) of Eq. 1, FP64-accurate
 * twiddle tables rounded once to FP32, data scale).
 *   psd      host float64 [n_psd], one-sided PSD on the rfft grid; must be
 *            finite and > 0 on every in-band bin (other bins are ignored).
 *   n_psd    must equal seg_len/2 + 1.
 *   f_low    low-frequency cutoff, 0 < f_low < fs/2.
 *   fs       sample rate (Hz), > 0.
 *   seg_len  N, a power of two in [2^10, 2^22].
 *   max_refs number of reference-series slots (1..4096); each holds the
 *            normalised series in FP32 and room for its hi/lo 16-bit planes,
 *            which the 16-bit FIR forms split from it (24 N bytes).
 *   stream   hipStream_t (NULL: the null stream).
 *   out      receives the plan.
 * Errors: RFD_E_INVALID for any violated range above, RFD_E_NOMEM,
 * RFD_E_DEVICE.
 */
int rfd_plan_create(const double* psd, int64_t n_psd, double f_low, double fs, int64_t seg_len,
                    int32_t max_refs, void* stream, rfd_plan** out);
int rfd_plan_info_get(const rfd_plan* plan, rfd_plan_info* out);
int rfd_plan_set_stream(rfd_plan* plan, void* stream);
int rfd_plan_destroy(rfd_plan* plan);

/*
 * rfd_plan_workspace_size - bytes of the per-call scratch of the filtering
 * calls (rfd_filter_bank, rfd_filter_range, findchirp_filter, the segment
 * graph): the window-peak slots of the fused epilogue (8 B per template and
 * cluster window, Table II's peak find), the compaction's per-block counts,
 * and with with_findchirp != 0 FINDCHIRP's four-step intermediate (N * 8 B
 * per template of a batch, up to 256 MiB; none when N <= 4096).  The size
 * grows with N / W, not with the tap count: tap storage belongs to the taps
 * object.
 *   max_templates       largest template count of a call (0 .. 2^31-1).
 *   min_cluster_window  smallest cluster window W of a call (1 .. N).
 *   bytes               receives the size (a multiple of 256).
 * Errors: RFD_E_INVALID for a NULL argument or a range violated above.
 */
int rfd_plan_workspace_size(const rfd_plan* plan, int64_t max_templates, int64_t min_cluster_window,
                            int32_t with_findchirp, size_t* bytes);
/*
 * rfd_plan_set_workspace - the filtering calls take their scratch from
 * caller-owned device memory [dev_ptr, dev_ptr + bytes) instead of growing
 * library-owned buffers: from then on they allocate none of it, and a call
 * needing more than the sizes given here (more templates, a smaller window,
 * FINDCHIRP when with_findchirp was 0) fails with RFD_E_NOMEM and changes
 * nothing.  The memory must stay valid, and unused by the caller, while the
 * plan may run work on its stream; the library never frees it.  Waits for the
 * plan's stream, releases library-owned scratch, and invalidates segment
 * graphs captured before (their replays return RFD_E_STATE).
 *   dev_ptr  device pointer, 256-byte aligned; NULL returns to library-owned
 *            scratch (the other arguments are then ignored).
 *   bytes    at least rfd_plan_workspace_size(max_templates,
 *            min_cluster_window, with_findchirp).
 * Errors: RFD_E_INVALID (misaligned pointer, bytes too small, ranges as in
 * rfd_plan_workspace_size), RFD_E_DEVICE.
 */
int rfd_plan_set_workspace(rfd_plan* plan, void* dev_ptr, size_t bytes, int64_t max_templates,
                           int64_t min_cluster_window, int32_t with_findchirp);

/*
 * rfd_dechirp - reference matched filter (Eq. 1 with h = h_ref; the
 * dechirped series of Eq. 3 and Fig. 2).
 *   data     dev float64 [N]: the segment's time series.  When non-NULL its
 *            transform is computed first (once per segment) and every
 *            reference series of the previous segment becomes stale.  NULL
 *            reuses the current segment's transform (RFD_E_STATE if none).
 *   h_ref    dev complex128 [N/2+1]: the reference template.
 *   ref_id   slot 0 <= ref_id < max_refs that receives
 *            z_ref[n]/sigma_ref, n = 0..N-1, where
 *            z_ref[n] = sum_i w_i s_i conj(h_ref,i) exp(+2 pi i i n / N) and
 *            sigma_ref^2 = sum_i w_i |h_ref,i|^2 (precision: rfd_dechirp_refs).
 *   sigma_ref_out  host double or NULL: receives sigma_ref (synchronises).
 * Errors: RFD_E_INVALID (NULL h_ref, ref_id out of range, sigma_ref = 0),
 * RFD_E_STATE (data NULL with no segment), RFD_E_DEVICE.
 */
int rfd_dechirp(rfd_plan* plan, const double* data, const double* h_ref, int32_t ref_id,
                double* sigma_ref_out);
/*
 * rfd_dechirp_refs - rfd_dechirp for several references of one segment:
 * the segment transform once (when data is non-NULL), then every
 * reference's series through batched launches (up to 32 references, or
 * 64 MiB of intermediates, per launch), each result identical to
 * rfd_dechirp's for that reference.
 *   n_refs     1 .. max_refs.
 *   ref_ids    host int32 [n_refs]: distinct slots 0 <= id < max_refs.
 *   h_refs     host array [n_refs] of dev complex128 [N/2+1] references.
 *   sigma_out  host double [n_refs] or NULL: sigma_ref of each (synchronises).
 * Errors: RFD_E_INVALID (NULL arrays or entries, ids out of range or
 * repeated, a reference with sigma_ref = 0), RFD_E_STATE, RFD_E_NOMEM,
 * RFD_E_DEVICE.
 *
 * Precision: the segment transform, the integrand w_i s_i conj(h_ref,i) /
 * sigma_ref and sigma_ref are FP64; the two transform passes of each
 * reference run in FP32 (twiddles rounded once from FP64), which adds about
 * 2e-7 of max |z_ref| to the series.  rfd_plan_set_dechirp_fp64(plan, 1)
 * runs them in FP64 instead (0 restores the default); changing it refuses
 * replays of graphs captured before.
 */
int rfd_dechirp_refs(rfd_plan* plan, const double* data, int32_t n_refs, const int32_t* ref_ids,
                     const double* const* h_refs, double* sigma_out);
int rfd_plan_set_dechirp_fp64(rfd_plan* plan, int32_t enable);

/* Copy slot ref_id's normalised series z_ref/sigma_ref (dev complex64 [N]). */
int rfd_get_zref(const rfd_plan* plan, int32_t ref_id, float* out);

/*
 * rfd_taps_create - storage for the ratio taps of a bank of sub-banks
 * (Sec. IV: each target template belongs to one reference's sub-bank).
 *   n_subbanks  >= 1.
 *   offsets     host int64 [n_subbanks+1]: templates of sub-bank b are the
 *               global indices offsets[b] .. offsets[b+1]-1; offsets[0] = 0,
 *               non-decreasing.
 *   ref_id      host int32 [n_subbanks]: reference slot filtered by sub-bank b.
 *   taps        host int32 [n_subbanks]: tap count T_b, 1..RFD_MAX_TAPS.
 *   k0          host int32 [n_subbanks]: lag of tap 0 (tap k sits at lag
 *               k0 + k samples), |k0| < N/2.
 * Errors: RFD_E_INVALID, RFD_E_NOMEM.
 */
int rfd_taps_create(rfd_plan* plan, int32_t n_subbanks, const int64_t* offsets, const int32_t* ref_id,
                    const int32_t* taps, const int32_t* k0, rfd_taps** out);

/*
 * rfd_make_taps - FP64 ratio taps for `count` templates of one sub-bank
 * (Sec. V.A), their fitted-template norms (Sec. VI.B) and the FIR operands.
 *   subbank    sub-bank index.
 *   h_ref      dev complex128 [N/2+1]: the sub-bank's reference template.
 *   h_tmpl     dev complex128 [count][N/2+1]: templates first..first+count-1
 *              of the sub-bank (indices relative to the sub-bank).
 *   method     RFD_TAPS_LS: minimise sum_i u_i |R_i - A_i|^2 + lam |a|^2 with
 *              R = h/h_ref, u_i = w_i |h_ref,i|^2, A_i = sum_k a_k
 *              exp(-2 pi i i (k0+k)/N), lam = ridge_eps * sum_i u_i, solved
 *              through the Hermitian Toeplitz normal equations by Cholesky
 *              (factor from the Toeplitz Schur recursion); RFD_E_INVALID when
 *              M + lam I is not positive definite (a reference zero in band).
 *              RFD_TAPS_WINDOW: a_k = tukey_k (1/N) sum_i R_i exp(+2 pi i i
 *              (k0+k)/N) (ridge_eps ignored).
 *              Either route may carry RFD_TAPS_CENTRE (per-template lag
 *              windows, see rfd_taps_method); re-making a template without
 *              it returns it to the sub-bank's k0.
 *   ridge_eps  >= 0 (LS); 1e-4 is the documented default (it bounds the
 *              normalised tap gain ||c||_2, which multiplies rounding noise).
 * The FIR applies c_k = conj(a_k) sigma_ref / sigma_fit to z_ref/sigma_ref,
 * sigma_fit^2 = a^H M a, M[l,k] = sum_i u_i exp(2 pi i i (l-k)/N).
 * Errors: RFD_E_INVALID (ranges, NULL pointers, first+count beyond the
 * sub-bank), RFD_E_DEVICE.
 */
int rfd_make_taps(rfd_plan* plan, rfd_taps* taps, int32_t subbank, const double* h_ref,
                  const double* h_tmpl, int64_t first, int64_t count, int32_t method, double ridge_eps);

/* Read back one template's FP64 taps a (host complex128 [T]), sigma_fit,
 * T and its own k0 (the sub-bank's, plus d_j under RFD_TAPS_CENTRE)
 * (synchronises).  Any output pointer may be NULL. */
int rfd_taps_get(const rfd_taps* taps, int64_t tmpl, double* a_out, double* sigma_fit_out,
                 int32_t* taps_out, int32_t* k0_out);
/* rfd_taps_destroy: RFD_E_STATE while a graph or stream uses the taps. */
int rfd_taps_destroy(rfd_taps* taps);

/*
 * rfd_filter_bank - the ratio FIR of Eq. 3 for every template of every
 * sub-bank, on the current segment's reference series, with the fused
 * epilogue.  For template j of sub-bank b:
 *     z_j[n] = sum_k c_j[k] zhat_ref[(n + k0_b + k) mod N],  rho = |z_j|,
 * computed as a complex GEMM on MFMA; in each window [qW, (q+1)W) the sample
 * of largest rho^2 (lowest n on ties) is a trigger when rho > threshold.
 *   precision       rfd_precision.
 *   threshold       >= 0, on rho (compared as rho^2 > threshold^2).
 *   cluster_window  W, 1 <= W <= N.
 *   out             dev rfd_trigger [capacity], sorted by (tmpl, sample).
 *   capacity        >= 0.
 *   n_out           host int64: number of triggers (synchronises).  On
 *                   RFD_E_OVERFLOW it is the required count and the first
 *                   `capacity` triggers are valid.
 * Errors: RFD_E_INVALID, RFD_E_STATE (a sub-bank's reference slot was not
 * dechirped on the current segment, or taps not made), RFD_E_OVERFLOW,
 * RFD_E_NOMEM, RFD_E_DEVICE.
 */
int rfd_filter_bank(rfd_plan* plan, const rfd_taps* taps, int32_t precision, float threshold,
                    int64_t cluster_window, rfd_trigger* out, int64_t capacity, int64_t* n_out);

/*
 * rfd_filter_bank_noalloc - rfd_filter_bank for callers that cannot allocate
 * device memory (code under stream capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, kernels, results and errors as
 * rfd_filter_bank, except:
 *   - every per-call scratch buffer (window-peak slots, compaction counts,
 *     the trigger total, overlap-save block spectra) lives in one static
 *     device array of 32 MiB inside the library, one copy per GPU, held
 *     until the process ends; the call allocates and frees nothing;
 *   - a call whose scratch exceeds 32 MiB fails with RFD_E_NOMEM
 *     (n_templates * ceil(N / W) * 8 B of slots, plus ceil(N / L) * K * 8 B
 *     of block spectra for RFD_OLS32);
 *   - direct forms run one launch per sub-bank (no persistent work queue);
 *   - RFD_OLS32 needs the taps' spectra to exist already (one earlier
 *     rfd_filter_bank call with RFD_OLS32 makes them), else RFD_E_STATE;
 *   - stage timing is not recorded.
 * The static array keeps the last call's contents; every call clears what it
 * reads before reading it.  Calls that overlap on one GPU (several host
 * threads or streams) share the array and race: serialise them.
 */
int rfd_filter_bank_noalloc(rfd_plan* plan, const rfd_taps* taps, int32_t precision, float threshold,
                            int64_t cluster_window, rfd_trigger* out, int64_t capacity, int64_t* n_out);

/*
 * rfd_findchirp_prepare - FINDCHIRP filters F_j = w_i conj(h_j,i) / sigma_j
 * (times the plan's data-scale compensation), FP64 on the device, stored in
 * complex64 over the band bins.
 *   h_tmpl     dev complex128 [count][N/2+1].
 *   filt_out   dev complex64 [count][n_band] (n_band from rfd_plan_info).
 *   sigma_out  dev float64 [count] or NULL: sigma_j.
 */
int rfd_findchirp_prepare(rfd_plan* plan, const double* h_tmpl, int64_t count, float* filt_out,
                          double* sigma_out);

/*
 * findchirp_filter - the standard matched filter per template (Eq. 1: one
 * pointwise product and one inverse FFT of length N per template) with the
 * same fused epilogue as rfd_filter_bank.
 *   data      dev float64 [N] or NULL (reuse the current segment transform).
 *   filt      dev complex64 [n_templates][n_band] from rfd_findchirp_prepare.
 *   Remaining arguments as rfd_filter_bank; triggers carry subbank = 0.
 */
int findchirp_filter(rfd_plan* plan, const double* data, const float* filt, int64_t n_templates,
                     float threshold, int64_t cluster_window, rfd_trigger* out, int64_t capacity,
                     int64_t* n_out);

/*
 * Stage timing with HIP events on the plan's stream (for profiling; the
 * paper's Table II reports the same stages on a CPU).  While enabled, every
 * entry point records an event pair around each of its stages; get returns
 * the summed milliseconds and the number of recorded intervals since the
 * previous get (synchronising on the recorded events), then resets them.
 */
typedef struct rfd_timing {
  double data_fft_ms;   /* segment transform */
  double dechirp_ms;    /* reference filters + reference-series transforms */
  double fir_ms;        /* ratio-FIR GEMM kernels with the fused epilogue */
  double compact_ms;    /* slot clearing, trigger compaction, z re-evaluation */
  double findchirp_ms;  /* FINDCHIRP transforms with the fused epilogue */
  double taps_ms;       /* tap construction */
  double sur_net_ms;    /* surrogate network forward pass (inference) */
  double sur_expand_ms; /* surrogate coefficients -> FP64 taps and sigma_fit */
  double sur_pack_ms;   /* surrogate taps: normalisation and MFMA packing */
  double match_ms;      /* fitted-template match of two tap sets */
  int64_t n_data_fft, n_dechirp, n_fir, n_compact, n_findchirp, n_taps, n_sur_net, n_sur_expand, n_sur_pack,
      n_match;
  double fir_kernel_ms; /* the main FIR kernel launches alone (one interval per launch), inside fir_ms */
  int64_t n_fir_kernel;
} rfd_timing;
int rfd_plan_set_timing(rfd_plan* plan, int32_t enable);
int rfd_plan_get_timing(rfd_plan* plan, rfd_timing* out);

/*
 * FIR launch configuration.  Output is identical for every setting; only
 * speed differs.  Fields:
 *   col_blocks  MFMA 16-column blocks per wave for the 16-bit forms: 8 or 16
 *               (the FP32 form always uses 16).
 *   mode        0 auto (one persistent launch when there is more than one
 *               sub-bank), 1 one launch per sub-bank, 2 always persistent:
 *               a fixed grid pulls (sub-bank, 32-template tile, tile group)
 *               work items from a counter, heaviest sub-banks first.
 *   max_tiles   most tiles one workgroup sweeps from one LDS window: 1, 2,
 *               4, 8 or 16 (fewer when the cluster window is shorter).
 *   wg_per_cu   persistent grid size in workgroups per CU (0: all that fit).
 *   ols_block   RFD_OLS32 block size K: 0 chooses per sub-bank the K in
 *               {1024, 2048, 4096} of least (5 log2 K + 6) K / (K - T + 1)
 *               divided by the measured relative speed of that K (1.25,
 *               1, 0.97); 1024, 2048 or 4096 forces it wherever K > T.
 *   ols_aligned 1 (default): RFD_OLS32 may keep L = 256 nf outputs per block
 *               (nf = floor((K - T + 1) / 256)) instead of all K - T + 1,
 *               when that costs less per output: the discarded outputs
 *               are then never computed and interior blocks skip
 *               per-sample range tests; 0: always K - T + 1.
 * RFD_E_INVALID for values outside these sets.
 */
typedef struct rfd_fir_config {
  int32_t col_blocks;
  int32_t mode;
  int32_t max_tiles;
  int32_t wg_per_cu;
  int32_t ols_block;
  int32_t ols_aligned;
} rfd_fir_config;
int rfd_plan_set_fir_config(rfd_plan* plan, const rfd_fir_config* cfg);
int rfd_plan_get_fir_config(const rfd_plan* plan, rfd_fir_config* cfg);
/*
 * rfd_ols_shape - the overlap-save shape the plan's configuration gives T
 * taps: block size K and outputs kept per block L (host int32 each).
 */
int rfd_ols_shape(const rfd_plan* plan, int32_t taps, int32_t* block, int32_t* outputs);

/*
 * rfd_autotune_fir - pick the FIR configuration by measurement on the
 * current segment (the project's own autotuner).  Every candidate of
 * {col_blocks 8, 16} x {max_tiles 4, 8, 16} x {per-sub-bank launches,
 * persistent with all / one workgroup per CU} (FP32: col_blocks 16 only) is
 * run `reps` times on `taps` with HIP events; the fastest becomes the plan's
 * configuration.  Requires the same state as rfd_filter_bank (slots and
 * triggers of the tuning runs are discarded).
 *   out  host: best configuration, its FIR time (ms, minimum over reps), the
 *        time of the configuration in force before the call, candidates run.
 */
typedef struct rfd_tune_result {
  rfd_fir_config best;
  double best_ms;
  double before_ms;
  int32_t n_candidates;
} rfd_tune_result;
int rfd_autotune_fir(rfd_plan* plan, const rfd_taps* taps, int32_t precision, int64_t cluster_window, int32_t reps,
                     rfd_tune_result* out);

/*
 * Segment graph: the whole per-segment pass (segment transform, the
 * dechirp of every listed reference, slot clearing, FIR with epilogue,
 * trigger compaction, complex-SNR re-evaluation) captured once into a HIP
 * graph and replayed per segment.  The graph reads `data` (dev float64 [N])
 * and the reference templates at the addresses given here: refill those
 * buffers between replays.  Captured on a private stream; replayed on the
 * plan's stream.  Arguments as rfd_dechirp / rfd_filter_bank; h_refs is a
 * host array of n_refs device pointers (complex128 [N/2+1]) for the slots
 * ref_ids.  Plan, taps and every captured buffer must outlive the graph:
 * rfd_plan_destroy and rfd_taps_destroy return RFD_E_STATE (and free
 * nothing) while a graph or stream created on them still exists.
 * rfd_segment_graph_launch replays it; with n_out non-NULL it synchronises
 * and returns the trigger count (RFD_E_OVERFLOW as rfd_filter_bank).  Taps
 * re-made after capture are picked up (RFD_OLS32 rebuilds its tap spectra in
 * place first).  If a later call reallocated a buffer the graph points at
 * (a filter call with more windows, another FIR configuration), the launch
 * returns RFD_E_STATE without running: create the graph again.
 */
typedef struct rfd_graph rfd_graph;
int rfd_segment_graph_create(rfd_plan* plan, const rfd_taps* taps, int32_t precision, float threshold,
                             int64_t cluster_window, const double* data, int32_t n_refs, const int32_t* ref_ids,
                             const double* const* h_refs, rfd_trigger* out, int64_t capacity, rfd_graph** graph);
int rfd_segment_graph_launch(rfd_graph* graph, int64_t* n_out);
int rfd_graph_destroy(rfd_graph* graph);

/*
 * Low-latency increment as one graph (Sec. VII.A: only the newest stretch of
 * the segment is filtered): the same capture as rfd_segment_graph_create, but
 * the FIR, window peaks and triggers cover only outputs [n_start, n_start +
 * n_len), exactly as rfd_filter_range (same range rules: 256-sample aligned,
 * non-empty, inside the segment, else RFD_E_INVALID).  The segment transform
 * and the dechirps still cover the whole segment, and the range is fixed at
 * capture: every replay filters the same output samples of whatever the
 * captured buffers hold (refill `data` to advance the stream by one
 * segment).  An advancing stream with incremental reference series is
 * rfd_stream_*.  Replayed with rfd_segment_graph_launch, freed with
 * rfd_graph_destroy.
 */
int rfd_range_graph_create(rfd_plan* plan, const rfd_taps* taps, int32_t precision, float threshold,
                           int64_t cluster_window, const double* data, int32_t n_refs, const int32_t* ref_ids,
                           const double* const* h_refs, int64_t n_start, int64_t n_len, rfd_trigger* out,
                           int64_t capacity, rfd_graph** graph);

/*
 * Learned tap surrogate (an extension to the method; the paper does not
 * define it).  A small MLP (4 -> hidden -> hidden -> n_basis, SiLU, BF16
 * weights, FP32 accumulation) maps scaled template parameters to
 * coefficients on an orthonormal basis of whitened ratio taps of ONE
 * sub-bank.  Each exact tap set a (Sec. V.A) is first given one global
 * phase so that z = ((M + lam I) a)[-k0] -- the normal equations'
 * right-hand side at zero lag, the weighted zero-lag overlap of template and
 * reference -- is real and positive (|z| of Eq. 3 and every match ignore a
 * global tap phase), then whitened: x = [Re v; Im v]/||v||, v = L^H a, with
 * L the sub-bank's Cholesky factor of M + lam I, so ||x_hat - x||^2 is a
 * mismatch proxy of the fitted template.  The exact taps are the training
 * data, the fallback and the yardstick of the SNR loss (rfd_taps_match).
 *
 * rfd_surrogate_create     whitens the exact taps of every template of
 *                          `subbank` in `taps` (all made by the LS route;
 *                          RFD_E_STATE otherwise).  The surrogate keeps
 *                          pointers to plan and taps: both must outlive it.
 *                          n_basis in [1, min(2T, 1024)], hidden in
 *                          [1, 4096]; seed fixes initial weights, the basis
 *                          start and the shuffles.
 * rfd_surrogate_set_feature_range
 *                          the network's input range from the training
 *                          set's physical parameters phys (dev float64
 *                          [n][4]: m1, m2, chi, e0): min and max of each
 *                          feature (chirp mass M eta^(3/5), eta = m1 m2 /
 *                          M^2, chi, e0).  Synchronises.
 * rfd_surrogate_features   network inputs for phys (dev float64 [n][4]):
 *                          each feature mapped linearly onto [-1, 1] over
 *                          that range (a constant feature maps to -1), into
 *                          out (dev float [n][4]): the params of train and
 *                          make_taps.  RFD_E_STATE before the range is set.
 * rfd_surrogate_fit_basis  subspace iteration (iters in [1, 100]) for the
 *                          basis; *captured_out (host, may be NULL) = mean
 *                          ||B^T x||^2 over the training set (<= 1).
 * rfd_surrogate_train      Adam (beta 0.9/0.999, eps 1e-8) on mean
 *                          ||c_hat - c||^2 over whole batches of a seeded
 *                          shuffle; params: dev float [count][4] (count =
 *                          training templates, same order); batch in
 *                          [1, 1024]; repeated calls continue the same
 *                          optimiser state (a learning-rate schedule is a
 *                          sequence of calls); loss_out: host float
 *                          [epochs] (mean loss per epoch) or NULL.
 *                          Each step's batch index and Adam step count live
 *                          on the device, so an epoch is one fixed launch
 *                          sequence: by default it is captured once per call
 *                          and replayed as a HIP graph every epoch.
 * rfd_surrogate_train_many the same epochs for count (1..32) surrogates of
 *                          one plan with equal training-set size, hidden
 *                          width and n_basis, launched together: each step
 *                          is one launch sequence for all of them (the grid's
 *                          third index or second selects the network), so the
 *                          small per-network GEMMs fill the device.  Each
 *                          network's arithmetic and shuffle are those of
 *                          rfd_surrogate_train on it alone, so the results
 *                          are identical.  params[i]: dev float [n][4] of
 *                          surrogate i; loss_out: host float [count][epochs]
 *                          or NULL.  A surrogate may not appear twice.
 *                          rfd_surrogate_train is this call with count 1.
 * rfd_surrogate_set_graphs enable != 0 (default): graph replay of epochs;
 *                          0: every step launched directly.  Results are
 *                          identical either way.
 * rfd_surrogate_loss_grad  loss and gradients (dev float [n_params], order
 *                          W1, b1, W2, b2, W3, b3; W row-major [out][in])
 *                          for the first n (<= 1024) rows of params;
 *                          targets dev [n][n_basis] or NULL for the
 *                          training targets.  The forward pass uses the
 *                          BF16-rounded weights, as training does.
 * rfd_surrogate_get_state  host copies of weights / basis [n_basis][2T] /
 *                          targets [count][n_basis] (each may be NULL);
 *                          sizes (host int64[6], may be NULL): n_params,
 *                          basis, targets, 2T, n_basis, hidden.
 * rfd_surrogate_set_state  replace weights and/or basis (host arrays, same
 *                          layouts; either may be NULL, not both); new
 *                          weights restart Adam (moments and step zeroed),
 *                          a new basis recomputes the training targets.
 * rfd_surrogate_make_taps  taps for templates first..first+count-1 of a
 *                          sub-bank of `target` with the same reference, T
 *                          and k0, from params dev float [count][4]:
 *                          c_hat, then a = L^-H (B^T c_hat) through the
 *                          folded FP64 matrix L^-H B (made when the basis
 *                          is fitted or set), then sigma_fit and packing as
 *                          rfd_make_taps.  Marks the templates made.
 *                          Training and inference before a basis exists
 *                          give RFD_E_STATE.
 * rfd_taps_match           dev double [count]: |a^H M b| / sqrt(a^H M a
 *                          b^H M b) between the FP64 taps of two objects of
 *                          one plan (same sub-bank index, T and size); M
 *                          from `a`'s sub-bank.
 * rfd_taps_fallback        copies the exact taps of `exact` into `target`
 *                          for every template of the range whose match
 *                          (dev double [count], e.g. from rfd_taps_match)
 *                          is below min_match or NaN, and re-normalises
 *                          and packs them; *n_fallback_out (host, may be
 *                          NULL) = templates replaced.  RFD_E_STATE if a
 *                          replaced template has no exact taps.
 * rfd_surrogate_destroy    frees the surrogate (NULL is a no-op).
 * All calls enqueue on the plan's stream and return after it drained,
 * except rfd_taps_match, which only enqueues.
 */
typedef struct rfd_surrogate rfd_surrogate;
int rfd_surrogate_create(rfd_plan* plan, rfd_taps* taps, int32_t subbank, int32_t n_basis, int32_t hidden,
                         uint64_t seed, rfd_surrogate** out);
int rfd_surrogate_fit_basis(rfd_surrogate* sur, int32_t iters, double* captured_out);
int rfd_surrogate_train(rfd_surrogate* sur, const float* params, int32_t epochs, int32_t batch, float lr,
                        float* loss_out);
int rfd_surrogate_train_many(rfd_surrogate* const* surs, const float* const* params, int32_t count, int32_t epochs,
                             int32_t batch, float lr, float* loss_out);
int rfd_surrogate_set_graphs(rfd_surrogate* sur, int32_t enable);
int rfd_surrogate_set_feature_range(rfd_surrogate* sur, const double* phys, int64_t n);
int rfd_surrogate_features(rfd_surrogate* sur, const double* phys, int64_t n, float* out);
int rfd_surrogate_loss_grad(rfd_surrogate* sur, const float* params, const float* targets, int32_t n, float* grads,
                            double* loss_out);
int rfd_surrogate_get_state(rfd_surrogate* sur, float* weights, float* basis, float* targets, int64_t* sizes);
int rfd_surrogate_set_state(rfd_surrogate* sur, const float* weights, const float* basis);
int rfd_surrogate_make_taps(rfd_surrogate* sur, const float* params, rfd_taps* target, int32_t subbank,
                            int64_t first, int64_t count);
int rfd_taps_match(const rfd_taps* a, const rfd_taps* b, int32_t subbank, int64_t first, int64_t count,
                   double* match_out);
int rfd_taps_fallback(rfd_taps* target, const rfd_taps* exact, int32_t subbank, int64_t first, int64_t count,
                      const double* match, double min_match, int64_t* n_fallback_out);
int rfd_surrogate_destroy(rfd_surrogate* sur);

/*
 * Ratio-filtered chi^2 signal-consistency test (Sec. VI.C): the time-frequency
 * chi^2 with each target's band SNRs taken from its reference's band SNR
 * series through the target's own taps.
 *
 * Bands: n_bands (2..64) contiguous bin ranges of the analysis band holding
 * equal reference power u_i = w_i |h_ref,i|^2: edge 0 = first band bin, edge
 * b = the first bin at which the sequential FP64 prefix sum of u (from the
 * first band bin) reaches (total * b) / n_bands, edge n_bands = last band bin
 * + 1.  RFD_E_INVALID if a band would be empty.
 *
 * rfd_dechirp_bands        after rfd_dechirp of slot ref_id on the current
 *                          segment (same h_ref): stores the slot's n_bands
 *                          band series zhat_b (FP32, normalised by
 *                          sigma_ref; they sum to the slot's series).
 *                          edges_out: host int64 [n_bands + 1] or NULL.
 * rfd_taps_band_fractions  for every template of `subbank` (taps made, any
 *                          route): shares f_b = a^H M_b a / sum_b a^H M_b a,
 *                          M_b the Toeplitz Gram of the band-restricted
 *                          reference power (FP64, stored FP32), with the
 *                          bands of h_ref (the sub-bank's reference).
 * rfd_taps_get_band_fractions  host float [n_bands] shares of one template.
 * rfd_chisq                chi^2 = sum_b |z_b - f_b z|^2 / f_b at each of n
 *                          triggers (device rfd_trigger [n], e.g. from
 *                          rfd_filter_bank), z_b = the FIR of zhat_b at the
 *                          trigger sample (FP32), z = sum_b z_b; chisq_out:
 *                          device float [n].  Mean 2 (n_bands - 1) in
 *                          Gaussian noise.  Every sub-bank needs shares and
 *                          its slot's band series on this segment with the
 *                          same edges (RFD_E_STATE otherwise); a trigger
 *                          naming no template of the bank gives NaN.
 */
int rfd_dechirp_bands(rfd_plan* plan, const double* h_ref, int32_t ref_id, int32_t n_bands, int64_t* edges_out);
int rfd_taps_band_fractions(rfd_plan* plan, rfd_taps* taps, int32_t subbank, const double* h_ref, int32_t n_bands);
int rfd_taps_get_band_fractions(const rfd_taps* taps, int64_t tmpl, float* f_out, int32_t* n_bands_out);
int rfd_chisq(rfd_plan* plan, const rfd_taps* taps, const rfd_trigger* triggers, int64_t n, float* chisq_out);

/*
 * rfd_select_taps - dynamic tap count (Sec. V.A tunes each template's number
 * of taps to a target match with the target template).  For each of `count`
 * templates (device complex128 [count][N/2+1], reference h_ref likewise):
 * the first T of the strictly ascending host `ladder` (n_ladder in [1, 64],
 * entries in [1, 2048]) whose least-squares taps with lags centred
 * (k0 = -floor(T/2), ridge ridge_eps) reach `target` in the match
 * |(h_j|h_fit)(0)| / (sigma_j sigma_fit) = |a^H b| / (sigma_j sigma_fit)
 * (the fitted template's phase-maximised overlap with the target at zero
 * lag), else the last T.  taps_out: host int32 [count]; match_out: host
 * double [count] (the match at the chosen T) or NULL.  Every ladder entry
 * builds the taps of all templates (n_ladder times the work of
 * rfd_make_taps); templates are then grouped by T into sub-banks.
 * flags: 0, or RFD_TAPS_CENTRE to centre each template's lags on its own
 * correlation peak (k0_j = l_peak - floor(T/2)) instead of on lag 0.
 * k0_out: host int32 [count] (the k0 at the chosen T) or NULL.
 */
int rfd_select_taps(rfd_plan* plan, const double* h_ref, const double* h_tmpl, int64_t count, double target,
                    const int32_t* ladder, int32_t n_ladder, double ridge_eps, int32_t flags, int32_t* taps_out,
                    double* match_out, int32_t* k0_out);

/*
 * PSD drift (Sec. VI.B): the template norm must follow the detector PSD.
 * rfd_plan_set_psd      replaces the plan's PSD weights w_i = 4 df / S_n(f_i)
 *                       (host psd [N/2+1], finite and > 0 in band); every
 *                       reference slot becomes stale (dechirp again).
 * rfd_taps_renormalize  recomputes a sub-bank's reference autocorrelation
 *                       g[m] under the current weights and, for every
 *                       template, sigma_fit^2 = a^H M a and the normalised
 *                       taps, leaving the taps a (designed under the old
 *                       PSD) unchanged: O(T^2) per template instead of a
 *                       full-band integral.  h_ref: the sub-bank's
 *                       reference (device complex128 [N/2+1]).  A cached
 *                       Cholesky factor is dropped (the next least-squares
 *                       rfd_make_taps refactors).
 */
int rfd_plan_set_psd(rfd_plan* plan, const double* psd, int64_t n_psd);
int rfd_taps_renormalize(rfd_plan* plan, rfd_taps* taps, int32_t subbank, const double* h_ref);

/*
 * rfd_filter_range - low-latency filtering (Sec. VII.A): the ratio FIR needs
 * only the reference series around the new samples (T - 1 of settling), so
 * a stream advancing by a few seconds filters just those samples.  As
 * rfd_filter_bank, restricted to output samples [n_start, n_start + n_len)
 * (both multiples of 256, inside the segment): windows keep their absolute
 * positions [qW, (q+1)W) and a window cut by the range reports the peak of
 * its part inside it.  Direct forms run one launch per sub-bank over the
 * range; RFD_OLS32 transforms and filters only the blocks that meet it.
 */
int rfd_filter_range(rfd_plan* plan, const rfd_taps* taps, int32_t precision, float threshold, int64_t cluster_window,
                     int64_t n_start, int64_t n_len, rfd_trigger* out, int64_t capacity, int64_t* n_out);

/* Thread-local description of the last error on this thread ("" if none). */
/*
 * Streaming (Sec. VII.A): the next stretch of SNR from the newest data.
 * The ratio FIR is short, so a new stretch of D samples needs the reference
 * series only over those samples plus the taps' span; the references (few,
 * Sec. IV) are still matched-filtered against the whole window.  The stream
 * keeps the last N data samples in a ring indexed by absolute sample number
 * mod N (trigger samples are such ring positions).  Each push:
 *   - writes D samples, transforms the ring once;
 *   - evaluates every reference series on the last zlen ring positions only
 *     (the correlation sum of Eq. 1 at those lags) into the plan's FP32
 *     series store (a 16-bit form splits its planes from it);
 *   - runs the ratio FIR of every template, with the fused epilogue, over the
 *     D outputs [head - D - lag, head - lag) mod N, lag = the taps' lead
 *     max(k0 + T) rounded up to 256, so every FIR input lies in the freshly
 *     evaluated stretch: zlen = D + lag + max(-k0), rounded up to 256.
 * A window [qW, (q+1)W) cut by the output range reports the peak of its part
 * inside (as rfd_filter_range).  After a push the series store is valid on
 * the last zlen positions only: rfd_filter_bank refuses (RFD_E_STATE) until
 * the references are dechirped again.
 *
 * rfd_stream_create - a stream over a plan and its taps.
 *   n_refs, ref_ids  host int32 [n_refs]: the reference slots the taps' sub-banks
 *                    use (every sub-bank's ref_id must be among them).
 *   h_refs           host array of n_refs dev pointers to complex128 [N/2+1]
 *                    reference spectra; copied into stream-owned memory.
 *   increment        D: a multiple of 256, at most N/4, and with the taps'
 *                    span zlen <= N/2.
 *   Allocates the ring (N float64), reference copies (n_refs (N/2+1) complex128),
 *   lag sums and their work buffer.  The plan and taps must outlive it.
 * rfd_stream_prime - fills the ring with a first window (dev float64 [N],
 *   ring positions 0..N-1, head = 0) and dechirps every stream reference on it.
 * rfd_stream_push - data: dev float64 [D], the samples at ring positions
 *   [head, head + D).  Remaining arguments as rfd_filter_bank; *out_start
 *   (host, may be NULL) receives the first output position.  Synchronises.
 * rfd_stream_info - head (next write position), lag, zlen.
 * Errors: RFD_E_INVALID, RFD_E_STATE (push before prime, taps not made),
 * RFD_E_NOMEM, RFD_E_OVERFLOW, RFD_E_DEVICE.
 */
typedef struct rfd_stream rfd_stream;
int rfd_stream_create(rfd_plan* plan, const rfd_taps* taps, int32_t n_refs, const int32_t* ref_ids,
                      const double* const* h_refs, int64_t increment, rfd_stream** out);
int rfd_stream_prime(rfd_stream* stream, const double* data);
int rfd_stream_push(rfd_stream* stream, const double* data, int32_t precision, float threshold,
                    int64_t cluster_window, rfd_trigger* out, int64_t capacity, int64_t* n_out,
                    int64_t* out_start);
int rfd_stream_info(const rfd_stream* stream, int64_t* head, int64_t* lag, int64_t* zlen);
int rfd_stream_destroy(rfd_stream* stream);

/*
 * rfd_measure_peaks - this GPU's ceilings measured by the library's own
 * microbenchmarks (a diagnostic beside the datasheet peaks that rooflines
 * are priced against; not part of the method):
 *   out[0] FP32 FMA issue, TFLOP/s (dependent chains, packed FP32 off as in
 *          every kernel here);  out[1] FP64 FMA, TFLOP/s;
 *   out[2] BF16 MFMA 16x16x32 with FP32 accumulation, TFLOP/s;
 *   out[3] device-to-device copy of 1 GiB, GB/s of read + write.
 *   stream  hipStream_t (NULL: the null stream); out host double [4].
 * Allocates 2 GiB + a small buffer for the duration of the call and
 * synchronises.  Errors: RFD_E_INVALID (NULL out), RFD_E_NOMEM, RFD_E_DEVICE.
 */
int rfd_measure_peaks(void* stream, double* out);

const char* rfd_last_error(void);

/*
 * rfd_debug_fail_allocation - failure injection for tests of the library's
 * out-of-memory paths: after `after` further successful device allocations
 * (process-wide, any plan), the next one fails once as if the device were
 * out of memory (the call reports RFD_E_NOMEM and releases what it had
 * allocated).  after < 0 disables it.  Not for production use.
 */
int rfd_debug_fail_allocation(int64_t after);

#ifdef __cplusplus
}
#endif
#endif /* RFD_H */
