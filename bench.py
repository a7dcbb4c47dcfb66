#!/usr/bin/env python
"""Throughput of the ratio-filter dechirping hot path on one MI355X.

Default workload ecc512s (the eccentric / subsolar search): one 512 s segment
(N = 2^20 samples at 2048 Hz, f_low = 15 Hz) of coloured Gaussian noise with
one SNR-12 injection; 16384 eccentric TaylorF2 templates (m1, m2 in
[0.2, 1.0] Msun, e0 in [0, 0.3] at 10 Hz) under 32 references (512
templates each); 1024 complex taps per template, each template's lags
centred on its own correlation peak (--no-lag-centre: on lag 0); threshold
rho > 6; 1 s cluster windows.

One step = one pass of the per-segment hot path with all inputs resident in
HBM: segment transform, dechirp of every reference, ratio FIR with the fused
|z|^2 / threshold / window-peak epilogue for every template, trigger
compaction, replayed as one captured graph.  The timed FIR form is the
faster of the workload's MFMA form (BF16 hi/lo split) and the overlap-save
FFT form, measured on this segment first (`--fir-form` forces one); the
plain FP32 direct FIR, both 16-bit split forms and FINDCHIRP (one full-length
FFT per template) run on the same segment and GPU beside it.  Taps are built
once before timing (the paper precomputes them with the bank); their
construction is timed separately.  The bank's waveforms are generated in
device memory (synth.device); the oracle legs use host waveforms.

The FP64 CPU oracle runs first, before the GPU is touched: a seeded sample of
templates (the injected one included) through its dechirp and direct-sum FIR
on every host core available to the process (worker processes, at most 16) and on one
core; its series are the parity reference for every FIR form, its matches
the tap-fidelity distribution.

Other workloads (--workload): spin256s (one reference, 4096 aligned-spin
templates, T = 256), tidal256s (64 uneven sub-banks, T 32..1024) and
surr512s (the learned tap surrogate end to end: 65536 templates whose taps
come from 32 trained networks, validated, with exact-tap fallback).

Prints one JSON line.  `--gpus` above 1 exits: the benchmark runs on one GPU.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"bf16x3": 2500.0, "fp16x3": 2500.0, "fp32": 157.3,   # dense MFMA TFLOP/s, MI355X datasheet
        "ols32": 157.3}                                          # FP32 vector TFLOP/s
TARGET = {"bf16x3": 1e-3, "fp16x3": 1e-3, "fp32": 1e-5, "ols32": 1e-5}   # stated max |drho|
# committed rocprofv3 counter summaries (HBM bytes per launch of the dominant kernel)
COUNTERS = {("ecc512s", "ols32"): "k_ols4096_ecc512s_counters.txt",
            ("spin256s", "ols32"): "fir_ols32_spin256s_counters.txt",
            ("spin256s", "bf16x3"): "fir_bf16x3_spin256s_counters.txt"}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def read_traffic(name):
    """HBM bytes per launch from a committed rocprofv3 counter summary, if present."""
    if not name:
        return None
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    for line in open(path):
        if line.startswith("traffic_bytes_per_launch:"):
            try:
                return float(line.split(":", 1)[1])
            except ValueError:
                return None
    return None


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_workers():
    """Worker processes for the all-core oracle leg: the CPUs this process may
    run on, at most 16 (the host share of one GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _oracle_fir_task(task):
    """One template through the oracle's direct-sum FIR (Eq. 3), normalised
    by its fitted norm: |z_j[n]| for every sample.  Runs in a worker process."""
    z_ref, a, k0, sigma_fit = task
    import numpy as np
    from oracle import fir as ofir
    return np.abs(ofir.fir_direct(z_ref, np.conj(a), k0)) / sigma_fit


def _oracle_match_task(task):
    """Tap fidelity (time-maximised match of the fitted template, Sec. VI.B
    norms) of one template.  Runs in a worker process."""
    psd, fs, f_low, h_j, h_ref, a, k0, sigma_fit = task
    import numpy as np
    from oracle import spectral as osp
    from oracle import taps as otaps
    n = 2 * (h_j.size - 1)
    w = osp.psd_weights(psd, n, fs, f_low)
    A = otaps.response_fft(a, k0, n)
    h_fit = h_ref * A
    z = osp.matched_filter(h_j, h_fit, w)
    return float(np.max(np.abs(z)) / np.sqrt(osp.sigma_sq(h_j, w) * osp.sigma_sq(h_fit, w)))


def oracle_leg(args, w, bank, psd, seg, hrefs, np, synth):
    """The FP64 oracle on a seeded template sample, before the GPU is touched.

    Taps (outside the timing), then the timed legs: dechirp of the sample's
    references and direct-sum FIR of every sampled template over the whole
    segment on all granted cores (one worker process per template), and the
    same for the first `--cpu-one-core` templates on one core.  Returns the
    oracle's rho series of the sample, its matches and the CPU baseline."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    from oracle import pipeline as orc
    from oracle import taps as otaps
    nt = bank.n_templates
    rng = np.random.default_rng(2601)
    pick = [seg.inj_template] + list(rng.choice(nt, size=max(0, args.cpu_sample - 1), replace=False))
    sample = sorted(set(int(j) for j in pick))
    sbi = [bank.subbank_of(j) for j in sample]
    t0 = time.perf_counter()
    Hs = synth.template_batch(w, [bank.params(j) for j in sample])
    p = orc.prepare(psd, seg.data, w.fs, w.f_low)
    grams = {b: otaps.gram(hrefs[b], p.w, bank.subbanks[b].taps) for b in sorted(set(sbi))}
    T_of = [bank.subbanks[b].taps for b in sbi]
    k0s = [otaps.centred_k0(Hs[i], hrefs[sbi[i]], p.w, T_of[i]) if not args.no_lag_centre
           else bank.subbanks[sbi[i]].k0 for i in range(len(sample))]
    tts = [orc.make_taps(p, Hs[i], hrefs[sbi[i]], T_of[i], k0s[i], M=grams[sbi[i]]) for i in range(len(sample))]
    shifts = np.array([k0s[i] - bank.subbanks[sbi[i]].k0 for i in range(len(sample))])
    log(f"oracle: taps of {len(sample)} sampled templates in {time.perf_counter() - t0:.1f} s (not timed)")
    nw = host_workers()
    ctx = mp.get_context("spawn")
    with ProcessPoolExecutor(max_workers=nw, mp_context=ctx) as ex:
        list(ex.map(abs, range(nw)))                  # start the workers outside the timing
        # all cores: dechirp of the sample's references here, FIR per template in the workers
        c0, w0 = time.process_time(), time.perf_counter()
        p2 = orc.prepare(psd, seg.data, w.fs, w.f_low)
        refs = {b: orc.dechirp(p2, hrefs[b]) for b in sorted(set(sbi))}
        tasks = [(refs[sbi[i]].z, tts[i].a, tts[i].k0, tts[i].sigma_fit) for i in range(len(sample))]
        rho = list(ex.map(_oracle_fir_task, tasks))
        wall_all = time.perf_counter() - w0
        log(f"oracle: {len(sample)} templates x {w.n} samples on {nw} worker processes in {wall_all:.1f} s")
        # fidelity of the sample (not timed)
        mtasks = [(psd, w.fs, w.f_low, Hs[i], hrefs[sbi[i]], tts[i].a, tts[i].k0, tts[i].sigma_fit)
                  for i in range(len(sample))]
        match = np.array(list(ex.map(_oracle_match_task, mtasks)))
    # one core: the first templates of the sample, in this process
    n1 = max(1, min(args.cpu_one_core, len(sample)))
    c1, w1 = time.process_time(), time.perf_counter()
    p3 = orc.prepare(psd, seg.data, w.fs, w.f_low)
    refs1 = {b: orc.dechirp(p3, hrefs[b]) for b in sorted(set(sbi[:n1]))}
    for i in range(n1):
        np.abs(orc.ratio_snr(refs1[sbi[i]], tts[i]))
    wall_one = time.perf_counter() - w1
    cpu_one = time.process_time() - c1
    log(f"oracle: {n1} templates on one core in {wall_one:.1f} s")
    taps_desc = sorted(set(bank.subbanks[b].taps for b in sbi))
    cpu = {"value": len(sample) * w.n / wall_all, "unit": "template*samples/s", "cores": nw, "kind": "oracle",
           "sample": f"{len(sample)} of {nt} templates (seeded, incl. the injected one), each over the full "
                     f"{w.n}-sample segment: FP64 dechirp of their {len(refs)} reference(s) in the parent, then the "
                     f"direct-sum FIR ({taps_desc} taps) of one template per task on {nw} worker processes; "
                     f"taps built outside the timing",
           "seconds": round(wall_all, 2),
           "one_core": {"value": n1 * w.n / wall_one, "cores": max(1, int(round(cpu_one / wall_one))),
                        "templates": n1, "seconds": round(wall_one, 2)},
           "host": {"nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)), "cpu_model": cpu_model()}}
    return dict(sample=sample, sbi=sbi, Hs=Hs, tts=tts, refs=refs, rho=np.array(rho), match=match,
                shifts=shifts, centre=not args.no_lag_centre), cpu


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="ecc512s", choices=["ecc512s", "spin256s", "tidal256s", "surr512s"])
    ap.add_argument("--subbanks", default="all", help="surr512s: references given a surrogate ('all' or a list)")
    ap.add_argument("--train", type=int, default=3125, help="surr512s: exact tap sets per reference (1e5 in all)")
    ap.add_argument("--epochs", type=int, default=36000, help="surr512s: training epochs")
    ap.add_argument("--batch", type=int, default=256, help="surr512s: training batch")
    ap.add_argument("--lr", type=float, default=4e-3, help="surr512s: first learning rate")
    ap.add_argument("--lr-end", type=float, default=5e-5, help="surr512s: last learning rate (geometric decay)")
    ap.add_argument("--cpu-sample", type=int, default=32, help="templates in the oracle sample (parity, all cores)")
    ap.add_argument("--cpu-one-core", type=int, default=3, help="templates of the sample timed on one core")
    ap.add_argument("--fir-form", default="auto", choices=["auto", "fp32", "bf16x3", "fp16x3", "ols32"],
                    help="FIR form of the timed run; auto: the faster of the workload's MFMA form and the "
                         "overlap-save form, measured on this segment")
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the oracle legs (no parity block)")
    ap.add_argument("--no-compare", action="store_true", help="skip the FP32 / FP16 / FINDCHIRP comparison legs")
    ap.add_argument("--no-low-latency", action="store_true")
    ap.add_argument("--no-lag-centre", action="store_true",
                    help="lags centred on 0 for every template (default: each template's lags centred on the peak "
                         "of its correlation with the reference)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 1 GiB read + 1 GiB write elementwise kernel (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this benchmark runs on one GPU only (no multi-GPU path); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np

    import synth
    if args.workload == "surr512s":
        return surrogate_main(args)
    w = synth.get_workload(args.workload)
    bank = synth.make_bank(w)
    psd = synth.psd_array(w.n, w.fs)
    seg = synth.make_segment(w, bank)
    hrefs = [synth.reference_waveform(w, sb) for sb in bank.subbanks]
    orc_out = cpu = None
    if not args.no_cpu_baseline:
        orc_out, cpu = oracle_leg(args, w, bank, psd, seg, hrefs, np, synth)

    import torch

    from paper_2601_18835_amd import rfd
    from paper_2601_18835_amd.driver import RatioFilterSearch, SubBankSpec
    from synth.device import template_batch_device

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    nt = bank.n_templates
    nsb = len(bank.subbanks)
    prec = w.precision
    multi = nsb > 1
    with_fc = args.workload in ("spin256s", "ecc512s") and not args.no_compare
    log(f"workload {w.name}: N={w.n} templates={nt} sub-banks={nsb} precision={prec}")

    specs = [SubBankSpec(b, sb.taps, sb.k0, sb.size) for b, sb in enumerate(bank.subbanks)]
    s = RatioFilterSearch(psd, w.f_low, w.fs, w.n, specs, max_refs=nsb)
    for b in range(nsb):
        s.set_reference(b, hrefs[b])
    info = s.info
    filt = fsig = None
    if with_fc:
        filt = torch.empty((nt, info["n_band"]), dtype=torch.complex64, device="cuda")
        fsig = torch.empty(nt, dtype=torch.float64, device="cuda")
    rfd.rfd_plan_set_timing(s.plan, True)
    taps_method = rfd.RFD_TAPS_LS | (0 if args.no_lag_centre else rfd.RFD_TAPS_CENTRE)
    batch = 256
    t_gen = 0.0
    Hd = None
    for b, sb in enumerate(bank.subbanks):
        g0 = int(bank.offsets[b])
        for b0 in range(0, sb.size, batch):
            ps = sb.params[b0:b0 + batch]
            tg = time.perf_counter()
            Hd = template_batch_device(w, ps, "cuda", out=Hd if Hd is not None and Hd.shape[0] == len(ps) else None)
            torch.cuda.synchronize()
            t_gen += time.perf_counter() - tg
            s.make_taps(b, Hd, first=b0, method=taps_method)
            if with_fc:
                k = len(ps)
                rfd.rfd_findchirp_prepare(s.plan, Hd, filt[g0 + b0:g0 + b0 + k], fsig[g0 + b0:g0 + b0 + k])
    del Hd
    torch.cuda.synchronize()
    tap_timing = rfd.rfd_plan_get_timing(s.plan)
    taps_per_s = nt / (tap_timing["taps_ms"] / 1e3)
    log(f"tap construction on GPU: {tap_timing['taps_ms']:.1f} ms for {nt} templates ({taps_per_s:.3g} taps/s); "
        f"waveform generation (device) {t_gen:.1f} s")

    data = torch.from_numpy(seg.data).to("cuda")
    s.set_segment(data)
    cap = 1 << 21
    out = torch.empty(cap * 32, dtype=torch.uint8, device="cuda")
    ts = nt * w.n
    flops_alg = 8.0 * w.n * sum(sb.size * sb.taps for sb in bank.subbanks)   # 8T flop per template*sample

    def eager_step(precision):
        rfd.rfd_dechirp_refs(s.plan, data, s.h_ref, False)     # transform + every reference, batched
        return rfd.rfd_filter_bank(s.plan, s.taps, precision, w.threshold, w.window, cap, out)[1]

    def timed(fn, steps, warmup):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        rfd.rfd_plan_get_timing(s.plan)          # discard warm-up marks
        t0 = time.perf_counter()
        for _ in range(steps):
            n = fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t0, n, rfd.rfd_plan_get_timing(s.plan)

    def ols_block(T):
        eff = {1024: 1.17, 2048: 1.0, 4096: 0.99}     # the library's block-size rule
        cands = [K for K in (1024, 2048, 4096) if K > T]
        return min(cands, key=lambda K: ((5 * np.log2(K) + 6) * K / (K - T + 1) / eff[K], K))

    def ols_flops_per_launch():
        """(5 log2 K + 6) K per (template, block) over one sub-bank's launch, averaged over the launches."""
        tot = []
        for sb in bank.subbanks:
            K = ols_block(sb.taps)
            nB = -(-w.n // (K - sb.taps + 1))
            tot.append(sb.size * nB * K * (5.0 * np.log2(K) + 6.0))
        return float(np.mean(tot)), float(np.sum(tot)), sorted(set(ols_block(sb.taps) for sb in bank.subbanks))

    selection = None
    if args.fir_form == "auto":
        s.dechirp_all()
        selection = {}
        for form in (prec, "ols32"):
            d, _, _ = timed(lambda: eager_step(form), 3, 1)
            selection[form] = d / 3 * 1e3
        mfma_form = prec
        prec = min(selection, key=selection.get)
        log(f"FIR form by measurement: {selection} -> {prec}")
    else:
        mfma_form = prec
        prec = args.fir_form

    tune = None
    if multi and prec != "ols32":
        s.dechirp_all()
        tune = rfd.rfd_autotune_fir(s.plan, s.taps, prec, w.window, reps=1)
        log(f"autotuner: {tune}")
    # the timed step replays the segment graph (transform, dechirps, FIR, compaction); the
    # per-stage times and the FIR kernel time for the roofline come from eager steps of the
    # same configuration, timed on the plan's stream with HIP events
    graph = rfd.rfd_segment_graph_create(s.plan, s.taps, prec, w.threshold, w.window, data, s.h_ref, out, cap)
    step = lambda: rfd.rfd_segment_graph_launch(graph)   # noqa: E731

    log(f"timing {args.steps} steps ({args.warmup} warm-up), {prec} (segment graph)")
    dt, ntrig, tim = timed(step, args.steps, args.warmup)
    ms_step = dt / args.steps * 1e3
    value = ts * args.steps / dt
    trig_main = rfd.triggers_to_numpy(out, min(ntrig, cap))
    ne = max(5, args.steps // 2)
    _, _, tfir = timed(lambda: eager_step(prec), ne, 2)
    n_launch = max(1, tfir["n_fir_kernel"])
    kernel_ms = tfir["fir_kernel_ms"] / n_launch
    stages = {k: tfir[k] / ne for k in ("data_fft_ms", "dechirp_ms", "fir_ms", "compact_ms", "fir_kernel_ms")
              if k in tfir}
    log(f"{prec}: {ms_step:.3f} ms/step, {value:.4g} t*s/s, FIR stage {stages['fir_ms']:.3f} ms, "
        f"{n_launch // ne} main FIR launches of {kernel_ms:.3f} ms, {ntrig} triggers")
    peak = PEAK[prec]
    if prec == "ols32":
        # the overlap-save algorithm's own work: per (template, block) a K-point
        # product and inverse FFT, (5 log2 K + 6) K flop
        fl, fl_step, ks = ols_flops_per_launch()
        achieved = fl / (kernel_ms * 1e-3) / 1e12
        roofline = {"bound": "alu", "achieved": round(achieved, 2), "peak": peak, "unit": "TFLOP/s",
                    "frac": round(achieved / peak, 4), "traffic": read_traffic(COUNTERS.get((w.name, prec))),
                    "kernel": "k_ols<" + ",".join(str(k) for k in ks) + ">", "flops_per_launch": fl,
                    "avg_launch_ms": round(kernel_ms, 4), "launches_per_step": n_launch // ne,
                    "direct_form_equivalent_TFLOPs": round(flops_alg / (stages["fir_ms"] * 1e-3) / 1e12, 2)}
    else:
        per_launch = flops_alg / (n_launch / ne)
        achieved = per_launch / (kernel_ms * 1e-3) / 1e12
        roofline = {"bound": "mfma", "achieved": round(achieved, 2), "peak": peak, "unit": "TFLOP/s",
                    "frac": round(achieved / peak, 4),
                    "traffic": read_traffic(COUNTERS.get((w.name, prec))),
                    "kernel": (f"k_fir16<{prec[:4]}>" if prec != "fp32" else "k_fir32") +
                              ("_persistent" if multi else ""),
                    "issued_frac": round(3 * achieved / peak, 4) if prec != "fp32" else round(achieved / peak, 4),
                    "flops_per_launch": per_launch, "avg_launch_ms": round(kernel_ms, 4),
                    "launches_per_step": n_launch // ne}

    compare = {}
    if not args.no_compare:
        k2 = max(3, args.steps // 4)
        others = [f for f in ("fp32", "bf16x3", "fp16x3", "ols32") if f != prec]
        for other in others:
            d2, n2, t2 = timed(lambda: eager_step(other), k2, 1)
            km = t2["fir_kernel_ms"] / max(1, t2["n_fir_kernel"])
            leg = {"value": ts * k2 / d2, "ms_per_step": d2 / k2 * 1e3,
                   "fir_stage_ms": t2["fir_ms"] / k2, "triggers": n2}
            if other in ("bf16x3", "fp16x3", "fp32"):
                # MFMA fraction of the direct form: 8T flop per template*sample (algorithmic;
                # the 16-bit split forms issue three MFMA terms per product)
                alg = flops_alg / (t2["fir_ms"] / k2 * 1e-3) / 1e12
                leg["mfma"] = {"achieved_TFLOPs": round(alg, 2), "peak": PEAK[other],
                               "frac": round(alg / PEAK[other], 4),
                               "issued_frac": round((3 if other != "fp32" else 1) * alg / PEAK[other], 4)}
            compare[f"fir_{other}"] = leg
            log(f"{other}: {d2 / k2 * 1e3:.3f} ms/step")
        if with_fc:
            d3, nfc, t3 = timed(lambda: rfd.findchirp_filter(s.plan, data, filt, w.threshold, w.window, cap, out)[1],
                                k2, 1)
            trig_fc = rfd.triggers_to_numpy(out, min(nfc, cap))
            fc_ms = t3["findchirp_ms"] / k2
            # HBM bytes of the two-pass transform per template: the filter over the
            # band (8 B per bin), then the [N2][N1] intermediate written and read back
            fc_bytes = nt * (info["n_band"] * 8 + 2 * w.n * 8)
            compare["findchirp_fp32"] = {"value": ts * k2 / d3, "ms_per_step": d3 / k2 * 1e3, "fft_ms": fc_ms,
                                         "triggers": nfc,
                                         "filter_stream_GBs": nt * info["n_band"] * 8 / (fc_ms * 1e-3) / 1e9,
                                         "two_pass_GBs": fc_bytes / (fc_ms * 1e-3) / 1e9,
                                         "two_pass_frac_of_8TBs": fc_bytes / (fc_ms * 1e-3) / 8e12}
            log(f"findchirp: {d3 / k2 * 1e3:.3f} ms/step")

    # the injection: recovered rho of the injected template in its window
    injection = None
    if seg.inj_template >= 0:
        q = seg.inj_sample // w.window

        def at_inj(tr):
            m = (tr["tmpl"] == seg.inj_template) & (tr["sample"] // w.window == q)
            return ({"sample": int(tr["sample"][m][0]), "rho": float(tr["rho"][m][0])} if m.any() else None)

        injection = {"template": seg.inj_template, "sample": seg.inj_sample, "optimal_snr": w.injection_snr,
                     "ratio_filter": at_inj(trig_main)}
        if "findchirp_fp32" in compare:
            injection["findchirp"] = at_inj(trig_fc)
        log(f"injection: {injection}")

    low_latency = None
    if not args.no_low_latency:
        low_latency = low_latency_leg(args, w, s, data, out, cap, prec, timed, rfd)
    crossover = None
    if not args.no_compare:
        crossover = crossover_leg(w, bank, psd, seg, hrefs, mfma_form, np, rfd, torch, template_batch_device)

    parity = fidelity = None
    if orc_out is not None:
        parity = parity_leg(w, bank, psd, seg, hrefs, orc_out, trig_main, prec, np, rfd)
        m = orc_out["match"]
        inj_i = orc_out["sample"].index(seg.inj_template) if seg.inj_template in orc_out["sample"] else None
        fidelity = {"templates": len(m), "match_mean": float(m.mean()), "match_min": float(m.min()),
                    "match_p10": float(np.quantile(m, 0.1)), "match_median": float(np.median(m)),
                    "match_max": float(m.max()),
                    "injected_template_match": float(m[inj_i]) if inj_i is not None else None,
                    "note": "oracle: time-maximised match of each sampled template with its fitted template "
                            "(reported, not gated); 1 - match is the ratio filter's SNR loss"}
        if injection is not None and inj_i is not None:
            r = orc_out["rho"][inj_i]
            q = seg.inj_sample // w.window
            seg_r = r[q * w.window:(q + 1) * w.window]
            injection["oracle_ratio_filter"] = {"sample": int(q * w.window + np.argmax(seg_r)),
                                                "rho": float(seg_r.max())}

    if graph is not None:
        rfd.rfd_graph_destroy(graph)
    s.close()
    if args.calibrate_copy:
        # plain streaming kernel of known traffic: reads 1 GiB, writes 1 GiB
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        log("copy calibration: 3 x (read 1073741824 B, write 1073741824 B) in elementwise_kernel")
        del src, dst
    # this GPU's ceilings from the library's own microbenchmarks (context beside the published peaks)
    peaks = {k: round(v, 2) for k, v in rfd.rfd_measure_peaks().items()}
    log(f"measured ceilings: {peaks}")
    # (the BF16 MFMA loop does not stand for an FP32-operand contraction)
    roofline["measured_ceiling"] = None if prec == "fp32" else {
        "alu": peaks["fp32_fma_TFLOPs"], "mfma": peaks["bf16_mfma_TFLOPs"], "hbm": peaks["copy_GBs"]}[roofline["bound"]]
    line = {
        "metric": "template*samples/s at SNR err <=1e-3 vs FP32 ratio-FIR and FINDCHIRP, 1 GPU",
        "value": value, "unit": "template*samples/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f16" if prec == "fp16x3" else ("bf16" if prec == "bf16x3" else "f32"),
        "precision": {"bf16x3": "bf16 hi/lo split operands (3 MFMA terms), fp32 accumulation",
                      "fp16x3": "fp16 hi/lo split operands (3 MFMA terms), fp32 accumulation",
                      "fp32": "fp32 operands, fp32 accumulation",
                      "ols32": "overlap-save FFT blocks in fp32 (tap spectra from fp64 sums)"}[prec],
        "data": "synthetic",
        "config": {"workload": w.name, "segment_samples": w.n, "fs": w.fs, "f_low": w.f_low, "templates": nt,
                   "references": nsb, "taps": sorted(set(sb.taps for sb in bank.subbanks))
                   if multi else bank.subbanks[0].taps, "threshold": w.threshold, "cluster_window": w.window,
                   "fir_form": prec, "segment_graph": True, "lag_centring": not args.no_lag_centre},
        "fir_form_selection_ms": selection, "mfma_form": mfma_form,
        "stages_ms": stages, "triggers": ntrig,
        "tap_construction": {"templates_per_s": taps_per_s, "gpu_ms": tap_timing["taps_ms"]},
        "autotune": tune, "roofline": roofline, "compare": compare, "injection": injection,
        "low_latency": low_latency, "fir_crossover": crossover, "parity": parity, "fidelity": fidelity,
        "cpu_baseline": cpu,
        "measured_peaks": peaks,
        # the paper's own speed-ups (context, other hardware) beside this GPU's measured ratios
        "paper_context": {
            "filtering_loop_speedup_vs_fft_matched_filter": {
                "value": 8.0, "kind": "measured", "hardware": "one CPU core of a Haswell-class cluster node",
                "source": "abstract; Sec. VI.A"},
            "low_latency_speedup": {"value": ">10", "kind": "projected, not measured", "source": "abstract"},
            "this_gpu_ratio_filter_vs_findchirp": (
                round(compare["findchirp_fp32"]["ms_per_step"] / ms_step, 3) if "findchirp_fp32" in compare else None),
            "this_gpu_hardware": "one MI355X; both forms on the same segment and GPU",
        },
    }
    print(json.dumps(line), flush=True)


def stream_check(w, s, data, prec, rfd, vbuf, nv, vstart, inc, vcap):
    """Window peaks (threshold 0) of one stream push against those of the
    range filter over the same outputs after a full re-dechirp: the same
    windows, every rho finite, the largest |rho difference| over them."""
    import numpy as np
    a = rfd.triggers_to_numpy(vbuf, nv)
    rfd.rfd_dechirp_refs(s.plan, data, s.h_ref, False)
    rbuf, nr = rfd.rfd_filter_range(s.plan, s.taps, prec, 0.0, w.window, vstart, inc, vcap)
    b = rfd.triggers_to_numpy(rbuf, nr)
    ka = np.sort(a["tmpl"].astype(np.int64) * (1 << 32) + a["sample"] // w.window)
    kb = np.sort(b["tmpl"].astype(np.int64) * (1 << 32) + b["sample"] // w.window)
    same_windows = bool(nv == nr and np.array_equal(ka, kb))
    finite = bool(np.isfinite(a["rho"]).all())
    oa = np.lexsort((a["sample"], a["tmpl"]))
    ob = np.lexsort((b["sample"], b["tmpl"]))
    drho = float(np.max(np.abs(a["rho"][oa] - b["rho"][ob]))) if same_windows and nv else None
    res = {"windows": int(nv), "same_windows": same_windows, "finite": finite, "max_abs_drho": drho}
    log(f"stream check against the range filter: {res}")
    if not (finite and same_windows and drho is not None and drho <= 1e-3):
        raise SystemExit(f"stream outputs disagree with the range filter: {res}")
    return res


def low_latency_leg(args, w, s, data, out, cap, prec, timed, rfd):
    """Sec. VII.A: the next second of SNR from the newest data.  The stream
    (rfd_stream_*) keeps the last N samples in a ring; each push of 1 s
    transforms the ring once, re-evaluates every reference series on the
    pushed stretch plus the taps' span only, and filters the templates over
    that second.  The pushes replay the segment's own samples, so the ring
    content (and every trigger) stays that of the segment.  Beside it, the
    earlier route: the whole segment transform and every full dechirp, then
    the last second filtered (as one graph)."""
    inc = int(w.fs)
    st = rfd.rfd_stream_create(s.plan, s.taps, s.h_ref, inc)
    info = rfd.rfd_stream_info(st)
    rfd.rfd_stream_prime(st, data)
    pos = [0]

    def push():
        _, n, _ = rfd.rfd_stream_push(st, data[pos[0]:pos[0] + inc], prec, w.threshold, w.window, cap, out)
        pos[0] = (pos[0] + inc) % w.n
        return n

    d4, n4, t4 = timed(push, 20, 3)
    # one more push with every window reported, against the range filter of
    # the same outputs after a full re-dechirp (the ring replays the segment)
    vcap = 1 << 22
    vbuf, nv, vstart = rfd.rfd_stream_push(st, data[pos[0]:pos[0] + inc], prec, 0.0, w.window, vcap)
    rfd.rfd_stream_destroy(st)
    check = stream_check(w, s, data, prec, rfd, vbuf, nv, vstart, inc, vcap)
    stream = {"ms_per_push": d4 / 20 * 1e3, "triggers_last_push": n4,
              "stages_ms_per_push": {k: t4[k] / 20 for k in ("data_fft_ms", "dechirp_ms", "fir_ms", "compact_ms")},
              "output_lag_samples": info["lag"], "reference_stretch_samples": info["zlen"],
              "check_vs_range_filter": check}
    log(f"low latency (stream): {d4 / 20 * 1e3:.3f} ms per 1 s push {stream['stages_ms_per_push']}")

    def increment():
        rfd.rfd_dechirp_refs(s.plan, data, s.h_ref, False)
        return rfd.rfd_filter_range(s.plan, s.taps, prec, w.threshold, w.window, w.n - inc, inc, cap, out)[1]

    d5, n5, t5 = timed(increment, 20, 3)
    ginc = rfd.rfd_range_graph_create(s.plan, s.taps, prec, w.threshold, w.window, data, s.h_ref, w.n - inc, inc,
                                      out, cap)
    dg, ng, _ = timed(lambda: rfd.rfd_segment_graph_launch(ginc), 20, 3)
    rfd.rfd_graph_destroy(ginc)
    log(f"low latency (full re-dechirp): {dg / 20 * 1e3:.3f} ms per 1 s increment as a graph, "
        f"{d5 / 20 * 1e3:.3f} ms eager ({prec})")
    return {"increment_samples": inc, "form": prec, "stream": stream,
            "full_redechirp": {"ms_per_increment_graph": dg / 20 * 1e3, "ms_per_increment_eager": d5 / 20 * 1e3,
                               "triggers": ng, "fir_ms_per_increment": t5["fir_ms"] / max(1, t5["n_fir"])},
            "note": "stream: ring transform + reference series on the pushed stretch only + FIR of that second "
                    "(host-synchronised per push); full_redechirp: the whole segment's transform and every "
                    "reference's full dechirp, then the same second filtered"}


def crossover_leg(w, bank, psd, seg, hrefs, mfma_form, np, rfd, torch, template_batch_device):
    """Where the direct MFMA form and the overlap-save form cross over: one
    sub-bank of 256 of the workload's templates (its first reference) at each
    tap count T, both forms timed on the segment (median of 5)."""
    from paper_2601_18835_amd.driver import RatioFilterSearch, SubBankSpec
    sb = bank.subbanks[0]
    ps = sb.params[:256]
    Hd = template_batch_device(w, ps, "cuda")
    data = torch.from_numpy(seg.data).cuda()
    out = {}
    for T in (16, 32, 64, 128, 256, 512, 1024):
        s = RatioFilterSearch(psd, w.f_low, w.fs, w.n, [SubBankSpec(0, T, -(T // 2), len(ps))], max_refs=1)
        try:
            s.set_reference(0, hrefs[0])
            s.make_taps(0, Hd)
            s.set_segment(data)
            s.dechirp_all()
            row = {}
            for form in (mfma_form, "ols32"):
                rfd.rfd_plan_set_timing(s.plan, True)
                for _ in range(6):
                    s.filter(form, w.threshold, w.window, 1 << 16)
                ts = []
                rfd.rfd_plan_get_timing(s.plan)
                for _ in range(5):
                    s.filter(form, w.threshold, w.window, 1 << 16)
                    ts.append(rfd.rfd_plan_get_timing(s.plan)["fir_ms"])
                row[form] = float(np.median(ts))
            out[T] = row
        finally:
            s.close()
    faster = [T for T in out if out[T]["ols32"] < out[T][mfma_form]]
    cross = min(faster) if faster else None
    log(f"crossover ({mfma_form} vs ols32, 256 templates, FIR stage ms): {out} -> ols32 faster from T = {cross}")
    return {"templates": len(ps), "fir_stage_ms": {str(T): v for T, v in out.items()},
            "ols32_faster_from_taps": cross, "mfma_form": mfma_form}


def parity_leg(w, bank, psd, seg, hrefs, orc_out, trig_main, prec, np, rfd):
    """Every FIR form on the oracle sample (validation mode: every sample's
    rho through the same kernels, each sampled template on its own
    reference slot, host waveforms as the oracle's) against the stated
    targets, and trigger identity of the timed run on the sample."""
    from oracle import cluster as ocl
    from paper_2601_18835_amd.driver import RatioFilterSearch, SubBankSpec
    sample, sbi, Hs, rho_o = orc_out["sample"], orc_out["sbi"], orc_out["Hs"], orc_out["rho"]
    shifts = orc_out["shifts"]
    centre = orc_out["centre"]
    tau = TARGET[prec]
    amb = mism = cmp = 0
    dmax = 0.0
    for i, j in enumerate(sample):
        d = int(shifts[i])
        rho = np.roll(rho_o[i], d)            # on the filter index m = n + d (lag-centred taps)
        want = {sm // w.window: (sm, r) for sm, r in ocl.cluster(rho, w.threshold, w.window)}
        sel = trig_main[trig_main["tmpl"] == j]
        got = {}
        for t in sel:
            m = (int(t["sample"]) + d) % w.n
            got[m // w.window] = (m, float(t["rho"]))
        fl = ocl.window_ambiguity(rho, w.threshold, w.window, tau)
        for q in range(len(fl)):
            if fl[q]:
                amb += 1
                continue
            cmp += 1
            if (q in want) != (q in got) or (q in want and want[q][0] != got[q][0]):
                mism += 1
            elif q in want:
                dmax = max(dmax, abs(want[q][1] - got[q][1]))
    specs = [SubBankSpec(i, bank.subbanks[sbi[i]].taps, bank.subbanks[sbi[i]].k0, 1) for i in range(len(sample))]
    s2 = RatioFilterSearch(psd, w.f_low, w.fs, w.n, specs, max_refs=len(sample))
    for i in range(len(sample)):
        s2.set_reference(i, hrefs[sbi[i]])
        s2.make_taps(i, Hs[i:i + 1], method=rfd.RFD_TAPS_LS | (rfd.RFD_TAPS_CENTRE if centre else 0))
    s2.set_segment(seg.data)
    s2.dechirp_all()
    full, ok = {}, {}
    for form in ("ols32", "fp32", "bf16x3", "fp16x3"):
        buf, n = s2.filter(form, 0.0, 1, len(sample) * w.n)
        tv = rfd.triggers_to_numpy(buf, n)
        r = np.zeros((len(sample), w.n))
        r[tv["tmpl"], tv["sample"]] = tv["rho"]
        full[form] = float(np.max(np.abs(r - rho_o)))
        ok[form] = bool(full[form] <= TARGET[form])
    s2.close()
    parity = {"templates": sample, "windows_compared": cmp, "ambiguous": amb, "mismatches": mism,
              "timed_form": prec, "max_drho_at_triggers": dmax, "max_drho_full_series": full,
              "target": TARGET, "within_target": ok,
              "ok": bool(mism == 0 and ok[prec] and dmax <= TARGET[prec])}
    log(f"parity: {parity}")
    if not parity["ok"]:
        log("PARITY FAILED for the timed form: its value does not meet the stated bar")
    return parity


def surrogate_main(args):
    """surr512s, the learned-surrogate configuration end to end: 65536
    (m1, m2, chi, e0) templates under 32 references (2048 each), N = 2^20,
    T = 1024, one coloured-noise segment with an injection.

    Set-up (untimed): the exact taps of the whole bank from waveforms made on
    the device (the yardstick and the fallback); --train exact training tap sets
    per reference (3125 by default: 1e5 in all) drawn over the reference's
    chirp-mass slice; one surrogate per reference, all trained together by
    rfd_surrogate_train_many; every bank template's surrogate taps validated
    against its exact taps (rfd_taps_match), fallback below 0.99.

    Timed step (one segment): the data transform and the 32 dechirps, the
    surrogate taps of all 65536 templates from parameters resident in HBM,
    the exact taps copied in wherever validation fell below 0.99, and the
    overlap-save FIR with threshold and window peaks over every template."""
    import numpy as np
    import torch

    import synth
    from paper_2601_18835_amd import rfd
    from paper_2601_18835_amd.driver import RatioFilterSearch, SubBankSpec, TapSurrogate
    from synth.device import template_batch_device

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    w = synth.get_workload("surr512s")
    bank = synth.make_bank(w)
    sel = (list(range(len(bank.subbanks))) if args.subbanks == "all"
           else [int(x) for x in args.subbanks.split(",")])
    sbs = [bank.subbanks[b] for b in sel]
    psd = synth.psd_array(w.n, w.fs)
    seg = synth.make_segment(w, bank)
    specs = [SubBankSpec(i, sb.taps, sb.k0, sb.size) for i, sb in enumerate(sbs)]
    s = RatioFilterSearch(psd, w.f_low, w.fs, w.n, specs, max_refs=len(sel))
    for i, sb in enumerate(sbs):
        s.set_reference(i, synth.reference_waveform(w, sb))
    T = sbs[0].taps
    nt = int(s.offsets[-1])
    phys = lambda ps: np.array([[p.m1, p.m2, p.chi1, p.e0] for p in ps])   # noqa: E731
    rfd.rfd_plan_set_timing(s.plan, True)
    log(f"workload surr512s: N={w.n}, {len(sel)} references, {nt} bank templates, T={T}; "
        f"{args.train} training tap sets per reference, {args.epochs} epochs")
    batch = 256
    Hd = None
    gen_s = 0.0

    def waveforms(ps):
        nonlocal Hd, gen_s
        tg = time.perf_counter()
        Hd = template_batch_device(w, ps, "cuda", out=Hd if Hd is not None and Hd.shape[0] == len(ps) else None)
        torch.cuda.synchronize()
        gen_s += time.perf_counter() - tg
        return Hd

    # exact taps of the bank (yardstick and fallback)
    rfd.rfd_plan_get_timing(s.plan)
    for i, sb in enumerate(sbs):
        for b0 in range(0, sb.size, batch):
            s.make_taps(i, waveforms(sb.params[b0:b0 + batch]), first=b0)
    torch.cuda.synchronize()
    exact_ms = rfd.rfd_plan_get_timing(s.plan)["taps_ms"]
    log(f"exact taps: {nt} in {exact_ms:.0f} ms of GPU time ({nt / exact_ms * 1e3:.3g}/s)")
    # training sets and surrogates
    surs = []
    t_sets = time.perf_counter()
    for i, (b, sb) in enumerate(zip(sel, sbs)):
        mc = [p.mchirp for p in sb.params]
        train = synth.workloads.draw_in_chirp_mass_range(w, min(mc), max(mc), args.train, stream=5 + b)
        sur = TapSurrogate(s, i, sb.taps, sb.k0, len(train), n_basis=64, hidden=256, seed=2601 + b)
        for b0 in range(0, len(train), batch):
            sur.add_training_waveforms(waveforms(train[b0:b0 + batch]), b0)
        torch.cuda.synchronize()
        sur.captured = sur.fit(phys(train))
        surs.append(sur)
        if i % 8 == 7 or i == len(sel) - 1:
            log(f"training sets and bases: {i + 1} of {len(sel)} references")
    del Hd
    t_sets = time.perf_counter() - t_sets
    rfd.rfd_plan_get_timing(s.plan)
    # all surrogates trained together, learning rate decayed geometrically over 10 calls
    handles, prm = [x.sur for x in surs], [x.params_dev for x in surs]
    stages, done, losses = 10, 0, []
    t0 = time.perf_counter()
    for st in range(stages):
        e = args.epochs // stages if st < stages - 1 else args.epochs - done
        rate = args.lr * (args.lr_end / args.lr) ** (st / (stages - 1))
        for g0 in range(0, len(handles), 32):
            losses.append((g0, rfd.rfd_surrogate_train_many(handles[g0:g0 + 32], prm[g0:g0 + 32], e, args.batch,
                                                           rate)))
        done += e
        last = np.concatenate([l[:, -1] for _, l in losses[-((len(handles) + 31) // 32):]])
        log(f"training: {done} epochs, loss mean {last.mean():.4f} (max {last.max():.4f})")
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    steps_per_net = done * (args.train // args.batch)
    log(f"trained {len(handles)} surrogates together in {train_s:.1f} s "
        f"({train_s / steps_per_net * 1e6:.0f} us per step of all {len(handles)})")
    # validation of every bank template, fallback flags at 0.99
    sur_taps = rfd.rfd_taps_create(s.plan, s.offsets, [sp.ref_id for sp in specs], [sp.taps for sp in specs],
                                   [sp.k0 for sp in specs])
    pdev = [x.scale_dev(phys(sb.params)) for x, sb in zip(surs, sbs)]
    for i in range(len(sel)):
        rfd.rfd_surrogate_make_taps(surs[i].sur, pdev[i], sur_taps, i, 0)
    matches = [rfd.rfd_taps_match(sur_taps, s.taps, i, 0, sb.size) for i, sb in enumerate(sbs)]
    mdev = [torch.from_numpy(m).cuda() for m in matches]
    m = np.concatenate(matches)
    thr = 0.99
    n_fb = [int(np.sum(~(x >= thr))) for x in matches]
    log(f"validation: match mean {m.mean():.4f}, median {np.median(m):.4f}, p01 {np.quantile(m, 0.01):.4f}, "
        f"min {m.min():.4f}; {np.mean(m >= thr):.1%} >= {thr}, {sum(n_fb)} fall back to exact taps")

    data = torch.from_numpy(seg.data).to("cuda")
    s.set_segment(data)
    cap = 1 << 22
    out = torch.empty(cap * 32, dtype=torch.uint8, device="cuda")

    def surrogate_taps():
        for i in range(len(sel)):
            rfd.rfd_surrogate_make_taps(surs[i].sur, pdev[i], sur_taps, i, 0)
            if n_fb[i]:
                rfd.rfd_taps_fallback(sur_taps, s.taps, i, 0, mdev[i], thr)

    def step():
        rfd.rfd_dechirp_refs(s.plan, data, s.h_ref, False)
        surrogate_taps()
        return rfd.rfd_filter_bank(s.plan, sur_taps, "ols32", w.threshold, w.window, cap, out)[1]

    def timed(fn, steps, warmup):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        rfd.rfd_plan_get_timing(s.plan)
        t1 = time.perf_counter()
        for _ in range(steps):
            n = fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t1, n, rfd.rfd_plan_get_timing(s.plan)

    log(f"timing {args.steps} steps ({args.warmup} warm-up): dechirps, surrogate taps with fallback and the "
        f"overlap-save FIR over {nt} templates")
    dt, ntrig, tim = timed(step, args.steps, args.warmup)
    ms_step = dt / args.steps * 1e3
    value = nt * w.n * args.steps / dt
    trig_sur = rfd.triggers_to_numpy(out, min(ntrig, cap))
    st_ms = {k: round(tim[k] / args.steps, 4) for k in ("data_fft_ms", "dechirp_ms", "sur_net_ms", "sur_expand_ms",
                                                       "sur_pack_ms", "fir_ms", "compact_ms") if k in tim}
    n_launch = max(1, tim["n_fir_kernel"] // args.steps)
    kernel_ms = tim["fir_kernel_ms"] / args.steps / n_launch
    # surrogate taps alone (with fallback), and the same filtering on exact taps
    d_tap, _, _ = timed(surrogate_taps, 3, 1)
    tap_rate = nt * 3 / d_tap
    d_ex, n_ex, _ = timed(lambda: (rfd.rfd_dechirp_refs(s.plan, data, s.h_ref, False),
                                   rfd.rfd_filter_bank(s.plan, s.taps, "ols32", w.threshold, w.window, cap,
                                                       out)[1])[1], 3, 1)
    trig_ex = rfd.triggers_to_numpy(out, min(n_ex, cap))
    log(f"surrogate step: {ms_step:.2f} ms ({value:.4g} t*s/s), {ntrig} triggers; taps alone "
        f"{d_tap / 3 * 1e3:.2f} ms ({tap_rate:.3g} tap sets/s); exact-tap filtering {d_ex / 3 * 1e3:.2f} ms, "
        f"{n_ex} triggers")
    # injection: recovered rho with surrogate taps and with exact taps
    injection = None
    if seg.inj_template >= 0 and len(sel) == len(bank.subbanks):   # bank numbering = search numbering
        q = seg.inj_sample // w.window

        def at_inj(tr):
            k = (tr["tmpl"] == seg.inj_template) & (tr["sample"] // w.window == q)
            return {"sample": int(tr["sample"][k][0]), "rho": float(tr["rho"][k][0])} if k.any() else None

        injection = {"template": seg.inj_template, "sample": seg.inj_sample, "optimal_snr": w.injection_snr,
                     "surrogate_taps": at_inj(trig_sur), "exact_taps": at_inj(trig_ex)}
        log(f"injection: {injection}")
    # per-window peaks present with both tap sets: relative rho difference
    key = lambda tr: tr["tmpl"].astype(np.int64) * (w.n // w.window + 1) + tr["sample"] // w.window   # noqa: E731
    ks, ke = key(trig_sur), key(trig_ex)
    common, i_s, i_e = np.intersect1d(ks, ke, return_indices=True)
    drho = np.abs(trig_sur["rho"][i_s] - trig_ex["rho"][i_e]) / np.maximum(trig_ex["rho"][i_e], 1e-30)
    after = np.concatenate([rfd.rfd_taps_match(sur_taps, s.taps, i, 0, sb.size) for i, sb in enumerate(sbs)])
    loss = 1.0 - after
    # roofline of the dominant kernel (the overlap-save FIR, K = 4096)
    K = 4096
    nB = -(-w.n // (K - T + 1))
    fl = (nt / n_launch) * nB * K * (5.0 * np.log2(K) + 6.0)
    achieved = fl / (kernel_ms * 1e-3) / 1e12
    roofline = {"bound": "alu", "achieved": round(achieved, 2), "peak": PEAK["ols32"], "unit": "TFLOP/s",
                "frac": round(achieved / PEAK["ols32"], 4), "traffic": None, "kernel": f"k_ols<{K}>",
                "flops_per_launch": fl, "avg_launch_ms": round(kernel_ms, 4), "launches_per_step": n_launch}
    cpu = None
    if not args.no_cpu_baseline:
        cpu = surrogate_cpu_baseline(w, sbs[0], psd, np)
    for x in surs:
        x.close()
    rfd.rfd_taps_destroy(sur_taps)
    s.close()
    line = {
        "metric": "template*samples/s with surrogate taps (validated, exact-tap fallback below 0.99), 1 GPU",
        "value": value, "unit": "template*samples/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "precision": "surrogate: bf16 weights, fp32 accumulation, fp64 expansion and norms; "
                                     "FIR: overlap-save FFT blocks in fp32",
        "data": "synthetic",
        "config": {"workload": "surr512s", "segment_samples": w.n, "fs": w.fs, "f_low": w.f_low,
                   "references": len(sel), "templates": nt, "taps": T, "n_basis": 64, "hidden": 256,
                   "train_sets_per_reference": args.train, "train_sets_total": args.train * len(sel),
                   "epochs": args.epochs, "batch": args.batch, "fir_form": "ols32", "threshold": w.threshold,
                   "cluster_window": w.window},
        "stages_ms": st_ms, "triggers": ntrig,
        "surrogate_taps": {"tap_sets_per_s": tap_rate, "ms_for_bank": d_tap / 3 * 1e3,
                           "exact_taps_per_s_gpu": nt / exact_ms * 1e3,
                           "gain_vs_exact_taps": tap_rate / (nt / exact_ms * 1e3),
                           "note": "exact taps also need one waveform per template; the surrogate needs none"},
        "validation": {"match_mean": float(m.mean()), "match_median": float(np.median(m)),
                       "match_p01": float(np.quantile(m, 0.01)), "match_min": float(m.min()),
                       "pass_0.99": float(np.mean(m >= thr)), "fallback": int(sum(n_fb)),
                       "fallback_fraction": float(sum(n_fb) / nt),
                       "per_reference_pass": [round(float(np.mean(x >= thr)), 4) for x in matches]},
        "snr_loss_after_fallback": {"mean": float(loss.mean()), "median": float(np.median(loss)),
                                    "p99": float(np.quantile(loss, 0.99)), "max": float(loss.max()),
                                    "note": "1 - match of each template's fitted surrogate taps to its exact "
                                            "taps (rfd_taps_match), after the fallback"},
        "filtering_vs_exact_taps": {"exact_ms_per_step": d_ex / 3 * 1e3, "triggers_exact": int(n_ex),
                                    "common_windows": int(common.size),
                                    "rel_rho_diff_max": float(drho.max()) if drho.size else None,
                                    "rel_rho_diff_median": float(np.median(drho)) if drho.size else None},
        "injection": injection,
        "training": {"seconds": round(train_s, 2), "networks_together": min(32, len(handles)),
                     "steps_per_network": steps_per_net, "us_per_step_all_networks":
                         round(train_s / steps_per_net * 1e6, 1),
                     "loss_last_mean": float(np.concatenate([l[:, -1] for _, l in losses[-1:]]).mean()),
                     "training_sets_and_bases_s": round(t_sets, 1),
                     "basis_captured_mean": float(np.mean([x.captured for x in surs]))},
        "waveform_generation_s": round(gen_s, 1),
        "roofline": roofline, "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def surrogate_cpu_baseline(w, sb, psd, np):
    """The oracle's surrogate inference (forward pass, basis expansion, FP64
    unwhitening, fitted norm) on this host for 256 templates of one sub-bank,
    with seeded random weights and basis of the same shapes."""
    import synth
    from oracle import spectral as osp
    from oracle import surrogate as osg
    from oracle import taps as otaps
    T, K, Hd, n = sb.taps, 64, 256, 256
    wts = osp.psd_weights(psd, w.n, w.fs, w.f_low)
    h_ref = synth.reference_waveform(w, sb)
    M = otaps.gram(h_ref, wts, T)
    L = np.linalg.cholesky(M + otaps.DEFAULT_RIDGE_EPS * M[0, 0].real * np.eye(T))
    rng = np.random.default_rng(5)
    params = osg.init_params([4, Hd, Hd, K], rng)
    B, _ = np.linalg.qr(rng.standard_normal((2 * T, K)))
    P = rng.uniform(-1, 1, size=(n, 4))
    c0, w0 = time.process_time(), time.perf_counter()
    y, _ = osg.forward(params, P)
    a = osg.unwhiten(y @ B.T, L)
    sig = np.sqrt(np.real(np.einsum("ij,jk,ik->i", np.conj(a), M, a)))
    wall = time.perf_counter() - w0
    cpu_t = time.process_time() - c0
    assert np.all(np.isfinite(sig))
    out = {"value": n / wall, "unit": "tap sets/s", "cores": max(1, int(round(cpu_t / wall))), "kind": "oracle",
           "sample": f"{n} templates of one sub-bank (T = {T}): FP64 forward pass, basis expansion, "
                     f"unwhitening solve and fitted norm; seeded random weights and basis",
           "seconds": round(wall, 2)}
    log(f"cpu oracle (surrogate inference): {out['value']:.4g} tap sets/s on {out['cores']} core(s)")
    return out


if __name__ == "__main__":
    main()
