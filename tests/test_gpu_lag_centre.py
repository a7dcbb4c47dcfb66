"""Per-template lag centring (Sec. V.A's tap tuning with each template's lag
window centred on its own correlation peak) on the GPU against the FP64
oracle: the chosen lags and taps, triggers of every FIR form on the filter
index m = n + d_j, the complex SNR and chi^2 at triggers, range filtering,
the selection of the tap count with centred lags, and the match gain.

Case: a 2^14-sample segment from 30 Hz with an SNR-15 injection; two
references; a least-squares sub-bank (T = 64) of templates spread in chirp
mass plus the reference delayed by +45 and -70 samples, and a windowed-route
sub-bank (T = 100) of templates of the second reference.
"""
import numpy as np
import pytest

import synth
from gpu_cases import SB, Case, compare_triggers, fir_tolerance, oracle_case
from oracle import chisq as ocq
from oracle import pipeline as orc
from oracle import spectral
from oracle import taps as otaps

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-5, "bf16x3": 1e-3, "ols32": 1e-5}


def _case():
    n, fs, f_low = 1 << 14, 2048.0, 30.0
    w = synth.Workload("lag-centre", 11, n, fs, f_low, 0, 2, 0, "fp32", "nonspin")
    rng = np.random.default_rng(23)
    psd = synth.psd_array(n, fs)
    s = synth.make_noise_spectrum(w, rng)
    refs = {0: synth.taylorf2(synth.WaveformParams(6.0, 5.0), n, fs, f_low),
            1: synth.taylorf2(synth.WaveformParams(9.0, 7.5), n, fs, f_low)}
    k = np.arange(n // 2 + 1)
    p0 = [synth.WaveformParams(*m) for m in rng.uniform(5.0, 7.0, size=(11, 2))]
    H0 = synth.template_batch(w, p0)
    delayed = [refs[0] * np.exp(-2j * np.pi * ((k * t) % n) / n) for t in (45, -70)]
    H0 = np.concatenate([H0, np.stack(delayed)])
    p1 = [synth.WaveformParams(*m) for m in rng.uniform(8.0, 10.0, size=(7, 2))]
    H1 = synth.template_batch(w, p1)
    # SNR-15 injection of template 3 of the first sub-bank at sample 9001
    amp = synth.workloads.optimal_snr_amplitude(H0[3], w, 15.0)
    s = s + amp * H0[3] * np.exp(-2j * np.pi * ((k * 9001) % n) / n)
    sbs = [SB(0, 64, -32, H0, "ls"), SB(1, 100, -50, H1, "window")]
    return Case("lag-centre", n, fs, f_low, psd, synth.spectrum_to_time(s, n, fs), refs, sbs)


def _oracle(case):
    """Oracle taps and series with each template's centred k0; shifts d_j."""
    p = orc.prepare(case.psd, case.data, case.fs, case.f_low)
    refs = {r: orc.dechirp(p, h) for r, h in case.refs.items()}
    taps, z, d = [], [], []
    for sb in case.subbanks:
        M = otaps.gram(case.refs[sb.ref], p.w, sb.T)
        for j in range(sb.H.shape[0]):
            k0j = otaps.centred_k0(sb.H[j], case.refs[sb.ref], p.w, sb.T)
            tt = orc.make_taps(p, sb.H[j], case.refs[sb.ref], sb.T, k0j, method=sb.method, M=M)
            taps.append(tt)
            z.append(orc.ratio_snr(refs[sb.ref], tt))
            d.append(k0j - sb.k0)
    case.oracle = dict(p=p, refs=refs, taps=taps, z=np.array(z))
    return np.array(d)


@pytest.fixture(scope="module")
def centred(rfd):
    from paper_2601_18835_amd.driver import RatioFilterSearch, SubBankSpec
    case = _case()
    d = _oracle(case)
    specs = [SubBankSpec(sb.ref, sb.T, sb.k0, sb.H.shape[0]) for sb in case.subbanks]
    s = RatioFilterSearch(case.psd, case.f_low, case.fs, case.n, specs, max_refs=2)
    for r, h in case.refs.items():
        s.set_reference(r, h)
    for b, sb in enumerate(case.subbanks):
        m = rfd.RFD_TAPS_LS if sb.method == "ls" else rfd.RFD_TAPS_WINDOW
        s.make_taps(b, sb.H, method=m | rfd.RFD_TAPS_CENTRE)
    s.set_segment(case.data)
    s.dechirp_all()
    print(f"\n[lag-centre] offsets d_j = {d.tolist()}", flush=True)
    yield case, s, d
    s.close()


def test_centred_lags_and_taps_match_oracle(rfd, centred):
    case, s, d = centred
    worst = 0.0
    j = 0
    for sb in case.subbanks:
        for _ in range(sb.H.shape[0]):
            a, sig, T, k0 = rfd.rfd_taps_get(s.taps, j)
            tt = case.oracle["taps"][j]
            assert T == sb.T and k0 == tt.k0, (j, k0, tt.k0)
            err = np.max(np.abs(a - tt.a)) / np.max(np.abs(tt.a))
            worst = max(worst, err)
            assert err <= 1e-8, (j, err)
            assert abs(sig - tt.sigma_fit) <= 1e-10 * tt.sigma_fit
            j += 1
    assert np.any(d != 0) and d[11] == 45 - 0 and d[12] == -70
    print(f"\n[lag-centre] {j} templates: lags identical, taps within {worst:.2e}")


@pytest.mark.parametrize("precision", ["fp32", "bf16x3", "ols32"])
def test_centred_triggers_and_z_match_oracle(rfd, centred, precision):
    case, s, d = centred
    thr, W = 3.0, 512
    buf, n = s.filter(precision, thr, W, 1 << 16)
    tr = rfd.triggers_to_numpy(buf, n)
    rho = np.abs(case.oracle["z"])
    tol = fir_tolerance(case, precision, TOL[precision])
    ncmp, namb, dmax = compare_triggers(tr, rho, thr, W, tol, shifts=d)
    assert dmax <= tol.max(), dmax
    # complex SNR at each trigger against the oracle series at its sample
    zo = case.oracle["z"][tr["tmpl"], tr["sample"]]
    zg = tr["z_re"] + 1j * tr["z_im"]
    zerr = np.abs(zg - zo)
    assert np.all(zerr <= 3 * tol[tr["tmpl"]] + 1e-5), zerr.max()
    # the injection is found by its template, at its sample
    hit = (tr["tmpl"] == 3) & (np.abs(tr["sample"] - 9001) <= 2)
    assert hit.any()
    print(f"\n[lag-centre] {precision}: {n} triggers, {ncmp} windows identical, {namb} ambiguous, "
          f"max |drho| {dmax:.2e}, max |dz| {zerr.max():.2e}; injection rho {tr['rho'][hit].max():.3f}")


def test_centred_range_filter_uses_the_filter_index(rfd, centred):
    """A range [lo, lo + len) of filter indices m: every reported sample is
    m - d_j of an m inside the range, and on whole windows the range gives
    the full filter's triggers."""
    case, s, d = centred
    lo, ln, W = 4096, 4096, 1024
    buf, n = s.filter_range("fp32", 3.0, W, lo, ln, 1 << 16)
    tr = rfd.triggers_to_numpy(buf, n)
    m = (tr["sample"] + d[tr["tmpl"]]) % case.n
    assert np.all((m >= lo) & (m < lo + ln))
    buf2, n2 = s.filter("fp32", 3.0, W, 1 << 16)
    full = rfd.triggers_to_numpy(buf2, n2)
    mf = (full["sample"] + d[full["tmpl"]]) % case.n
    keep = (mf >= lo) & (mf < lo + ln)
    assert np.array_equal(full[keep], tr)
    print(f"\n[lag-centre] range [{lo}, {lo + ln}): {n} triggers = the full filter's on those windows")


def test_centred_chisq_at_triggers_matches_oracle(rfd, centred):
    case, s, d = centred
    P = 4
    edges = s.bands(P)
    buf, n = s.filter("fp32", 3.0, 512, 1 << 16)
    tr = rfd.triggers_to_numpy(buf, n)
    got = s.chisq(buf, n)
    p = case.oracle["p"]
    i_low, i_high = spectral.band_limits(case.n, case.fs, case.f_low)
    want = []
    first = np.cumsum([0] + [sb.H.shape[0] for sb in case.subbanks])
    for t, smp in zip(tr["tmpl"], tr["sample"]):
        b = int(np.searchsorted(first, t, side="right") - 1)
        sb = case.subbanks[b]
        e = ocq.band_edges(case.refs[sb.ref], p.w, i_low, i_high, P)
        np.testing.assert_array_equal(edges[sb.ref], e)
        tt = case.oracle["taps"][t]
        zb = ocq.fitted_band_snr(p.stilde, case.refs[sb.ref], p.w, tt.a, tt.k0, e)
        f = ocq.band_fractions(case.refs[sb.ref], p.w, tt.a, tt.k0, e)
        want.append(ocq.chisq(zb, f)[smp])
    want = np.array(want)
    err = np.abs(got - want) / np.maximum(1.0, want)
    assert n > 0 and np.all(err <= 1e-3), err.max()
    print(f"\n[lag-centre] chi^2 at {n} triggers: max relative error {err.max():.2e}")


def test_centred_selection_matches_oracle_and_gains(rfd, centred):
    """rfd_select_taps with centred lags: the oracle's tap count, match and k0
    per template; at T = 64 centring lifts the zero-lag match of the delayed
    references far above that of lags centred on 0 (the mean gain over the
    sub-bank is printed)."""
    case, s, _ = centred
    p = case.oracle["p"]
    sb = case.subbanks[0]
    ladder = [16, 32, 64, 128]
    href = case.refs[sb.ref]
    T, m, k0 = rfd.rfd_select_taps(s.plan, s.to_dev(href), s.to_dev(sb.H), 0.99, ladder, centre=True)
    T0, m0 = rfd.rfd_select_taps(s.plan, s.to_dev(href), s.to_dev(sb.H), 0.99, ladder)
    for j in range(sb.H.shape[0]):
        Tw, mw = otaps.select_taps(sb.H[j], href, p.w, 0.99, ladder, centre=True)
        assert T[j] == Tw and abs(m[j] - mw) <= 1e-9, (j, T[j], Tw, m[j], mw)
        assert k0[j] == otaps.centred_k0(sb.H[j], href, p.w, Tw)
    gain = []
    for j in range(sb.H.shape[0]):
        kc = otaps.centred_k0(sb.H[j], href, p.w, 64)
        ac = otaps.ls_taps_normal(sb.H[j], href, p.w, 64, kc)
        a0 = otaps.ls_taps_normal(sb.H[j], href, p.w, 64, -32)
        gain.append(otaps.zero_lag_match(sb.H[j], href, p.w, ac, kc) - otaps.zero_lag_match(sb.H[j], href, p.w, a0, -32))
    gain = np.array(gain)
    assert gain[11] > 0.1 and gain[12] > 0.1
    print(f"\n[lag-centre] T = 64 zero-lag match gain from centring: mean {gain.mean():.4f}, "
          f"min {gain.min():.4f}, max {gain.max():.4f}; centred T {T.tolist()} vs lag-0 T {T0.tolist()}")


def test_graph_captured_before_centring_follows_the_taps(rfd, centred):
    """A segment graph captured while sub-bank 0 had lags centred on 0, then
    replayed after its taps were re-made with centred lags (same buffers),
    reports the centred taps' triggers: the lag offsets are read at replay."""
    import torch
    case, s, d = centred
    thr, W, cap = 3.0, 512, 1 << 16
    H0 = case.subbanks[0].H
    out = torch.empty(cap * 32, dtype=torch.uint8, device="cuda")
    s.make_taps(0, H0, method=rfd.RFD_TAPS_LS)
    graph = rfd.rfd_segment_graph_create(s.plan, s.taps, "fp32", thr, W, s.data, s.h_ref, out, cap)
    try:
        s.make_taps(0, H0, method=rfd.RFD_TAPS_LS | rfd.RFD_TAPS_CENTRE)
        n = rfd.rfd_segment_graph_launch(graph)
        got = rfd.triggers_to_numpy(out, n)
    finally:
        rfd.rfd_graph_destroy(graph)
    buf, n2 = s.filter("fp32", thr, W, cap)
    want = rfd.triggers_to_numpy(buf, n2)
    assert n == n2 and np.array_equal(got, want)
    print(f"\n[lag-centre] graph captured before centring: {n} triggers = eager with centred taps")
