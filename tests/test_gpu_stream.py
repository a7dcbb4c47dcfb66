"""Low-latency and PSD-drift paths (Sec. VII.A, Sec. VI.B): range filtering
against the oracle restricted to the range, for every FIR form and for
aligned and cut windows; renormalisation after a PSD change against the
oracle's ratio SNR with the old taps under the new PSD."""
import numpy as np
import pytest

from gpu_cases import check_target_ambiguity, compare_triggers, fir_tolerance, gpu_search, oracle_case, ragged_case, workload_case
from oracle import fir, pipeline
from oracle import taps as otaps

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-5, "bf16x3": 1e-3, "fp16x3": 1e-3, "ols32": 1e-5}


@pytest.fixture(scope="module")
def ragged(rfd):
    case = ragged_case()
    oracle_case(case)
    s = gpu_search(case)
    yield case, s
    s.close()


@pytest.mark.parametrize("precision", ["fp32", "bf16x3", "fp16x3", "ols32"])
@pytest.mark.parametrize("n_start,n_len,window", [(2048, 2048, 512), (2304, 1792, 512), (0, 8192, 300),
                                                  (7936, 256, 1024)])
def test_range_matches_oracle_on_the_range(rfd, ragged, precision, n_start, n_len, window):
    case, s = ragged
    want = np.abs(case.oracle["z"]).copy()
    outside = np.ones(case.n, dtype=bool)
    outside[n_start:n_start + n_len] = False
    want[:, outside] = 0.0                      # the range's samples only
    tol = fir_tolerance(case, precision, TOL[precision])
    buf, n = s.filter_range(precision, 2.5, window, n_start, n_len, 1 << 16)
    tr = rfd.triggers_to_numpy(buf, n)
    assert np.all((tr["sample"] >= n_start) & (tr["sample"] < n_start + n_len))
    ncmp, namb, dmax = compare_triggers(tr, want, 2.5, window, tol)
    check_target_ambiguity(tr, want, 2.5, window, tol, TOL[precision])
    assert dmax <= tol.max(), dmax
    print(f"\n[ragged] {precision} range [{n_start}, {n_start + n_len}) W={window}: {n} triggers, "
          f"{ncmp} windows identical, {namb} ambiguous")
    if precision != "ols32" and window % 256 == 0 and n_start % window == 0 and n_len % window == 0:
        # whole windows: the direct forms give the full filter's triggers bit for bit
        buf2, n2 = s.filter(precision, 2.5, window, 1 << 16)
        full = rfd.triggers_to_numpy(buf2, n2)
        keep = (full["sample"] >= n_start) & (full["sample"] < n_start + n_len)
        assert np.array_equal(full[keep], tr)


def test_range_arguments_are_checked(rfd, ragged):
    case, s = ragged
    for n_start, n_len in [(100, 256), (0, 300), (0, 0), (8192 - 256, 512), (-256, 512)]:
        with pytest.raises(rfd.RfdError) as e:
            s.filter_range("fp32", 3.0, 512, n_start, n_len, 1024)
        assert e.value.code == rfd.RFD_E_INVALID


def test_renormalisation_follows_a_psd_change(rfd):
    case = workload_case("bns64s")
    oracle_case(case)
    s = gpu_search(case)
    try:
        f = np.arange(case.psd.size) * case.fs / case.n
        psd2 = case.psd * (1.0 + 0.3 * np.sin(2 * np.pi * f / 200.0))
        a_before = [s.tap(j)[0] for j in range(case.n_templates)]
        rfd.rfd_plan_set_psd(s.plan, psd2)
        with pytest.raises(rfd.RfdError):          # the reference series are stale now
            s.filter("fp32", 0.0, 1, case.n_templates * case.n)
        for b, sb in enumerate(case.subbanks):
            rfd.rfd_taps_renormalize(s.plan, s.taps, b, s.h_ref[sb.ref])
        s.dechirp_all()
        buf, n = s.filter("fp32", 0.0, 1, case.n_templates * case.n)
        tr = rfd.triggers_to_numpy(buf, n)
        rho = np.zeros((case.n_templates, case.n))
        rho[tr["tmpl"], tr["sample"]] = tr["rho"]
        # oracle: the same taps, the new PSD in the reference filter and in the norm
        p2 = pipeline.prepare(psd2, case.data, case.fs, case.f_low)
        sb = case.subbanks[0]
        ref2 = pipeline.dechirp(p2, case.refs[sb.ref])
        M2 = otaps.gram(case.refs[sb.ref], p2.w, sb.T)
        worst = worst_s = 0.0
        for j in range(case.n_templates):
            a, sig, _, _ = s.tap(j)
            assert np.array_equal(a, a_before[j]), "renormalisation must not change the taps"
            a_o = case.oracle["taps"][j].a
            sig2 = np.sqrt(otaps.fitted_sigma_sq_lag(a_o, M2))
            worst_s = max(worst_s, abs(sig - sig2) / sig2)
            z = fir.fir_direct(ref2.z, np.conj(a_o), sb.k0) / sig2
            worst = max(worst, np.max(np.abs(rho[j] - np.abs(z))))
        print(f"\n[bns64s] PSD drift: max rel dsigma_fit {worst_s:.2e}, max |drho| {worst:.2e}")
        assert worst_s <= 1e-9 and worst <= 1e-5
    finally:
        s.close()


@pytest.mark.parametrize("precision", ["ols32", "fp32", "bf16x3"])
def test_range_graph_replays_match_eager_range(rfd, ragged, precision):
    """The low-latency increment captured as one graph (transform, dechirps,
    range FIR, compaction) gives the eager range filter's triggers on every
    replay, with eager work between the replays."""
    import torch
    case, s = ragged
    th, W, cap = 2.5, 512, 1 << 16
    n_start, n_len = case.n - 2048, 2048
    s.dechirp_all()
    buf, n = s.filter_range(precision, th, W, n_start, n_len, cap)
    eager = rfd.triggers_to_numpy(buf, n)
    assert len(eager) > 0
    out = torch.empty(cap * 32, dtype=torch.uint8, device="cuda")
    g = rfd.rfd_range_graph_create(s.plan, s.taps, precision, th, W, s.data, s.h_ref, n_start, n_len, out, cap)
    try:
        for rep in range(3):
            n2 = rfd.rfd_segment_graph_launch(g)
            assert np.array_equal(rfd.triggers_to_numpy(out, n2), eager), f"replay {rep}"
            s.dechirp_all()
            buf, n3 = s.filter_range(precision, th, W, n_start, n_len, cap)
            assert np.array_equal(rfd.triggers_to_numpy(buf, n3), eager)
            torch.cuda.synchronize()
    finally:
        rfd.rfd_graph_destroy(g)
        s.dechirp_all()


def test_range_graph_arguments_are_checked(rfd, ragged):
    import torch
    case, s = ragged
    out = torch.empty(1024 * 32, dtype=torch.uint8, device="cuda")
    for n_start, n_len in [(100, 256), (0, 0), (0, 100), (case.n - 256, 512), (-256, 256)]:
        with pytest.raises(rfd.RfdError) as e:
            rfd.rfd_range_graph_create(s.plan, s.taps, "ols32", 2.5, 512, s.data, s.h_ref, n_start, n_len, out, 1024)
        assert e.value.code == rfd.RFD_E_INVALID
