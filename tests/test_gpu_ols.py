"""Overlap-save FFT form of the ratio FIR (RFD_OLS32) against the FP64 oracle
and against the direct forms: every block size, windows shorter and longer
than a block, the tap spectra following new taps, graph replays and the
block-size autotuner."""
import numpy as np
import pytest

from gpu_cases import check_target_ambiguity, compare_triggers, fir_tolerance, gpu_search, oracle_case, ragged_case, rho_matrix

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ragged(rfd):
    case = ragged_case()
    oracle_case(case)
    s = gpu_search(case)
    yield case, s
    s.close()


def _rho(rfd, s, case, precision):
    buf, n = s.filter(precision, 0.0, 1, case.n_templates * case.n)
    trig = rfd.triggers_to_numpy(buf, n)
    return trig, rho_matrix(trig, case.n_templates, case.n)


@pytest.mark.parametrize("block", [0, 1024, 2048, 4096])
def test_block_sizes_match_oracle(rfd, ragged, block):
    case, s = ragged
    rfd.rfd_plan_set_fir_config(s.plan, ols_block=block)
    try:
        trig, rho = _rho(rfd, s, case, "ols32")
        assert not np.isnan(rho).any(), "validation mode must report every sample"
        want = np.abs(case.oracle["z"])
        err_t = np.max(np.abs(rho - want), axis=1)
        tol = fir_tolerance(case, "ols32", 1e-5, ols_forced=block)
        print(f"\n[ragged] ols32 K={block or 'auto'}: max |drho| = {err_t.max():.3e}, "
              f"worst err/tol = {np.max(err_t / tol):.2f}")
        assert (err_t <= tol).all()
        # windows much shorter than a block (per-sample keys), about a block, longer than the segment part
        for threshold, window in [(3.0, 17), (3.0, 300), (2.5, 8192)]:
            buf, n = s.filter("ols32", threshold, window, 1 << 16)
            tr = rfd.triggers_to_numpy(buf, n)
            compare_triggers(tr, want, threshold, window, tol)
            check_target_ambiguity(tr, want, threshold, window, tol, 1e-5)
    finally:
        rfd.rfd_plan_set_fir_config(s.plan)


def test_tap_spectra_follow_new_taps(rfd, ragged):
    """Re-made taps (templates of a sub-bank in reverse order) must reach the
    overlap-save form: its rows follow the permutation, as the direct form's do."""
    case, s = ragged
    b = 1
    sb = case.subbanks[b]
    first = case.first(b)
    rows = slice(first, first + sb.H.shape[0])
    _, before = _rho(rfd, s, case, "ols32")
    s.make_taps(b, sb.H[::-1].copy())
    try:
        _, after = _rho(rfd, s, case, "ols32")
        _, direct = _rho(rfd, s, case, "fp32")
        assert np.array_equal(after[:first], before[:first])
        np.testing.assert_allclose(after[rows], before[rows][::-1], rtol=0, atol=1e-6)
        # both forms within their own bounds of the oracle, so within the sum of
        # those bounds of each other (the largest over the permuted rows)
        both = (fir_tolerance(case, "fp32", 1e-5) + fir_tolerance(case, "ols32", 1e-5))[rows].max()
        assert np.max(np.abs(after[rows] - direct[rows])) <= both
    finally:
        s.make_taps(b, sb.H)
    _, again = _rho(rfd, s, case, "ols32")
    assert np.array_equal(again, before)


def test_segment_graph_replays_match_eager(rfd, ragged):
    import torch
    case, s = ragged
    th, W, cap = 2.5, 300, 1 << 16
    s.dechirp_all()
    buf, n = s.filter("ols32", th, W, cap)
    eager = rfd.triggers_to_numpy(buf, n)
    out = torch.empty(cap * 32, dtype=torch.uint8, device="cuda")
    g = rfd.rfd_segment_graph_create(s.plan, s.taps, "ols32", th, W, s.data, s.h_ref, out, cap)
    try:
        for rep in range(3):
            n2 = rfd.rfd_segment_graph_launch(g)
            assert np.array_equal(rfd.triggers_to_numpy(out, n2), eager), f"replay {rep}"
            s.dechirp_all()
            buf, n3 = s.filter("ols32", th, W, cap)
            assert np.array_equal(rfd.triggers_to_numpy(buf, n3), eager)
            torch.cuda.synchronize()
    finally:
        rfd.rfd_graph_destroy(g)
        s.dechirp_all()


def test_autotuner_picks_a_block_size(rfd, ragged):
    case, s = ragged
    buf, n = s.filter("ols32", 0.0, 1, case.n_templates * case.n)
    before = rfd.triggers_to_numpy(buf, n)
    res = rfd.rfd_autotune_fir(s.plan, s.taps, "ols32", 1, reps=2)
    print(f"\n[ragged] autotune ols32: {res}")
    assert res["n_candidates"] == 9       # the current one, then 4 block sizes x (general, aligned outputs)
    assert res["best"]["ols_block"] in (0, 1024, 2048, 4096) and res["best"]["ols_aligned"] in (0, 1)
    assert res["best_ms"] <= res["before_ms"] + 1e-9
    buf, n = s.filter("ols32", 0.0, 1, case.n_templates * case.n)
    after = rfd.triggers_to_numpy(buf, n)
    assert np.array_equal(after["sample"], before["sample"])
    # the tuned block size may differ from the automatic one: both lie within
    # their own bounds of the oracle, so within the sum of the two of each other
    both = fir_tolerance(case, "ols32", 1e-5) + fir_tolerance(case, "ols32", 1e-5,
                                                              ols_forced=res["best"]["ols_block"])
    assert np.all(np.abs(after["rho"] - before["rho"]) <= both[after["tmpl"]])
    rfd.rfd_plan_set_fir_config(s.plan)

