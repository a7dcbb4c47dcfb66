"""Ratio-filtered chi^2 (Sec. VI.C) on the GPU against the FP64 oracle
(oracle/chisq.py): band edges (exact), band shares, chi^2 at every sample of
every template of the uneven-sub-bank case, triggers, and the error paths."""
import numpy as np
import pytest

from gpu_cases import UNIT, gpu_search, oracle_case, ragged_case, rho_matrix, tap_gain
from oracle import chisq as ocq
from oracle import spectral

pytestmark = pytest.mark.gpu

P = 8


@pytest.fixture(scope="module")
def banded(rfd):
    case = ragged_case()
    oracle_case(case)
    s = gpu_search(case)
    edges = s.bands(P)
    yield case, s, edges
    s.close()


def _oracle_edges(case, r):
    p = case.oracle["p"]
    i_low, i_high = spectral.band_limits(case.n, case.fs, case.f_low)
    return ocq.band_edges(case.refs[r], p.w, i_low, i_high, P)


def test_band_edges_are_exact(rfd, banded):
    case, s, edges = banded
    for r in case.refs:
        np.testing.assert_array_equal(edges[r], _oracle_edges(case, r))


def _oracle_shares_and_chisq(case):
    p = case.oracle["p"]
    shares, chis, zbs = [], [], []
    j = 0
    for sb in case.subbanks:
        e = _oracle_edges(case, sb.ref)
        for _ in range(sb.H.shape[0]):
            tt = case.oracle["taps"][j]
            f = ocq.band_fractions(case.refs[sb.ref], p.w, tt.a, tt.k0, e)
            zb = ocq.fitted_band_snr(p.stilde, case.refs[sb.ref], p.w, tt.a, tt.k0, e)
            shares.append(f)
            zbs.append(zb)
            chis.append(ocq.chisq(zb, f))
            j += 1
    return np.array(shares), np.array(chis), zbs


def test_band_shares_match_oracle(rfd, banded):
    case, s, _ = banded
    want, _, _ = _oracle_shares_and_chisq(case)
    got = np.array([rfd.rfd_taps_get_band_fractions(s.taps, j) for j in range(case.n_templates)])
    err = np.max(np.abs(got - want))
    print(f"\n[ragged] band shares (p={P}): max |df| = {err:.3e}")
    assert err <= 4 * 2.0 ** -24
    np.testing.assert_allclose(got.sum(axis=1), 1.0, atol=P * 2.0 ** -24)


def test_chisq_every_sample_matches_oracle(rfd, banded):
    case, s, _ = banded
    cap = case.n_templates * case.n
    buf, n = s.filter("fp32", 0.0, 1, cap)
    trig = rfd.triggers_to_numpy(buf, n)
    got = s.chisq(buf, n)
    f, want_full, zbs = _oracle_shares_and_chisq(case)
    want = want_full[trig["tmpl"], trig["sample"]]
    # bound: FP32 band FIR errors e_b (operand rounding over ||c||_1 and
    # accumulation of 2T products, as for the FIR itself), propagated through
    # sum_b |z_b - f_b z|^2 / f_b to first order, plus FP32 rounding of f_b
    u = UNIT["fp32"]
    gain = tap_gain(case)
    taps = np.concatenate([[sb.T] * sb.H.shape[0] for sb in case.subbanks])
    po = case.oracle["p"]
    zref_max = {r: np.max(np.abs(ocq.reference_band_series(po.stilde, h, po.w, _oracle_edges(case, r))))
                for r, h in case.refs.items()}
    zmax = np.concatenate([[zref_max[sb.ref]] * sb.H.shape[0] for sb in case.subbanks])
    e_band = 3.0 * zmax * (u * gain + u * np.sqrt(2.0 * taps))                    # per template
    zb_t = np.stack([zbs[j][:, sm] for j, sm in zip(trig["tmpl"], trig["sample"])])   # [n, P]
    ft = f[trig["tmpl"]]
    z_t = zb_t.sum(axis=1, keepdims=True)
    r = np.abs(zb_t - ft * z_t)
    e = e_band[trig["tmpl"]][:, None] * (1.0 + ft * P)
    bound = (np.sum((2.0 * r * e + e * e) / ft, axis=1) + np.sum((2 * r * np.abs(z_t) + r ** 2 / ft), axis=1) * 8 * u
             + 4 * P * u * want)                                     # and the FP32 sum of the statistic
    err = np.abs(got.astype(np.float64) - want)
    print(f"\n[ragged] chi^2 at {n} samples: max |dchi2| = {err.max():.3e}, worst err/bound = "
          f"{np.max(err / bound):.3f}; mean chi^2 {got.mean():.3f} (2(p-1) = {2 * (P - 1)} in pure noise; this "
          f"segment holds an SNR-15 injection)")
    assert np.all(err <= bound)


def test_chisq_at_triggers_equals_series(rfd, banded):
    case, s, _ = banded
    cap = case.n_templates * case.n
    buf, n = s.filter("fp32", 0.0, 1, cap)
    full = s.chisq(buf, n)
    trig_all = rfd.triggers_to_numpy(buf, n)
    table = np.full((case.n_templates, case.n), np.nan, dtype=np.float32)
    table[trig_all["tmpl"], trig_all["sample"]] = full
    for form in ("fp32", "bf16x3", "ols32"):
        buf2, n2 = s.filter(form, 3.0, 300, 1 << 16)
        tr = rfd.triggers_to_numpy(buf2, n2)
        x = s.chisq(buf2, n2)
        assert n2 > 0
        np.testing.assert_array_equal(x, table[tr["tmpl"], tr["sample"]])


def test_error_paths(rfd, banded):
    import torch
    case, s, _ = banded
    # a trigger naming no template of the bank gives NaN
    bad = np.zeros(2, dtype=rfd.TRIGGER_DTYPE)
    bad[0]["subbank"], bad[0]["tmpl"], bad[0]["sample"] = 99, 0, 0
    bad[1]["subbank"], bad[1]["tmpl"], bad[1]["sample"] = 0, 0, case.n + 5
    dev = torch.from_numpy(bad.view(np.uint8).copy()).cuda()
    x = s.chisq(dev, 2)
    assert np.isnan(x).all()
    # a taps object without shares is a state error (nothing runs)
    from paper_2601_18835_amd.driver import RatioFilterSearch, SubBankSpec
    sb = case.subbanks[0]
    s2 = RatioFilterSearch(case.psd, case.f_low, case.fs, case.n, [SubBankSpec(sb.ref, sb.T, sb.k0, 2)],
                           max_refs=max(case.refs) + 1)
    try:
        for r, h in case.refs.items():
            s2.set_reference(r, h)
        s2.make_taps(0, sb.H[:2])
        s2.set_segment(case.data)
        s2.dechirp_all()
        buf, n = s2.filter("fp32", 0.0, 1, 2 * case.n)
        with pytest.raises(rfd.RfdError) as e:
            s2.chisq(buf, n)
        assert e.value.code == rfd.RFD_E_STATE
    finally:
        s2.close()
