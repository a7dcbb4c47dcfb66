"""Dynamic tap count (Sec. V.A) on the GPU against the oracle's selection:
identical T per template (decisions closer than 1e-9 to the target are
counted as ambiguous), matches to 1e-9, and a search over the sub-banks the
selection forms (one per selected T) against the oracle's ratio SNR."""
import numpy as np
import pytest

import synth
from gpu_cases import SB, Case, ambiguity_bound, compare_triggers, fir_tolerance, gpu_search, oracle_case
from oracle import spectral
from oracle import taps as otaps

pytestmark = pytest.mark.gpu

N, FS, F_LOW = 8192, 2048.0, 30.0
LADDER = [16, 32, 64, 128, 256, 512, 1024]


@pytest.fixture(scope="module")
def bank():
    rng = np.random.default_rng(21)
    w_ = synth.Workload("select", 9, N, FS, F_LOW, 0, 1, 0, "fp32", "nonspin")
    psd = synth.psd_array(N, FS)
    h_ref = synth.taylorf2(synth.WaveformParams(6.0, 5.0), N, FS, F_LOW)
    params = [synth.WaveformParams(*m) for m in rng.uniform([5.5, 4.4], [6.6, 5.6], size=(40, 2))]
    H = synth.template_batch(w_, params)
    s = synth.make_noise_spectrum(w_, rng)
    amp = synth.workloads.optimal_snr_amplitude(H[3], w_, 14.0)
    k = np.arange(N // 2 + 1)
    s = s + amp * H[3] * np.exp(-2j * np.pi * ((k * 2500) % N) / N)
    return dict(psd=psd, h_ref=h_ref, H=H, data=synth.spectrum_to_time(s, N, FS))


@pytest.mark.parametrize("target", [0.99, 0.9999])
def test_selection_matches_oracle(rfd, bank, target):
    from paper_2601_18835_amd.driver import RatioFilterSearch, SubBankSpec
    s = RatioFilterSearch(bank["psd"], F_LOW, FS, N, [SubBankSpec(0, 16, -8, 1)], max_refs=1)
    try:
        T, m = rfd.rfd_select_taps(s.plan, s.to_dev(bank["h_ref"]), s.to_dev(bank["H"]), target, LADDER)
    finally:
        s.close()
    w = spectral.psd_weights(bank["psd"], N, FS, F_LOW)
    amb = 0
    for j, h in enumerate(bank["H"]):
        T_o, m_o = otaps.select_taps(h, bank["h_ref"], w, target, LADDER)
        if T[j] != T_o:
            # only a decision at the threshold may differ
            lad = [otaps.zero_lag_match(h, bank["h_ref"], w, otaps.ls_taps_normal(h, bank["h_ref"], w, t, -(t // 2)),
                                        -(t // 2)) for t in LADDER]
            assert min(abs(x - target) for x in lad) <= 1e-9, (j, T[j], T_o)
            amb += 1
            continue
        assert abs(m[j] - m_o) <= 1e-9
    print(f"\n[select] target {target}: T histogram {dict(zip(*np.unique(T, return_counts=True)))}, "
          f"{amb} ambiguous; min match {m.min():.6f}")


def test_search_over_selected_subbanks(rfd, bank):
    """Templates grouped by their selected T run as uneven sub-banks (persistent
    launch), in parity with the oracle's ratio SNR for the same taps."""
    from paper_2601_18835_amd.driver import RatioFilterSearch, SubBankSpec
    s = RatioFilterSearch(bank["psd"], F_LOW, FS, N, [SubBankSpec(0, 16, -8, 1)], max_refs=1)
    try:
        T, _ = rfd.rfd_select_taps(s.plan, s.to_dev(bank["h_ref"]), s.to_dev(bank["H"]), 0.999, LADDER)
    finally:
        s.close()
    subbanks = [SB(0, int(t), -(int(t) // 2), bank["H"][T == t]) for t in np.unique(T)]
    case = Case("select", N, FS, F_LOW, bank["psd"], bank["data"], {0: bank["h_ref"]}, subbanks)
    oracle_case(case)
    g = gpu_search(case)
    try:
        want = np.abs(case.oracle["z"])
        for form in ("fp32", "bf16x3", "ols32"):
            tol = fir_tolerance(case, form, 1e-5 if form != "bf16x3" else 1e-3)
            buf, n = g.filter(form, 5.0, 1024, 1 << 14)
            tr = rfd.triggers_to_numpy(buf, n)
            ncmp, namb, dmax = compare_triggers(tr, want, 5.0, 1024, tol)
            assert namb <= ambiguity_bound(ncmp + namb, float(tol.min())) and dmax <= tol.max()
            print(f"\n[select] {len(subbanks)} sub-banks T={[sb.T for sb in subbanks]}, {form}: {n} triggers, "
                  f"{ncmp} windows identical, {namb} ambiguous")
            assert n >= 1
    finally:
        g.close()
