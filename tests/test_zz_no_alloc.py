"""rfd_filter_bank_noalloc (static per-GPU scratch, no device allocation in
the call) against rfd_filter_bank on the same taps and segment: the same
kernels on the same inputs, so the triggers must agree bit for bit.  Two
calls in a row, the second with a smaller input (fewer templates and a
longer cluster window), each checked; then a call whose scratch would exceed
the static array is refused with RFD_E_NOMEM."""
import numpy as np
import pytest

from gpu_cases import SB, Case, gpu_search, ragged_case

pytestmark = pytest.mark.gpu


def _both(rfd, s, form, threshold, window, cap):
    import torch
    ref_buf, n_ref = s.filter(form, threshold, window, cap)
    want = rfd.triggers_to_numpy(ref_buf, n_ref)
    out = torch.empty(cap * 32, dtype=torch.uint8, device="cuda")
    out.fill_(0xAB)                      # stale bytes must not leak into the result
    _, n = rfd.rfd_filter_bank_noalloc(s.plan, s.taps, form, threshold, window, cap, out)
    got = rfd.triggers_to_numpy(out, n)
    return want, got


@pytest.mark.parametrize("form", ["fp32", "bf16x3", "fp16x3", "ols32"])
def test_noalloc_equals_filter_bank_twice(rfd, form):
    case = ragged_case()
    big = gpu_search(case)
    small_case = Case("ragged-small", case.n, case.fs, case.f_low, case.psd, case.data, case.refs,
                      [SB(sb.ref, sb.T, sb.k0, sb.H[:2], sb.method) for sb in case.subbanks[:2]])
    small = gpu_search(small_case)
    try:
        # first call: every template, validation mode (every sample is a trigger)
        want, got = _both(rfd, big, form, 0.0, 1, case.n_templates * case.n)
        print(f"\n[noalloc] {form} call 1: {len(got)} triggers ({case.n_templates} templates, W = 1)")
        assert len(got) == case.n_templates * case.n
        assert np.array_equal(got, want)
        # second call, smaller input: 4 templates, W = 300, a threshold
        want, got = _both(rfd, small, form, 2.5, 300, 1 << 12)
        print(f"[noalloc] {form} call 2: {len(got)} triggers ({small_case.n_templates} templates, W = 300)")
        assert len(got) >= 1
        assert np.array_equal(got, want)
    finally:
        small.close()
        big.close()


def test_noalloc_refuses_scratch_beyond_its_maximum(rfd):
    import torch
    from paper_2601_18835_amd.driver import RatioFilterSearch, SubBankSpec
    case = ragged_case()
    n = 1 << 20                   # 2^20 slots per template at W = 1: 8 MiB each, 5 templates exceed 32 MiB
    import synth
    w = synth.Workload("noalloc-big", 9, n, case.fs, case.f_low, 0, 1, 0, "fp32", "nonspin")
    psd = synth.psd_array(n, case.fs)
    h_ref = synth.taylorf2(synth.WaveformParams(6.0, 5.0), n, case.fs, case.f_low)
    H = synth.template_batch(w, [synth.WaveformParams(5.0 + 0.1 * k, 5.0) for k in range(5)])
    s = RatioFilterSearch(psd, case.f_low, case.fs, n, [SubBankSpec(0, 16, -8, 5)])
    try:
        s.set_reference(0, h_ref)
        s.make_taps(0, H)
        s.set_segment(synth.spectrum_to_time(synth.make_noise_spectrum(w, np.random.default_rng(1)), n, case.fs))
        s.dechirp_all()
        out = torch.empty(32 * 16, dtype=torch.uint8, device="cuda")
        with pytest.raises(rfd.RfdError) as e:
            rfd.rfd_filter_bank_noalloc(s.plan, s.taps, "fp32", 0.0, 1, 16, out)
        assert e.value.code == rfd.RFD_E_NOMEM
        # the same bank with 4 s windows fits, and agrees with rfd_filter_bank
        buf, n_ref = s.filter("fp32", 3.0, 8192, 1 << 12)
        out = torch.empty(32 * (1 << 12), dtype=torch.uint8, device="cuda")
        _, n_got = rfd.rfd_filter_bank_noalloc(s.plan, s.taps, "fp32", 3.0, 8192, 1 << 12, out)
        assert np.array_equal(rfd.triggers_to_numpy(out, n_got), rfd.triggers_to_numpy(buf, n_ref))
    finally:
        s.close()
