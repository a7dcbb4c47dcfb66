"""Batched dechirp (rfd_dechirp_refs): 40 references in shuffled,
non-contiguous slots (two launches of at most 32), each series bit-identical
to the one-reference call and within the FP32 target of the FP64 oracle,
sigma_ref to FP64 accuracy, and its argument errors."""
import numpy as np
import pytest

import synth
from oracle import pipeline as orc

pytestmark = pytest.mark.gpu

N, FS, F_LOW, MAX_REFS, NREF = 8192, 2048.0, 30.0, 64, 40


@pytest.fixture(scope="module")
def setup(rfd):
    import torch
    rng = np.random.default_rng(17)
    w = synth.Workload("dechirp-batch", 9, N, FS, F_LOW, 0, NREF, 0, "fp32", "nonspin")
    psd = synth.psd_array(N, FS)
    data = synth.spectrum_to_time(synth.make_noise_spectrum(w, rng), N, FS)
    params = [synth.WaveformParams(*m) for m in rng.uniform(1.2, 3.0, size=(NREF, 2))]
    H = synth.template_batch(w, params)
    slots = rng.permutation(MAX_REFS)[:NREF].tolist()
    plan = rfd.rfd_plan_create(psd, F_LOW, FS, N, MAX_REFS)
    d = torch.from_numpy(data).to("cuda")
    refs = {slot: torch.from_numpy(H[i]).to("cuda") for i, slot in enumerate(slots)}
    yield dict(plan=plan, data=data, d=d, H=H, slots=slots, refs=refs, psd=psd)
    rfd.rfd_plan_destroy(plan)


def test_batched_series_equal_single_calls_and_oracle(rfd, setup):
    c = setup
    plan = c["plan"]
    sig = rfd.rfd_dechirp_refs(plan, c["d"], c["refs"], True)
    batched = {r: rfd.rfd_get_zref(plan, r).cpu().numpy() for r in c["slots"]}
    single = {}
    for r in c["slots"]:
        rfd.rfd_dechirp(plan, None, c["refs"][r], r, False)
        single[r] = rfd.rfd_get_zref(plan, r).cpu().numpy()
    p = orc.prepare(c["psd"], c["data"], FS, F_LOW)
    worst = 0.0
    for i, r in enumerate(c["slots"]):
        assert np.array_equal(batched[r], single[r]), f"slot {r}"
        ref = orc.dechirp(p, c["H"][i])
        worst = max(worst, float(np.max(np.abs(batched[r].astype(np.complex128) - ref.z / ref.sigma))))
        assert abs(sig[r] - ref.sigma) <= 1e-12 * ref.sigma
    print(f"\n[dechirp batch] {NREF} references: max |dz_ref| = {worst:.3e}")
    assert worst <= 1e-5


def test_batched_dechirp_argument_errors(rfd, setup):
    import ctypes as C
    c = setup
    plan = c["plan"]
    h = c["refs"][c["slots"][0]]
    ptrs = (C.c_void_p * 2)(h.data_ptr(), h.data_ptr())
    for ids in ([3, 3], [3, MAX_REFS], [-1, 2]):
        arr = (C.c_int32 * 2)(*ids)
        assert rfd.rfd._lib.rfd_dechirp_refs(plan, None, 2, arr, ptrs, None) == rfd.RFD_E_INVALID
    arr = (C.c_int32 * 2)(1, 2)
    assert rfd.rfd._lib.rfd_dechirp_refs(plan, None, 0, arr, ptrs, None) == rfd.RFD_E_INVALID
    assert rfd.rfd._lib.rfd_dechirp_refs(plan, None, 2, None, ptrs, None) == rfd.RFD_E_INVALID
    nulls = (C.c_void_p * 2)(h.data_ptr(), None)
    assert rfd.rfd._lib.rfd_dechirp_refs(plan, None, 2, arr, nulls, None) == rfd.RFD_E_INVALID


def test_fp32_and_fp64_transform_passes_against_oracle(rfd, setup):
    """The default FP32 transform passes and the FP64 ones both meet 1e-5 on
    the normalised series; the FP32 error stays within a few units of FP32
    rounding of max |z_ref| (log2 N butterfly levels)."""
    c = setup
    plan = c["plan"]
    p = orc.prepare(c["psd"], c["data"], FS, F_LOW)
    errs = {}
    try:
        for fp64 in (False, True):
            rfd.rfd_plan_set_dechirp_fp64(plan, fp64)
            rfd.rfd_dechirp_refs(plan, c["d"], c["refs"], False)
            worst = 0.0
            for i, r in enumerate(c["slots"]):
                ref = orc.dechirp(p, c["H"][i])
                want = ref.z / ref.sigma
                got = rfd.rfd_get_zref(plan, r).cpu().numpy().astype(np.complex128)
                worst = max(worst, float(np.max(np.abs(got - want)) / np.max(np.abs(want))))
            errs[fp64] = worst
    finally:
        rfd.rfd_plan_set_dechirp_fp64(plan, False)
    print(f"\n[dechirp] max |dz|/max|z|: FP32 passes {errs[False]:.2e}, FP64 passes {errs[True]:.2e}")
    assert errs[True] <= 2.0 ** -23
    assert errs[False] <= 2.0 ** -24 * 4 * np.log2(N)


@pytest.mark.parametrize("log2n", [21, 22])
def test_long_segment_series_match_oracle(rfd, log2n):
    """Reference series at N = 2^21 and 2^22, where the row transforms of the
    FP32 passes are 2048 points long (four columns per workgroup there): three
    references in one batched call against the FP64 oracle."""
    import torch
    n = 1 << log2n
    rng = np.random.default_rng(log2n)
    w = synth.Workload(f"dechirp{log2n}", 9, n, FS, F_LOW, 0, 3, 0, "fp32", "nonspin")
    psd = synth.psd_array(n, FS)
    data = synth.spectrum_to_time(synth.make_noise_spectrum(w, rng), n, FS)
    params = [synth.WaveformParams(*m) for m in rng.uniform(2.0, 3.0, size=(3, 2))]
    H = synth.template_batch(w, params)
    plan = rfd.rfd_plan_create(psd, F_LOW, FS, n, 3)
    try:
        refs = {r: torch.from_numpy(H[r]).to("cuda") for r in range(3)}
        rfd.rfd_dechirp_refs(plan, torch.from_numpy(data).to("cuda"), refs, False)
        p = orc.prepare(psd, data, FS, F_LOW)
        worst = 0.0
        for r in range(3):
            ref = orc.dechirp(p, H[r])
            got = rfd.rfd_get_zref(plan, r).cpu().numpy().astype(np.complex128)
            worst = max(worst, float(np.max(np.abs(got - ref.z / ref.sigma))))
        print(f"\n[dechirp N=2^{log2n}] max |dz_ref| = {worst:.3e}")
        assert worst <= 1e-5
    finally:
        rfd.rfd_plan_destroy(plan)
