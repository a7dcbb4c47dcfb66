"""Out-of-memory paths, forced from the host: rfd_debug_fail_allocation
makes the k-th device allocation of the library fail.  For every k up to the
number of allocations a whole search makes (plan, taps, dechirp, direct and
overlap-save filtering, FINDCHIRP, a stream), the call that meets the failure
reports RFD_E_NOMEM, everything created so far is destroyed, and no device
memory stays behind; the same search then runs to the same triggers."""
import numpy as np
import pytest

from gpu_cases import ragged_case

pytestmark = pytest.mark.gpu


def _search(rfd, case, torch):
    """A whole search through the C ABI; returns its triggers.  Destroys
    whatever it created, also when a call fails."""
    plan = taps = st = None
    offsets = np.concatenate([[0], np.cumsum([sb.H.shape[0] for sb in case.subbanks])]).astype(np.int64)
    try:
        plan = rfd.rfd_plan_create(case.psd, case.f_low, case.fs, case.n, 2)
        taps = rfd.rfd_taps_create(plan, offsets, [sb.ref for sb in case.subbanks], [sb.T for sb in case.subbanks],
                                   [sb.k0 for sb in case.subbanks])
        h_ref = {r: torch.from_numpy(h).cuda() for r, h in case.refs.items()}
        for b, sb in enumerate(case.subbanks):
            rfd.rfd_make_taps(plan, taps, b, h_ref[sb.ref], torch.from_numpy(sb.H).cuda(), 0,
                              rfd.RFD_TAPS_LS if sb.method == "ls" else rfd.RFD_TAPS_WINDOW)
        data = torch.from_numpy(case.data).cuda()
        rfd.rfd_dechirp_refs(plan, data, h_ref, False)
        out = {}
        for form in ("fp32", "ols32", "bf16x3"):
            buf, n = rfd.rfd_filter_bank(plan, taps, form, 3.0, 300, 1 << 14)
            out[form] = rfd.triggers_to_numpy(buf, n)
        filt, _ = rfd.rfd_findchirp_prepare(plan, torch.from_numpy(case.subbanks[0].H).cuda())
        buf, n = rfd.findchirp_filter(plan, data, filt, 3.0, 300, 1 << 14)
        out["findchirp"] = rfd.triggers_to_numpy(buf, n)
        st = rfd.rfd_stream_create(plan, taps, h_ref, 1024)
        rfd.rfd_stream_prime(st, data)
        buf, n, _ = rfd.rfd_stream_push(st, data[:1024], "ols32", 3.0, 300, 1 << 14)
        out["stream"] = rfd.triggers_to_numpy(buf, n)
        return out
    finally:
        if st is not None:
            rfd.rfd_stream_destroy(st)
        if taps is not None:
            rfd.rfd_taps_destroy(taps)
        if plan is not None:
            rfd.rfd_plan_destroy(plan)


def test_every_allocation_failure_is_reported_and_released(rfd):
    import torch
    case = ragged_case()
    want = _search(rfd, case, torch)
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    free0 = torch.cuda.mem_get_info()[0]
    failed = 0
    k = 0
    try:
        while k < 400:
            rfd.rfd_debug_fail_allocation(k)
            try:
                _search(rfd, case, torch)
            except rfd.RfdError as e:
                assert e.code == rfd.RFD_E_NOMEM, (k, e)
                failed += 1
                k += 1
                continue
            finally:
                rfd.rfd_debug_fail_allocation(-1)
            break                       # k is past the last allocation: the search completed
    finally:
        rfd.rfd_debug_fail_allocation(-1)
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    free1 = torch.cuda.mem_get_info()[0]
    print(f"\n[alloc failure] {failed} allocation sites failed in turn; device memory "
          f"{(free0 - free1) / 2**20:+.1f} MiB after all of them")
    assert failed >= 20
    assert free0 - free1 <= 64 << 20, "device memory left behind by failed calls"
    got = _search(rfd, case, torch)
    for key in want:
        assert np.array_equal(got[key], want[key]), key
