"""Caller-owned workspace (rfd_plan_workspace_size / rfd_plan_set_workspace):
the filtering calls give the same triggers from a torch-owned buffer as from
library-owned scratch, refuse calls that need more than the sizes given,
refuse replays of graphs captured before the switch, and return to
library-owned scratch on NULL."""
import numpy as np
import pytest

from gpu_cases import gpu_search, ragged_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ragged(rfd):
    case = ragged_case()
    s = gpu_search(case)
    yield case, s
    rfd.rfd_plan_set_workspace(s.plan, None)
    s.close()


def _all(rfd, s, case, filt):
    out = {}
    for form in ("fp32", "bf16x3", "ols32"):
        buf, n = s.filter(form, 3.0, 300, 1 << 16)
        out[form] = rfd.triggers_to_numpy(buf, n)
    buf, n = s.filter("fp32", 0.0, 1, case.n_templates * case.n)
    out["series"] = rfd.triggers_to_numpy(buf, n)
    buf, n = rfd.findchirp_filter(s.plan, None, filt, 3.0, 300, 1 << 16)
    out["findchirp"] = rfd.triggers_to_numpy(buf, n)
    return out


def test_workspace_gives_identical_triggers(rfd, ragged):
    import torch
    case, s = ragged
    H = torch.from_numpy(np.concatenate([sb.H for sb in case.subbanks])).to("cuda")
    filt, _ = rfd.rfd_findchirp_prepare(s.plan, H)
    owned = _all(rfd, s, case, filt)
    nbytes = rfd.rfd_plan_workspace_size(s.plan, case.n_templates, 1, True)
    assert nbytes % 256 == 0 and nbytes >= case.n_templates * case.n * 8
    ws = torch.full((nbytes,), 0xAB, dtype=torch.uint8, device="cuda")
    rfd.rfd_plan_set_workspace(s.plan, ws, case.n_templates, 1, True)
    try:
        ext = _all(rfd, s, case, filt)
        for k in owned:
            assert np.array_equal(owned[k], ext[k]), k
        # the slots really live in the caller's buffer: validation mode writes every one
        s.filter("fp32", 0.0, 1, case.n_templates * case.n)
        torch.cuda.synchronize()
        slots = ws[:case.n_templates * case.n * 8].view(torch.int64)
        assert int((slots == 0).sum()) == 0
    finally:
        rfd.rfd_plan_set_workspace(s.plan, None)
    again = _all(rfd, s, case, filt)
    for k in owned:
        assert np.array_equal(owned[k], again[k]), k


def test_workspace_limits_are_enforced(rfd, ragged):
    import torch
    case, s = ragged
    W = 300
    nbytes = rfd.rfd_plan_workspace_size(s.plan, case.n_templates, W, False)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    with pytest.raises(rfd.RfdError) as e:            # too small for the sizes asked
        rfd.rfd_plan_set_workspace(s.plan, ws[:nbytes - 256], case.n_templates, W, False)
    assert e.value.code == rfd.RFD_E_INVALID
    with pytest.raises(rfd.RfdError) as e:            # misaligned
        rfd.rfd_plan_set_workspace(s.plan, ws[8:], case.n_templates, W, False)
    assert e.value.code == rfd.RFD_E_INVALID
    rfd.rfd_plan_set_workspace(s.plan, ws, case.n_templates, W, False)
    try:
        buf, n = s.filter("fp32", 3.0, W, 1 << 16)     # fits
        with pytest.raises(rfd.RfdError) as e:        # a smaller window needs more slots
            s.filter("fp32", 3.0, 17, 1 << 16)
        assert e.value.code == rfd.RFD_E_NOMEM and "workspace" in str(e.value)
        H = torch.from_numpy(case.subbanks[0].H).to("cuda")
        filt, _ = rfd.rfd_findchirp_prepare(s.plan, H)
        if rfd.rfd_plan_info_get(s.plan)["n"] > 4096:   # FINDCHIRP needs its intermediate
            with pytest.raises(rfd.RfdError) as e:
                rfd.findchirp_filter(s.plan, None, filt, 3.0, W, 1 << 16)
            assert e.value.code == rfd.RFD_E_NOMEM
        buf2, n2 = s.filter("fp32", 3.0, W, 1 << 16)  # the refused calls changed nothing
        assert np.array_equal(rfd.triggers_to_numpy(buf, n), rfd.triggers_to_numpy(buf2, n2))
    finally:
        rfd.rfd_plan_set_workspace(s.plan, None)


def test_graph_captured_before_the_switch_is_refused(rfd, ragged):
    import torch
    case, s = ragged
    cap = 1 << 16
    out = torch.empty(cap * 32, dtype=torch.uint8, device="cuda")
    g = rfd.rfd_segment_graph_create(s.plan, s.taps, "fp32", 3.0, 300, s.data, s.h_ref, out, cap)
    try:
        n0 = rfd.rfd_segment_graph_launch(g)
        want = rfd.triggers_to_numpy(out, n0)
        nbytes = rfd.rfd_plan_workspace_size(s.plan, case.n_templates, 300, False)
        ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        rfd.rfd_plan_set_workspace(s.plan, ws, case.n_templates, 300, False)
        try:
            with pytest.raises(rfd.RfdError) as e:
                rfd.rfd_segment_graph_launch(g)
            assert e.value.code == rfd.RFD_E_STATE
            g2 = rfd.rfd_segment_graph_create(s.plan, s.taps, "fp32", 3.0, 300, s.data, s.h_ref, out, cap)
            try:
                for _ in range(2):
                    n2 = rfd.rfd_segment_graph_launch(g2)
                    assert np.array_equal(rfd.triggers_to_numpy(out, n2), want)
            finally:
                rfd.rfd_graph_destroy(g2)
        finally:
            rfd.rfd_plan_set_workspace(s.plan, None)
    finally:
        rfd.rfd_graph_destroy(g)
        s.dechirp_all()
