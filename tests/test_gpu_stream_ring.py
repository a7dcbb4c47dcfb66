"""Streaming (Sec. VII.A) against the FP64 oracle: a ring of N samples primed
with one segment, then increments of a second segment pushed one by one.
After every push the ring holds a known mix of the two segments; the oracle
evaluates the whole circular series of that content, and the stream must
match it on the stretch it re-evaluated (reference series) and on the D
outputs it filtered (every FIR form, validation mode and thresholded
triggers).  The first push's output range wraps the ring's end."""
import numpy as np
import pytest

import synth
from gpu_cases import SB, Case, compare_triggers, fir_tolerance, oracle_case

pytestmark = pytest.mark.gpu

N, FS, F_LOW = 1 << 15, 2048.0, 30.0
TOL = {"fp32": 1e-5, "ols32": 1e-5, "bf16x3": 1e-3, "fp16x3": 1e-3}
# (reference, T, k0, templates): centred, off-centre and all-future lags
SPECS = [(0, 64, -32, 3), (1, 200, -100, 3), (0, 37, 5, 2), (1, 130, -129, 2)]


def _case(N=N):
    w = synth.Workload("stream", 11, N, FS, F_LOW, 0, 2, 0, "fp32", "nonspin")
    rng = np.random.default_rng(31)
    psd = synth.psd_array(N, FS)
    refs = {0: synth.taylorf2(synth.WaveformParams(8.0, 7.0), N, FS, F_LOW),
            1: synth.taylorf2(synth.WaveformParams(11.0, 9.5), N, FS, F_LOW)}
    H = []
    for ref, T, k0, count in SPECS:
        m = 8.0 if ref == 0 else 10.5
        H.append(synth.template_batch(w, [synth.WaveformParams(*x) for x in
                                          rng.uniform(m - 1.2, m + 1.2, size=(count, 2))]))
    seg = []
    for k in range(2):
        s = synth.make_noise_spectrum(w, np.random.default_rng(100 + k))
        h = H[1][0] if k == 1 else H[0][0]
        amp = synth.workloads.optimal_snr_amplitude(h, w, 14.0)
        n0 = 3000 + 2500 * k
        kk = np.arange(N // 2 + 1)
        s = s + amp * h * np.exp(-2j * np.pi * ((kk * n0) % N) / N)
        seg.append(synth.spectrum_to_time(s, N, FS))
    return psd, refs, H, seg


def _oracle(psd, refs, H, data, form, N=N):
    """The oracle's whole circular series of the ring content: reference
    series, each template's rho, and each template's tolerance (the stated
    target, or where larger the first-order rounding bound of its taps: the
    off-centre and all-past tap windows here have gains the ridge does not
    keep small)."""
    case = Case("stream", N, FS, F_LOW, psd, data, refs,
                [SB(ref, T, k0, Hb) for (ref, T, k0, _), Hb in zip(SPECS, H)])
    o = oracle_case(case)
    return o["refs"], np.abs(o["z"]), fir_tolerance(case, form, TOL[form])


@pytest.fixture(scope="module")
def stream_case(rfd):
    import torch
    from paper_2601_18835_amd.driver import RatioFilterSearch, SubBankSpec
    psd, refs, H, seg = _case()
    specs = [SubBankSpec(r, T, k0, c) for r, T, k0, c in SPECS]
    s = RatioFilterSearch(psd, F_LOW, FS, N, specs, max_refs=2)
    for r, h in refs.items():
        s.set_reference(r, h)
    for b, Hb in enumerate(H):
        s.make_taps(b, Hb)
    yield psd, refs, H, seg, s
    s.close()


@pytest.mark.parametrize("D", [2048, 1024])
@pytest.mark.parametrize("form", ["fp32", "ols32", "bf16x3", "fp16x3"])
def test_stream_pushes_match_whole_window_oracle(rfd, stream_case, form, D):
    import torch
    psd, refs, H, seg, s = stream_case
    st = rfd.rfd_stream_create(s.plan, s.taps, s.h_ref, D)
    try:
        info = rfd.rfd_stream_info(st)
        assert info["lag"] >= max(k0 + T for _, T, k0, _ in SPECS) and info["lag"] % 256 == 0
        assert info["zlen"] >= D + info["lag"] + max(-k0 for _, _, k0, _ in SPECS)
        ring = seg[0].copy()
        rfd.rfd_stream_prime(st, torch.from_numpy(ring).cuda())
        B = torch.from_numpy(seg[1]).cuda()
        nt = sum(c for *_, c in SPECS)
        for push in range(4):
            head = push * D
            ring[head:head + D] = seg[1][head:head + D]
            buf, n, start = rfd.rfd_stream_push(st, B[head:head + D], form, 0.0, 1, nt * D)
            new_head = head + D
            assert start == (new_head - D - info["lag"]) % N and n == nt * D
            zr, rho, tol = _oracle(psd, refs, H, ring, form)
            # reference series on the re-evaluated stretch
            pos = (new_head - info["zlen"] + np.arange(info["zlen"])) % N
            for r in refs:
                z = s.zref(r).cpu().numpy().astype(np.complex128)
                err = np.max(np.abs(z[pos] - zr[r].z[pos] / zr[r].sigma))
                assert err <= 1e-5, (push, r, err)
            # every output sample of the pushed stretch (validation mode)
            tr = rfd.triggers_to_numpy(buf, n)
            outs = (start + np.arange(D)) % N
            got = np.full((nt, N), np.nan)
            got[tr["tmpl"], tr["sample"]] = tr["rho"]
            assert not np.isnan(got[:, outs]).any()
            err_t = np.max(np.abs(got[:, outs] - rho[:, outs]), axis=1)
            print(f"\n[stream] {form} D={D} push {push}: outputs [{start}, +{D}) max |drho| {err_t.max():.2e} "
                  f"(worst err/tol {np.max(err_t / tol):.2f})")
            assert (err_t <= tol).all()
        # thresholded triggers of one more push against the oracle on its range
        head = 4 * D
        ring[head:head + D] = seg[1][head:head + D]
        buf, n, start = rfd.rfd_stream_push(st, B[head:head + D], form, 2.5, 512, 1 << 14)
        _, rho, tol = _oracle(psd, refs, H, ring, form)
        outs = (start + np.arange(D)) % N
        want = np.zeros_like(rho)
        want[:, outs] = rho[:, outs]
        tr = rfd.triggers_to_numpy(buf, n)
        assert np.isin(tr["sample"], outs).all()
        ncmp, namb, dmax = compare_triggers(tr, want, 2.5, 512, tol)
        print(f"[stream] {form} D={D}: {n} triggers, {ncmp} windows identical, {namb} ambiguous")
        assert n >= 1 and dmax <= tol.max()
        # the series store is now a mix of pushes: whole-segment filtering is refused
        with pytest.raises(rfd.RfdError) as e:
            s.filter(form, 6.0, 2048, 16)
        assert e.value.code == rfd.RFD_E_STATE
    finally:
        rfd.rfd_stream_destroy(st)


def test_stream_arguments_are_checked(rfd, stream_case):
    import torch
    psd, refs, H, seg, s = stream_case
    for D in (100, 0, N // 2):
        with pytest.raises(rfd.RfdError) as e:
            rfd.rfd_stream_create(s.plan, s.taps, s.h_ref, D)
        assert e.value.code == rfd.RFD_E_INVALID
    with pytest.raises(rfd.RfdError) as e:        # sub-banks use reference 1, which is missing
        rfd.rfd_stream_create(s.plan, s.taps, {0: s.h_ref[0]}, 2048)
    assert e.value.code == rfd.RFD_E_INVALID
    st = rfd.rfd_stream_create(s.plan, s.taps, s.h_ref, 2048)
    try:
        x = torch.zeros(2048, dtype=torch.float64, device="cuda")
        with pytest.raises(rfd.RfdError) as e:
            rfd.rfd_stream_push(st, x, "fp32", 6.0, 2048, 16)
        assert e.value.code == rfd.RFD_E_STATE      # not primed
    finally:
        rfd.rfd_stream_destroy(st)


def test_plan_and_taps_outlive_their_graphs_and_streams(rfd, stream_case):
    """Destroying a plan or taps object that a graph or stream still points at
    is refused (nothing freed); after the graph and stream go, it works."""
    import torch
    psd, refs, H, seg, s = stream_case
    data = torch.from_numpy(seg[0]).cuda()
    out = torch.empty(32 * 64, dtype=torch.uint8, device="cuda")
    st = rfd.rfd_stream_create(s.plan, s.taps, s.h_ref, 1024)
    g = rfd.rfd_range_graph_create(s.plan, s.taps, "fp32", 6.0, 2048, data, s.h_ref, N - 2048, 2048, out, 64)
    try:
        for destroy, obj in ((rfd.rfd_taps_destroy, s.taps), (rfd.rfd_plan_destroy, s.plan)):
            with pytest.raises(rfd.RfdError) as e:
                destroy(obj)
            assert e.value.code == rfd.RFD_E_STATE
        rfd.rfd_graph_destroy(g)
        g = None
        with pytest.raises(rfd.RfdError) as e:       # the stream still holds them
            rfd.rfd_taps_destroy(s.taps)
        assert e.value.code == rfd.RFD_E_STATE
    finally:
        if g is not None:
            rfd.rfd_graph_destroy(g)
        rfd.rfd_stream_destroy(st)
    # both usable again
    s.dechirp_all()
    s.filter("fp32", 6.0, 2048, 64)


@pytest.mark.parametrize("fp64", [False, True])
def test_stream_long_segment_matches_whole_window_oracle(rfd, fp64):
    """At N = 2^18 the stretch of 3072 lags takes the fused share path of the
    lag-restricted transform (N1 / C column groups times the lags fit the work
    buffer) with FP32 column transforms, and the direct path with FP64 ones;
    at N = 2^15 above only the direct path runs.  Reference series on the
    stretch and every output of the pushed second against the oracle."""
    import torch
    from paper_2601_18835_amd.driver import RatioFilterSearch, SubBankSpec
    n = 1 << 18
    D = 2048
    psd, refs, H, seg = _case(n)
    specs = [SubBankSpec(r, T, k0, c) for r, T, k0, c in SPECS]
    s = RatioFilterSearch(psd, F_LOW, FS, n, specs, max_refs=2)
    try:
        rfd.rfd_plan_set_dechirp_fp64(s.plan, fp64)
        for r, h in refs.items():
            s.set_reference(r, h)
        for b, Hb in enumerate(H):
            s.make_taps(b, Hb)
        st = rfd.rfd_stream_create(s.plan, s.taps, s.h_ref, D)
        try:
            info = rfd.rfd_stream_info(st)
            ring = seg[0].copy()
            rfd.rfd_stream_prime(st, torch.from_numpy(ring).cuda())
            B = torch.from_numpy(seg[1]).cuda()
            nt = sum(c for *_, c in SPECS)
            for push in range(3):
                head = push * D
                ring[head:head + D] = seg[1][head:head + D]
                buf, nn, start = rfd.rfd_stream_push(st, B[head:head + D], "ols32", 0.0, 1, nt * D)
                assert start == (head - info["lag"]) % n and nn == nt * D
                if push == 1:
                    continue
                zr, rho, tol = _oracle(psd, refs, H, ring, "ols32", n)
                pos = (head + D - info["zlen"] + np.arange(info["zlen"])) % n
                for r in refs:
                    z = s.zref(r).cpu().numpy().astype(np.complex128)
                    assert np.isfinite(z[pos]).all(), (push, r)
                    err = np.max(np.abs(z[pos] - zr[r].z[pos] / zr[r].sigma))
                    print(f"\n[stream 2^18] fp64={fp64} push {push} ref {r}: stretch max |dz| {err:.2e}")
                    assert err <= 1e-5, (push, r, err)
                tr = rfd.triggers_to_numpy(buf, nn)
                outs = (start + np.arange(D)) % n
                got = np.full((nt, n), np.nan)
                got[tr["tmpl"], tr["sample"]] = tr["rho"]
                assert not np.isnan(got[:, outs]).any()
                err_t = np.max(np.abs(got[:, outs] - rho[:, outs]), axis=1)
                assert (err_t <= tol).all(), err_t / tol
        finally:
            rfd.rfd_stream_destroy(st)
    finally:
        s.close()
