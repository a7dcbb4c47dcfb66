"""Learned tap surrogate at the learned-parts workload's own shape: N = 2^20
samples from 20 Hz, T = 1024 taps (four 256-tap blocks in the expansion, so
the per-block norm partials and their fixed-order sum are exercised), on one
sub-bank of the 65536-template (m1, m2, chi, e0) bank.  Inference (taps and
fitted norms), the match kernel and the exact-tap fallback against the FP64
oracle, with the oracle's basis and one set of BF16-exact weights."""
import numpy as np
import pytest

import synth
from oracle import spectral as osp
from oracle import surrogate as osg
from oracle import taps as otaps
from test_gpu_surrogate import H, K, U32, _phys, bf16_round, unpack

pytestmark = pytest.mark.gpu

N_TRAIN, N_TEST = 128, 96


@pytest.fixture(scope="module")
def long_case(rfd):
    import torch
    from paper_2601_18835_amd.driver import RatioFilterSearch, SubBankSpec, TapSurrogate
    w = synth.get_workload("surr512s")
    bank = synth.make_bank(w)
    sb = bank.subbanks[9]
    T, k0 = sb.taps, sb.k0
    assert T == 1024
    mc = [p.mchirp for p in sb.params]
    train = synth.workloads.draw_in_chirp_mass_range(w, min(mc), max(mc), N_TRAIN, stream=40)
    test = sb.params[:N_TEST]
    psd = synth.psd_array(w.n, w.fs)
    h_ref = synth.reference_waveform(w, sb)
    Htr = synth.template_batch(w, train)
    Hte = synth.template_batch(w, test)
    print(f"\n[surrogate T=1024] N={w.n}, ref {sb.ref}", flush=True)
    s = RatioFilterSearch(psd, w.f_low, w.fs, w.n, [SubBankSpec(0, T, k0, N_TEST)], max_refs=1)
    s.set_reference(0, h_ref)
    s.make_taps(0, s.to_dev(Hte))
    sur = TapSurrogate(s, 0, T, k0, N_TRAIN, n_basis=K, hidden=H, seed=5)
    sur.add_training_waveforms(Htr, 0)
    sur_taps = rfd.rfd_taps_create(s.plan, np.array([0, N_TEST], np.int64), [0], [T], [k0])
    wts = osp.psd_weights(psd, w.n, w.fs, w.f_low)
    M = otaps.gram(h_ref, wts, T)
    lam = otaps.DEFAULT_RIDGE_EPS * float(M[0, 0].real)
    L = np.linalg.cholesky(M + lam * np.eye(T))
    A_train = np.stack([otaps.ls_taps_normal(h, h_ref, wts, T, k0, M=M) for h in Htr])
    A_test = np.stack([otaps.ls_taps_normal(h, h_ref, wts, T, k0, M=M) for h in Hte])
    del Htr, Hte
    X = osg.whiten(osg.phase_align(A_train, M, lam, k0), L)
    B = osg.basis_svd(X, K).T.astype(np.float32)
    sur.fit(_phys(train))
    w0 = bf16_round(rfd.rfd_surrogate_state(sur.sur)["weights"])
    rfd.rfd_surrogate_set_state(sur.sur, weights=w0, basis=B)
    sur.make_taps(sur_taps, 0, _phys(test))
    torch.cuda.synchronize()
    P = sur.scale(_phys(test)).astype(np.float64)
    y, _ = osg.forward(unpack(w0), P)
    a_or = osg.unwhiten(y @ B.astype(np.float64), L)
    yield dict(s=s, sur=sur, sur_taps=sur_taps, M=M, lam=lam, A_test=A_test, a_or=a_or, T=T)
    rfd.rfd_taps_destroy(sur_taps)
    sur.close()
    s.close()


def test_long_inference_taps_and_norms(rfd, long_case):
    c = long_case
    T = c["T"]
    a_gpu = np.stack([rfd.rfd_taps_get(c["sur_taps"], j)[0] for j in range(N_TEST)])
    sig_gpu = np.array([rfd.rfd_taps_get(c["sur_taps"], j)[1] for j in range(N_TEST)])
    ev = np.linalg.eigvalsh(c["M"] + c["lam"] * np.eye(T))
    cond = float(np.sqrt(ev[-1] / ev[0]))
    tol = cond * 4 * np.sqrt(2 * H + K) * U32
    a_or = c["a_or"]
    rel = np.linalg.norm(a_gpu - a_or, axis=1) / np.linalg.norm(a_or, axis=1)
    sig_or = np.sqrt(np.real(np.einsum("ij,jk,ik->i", np.conj(a_or), c["M"], a_or)))
    srel = np.abs(sig_gpu - sig_or) / sig_or
    print(f"\n[surrogate T=1024] taps: max rel error {rel.max():.3e}; sigma_fit: max rel error {srel.max():.3e} "
          f"(cond(L) {cond:.1f}, tol {tol:.3e})")
    assert rel.max() <= tol
    assert srel.max() <= 2 * tol
    # every 256-tap block carries taps (the expansion really spans four blocks)
    for blk in range(T // 256):
        assert np.abs(a_gpu[:, 256 * blk:256 * (blk + 1)]).max() > 0


def test_long_match_and_fallback(rfd, long_case):
    import torch
    c = long_case
    m_gpu = rfd.rfd_taps_match(c["sur_taps"], c["s"].taps, 0, 0, N_TEST)
    m_or = osg.match(c["a_or"], c["A_test"], c["M"])
    err = float(np.max(np.abs(m_gpu - m_or)))
    print(f"\n[surrogate T=1024] match vs oracle: max |dm| = {err:.3e} (untrained mean {m_or.mean():.3f})")
    assert err <= 1e-3
    thr = float(np.median(m_gpu))
    n_fb = rfd.rfd_taps_fallback(c["sur_taps"], c["s"].taps, 0, 0, torch.from_numpy(m_gpu).cuda(), thr)
    fb = m_gpu < thr
    assert n_fb == int(fb.sum())
    after = rfd.rfd_taps_match(c["sur_taps"], c["s"].taps, 0, 0, N_TEST)
    np.testing.assert_allclose(after[fb], 1.0, atol=1e-12)
    assert np.array_equal(after[~fb], m_gpu[~fb])
