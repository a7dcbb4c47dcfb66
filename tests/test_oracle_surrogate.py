"""Pins for the FP64 surrogate oracle: gradients against central finite
differences, Adam against a hand-computed first step, whitening round trip,
the basis against the Eckart-Young optimum, the match bounds."""
import numpy as np
import pytest

from oracle import surrogate as sg

RNG = np.random.default_rng(99)


def small_net():
    params = sg.init_params([4, 7, 6, 5], RNG)
    params = [(W, RNG.standard_normal(b.shape) * 0.1) for W, b in params]
    x = RNG.uniform(-1, 1, size=(9, 4))
    c = RNG.standard_normal((9, 5))
    return params, x, c


def test_gradients_match_central_finite_differences():
    params, x, c = small_net()
    loss, grads = sg.loss_and_grads(params, x, c)
    h = 1e-6
    for li in range(3):
        for wi in range(2):
            P = params[li][wi]
            G = grads[li][wi]
            it = np.nditer(P, flags=["multi_index"])
            for _ in it:
                idx = it.multi_index
                old = P[idx]
                P[idx] = old + h
                lp, _ = sg.loss_and_grads(params, x, c)
                P[idx] = old - h
                lm, _ = sg.loss_and_grads(params, x, c)
                P[idx] = old
                fd = (lp - lm) / (2 * h)
                assert abs(fd - G[idx]) <= 1e-7 * max(1.0, abs(fd)), (li, wi, idx, fd, G[idx])


def test_silu_derivative():
    z = np.linspace(-6, 6, 101)
    h = 1e-6
    assert np.allclose((sg.silu(z + h) - sg.silu(z - h)) / (2 * h), sg.silu_grad(z), atol=1e-9)
    assert sg.silu(0.0) == 0.0 and abs(sg.silu(50.0) - 50.0) < 1e-12


def test_adam_first_step_moves_each_weight_by_lr_times_sign():
    params, x, c = small_net()
    loss, grads = sg.loss_and_grads(params, x, c)
    new, st = sg.adam_step(params, grads, sg.adam_init(params), lr=1e-3)
    for (P, _), (Q, _), (G, _) in zip(params, new, grads):
        # bias-corrected first step: m_hat = g, v_hat = g^2  ->  delta = -lr g / (|g| + eps)
        want = -1e-3 * G / (np.abs(G) + 1e-8)
        assert np.allclose(Q - P, want, atol=1e-15)
    assert st[0] == 1


def test_training_reduces_loss():
    params = sg.init_params([4, 32, 32, 3], RNG)
    x = RNG.uniform(-1, 1, size=(64, 4))
    c = np.stack([np.sin(x[:, 0]) + x[:, 1], x[:, 2] * x[:, 3], np.cos(x.sum(1))], axis=1)
    st = sg.adam_init(params)
    l0, _ = sg.loss_and_grads(params, x, c)
    for _ in range(300):
        l, g = sg.loss_and_grads(params, x, c)
        params, st = sg.adam_step(params, g, st, lr=3e-3)
    assert l < 0.05 * l0


def test_whitening_round_trip_and_norm():
    T = 12
    A = RNG.standard_normal((T, T)) + 1j * RNG.standard_normal((T, T))
    M = A @ np.conj(A).T + T * np.eye(T)
    L = np.linalg.cholesky(M)
    a = RNG.standard_normal((5, T)) + 1j * RNG.standard_normal((5, T))
    x = sg.whiten(a, L)
    assert np.allclose(np.linalg.norm(x, axis=1), 1.0)
    # ||L^H a||^2 = a^H M a
    v = a @ np.conj(L)
    assert np.allclose(np.sum(np.abs(v) ** 2, axis=1), np.real(np.einsum("ij,jk,ik->i", np.conj(a), M, a)))
    back = sg.unwhiten(x, L)
    ratio = back / a
    assert np.allclose(ratio, ratio[:, :1])            # same taps up to one real positive scale per row
    assert np.allclose(ratio.imag, 0, atol=1e-12) and (ratio.real > 0).all()


def test_basis_is_the_best_rank_k_subspace():
    X = RNG.standard_normal((200, 30)) @ RNG.standard_normal((30, 30))
    B = sg.basis_svd(X, 8)
    assert np.allclose(B.T @ B, np.eye(8), atol=1e-12)
    err_opt = np.linalg.norm(X - X @ B @ B.T) ** 2
    s = np.linalg.svd(X, compute_uv=False)
    assert abs(err_opt - np.sum(s[8:] ** 2)) <= 1e-9 * np.sum(s ** 2)     # Eckart-Young
    Q, _ = np.linalg.qr(RNG.standard_normal((30, 8)))
    assert np.linalg.norm(X - X @ Q @ Q.T) ** 2 >= err_opt


def test_match_bounds():
    T = 10
    A = RNG.standard_normal((T, T)) + 1j * RNG.standard_normal((T, T))
    M = A @ np.conj(A).T
    a = RNG.standard_normal((4, T)) + 1j * RNG.standard_normal((4, T))
    assert np.allclose(sg.match(a, a, M), 1.0)
    assert np.allclose(sg.match(3j * a, a, M), 1.0)           # phase and scale free
    b = RNG.standard_normal((4, T)) + 1j * RNG.standard_normal((4, T))
    m = sg.match(b, a, M)
    assert (m <= 1.0 + 1e-12).all() and (m >= 0).all()


def test_phase_align_is_the_zero_lag_overlap_phase():
    """For least-squares taps (M + lam I) a = b, so z = b[-k0], the weighted
    zero-lag inner product sum_i w_i h_j conj(h_ref) of Eq. 1's weights: the
    rotation follows from the spectra alone."""
    from oracle import spectral, taps as tp
    from synth.waveforms import WaveformParams, taylorf2
    from synth.psd import psd_array
    n, fs, f_low, T = 8192, 2048.0, 20.0, 32
    k0 = -(T // 2)
    w = spectral.psd_weights(psd_array(n, fs), n, fs, f_low)
    h_ref = taylorf2(WaveformParams(1.4, 1.4), n, fs, f_low)
    M = tp.gram(h_ref, w, T)
    lam = tp.DEFAULT_RIDGE_EPS * M[0, 0].real
    hs = [taylorf2(WaveformParams(1.4 + 0.01 * k, 1.39, e0=0.02 * k), n, fs, f_low) for k in range(4)]
    a = np.stack([tp.ls_taps_normal(h, h_ref, w, T, k0, M=M) for h in hs])
    al = sg.phase_align(a, M, lam, k0)
    zero_lag = np.array([np.sum(w * h * np.conj(h_ref)) for h in hs])
    rot = al / a
    assert np.allclose(np.abs(rot), 1.0, atol=1e-12)
    assert np.allclose(rot, rot[:, :1], atol=1e-12)
    assert np.allclose(rot[:, 0], np.exp(-1j * np.angle(zero_lag)), atol=1e-9)
    z = (al @ (M + lam * np.eye(T)).T)[:, -k0]
    assert np.allclose(z.imag, 0, atol=1e-9 * np.abs(z).max()) and (z.real > 0).all()
    assert np.allclose(sg.match(al, a, M), 1.0, atol=1e-12)


@pytest.mark.parametrize("T,k0", [(32, 5), (32, -40), (16, -16), (8, 0), (24, -23)])
def test_phase_align_outside_the_window_uses_the_nearest_lag(T, k0):
    """When the tap window [k0, k0 + T) does not contain lag 0, the phase
    reference is the weighted overlap at the window's lag nearest zero:
    m* = k0 for k0 > 0, m* = k0 + T - 1 for k0 + T - 1 < 0.  For least-squares
    taps (M + lam I) a = b, so that overlap is the cross-correlation
    sum_i w_i h_j conj(h_ref) exp(+2 pi i i m*/N) of the spectra, computed here
    directly by a loop over bins, independent of the taps."""
    from oracle import spectral, taps as tp
    from synth.waveforms import WaveformParams, taylorf2
    from synth.psd import psd_array
    n, fs, f_low = 4096, 2048.0, 20.0
    w = spectral.psd_weights(psd_array(n, fs), n, fs, f_low)
    h_ref = taylorf2(WaveformParams(1.4, 1.4), n, fs, f_low)
    M = tp.gram(h_ref, w, T)
    lam = tp.DEFAULT_RIDGE_EPS * M[0, 0].real
    hs = [taylorf2(WaveformParams(1.4 + 0.013 * k, 1.38, e0=0.03 * k), n, fs, f_low) for k in range(3)]
    a = np.stack([tp.ls_taps_normal(h, h_ref, w, T, k0, M=M) for h in hs])
    al = sg.phase_align(a, M, lam, k0)
    if k0 <= 0 <= k0 + T - 1:
        m_star = 0
    elif k0 > 0:
        m_star = k0
    else:
        m_star = k0 + T - 1
    bins = np.arange(w.size)
    want = []
    for h in hs:
        acc = 0j
        for i in bins[w > 0]:
            acc += w[i] * h[i] * np.conj(h_ref[i]) * np.exp(2j * np.pi * ((i * m_star) % n) / n)
        want.append(acc)
    rot = al / a
    assert np.allclose(np.abs(rot), 1.0, atol=1e-12)
    assert np.allclose(rot, rot[:, :1], atol=1e-12)
    assert np.allclose(rot[:, 0], np.exp(-1j * np.angle(np.array(want))), atol=1e-8)


def test_input_features_closed_forms():
    """Equal masses m: chirp mass m 2^(-1/5), eta = 1/4; swapping the masses
    changes nothing; training extremes map to -1 and +1, a constant feature
    to -1."""
    phys = np.array([[1.4, 1.4, 0.01, 0.1], [2.0, 1.0, -0.02, 0.0], [1.0, 2.0, -0.02, 0.0], [3.0, 3.0, 0.03, 0.2]])
    f = sg.input_features(phys)
    assert np.allclose(f[0, :2], [1.4 * 2 ** -0.2, 0.25], rtol=1e-15)
    assert np.allclose(f[3, :2], [3.0 * 2 ** -0.2, 0.25], rtol=1e-15)
    assert np.allclose(f[1], f[2]) and np.isclose(f[1, 1], 2.0 / 9.0)
    # chirp mass from the definition (m1 m2)^(3/5) / M^(1/5)
    assert np.isclose(f[1, 0], (2.0 * 1.0) ** 0.6 / 3.0 ** 0.2, rtol=1e-14)
    x = sg.scaled_inputs(phys, phys)
    assert np.allclose(x.min(axis=0)[:2], -1.0) and np.allclose(x.max(axis=0)[:2], 1.0)
    const = phys.copy()
    const[:, 3] = 0.3
    assert np.all(sg.scaled_inputs(const, const)[:, 3] == -1.0)
