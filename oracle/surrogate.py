"""FP64 oracle of the learned tap surrogate (an extension; not in the paper).

Test infrastructure only (see package header).

The surrogate maps template parameters p (4 numbers, scaled to [-1, 1]) to
coefficients on an orthonormal basis of whitened ratio taps:
    a'     = a exp(-i arg z),  z = ((M + lam I) a)[-k0]
             (a global phase, so that the fitted template's zero-lag overlap
             with the reference, the right-hand side b[-k0] of Sec. V.A's
             normal equations, is real and positive; the ratio filter's |z|
             and every match are unchanged by it, and it removes the fast
             phase rotation of the taps across a sub-bank),
    x(a')  = [Re v; Im v] / ||v||,   v = L^H a',  M + lam I = L L^H
             (whitening makes ||x_hat - x||^2 the fitted-template mismatch
             proxy of Sec. V.A's chi^2 metric),
    c      = B^T x                        (B: 2T x K, orthonormal columns),
    MLP    h1 = silu(W1 p + b1), h2 = silu(W2 h1 + b2), c_hat = W3 h2 + b3,
    loss   = mean over the batch of ||c_hat - c||^2,
    silu(z) = z / (1 + exp(-z)).
Weights are row-major [out, in].  Adam: the published update of Kingma & Ba
(2015) with bias correction.
"""
import numpy as np


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def init_params(sizes, rng):
    """He-style uniform init; returns [(W, b), ...] with W [out, in]."""
    out = []
    for fan_in, fan_out in zip(sizes[:-1], sizes[1:]):
        lim = np.sqrt(6.0 / fan_in)
        out.append((rng.uniform(-lim, lim, size=(fan_out, fan_in)), np.zeros(fan_out)))
    return out


def forward(params, x):
    """x [n, 4] -> (y [n, K], cache)."""
    (W1, b1), (W2, b2), (W3, b3) = params
    z1 = x @ W1.T + b1
    h1 = silu(z1)
    z2 = h1 @ W2.T + b2
    h2 = silu(z2)
    y = h2 @ W3.T + b3
    return y, (x, z1, h1, z2, h2)


def loss_and_grads(params, x, c):
    """Loss mean_i ||y_i - c_i||^2 and its gradients by the chain rule."""
    (W1, b1), (W2, b2), (W3, b3) = params
    y, (x, z1, h1, z2, h2) = forward(params, x)
    n = x.shape[0]
    r = y - c
    loss = float(np.sum(r * r) / n)
    dy = 2.0 * r / n
    dW3 = dy.T @ h2
    db3 = dy.sum(axis=0)
    dh2 = dy @ W3
    dz2 = dh2 * silu_grad(z2)
    dW2 = dz2.T @ h1
    db2 = dz2.sum(axis=0)
    dh1 = dz2 @ W2
    dz1 = dh1 * silu_grad(z1)
    dW1 = dz1.T @ x
    db1 = dz1.sum(axis=0)
    return loss, [(dW1, db1), (dW2, db2), (dW3, db3)]


def adam_step(params, grads, state, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (in place on copies); state = (step, m, v)."""
    step, m, v = state
    step += 1
    out_p, out_m, out_v = [], [], []
    for (P, G, Mm, Vv) in zip([q for pair in params for q in pair], [g for pair in grads for g in pair],
                              m, v):
        Mn = beta1 * Mm + (1 - beta1) * G
        Vn = beta2 * Vv + (1 - beta2) * G * G
        mh = Mn / (1 - beta1 ** step)
        vh = Vn / (1 - beta2 ** step)
        out_p.append(P - lr * mh / (np.sqrt(vh) + eps))
        out_m.append(Mn)
        out_v.append(Vn)
    new_params = [(out_p[0], out_p[1]), (out_p[2], out_p[3]), (out_p[4], out_p[5])]
    return new_params, (step, out_m, out_v)


def adam_init(params):
    flat = [q for pair in params for q in pair]
    return (0, [np.zeros_like(q) for q in flat], [np.zeros_like(q) for q in flat])


def input_features(phys):
    """(m1, m2, chi, e0) [n, 4] -> (chirp mass M eta^(3/5), eta = m1 m2 / M^2,
    chi, e0): the network's input coordinates."""
    p = np.asarray(phys, dtype=np.float64).reshape(-1, 4)
    m1, m2 = p[:, 0], p[:, 1]
    mt = m1 + m2
    eta = m1 * m2 / mt ** 2
    return np.stack([mt * eta ** 0.6, eta, p[:, 2], p[:, 3]], axis=1)


def scaled_inputs(phys, phys_train):
    """Features of phys mapped linearly onto [-1, 1] over the training set's
    range of each feature (a constant feature maps to -1)."""
    f = input_features(phys)
    ft = input_features(phys_train)
    lo, hi = ft.min(axis=0), ft.max(axis=0)
    span = np.where(hi > lo, hi - lo, 1.0)
    return 2.0 * (f - lo) / span - 1.0


def phase_align(a, M, lam, k0):
    """a exp(-i arg z) with z = ((M + lam I) a)[i0] (a: [n, T] complex);
    i0 = -k0 is the zero-lag tap, clamped into [0, T) when the tap window
    does not contain lag 0."""
    T = M.shape[0]
    i0 = min(max(-k0, 0), T - 1)
    z = (a @ (M + lam * np.eye(T)).T)[:, i0]
    return a * np.exp(-1j * np.angle(z))[:, None]


def whiten(a, L):
    """x = [Re v; Im v] / ||v|| with v = L^H a (a: [n, T] complex)."""
    v = a @ np.conj(L)          # rows: (L^H a)^T = a^T conj(L)
    x = np.concatenate([v.real, v.imag], axis=1)
    return x / np.linalg.norm(x, axis=1, keepdims=True)


def unwhiten(x, L):
    """a with L^H a = Re x + i Im x (scale irrelevant: taps are normalised later)."""
    T = L.shape[0]
    v = x[:, :T] + 1j * x[:, T:]
    return np.linalg.solve(np.conj(L).T, v.T).T


def basis_svd(X, K):
    """Top-K right singular vectors of the stacked whitened taps (2T x K)."""
    _, _, Vt = np.linalg.svd(X, full_matrices=False)
    return Vt[:K].T


def match(a_hat, a, M):
    """|a_hat^H M a| / sqrt(a_hat^H M a_hat * a^H M a) (the fitted templates'
    normalised overlap, maximised over phase, at zero lag)."""
    num = np.abs(np.einsum("ij,jk,ik->i", np.conj(a_hat), M, a))
    d1 = np.real(np.einsum("ij,jk,ik->i", np.conj(a_hat), M, a_hat))
    d2 = np.real(np.einsum("ij,jk,ik->i", np.conj(a), M, a))
    return num / np.sqrt(d1 * d2)
