"""Peak find and trigger accumulation (the last two stages of Table II).

Test infrastructure only (see package header).

Reading (the paper names the stages only): windows are fixed, non-overlapping
[qW, (q+1)W) aligned to n = 0; in each window the sample of largest rho^2 is
the peak (lowest index on exact ties); a trigger is emitted when that peak's
rho exceeds the threshold strictly.  Triggers are ordered by (template,
sample).
"""
import numpy as np


def cluster(rho, threshold, window):
    """[(sample, rho)] for one template's normalised SNR series (float64)."""
    rho = np.asarray(rho, dtype=np.float64)
    n = rho.size
    out = []
    for q0 in range(0, n, window):
        seg = rho[q0:q0 + window]
        r2 = seg * seg
        k = int(np.argmax(r2))            # first maximum = lowest index
        if seg[k] > threshold:
            out.append((q0 + k, float(seg[k])))
    return out


def cluster_brute(rho, threshold, window):
    """Pure-Python loop version (for pinning cluster() on small arrays)."""
    out = []
    n = len(rho)
    q0 = 0
    while q0 < n:
        best, bi = -1.0, -1
        for m in range(q0, min(n, q0 + window)):
            v = float(rho[m]) ** 2
            if v > best:
                best, bi = v, m
        if float(rho[bi]) > threshold:
            out.append((bi, float(rho[bi])))
        q0 += window
    return out


def window_ambiguity(rho, threshold, window, tau):
    """Per-window flag: True when a tolerance tau could change the outcome.

    A window is ambiguous when |rho_max - threshold| <= tau (the threshold
    decision may flip), or when it holds a trigger and the gap from rho_max
    to the largest rho at any other index of the window is <= 2 tau (a
    different sample may win).  Below threshold by more than tau, near-ties
    do not matter: no trigger either way.
    """
    rho = np.asarray(rho, dtype=np.float64)
    n = rho.size
    flags = []
    for q0 in range(0, n, window):
        seg = rho[q0:q0 + window]
        k = int(np.argmax(seg))
        top = seg[k]
        if seg.size > 1:
            rest = np.delete(seg, k)
            gap = top - rest.max()
        else:
            gap = np.inf
        flags.append(bool(abs(top - threshold) <= tau or (top > threshold and gap <= 2 * tau)))
    return np.array(flags, dtype=bool)
