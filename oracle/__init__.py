"""FP64 CPU oracle for ratio-filter dechirping (arXiv:2601.18835).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the GPU
library (no kernels, headers, tables or helpers); it consumes the same seeded
inputs from ``synth`` and nothing else.

Everything is plain numpy in float64 / complex128.  Library primitives used as
single steps: ``numpy.fft`` (a discrete Fourier transform), ``numpy.linalg``
(least squares, Cholesky, triangular solves).  Each function cites the part of
the paper it follows.  Readings where the paper is silent are marked
"Reading:" in the docstrings.

Modules
-------
spectral   Eq. 1 discretised: PSD weights, data transform, matched filter
           (the FINDCHIRP definition), sigma^2.
taps       Sec. V.A: weighted ridge least-squares ratio taps (direct chi^2
           form and normal-equation form), the windowed variant,
           Sec. VI.B fitted-template norms in both forms.
fir        Eq. 3: the ratio FIR by direct summation.
cluster    Table II peak find / trigger accumulation: threshold and one
           trigger per fixed window.
pipeline   End-to-end helpers per workload (used by tests and the CPU
           baseline timing).
surrogate  The learned tap surrogate (MLP forward / backward / Adam, SVD basis)
           in FP64.
chisq      Sec. VI.C: the ratio-filtered chi^2 consistency test (equal
           reference-power bands, band SNRs of the fitted template, shares).
"""
