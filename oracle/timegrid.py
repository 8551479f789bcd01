"""Frequency grid and the real inverse Fourier quadrature to time samples (FP64).

The weighting field is driven by a voltage impulse on the readout contact, so
its spectrum is the per-frequency response to a unit applied voltage.  With
the convention exp(+i w t) and a real response (X(-f) = conj X(f)), the time
signal on the grid f_j = j df, t_n = n dt is

    x(t_n) = df sum_j c_j Re[ X(f_j) exp(+2 pi i f_j t_n) ]

with c_0 = 1, c_j = 2 inside the band, and c_last = 1 when the last frequency
is the Nyquist frequency 1/(2 dt) (else 2).  When df = 1/(2 (n_freq - 1) dt)
this is exactly a length-2(n_freq-1) real inverse DFT; the result is periodic
with period 1/df.
"""
from __future__ import annotations

import numpy as np


def frequencies(spectrum) -> np.ndarray:
    return spectrum["df"] * np.arange(spectrum["n_freq"])


def quadrature_weights(spectrum) -> np.ndarray:
    nf = spectrum["n_freq"]
    c = np.full(nf, 2.0)
    c[0] = 1.0
    if nf > 1:
        f_last = spectrum["df"] * (nf - 1)
        nyq = 0.5 / spectrum["dt"]
        if abs(f_last - nyq) <= 1e-9 * nyq:
            c[-1] = 1.0
    return c


def to_time(values, spectrum) -> np.ndarray:
    """Map a spectrum (n_freq, ...) to time samples (n_time, ...)."""
    f = frequencies(spectrum)
    t = spectrum["dt"] * np.arange(spectrum["n_time"])
    c = quadrature_weights(spectrum)
    ker = spectrum["df"] * c[None, :] * np.exp(2j * np.pi * np.outer(t, f))   # (nt, nf)
    v = np.asarray(values).reshape(f.size, -1)
    out = (ker @ v).real
    return out.reshape((t.size,) + np.asarray(values).shape[1:])
