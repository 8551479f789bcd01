"""Readout electronics and timing features (workflow step "simulate
electronics and DAQ", Section 2): the induced current convolved with the
impulse response of the front end, plus noise, then per-track features.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain FP64 numpy.

Definitions (the paper names the step, not its model; the readings are the
caller's sampled impulse response g and noise samples):
* signal   v[n] = dt * sum_{m <= n} g[n - m] i[m] + sigma * noise[n]
           (causal rectangle-rule convolution on the time grid);
* peak     n_p = the first index of max |v|; amplitude A = v[n_p] (signed);
           with s = sign(A) and u = s v, the peak time is (n_p + d) dt with
           d = (u[n_p-1] - u[n_p+1]) / (2 (u[n_p-1] - 2 u[n_p] + u[n_p+1]))
           for 0 < n_p < N-1 and a negative denominator (the vertex of the
           parabola through the three samples), else d = 0;
* CFD time the last n_c < n_p with u[n_c] < f |A| (scanning back from the
           peak); t = (n_c + (f |A| - u[n_c]) / (u[n_c+1] - u[n_c])) dt; NaN
           if there is none, or if A = 0.
"""
import numpy as np


def shape_signal(current, response, dt, noise=None, sigma=0.0):
    """v[k][n] for currents (n_tracks, N), response (N,), noise (n_tracks, N)."""
    i = np.atleast_2d(np.asarray(current, dtype=np.float64))
    g = np.asarray(response, dtype=np.float64)
    n_t = i.shape[1]
    v = np.zeros_like(i)
    for n in range(n_t):
        # explicit causal sum over m <= n
        v[:, n] = dt * (i[:, :n + 1] @ g[n::-1])
    if noise is not None:
        v = v + sigma * np.asarray(noise, dtype=np.float64)
    return v


def features(v, dt, fraction):
    """(amplitude, t_peak, t_cfd) per row of v."""
    v = np.atleast_2d(np.asarray(v, dtype=np.float64))
    out = np.empty((v.shape[0], 3))
    n_t = v.shape[1]
    for k, row in enumerate(v):
        n_p = int(np.argmax(np.abs(row)))
        a = row[n_p]
        out[k, 0] = a
        if a == 0.0:
            out[k, 1] = n_p * dt
            out[k, 2] = np.nan
            continue
        u = np.sign(a) * row
        d = 0.0
        if 0 < n_p < n_t - 1:
            den = u[n_p - 1] - 2.0 * u[n_p] + u[n_p + 1]
            if den < 0.0:
                d = (u[n_p - 1] - u[n_p + 1]) / (2.0 * den)
        out[k, 1] = (n_p + d) * dt
        thr = fraction * abs(a)
        t_cfd = np.nan
        for n_c in range(n_p - 1, -1, -1):
            if u[n_c] < thr:
                t_cfd = (n_c + (thr - u[n_c]) / (u[n_c + 1] - u[n_c])) * dt
                break
        out[k, 2] = t_cfd
    return out
