"""Periodic Green's functions of the diamond cell (FP64, direct mode sums).

The paper's solver uses fundamental solutions to impose the boundary
conditions and a spectral method to extend the solution to the bulk
(abstract); the bulk step multiplies spectra by the squared wave-vector
(Section 3).  Both use the Fourier series of the periodic potential of a
Gaussian charge of unit magnitude in a uniform neutralising background:

    G(d)   = 1/(eps V) sum_{k in K} S(k) cos(k.d) / |k|^2         [V/C]
    E_G(d) = -grad G = 1/(eps V) sum_{k in K} S(k) k sin(k.d) / |k|^2
    S(k)   = exp(-(k_x^2 s_x^2 + k_y^2 s_y^2 + k_z^2 s_z^2)/2)

with k = 2 pi (m_x/L_x, m_y/L_y, m_z/L_z), k = 0 left out.  Two mode sets:

* the grid set (bulk field): |m_a| < N_a/2, i.e. the modes an N_a-node grid
  resolves, Nyquist planes left out; widths s = (1.5 h_x, 1.5 h_y,
  max(1.5 h_z, column node spacing));
* the converged set (boundary fit): an isotropic width s_c = r/4 of the source
  column and every mode with |m_a| <= floor(k_c L_a / 2 pi) + 1, k_c^2 s_c^2/2
  = 40, beyond which the terms are below exp(-40) of the leading ones; this is
  the full periodic sum to double precision and does not depend on the grid.
"""
from __future__ import annotations

import numpy as np

EPS0 = 8.8541878128e-12      # vacuum permittivity, F/m (CODATA 2018)
CUTOFF_EXPONENT = 40.0       # converged set: keep k^2 s^2 / 2 <= 40 (box)
COLLOCATION_WIDTH_FRACTION = 0.25


def axis_modes(n: int) -> np.ndarray:
    """Signed mode numbers m with |m| < n/2 along one axis (grid set)."""
    return np.arange(-(n // 2) + 1, n // 2)


def converged_axis_modes(length: float, width: float) -> np.ndarray:
    kc = np.sqrt(2.0 * CUTOFF_EXPONENT) / width
    mmax = int(np.floor(kc * length / (2.0 * np.pi))) + 1
    return np.arange(-mmax, mmax + 1)


def spacing(cell):
    L, N = cell["L"], cell["N"]
    return tuple(L[a] / N[a] for a in range(3))


def node_spacing(col) -> float:
    return abs(col["z_free"] - col["z_contact"]) / (col["n_colloc"] - 1)


def smoothing_widths(cell, columns):
    """Bulk-field Gaussian widths (s_x, s_y, s_z).

    1.5 h in-plane; along z at least the largest column node spacing, so that
    a column's row of point charges radiates like a smooth line charge.
    """
    h = spacing(cell)
    dz = max(node_spacing(c) for c in columns)
    return (1.5 * h[0], 1.5 * h[1], max(1.5 * h[2], dz))


def collocation_width(col) -> float:
    """Isotropic width of a column's source charges in the boundary fit."""
    return COLLOCATION_WIDTH_FRACTION * col["radius"]


def _as_wavevectors(cell, mx, my, mz):
    L = cell["L"]
    gx, gy, gz = np.meshgrid(mx, my, mz, indexing="ij")
    m = np.stack([gx.ravel(), gy.ravel(), gz.ravel()], axis=1)
    m = m[np.any(m != 0, axis=1)]
    return 2.0 * np.pi * m / np.asarray(L, dtype=np.float64)


def grid_mode_set(cell):
    """Wave-vectors of the grid set, (n_modes, 3)."""
    N = cell["N"]
    return _as_wavevectors(cell, *(axis_modes(N[a]) for a in range(3)))


def converged_mode_set(cell, width):
    L = cell["L"]
    return _as_wavevectors(cell, *(converged_axis_modes(L[a], width) for a in range(3)))


def permittivity(cell):
    return cell["eps_r"] * EPS0


def _spectral_weight(k, s):
    k2 = np.sum(k * k, axis=1)
    return np.exp(-0.5 * np.sum((k * np.asarray(s, dtype=np.float64)) ** 2, axis=1)) / k2


def potential(d, cell, s, k=None, chunk=1 << 22):
    """G(d) for displacements d (n, 3); mode set k (default: grid set)."""
    d = np.atleast_2d(np.asarray(d, dtype=np.float64))
    if k is None:
        k = grid_mode_set(cell)
    if np.isscalar(s):
        s = (s, s, s)
    w = _spectral_weight(k, s)
    vol = float(np.prod(cell["L"]))
    out = np.empty(d.shape[0])
    step = max(1, chunk // k.shape[0])
    for i in range(0, d.shape[0], step):
        out[i:i + step] = np.cos(d[i:i + step] @ k.T) @ w
    return out / (permittivity(cell) * vol)


def field(d, cell, s, k=None, chunk=1 << 22):
    """E_G(d) = -grad G(d) for displacements d (n, 3); mode set k (default: grid set)."""
    d = np.atleast_2d(np.asarray(d, dtype=np.float64))
    if k is None:
        k = grid_mode_set(cell)
    if np.isscalar(s):
        s = (s, s, s)
    w = _spectral_weight(k, s)
    vol = float(np.prod(cell["L"]))
    out = np.empty((d.shape[0], 3))
    step = max(1, chunk // k.shape[0])
    for i in range(0, d.shape[0], step):
        out[i:i + step] = (np.sin(d[i:i + step] @ k.T) * w) @ k
    return out / (permittivity(cell) * vol)
