"""Pins of the oracle's Green's functions against Ewald sums (closed form)."""
import numpy as np
import pytest

import ewald
from oracle import collocation, green

UM = 1e-6


def _points(L, rng, n=12, r=5 * UM):
    pts = [np.zeros(3), np.array([r, 0, 0]), np.array([r, 0, 37 * UM]),
           np.array([0.5 * L[0], 0.5 * L[1], 0.5 * L[2]]), np.array([-0.3 * L[0], 0.45 * L[1], -0.49 * L[2]])]
    pts += list((rng.random((n, 3)) - 0.5) * np.asarray(L))
    return np.array(pts)


def test_ewald_helper_is_split_independent():
    L = (50 * UM, 50 * UM, 300 * UM)
    d = _points(L, np.random.default_rng(0))
    g1 = ewald.potential(d, L, 5.7, 1.25 * UM, b=10 * UM)
    g2 = ewald.potential(d, L, 5.7, 1.25 * UM, b=7 * UM)
    assert np.max(np.abs(g1 - g2)) <= 1e-13 * np.max(np.abs(g1))
    e1 = ewald.field(d, L, 5.7, 1.25 * UM, b=10 * UM)
    e2 = ewald.field(d, L, 5.7, 1.25 * UM, b=7 * UM)
    assert np.max(np.abs(e1 - e2)) <= 1e-12 * np.max(np.abs(e1))


def test_collocation_green_matches_ewald():
    """Converged mode sum of a width-r/4 Gaussian charge == Ewald sum, anisotropic cell."""
    cell = dict(L=(50 * UM, 50 * UM, 300 * UM), N=(32, 32, 64), eps_r=5.7, sigma_bulk=0.0)
    col = dict(radius=5 * UM)
    s = green.collocation_width(col)
    k = green.converged_mode_set(cell, s)
    d = _points(cell["L"], np.random.default_rng(1))
    g = green.potential(d, cell, s, k=k)
    ge = ewald.potential(d, cell["L"], cell["eps_r"], s)
    assert np.max(np.abs(g - ge)) <= 1e-12 * np.max(np.abs(ge))
    e = green.field(d, cell, s, k=k)
    ee = ewald.field(d, cell["L"], cell["eps_r"], s)
    assert np.max(np.abs(e - ee)) <= 1e-11 * np.max(np.abs(ee))


def test_grid_green_matches_ewald_within_band_leakage():
    """Grid-band-limited G and E_G (cubic box, s = 1.5 h) vs Ewald: only the
    modes beyond the grid's band differ, each damped by exp(-(1.5 pi)^2/2)."""
    n = 32
    Lc = 20 * UM
    cell = dict(L=(Lc, Lc, Lc), N=(n, n, n), eps_r=5.7, sigma_bulk=0.0)
    s = 1.5 * Lc / n
    d = _points(cell["L"], np.random.default_rng(2), r=2 * UM)
    g = green.potential(d, cell, s)
    ge = ewald.potential(d, cell["L"], cell["eps_r"], s)
    assert np.max(np.abs(g - ge)) <= 1e-4 * np.max(np.abs(ge))
    e = green.field(d, cell, s)
    ee = ewald.field(d, cell["L"], cell["eps_r"], s)
    assert np.max(np.abs(e - ee)) <= 2e-4 * np.max(np.abs(ee))
    # and the difference is real: dropping the band edge is visible at 1e-9
    assert np.max(np.abs(e - ee)) > 1e-9 * np.max(np.abs(ee))


def test_nested_collocation_matrix_equals_direct_sum(px32):
    A = collocation.collocation_matrix(px32["cell"], px32["columns"])
    rows = [0, 1, 31, 63, 64, 100, 127]
    cols = [0, 2, 40, 64, 65, 127]
    Ad = collocation.collocation_matrix_direct(px32["cell"], px32["columns"], rows, cols)
    assert np.max(np.abs(A[np.ix_(rows, cols)] - Ad)) <= 1e-12 * np.max(np.abs(Ad))


def test_collocation_matrix_entries_match_ewald(px32):
    A = collocation.collocation_matrix(px32["cell"], px32["columns"])
    x = collocation.collocation_points(px32["columns"])
    y = collocation.sources(px32["columns"])
    rng = np.random.default_rng(3)
    pairs = rng.integers(0, A.shape[0], size=(16, 2))
    for i, j in pairs:
        col = px32["columns"][0 if j < 64 else 1]
        ge = ewald.potential(x[i] - y[j], px32["cell"]["L"], px32["cell"]["eps_r"], green.collocation_width(col))
        assert abs(A[i, j] - ge[0]) <= 1e-12 * abs(A[0, 0])


def test_full_collocation_matrix_matches_ewald(px32):
    """Every entry of the oracle's A (in-plane lattice sums times a k_z
    series) against an Ewald sum of the same width-r/4 Gaussian charges,
    which shares none of that structure: A_ij = G(x_i - y_j) exactly."""
    cell, columns = px32["cell"], px32["columns"]
    A = collocation.collocation_matrix(cell, columns)
    x = collocation.collocation_points(columns)
    y = collocation.sources(columns)
    n = A.shape[0]
    assert n % len(columns) == 0
    m = n // len(columns)                               # sources per column, column by column
    Ae = np.empty_like(A)
    for w, col in enumerate(columns):
        js = np.arange(w * m, (w + 1) * m)
        d = (x[:, None, :] - y[None, js, :]).reshape(-1, 3)
        Ae[:, js] = ewald.potential(d, cell["L"], cell["eps_r"], green.collocation_width(col)).reshape(n, m)
    assert np.max(np.abs(A - Ae)) <= 1e-12 * np.max(np.abs(Ae))
