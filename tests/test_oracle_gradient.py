"""Pins of the oracle's forward-mode derivatives: central differences of the
oracle's own forward pipeline (the FP64 reference the GPU adjoint is checked
against)."""
import numpy as np
import pytest

from oracle import collocation, field, gradient, green, pipeline, timegrid
from paper_2605_13987_amd import workloads


@pytest.fixture(scope="module")
def tiny():
    return workloads.small_pixel(k=21, n_xy=8, n_z=16, n_freq=6, n_time=12, n_pairs=4, n_colloc=6)


def _currents(cfg, columns, A=None):
    cell, spec = cfg["cell"], cfg["spectrum"]
    sol = collocation.solve_spectrum(cell, columns, spec, A=A)
    s = green.smoothing_widths(cell, columns)
    H = field.field_fft(cell, s, collocation.sources(columns), timegrid.to_time(sol["q"], spec))
    return pipeline.induced_current(H, cell, cfg["carriers"])


def test_radius_derivative_of_collocation_matrix_matches_central_differences(tiny):
    cell, cols = tiny["cell"], tiny["columns"]
    for w in range(len(cols)):
        r = cols[w]["radius"]
        h = 1e-4 * r
        prm = (w, "radius", 0)
        Ap = collocation.collocation_matrix(cell, gradient.perturbed_columns(cols, prm, r + h))
        Am = collocation.collocation_matrix(cell, gradient.perturbed_columns(cols, prm, r - h))
        fd = (Ap - Am) / (2 * h)
        dA = gradient.collocation_matrix_radius_derivative(cell, cols, w)
        assert np.linalg.norm(dA - fd) <= 1e-6 * np.linalg.norm(fd)
        # the radius moves only the rows and columns of its own column
        n0 = cols[0]["n_colloc"]
        other = slice(n0, None) if w == 0 else slice(0, n0)
        assert np.all(dA[other, other] == 0.0)


def test_current_jacobian_matches_central_differences(tiny):
    cell, cols = tiny["cell"], tiny["columns"]
    params = gradient.parameter_names(cols)
    assert len(params) == 7                     # readout: 1 rho + r; bias: 4 rho + r
    jac, i0 = gradient.current_jacobian(cell, cols, tiny["spectrum"], tiny["carriers"], params)
    A = collocation.collocation_matrix(cell, cols)
    assert np.allclose(_currents(tiny, cols, A), i0, rtol=0, atol=1e-14 * np.abs(i0).max())
    for prm in params:
        v = gradient.parameter_value(cols, prm)
        h = 1e-4 * v
        Ause = A if prm[1] == "rho" else None
        ip = _currents(tiny, gradient.perturbed_columns(cols, prm, v + h), Ause)
        im = _currents(tiny, gradient.perturbed_columns(cols, prm, v - h), Ause)
        fd = (ip - im) / (2 * h)
        err = np.linalg.norm(jac[prm] - fd) / np.linalg.norm(fd)
        assert err <= 1e-6, (prm, err)


def test_parallel_quarter_columns_share_one_conductivity_derivative(tiny):
    """The bias column's conductivity is the mean of 1/rho over its quarters, so
    rho_p^2 di/drho_p is the same for every quarter (all equal to -n d i/d sigma)."""
    cell, cols = tiny["cell"], tiny["columns"]
    params = [(1, "rho", p) for p in range(4)]
    jac, _ = gradient.current_jacobian(cell, cols, tiny["spectrum"], tiny["carriers"], params)
    scaled = [jac[prm] * cols[1]["resistivity"][prm[2]] ** 2 for prm in params]
    for s in scaled[1:]:
        assert np.linalg.norm(s - scaled[0]) <= 1e-12 * np.linalg.norm(scaled[0])


def test_pitch_central_difference_is_converged(tiny):
    """The pitch reference (central differences of the FP64 pipeline) does not
    move when the step is halved: its truncation and rounding errors are far
    below the GPU tolerances it is used with."""
    cell, cols = tiny["cell"], tiny["columns"]
    d1 = gradient.pitch_derivative(cell, cols, tiny["spectrum"], tiny["carriers"], 2e-4)
    d2 = gradient.pitch_derivative(cell, cols, tiny["spectrum"], tiny["carriers"], 1e-4)
    assert np.linalg.norm(d1 - d2) <= 1e-7 * np.linalg.norm(d2)
    # scaling by 1 reproduces the unscaled pipeline
    i1 = gradient.currents_at_scale(cell, cols, tiny["spectrum"], tiny["carriers"], 1.0)
    assert np.allclose(i1, _currents(tiny, cols), rtol=0, atol=1e-14 * np.abs(i1).max())

