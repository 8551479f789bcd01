"""The paper's time-domain scheme (forward-Euler stepping of the boundary
charges, Section 3) on the same RC-line model, against the frequency-domain
solve: the time-domain system's transfer function is the collocation system
at every frequency; its step response starts at the capacitive (infinite
frequency) solution and settles at the DC solution; forward Euler converges
to the exact (eigen-decomposition) step response at first order."""
import numpy as np
import pytest

from oracle import collocation, green, timedomain
from paper_2605_13987_amd import workloads


@pytest.fixture(scope="module")
def system():
    cfg = workloads.uniform_pixel_32x32x64()
    cell, cols = cfg["cell"], cfg["columns"]
    A = collocation.collocation_matrix(cell, cols)
    eps = green.permittivity(cell)
    return A, cols, eps, timedomain.rc_line_system(A, cols, eps)


def test_transfer_function_is_the_collocation_system(system):
    A, cols, eps, (K, G, bs, be) = system
    for f in (0.0, 0.3e9, 1.25e9, 7e9, 19.9e9, 120e9):
        w = 2 * np.pi * f
        x = timedomain.transfer(K, G, bs, be, w)
        q, c = collocation.solve_frequency(A, cols, w, eps)
        assert np.linalg.norm(x[:-1] - q) <= 1e-12 * np.linalg.norm(q)
        assert abs(x[-1] - c) <= 1e-12 * abs(c)


def test_step_response_limits(system):
    A, cols, eps, (K, G, bs, be) = system
    x0, x_inf = timedomain.step_limits(K, G, bs, be)
    # x(0+): the infinite-frequency response; x(inf): the DC response
    hf = timedomain.transfer(K, G, bs, be, 2 * np.pi * 1e19)
    assert np.linalg.norm(hf.real - x0) <= 1e-6 * np.linalg.norm(x0)
    q0, c0 = collocation.solve_frequency(A, cols, 0.0, eps)
    assert np.linalg.norm(x_inf[:-1] - q0.real) <= 1e-12 * np.linalg.norm(q0)
    x, lam = timedomain.step_response_exact(K, G, bs, be, [0.0, 5e-9])
    assert np.linalg.norm(x[0] - x0) <= 1e-9 * np.linalg.norm(x0)
    assert np.linalg.norm(x[1] - x_inf) <= 1e-9 * np.linalg.norm(x_inf)
    assert np.all(lam.real <= 1e-6 * np.max(np.abs(lam)))          # passive: no growing mode
    assert abs(np.sum(x[1][:-1])) <= 1e-12 * np.sum(np.abs(x[1][:-1]))   # neutrality kept


def test_forward_euler_converges_to_the_exact_step_response(system):
    A, cols, eps, (K, G, bs, be) = system
    t_rec = 20e-12
    errs = []
    for dt in (0.04e-12, 0.02e-12):
        every = int(round(t_rec / dt))
        xe = timedomain.step_response_euler(K, G, bs, be, dt, 10 * every, record_every=every)
        times = np.arange(xe.shape[0]) * t_rec
        xx, _ = timedomain.step_response_exact(K, G, bs, be, times)
        q_scale = np.max(np.abs(xx[:, :-1]))
        errs.append(np.max(np.abs(xe[1:, :-1] - xx[1:, :-1])) / q_scale)
    # first order: halving the step halves the error
    assert errs[1] <= 0.6 * errs[0] and errs[1] >= 0.4 * errs[0]
    assert errs[1] <= 1e-4
