"""Pins of the electronics oracle (front-end convolution, noise, features)
against closed forms: the discrete convolution of two sampled exponentials is
a geometric sum; an identity response returns the current; the parabola
through three samples of a parabola is the parabola itself (its vertex is
recovered exactly); linear interpolation on a line is exact."""
import numpy as np
import pytest

from oracle import electronics


def test_convolution_of_sampled_exponentials_is_a_geometric_sum():
    dt, a, b, n_t = 10e-12, 130e-12, 47e-12, 200
    n = np.arange(n_t)
    cur = np.exp(-n * dt / a)
    g = np.exp(-n * dt / b)
    v = electronics.shape_signal(cur, g, dt)[0]
    r = np.exp(dt / b - dt / a)
    closed = dt * np.exp(-n * dt / b) * (1.0 - r ** (n + 1)) / (1.0 - r)
    assert np.max(np.abs(v - closed) / np.abs(closed)) <= 1e-12


def test_identity_response_and_noise():
    rng = np.random.default_rng(5)
    dt = 10e-12
    cur = rng.standard_normal((3, 64))
    noise = rng.standard_normal((3, 64))
    g = np.zeros(64)
    g[0] = 1.0 / dt
    v = electronics.shape_signal(cur, g, dt, noise=noise, sigma=0.25)
    assert np.max(np.abs(v - (cur + 0.25 * noise))) <= 1e-14


def test_peak_time_is_the_vertex_of_a_sampled_parabola():
    dt, t0, c = 10e-12, 1.237e-9, 3.0
    n = np.arange(300)
    v = c - ((n * dt - t0) / 1e-9) ** 2
    f = electronics.features(v, dt, 0.5)[0]
    assert f[1] == pytest.approx(t0, rel=0, abs=1e-21)
    # the sign is taken from the extremum: the mirrored signal has the same times
    g = electronics.features(-v, dt, 0.5)[0]
    assert g[0] == pytest.approx(-f[0]) and g[1] == f[1] and g[2] == f[2]


def test_constant_fraction_time_on_a_linear_ramp():
    dt, slope, n_p = 10e-12, 2.0e9, 120
    n = np.arange(200)
    v = np.where(n <= n_p, slope * n * dt, slope * n_p * dt - 0.5 * slope * (n - n_p) * dt)
    for frac in (0.2, 0.5, 0.77):
        amp, t_peak, t_cfd = electronics.features(v, dt, frac)[0]
        assert amp == pytest.approx(slope * n_p * dt)
        assert t_cfd == pytest.approx(frac * amp / slope, rel=1e-12)


def test_no_crossing_and_zero_signal():
    dt = 10e-12
    v = np.array([5.0, 6.0, 7.0, 3.0])                   # already above half the peak at n = 0
    assert np.isnan(electronics.features(v, dt, 0.5)[0][2])
    z = electronics.features(np.zeros(16), dt, 0.5)[0]
    assert z[0] == 0.0 and np.isnan(z[2])


def test_nan_samples_name_the_first_nan():
    # a NaN in |v| counts as the largest value: the peak is the first NaN
    # sample, the amplitude NaN, the peak time that sample's time (no parabola
    # through NaN), and there is no constant-fraction crossing
    dt = 10e-12
    v = np.array([[1.0, 3.0, np.nan, 9.0, np.nan, 2.0], [np.nan] * 6])
    f = electronics.features(v, dt, 0.5)
    assert np.isnan(f[0, 0]) and f[0, 1] == 2 * dt and np.isnan(f[0, 2])
    assert np.isnan(f[1, 0]) and f[1, 1] == 0.0 and np.isnan(f[1, 2])
