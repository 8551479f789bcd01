"""Pins of the frequency-to-time quadrature."""
import numpy as np

from oracle import timegrid


def test_full_period_identity(px32, px32_oracle):
    """Summing a full period (1/df = 40 dt at 1.25 GHz, 20 ps) of the time
    charges times dt returns the zero-frequency charges exactly."""
    spec = px32["spectrum"]
    period = int(round(1.0 / (spec["df"] * spec["dt"])))
    assert period == 40 and spec["n_time"] >= period
    qt = px32_oracle["q_t"]
    lhs = qt[:period].sum(axis=0) * spec["dt"]
    q0 = px32_oracle["q"][0].real
    assert np.max(np.abs(lhs - q0)) <= 1e-12 * np.max(np.abs(q0))


def test_nyquist_grid_is_a_real_inverse_dft():
    """With df = 1/(2 (n_f - 1) dt) the quadrature is a length-2(n_f-1) irfft."""
    rng = np.random.default_rng(5)
    nf, dt = 33, 10e-12
    spec = dict(n_freq=nf, df=1.0 / (2 * (nf - 1) * dt), n_time=2 * (nf - 1), dt=dt)
    X = rng.standard_normal(nf) + 1j * rng.standard_normal(nf)
    X[0] = X[0].real
    X[-1] = X[-1].real
    ref = np.fft.irfft(X, n=2 * (nf - 1)) * (2 * (nf - 1)) * spec["df"]
    got = timegrid.to_time(X, spec)
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_impulse_response_is_causal(px32, px32_oracle):
    """exp(+i w t) with a passive network gives a response concentrated after
    t = 0: over one period the readout charge's energy in the first half
    (0 < t < P/2) exceeds the wrapped negative-time half by a wide margin."""
    spec = px32["spectrum"]
    period = 40
    Q = px32_oracle["q_t"][:period, :64].sum(axis=1)
    pos = np.sum(Q[1:period // 2] ** 2)
    neg = np.sum(Q[period // 2 + 1:] ** 2)
    assert neg < 0.2 * pos
