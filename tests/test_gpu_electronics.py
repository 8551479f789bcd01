"""GPU parity of the electronics step (front-end response, noise, features).

The signal is compared with the FP64 oracle (1e-12 relative L2 for the double
instantiation, 1e-5 for float).  The features take integer decisions (the
peak sample, the crossing sample); as the oracle and the kernel would take
them on differently rounded signals, the oracle extracts them from the GPU's
own signal, and the times agree to 1e-9 dt (double) / 1e-3 dt (float).
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_common import context, rel_l2, rounded_carriers, say
from oracle import electronics as oel
from paper_2605_13987_amd import workloads, wt

pytestmark = pytest.mark.gpu

DT = 10e-12


@pytest.fixture(scope="module")
def ctx():
    c = context()
    yield c
    wt.wt_context_destroy(c)


def _run(ctx, precision, cur, g, noise, sigma, frac, raise_on_error=True, dt=DT):
    dt_ = torch.float64 if precision == wt.WT_F64 else torch.float32
    n_tr, n_t = cur.shape
    d_i = torch.from_numpy(np.ascontiguousarray(cur)).to("cuda", dt_)
    d_g = torch.from_numpy(np.ascontiguousarray(g)).to("cuda", dt_)
    d_n = None if noise is None else torch.from_numpy(np.ascontiguousarray(noise)).to("cuda", dt_)
    v = torch.empty((n_tr, n_t), dtype=dt_, device="cuda")
    f = torch.empty((n_tr, 3), dtype=dt_, device="cuda")
    st = wt.wt_electronics(ctx, precision, n_tr, n_t, dt, d_i.data_ptr(), d_g.data_ptr(),
                           0 if d_n is None else d_n.data_ptr(), sigma, frac, v.data_ptr(), f.data_ptr(),
                           raise_on_error=raise_on_error)
    torch.cuda.synchronize()
    return st, v.cpu().numpy().astype(np.float64), f.cpu().numpy().astype(np.float64)


def _pulses(k, n_tracks, n_time):
    """Seeded bipolar-free pulses of different heights, widths and delays, one
    negative, plus a zero track."""
    rng = np.random.default_rng(k)
    t = np.arange(n_time) * DT
    out = np.zeros((n_tracks, n_time))
    for j in range(n_tracks - 1):
        t0, w, a = rng.uniform(0.2e-9, 1.0e-9), rng.uniform(50e-12, 300e-12), rng.uniform(0.5e-6, 3e-6)
        out[j] = a * np.where(t > t0, (t - t0) / w * np.exp(1 - (t - t0) / w), 0.0)
    out[1] *= -1.0
    return out


@pytest.mark.parametrize("precision", [wt.WT_F64, wt.WT_F32], ids=["f64", "f32"])
def test_electronics_on_pulses(ctx, precision):
    say(f"test_electronics_on_pulses precision={precision}")
    n_tr, n_t = 6, 200
    cur = _pulses(7, n_tr, n_t)
    g = workloads.cr_rc_response(n_t, DT)
    noise = workloads.noise_samples(8, n_tr, n_t)
    sigma, frac = 2e-5, 0.3
    if precision == wt.WT_F32:
        cur, g, noise = (a.astype(np.float32).astype(np.float64) for a in (cur, g, noise))
    st, v, f = _run(ctx, precision, cur, g, noise, sigma, frac)
    assert st == wt.WT_OK
    v_ref = oel.shape_signal(cur, g, DT, noise=noise, sigma=sigma)
    err = rel_l2(v, v_ref)
    say(f"  signal rel L2 {err:.2e}")
    assert err <= (1e-12 if precision == wt.WT_F64 else 1e-5)
    f_ref = oel.features(v, DT, frac)
    tol_t = (1e-9 if precision == wt.WT_F64 else 1e-3) * DT
    assert np.array_equal(f[:, 0], f_ref[:, 0])
    assert np.allclose(f[:, 1], f_ref[:, 1], rtol=0, atol=tol_t)
    assert np.array_equal(np.isnan(f[:, 2]), np.isnan(f_ref[:, 2]))
    ok = ~np.isnan(f_ref[:, 2])
    assert np.allclose(f[ok, 2], f_ref[ok, 2], rtol=0, atol=tol_t)
    assert f[1, 0] < 0                                       # the negative pulse keeps its sign


def test_electronics_on_the_c1_current_without_noise(ctx, px32, px32_oracle):
    say("test_electronics_on_the_c1_current_without_noise")
    car = rounded_carriers(px32["carriers"], wt.WT_F64)
    cur = oracle.induced_current(px32_oracle["H"], px32["cell"], car)
    n_t = cur.shape[1]
    dt = px32["spectrum"]["dt"]
    g = workloads.cr_rc_response(n_t, dt)
    st, v, f = _run(ctx, wt.WT_F64, cur, g, None, 0.0, 0.5, dt=dt)
    assert st == wt.WT_OK
    assert rel_l2(v, oel.shape_signal(cur, g, dt)) <= 1e-12
    f_ref = oel.features(v, dt, 0.5)
    assert np.allclose(f, f_ref, rtol=0, atol=1e-9 * dt, equal_nan=True)


def test_electronics_edge_cases(ctx):
    say("test_electronics_edge_cases")
    g = workloads.cr_rc_response(64, DT)
    # a zero current: amplitude 0, no crossing
    st, v, f = _run(ctx, wt.WT_F64, np.zeros((2, 64)), g, None, 0.0, 0.5)
    assert st == wt.WT_OK and np.all(v == 0) and np.all(f[:, 0] == 0) and np.all(np.isnan(f[:, 2]))
    # a single sample
    st, v, f = _run(ctx, wt.WT_F64, np.array([[2e-6]]), g[:1] + 1.0, None, 0.0, 0.5)
    assert st == wt.WT_OK and v[0, 0] == pytest.approx(DT * 2e-6 * (g[0] + 1.0)) and np.isnan(f[0, 2])
    # invalid arguments are rejected before any launch
    bad = dict(frac=1.0), dict(frac=0.0), dict(sigma=-1.0)
    for b in bad:
        st, _, _ = _run(ctx, wt.WT_F64, np.ones((1, 8)), g[:8], None, b.get("sigma", 0.0), b.get("frac", 0.5),
                        raise_on_error=False)
        assert st == wt.WT_E_INVALID_ARG
    st, _, _ = _run(ctx, wt.WT_F64, np.ones((1, 600)), np.ones(600), None, 0.0, 0.5, raise_on_error=False)
    assert st == wt.WT_E_UNSUPPORTED_SIZE


@pytest.mark.parametrize("precision", [wt.WT_F64, wt.WT_F32])
def test_electronics_nan_currents(ctx, precision):
    """Rows of NaN currents (all NaN, and NaN from some sample on, at the
    longest record): the features are those the oracle extracts from the
    same signal, the peak at the first NaN sample."""
    say(f"test_electronics_nan_currents precision={precision}")
    n_t = 512
    g = workloads.cr_rc_response(n_t, DT)
    cur = np.full((3, n_t), 1e-6)
    cur[0, :] = np.nan
    cur[1, 300:] = np.nan
    cur[2, :] = np.sin(np.arange(n_t) * 0.05) * 1e-6
    st, v, f = _run(ctx, precision, cur, g, None, 0.0, 0.5)
    assert st == wt.WT_OK
    f_ref = oel.features(v, DT, 0.5)
    assert np.array_equal(np.isnan(f), np.isnan(f_ref))
    assert f[0, 1] == 0.0 and f[1, 1] == pytest.approx(300 * DT, rel=1e-6)
    tol = 1e-9 if precision == wt.WT_F64 else 1e-3
    assert np.allclose(f[:, 1:2], f_ref[:, 1:2], rtol=0, atol=tol * DT, equal_nan=True)
