"""GPU parity of the adjoint (wt_h_gradient, behind torch.autograd):

* small multi-tile case, both precisions: the adjoint gradient of a seeded
  loss against the FP64 oracle's forward-mode derivatives, and for the pitch
  against the oracle's central differences (FP64 path 1e-6, FP32 path 1e-3,
  relative to the largest log-derivative);
* the 128x128x256 pixel with its MIP track: the FP64 adjoint against central
  differences of the GPU's own FP64 forward (1e-5), and the FP32 adjoint
  against the FP64 one (1e-3);
* the peak-time and windowed-charge features through torch autograd.

Compared quantities are log-derivatives theta_k dL/dtheta_k (dimensionless),
so that resistivities (ohm m) and radii (m) share one scale.
"""
import numpy as np
import pytest
import torch

from gpu_common import rounded_carriers, say
from oracle import gradient as ograd
from paper_2605_13987_amd import workloads, wt
from paper_2605_13987_amd.grad import ColumnModel, signal_features

pytestmark = pytest.mark.gpu


def _slots(columns):
    """(w, slot) of every live parameter, in the oracle's parameter order."""
    out = []
    for w, c in enumerate(columns):
        out += [(w, p) for p in range(len(c["resistivity"]))] + [(w, 4)]
    return out


def _log_grad(theta, grad, columns):
    return np.array([theta[w, s] * grad[w, s] for w, s in _slots(columns)])


def _seeded_loss_weights(n_tracks, n_time, k):
    rng = workloads.rng_for(k)
    return rng.standard_normal((n_tracks, n_time))


@pytest.fixture(scope="module")
def small():
    return workloads.small_pixel(k=23, n_xy=16, n_z=32, n_freq=10, n_time=24, n_pairs=10, n_colloc=12)


@pytest.mark.parametrize("precision,tol", [(wt.WT_F64, 1e-6), (wt.WT_F32, 1e-3)])
def test_adjoint_matches_oracle_forward_mode(small, precision, tol):
    cfg = small
    say(f"  gradient parity {cfg['name']} precision={precision}")
    car = rounded_carriers(cfg["carriers"], precision)
    model = ColumnModel(cfg["cell"], cfg["columns"], cfg["spectrum"], car, precision=precision)
    theta = model.theta0()
    G = _seeded_loss_weights(car["n_tracks"], cfg["spectrum"]["n_time"], 61)
    plan, cur = model.solve(theta)
    g, gp = model.gradient(plan, torch.as_tensor(G, device="cuda"))
    torch.cuda.synchronize()
    jac, i0 = ograd.current_jacobian(cfg["cell"], cfg["columns"], cfg["spectrum"], car)
    ref = np.array([np.sum(G * jac[prm]) for prm in ograd.parameter_names(cfg["columns"])])
    ref_p = np.sum(G * ograd.pitch_derivative(cfg["cell"], cfg["columns"], cfg["spectrum"], car))
    th = theta.numpy()
    p0 = cfg["cell"]["L"][0]
    ref_log = np.array([th[w, s] * r for (w, s), r in zip(_slots(cfg["columns"]), ref)] + [p0 * ref_p])
    got_log = np.concatenate([_log_grad(th, g.numpy(), cfg["columns"]), [p0 * float(gp)]])
    err = np.max(np.abs(got_log - ref_log)) / np.max(np.abs(ref_log))
    say(f"    log-gradient ref {ref_log}\n    got {got_log}\n    max err / max = {err:.3e}")
    assert err <= tol
    # unused resistivity slots get exactly zero
    assert np.all(g.numpy()[0, 1:4] == 0.0)
    # the currents themselves came from the same forward
    assert np.linalg.norm(cur.cpu().numpy() - i0) <= (1e-9 if precision == wt.WT_F64 else 1e-4) * np.linalg.norm(i0)


@pytest.fixture(scope="module")
def px128():
    return workloads.mip_pixel_128x128x256()


def test_full_size_adjoint_against_central_differences(px128):
    cfg = px128
    say(f"  full-size gradient {cfg['name']}: FP64 adjoint vs FP64 central differences")
    model = ColumnModel(cfg["cell"], cfg["columns"], cfg["spectrum"], cfg["carriers"], precision=wt.WT_F64)
    theta = model.theta0()
    G = torch.as_tensor(_seeded_loss_weights(1, cfg["spectrum"]["n_time"], 62), device="cuda")
    plan, _ = model.solve(theta)
    g64, gp64 = model.gradient(plan, G)
    g64 = g64.numpy()
    del plan
    fd = np.zeros_like(g64)
    for w, s in _slots(cfg["columns"]):
        h = 1e-4 * theta[w, s].item()
        vals = []
        for sign in (1.0, -1.0):
            th = theta.clone()
            th[w, s] += sign * h
            p, cur = model.solve(th)
            vals.append(float((cur * G).sum().item()))
            del p
        fd[w, s] = (vals[0] - vals[1]) / (2 * h)
    p0 = float(model.pitch0())
    vals = []
    for sign in (1.0, -1.0):
        p, cur = model.solve(theta, torch.tensor(p0 * (1.0 + sign * 1e-4), dtype=torch.float64))
        vals.append(float((cur * G).sum().item()))
        del p
    fdp = (vals[0] - vals[1]) / (2e-4 * p0)
    th = theta.numpy()
    a = np.concatenate([_log_grad(th, g64, cfg["columns"]), [p0 * float(gp64)]])
    b = np.concatenate([_log_grad(th, fd, cfg["columns"]), [p0 * fdp]])
    err = np.max(np.abs(a - b)) / np.max(np.abs(b))
    say(f"    adjoint {a}\n    central differences {b}\n    max err / max = {err:.3e}")
    assert err <= 1e-5

    say("  full-size gradient: FP32 adjoint vs FP64 adjoint")
    m32 = ColumnModel(cfg["cell"], cfg["columns"], cfg["spectrum"], cfg["carriers"], precision=wt.WT_F32)
    p32, _ = m32.solve(theta)
    g32, gp32 = m32.gradient(p32, G)
    c = np.concatenate([_log_grad(th, g32.numpy(), cfg["columns"]), [p0 * float(gp32)]])
    err32 = np.max(np.abs(c - a)) / np.max(np.abs(a))
    say(f"    FP32 adjoint {c}\n    max err / max = {err32:.3e}")
    assert err32 <= 1e-3


def test_signal_features_through_autograd(px128):
    """Peak time and windowed charge of the MIP track's current, differentiated
    by the adjoint (FP32 path) and by FP64 central differences."""
    cfg = px128
    dt = cfg["spectrum"]["dt"]
    rng = workloads.rng_for(63)
    t_c, t_s = rng.uniform(0.5e-9, 1.5e-9), rng.uniform(0.1e-9, 0.4e-9)
    m32 = ColumnModel(cfg["cell"], cfg["columns"], cfg["spectrum"], cfg["carriers"], precision=wt.WT_F32)
    theta = m32.theta0().requires_grad_(True)
    pitch = m32.pitch0().requires_grad_(True)
    t_peak, q_w = signal_features(m32.currents(theta, pitch), dt, t_c, t_s, 2e-9)
    gp, gpp = (g.numpy() for g in torch.autograd.grad(t_peak.sum(), (theta, pitch), retain_graph=True))
    gq, gqp = (g.numpy() for g in torch.autograd.grad(q_w.sum(), (theta, pitch)))
    m64 = ColumnModel(cfg["cell"], cfg["columns"], cfg["spectrum"], cfg["carriers"], precision=wt.WT_F64)
    th0 = m64.theta0()
    fp, fq = np.zeros_like(gp), np.zeros_like(gq)
    for w, s in _slots(cfg["columns"]):
        h = 1e-4 * th0[w, s].item()
        vals = []
        for sign in (1.0, -1.0):
            th = th0.clone()
            th[w, s] += sign * h
            p, cur = m64.solve(th)
            tp, qw = signal_features(cur, dt, t_c, t_s, 2e-9)
            vals.append((tp.sum().item(), qw.sum().item()))
            del p
        fp[w, s] = (vals[0][0] - vals[1][0]) / (2 * h)
        fq[w, s] = (vals[0][1] - vals[1][1]) / (2 * h)
    p0 = float(m64.pitch0())
    vals = []
    for sign in (1.0, -1.0):
        p, cur = m64.solve(th0, torch.tensor(p0 * (1.0 + sign * 1e-4), dtype=torch.float64))
        tp, qw = signal_features(cur, dt, t_c, t_s, 2e-9)
        vals.append((tp.sum().item(), qw.sum().item()))
        del p
    fpp = (vals[0][0] - vals[1][0]) / (2e-4 * p0)
    fqp = (vals[0][1] - vals[1][1]) / (2e-4 * p0)
    th = th0.numpy()
    for name, got, ref, gpitch, fpitch in (("t_peak", gp, fp, gpp, fpp), ("q_w", gq, fq, gqp, fqp)):
        a = np.concatenate([_log_grad(th, got, cfg["columns"]), [p0 * float(gpitch)]])
        b = np.concatenate([_log_grad(th, ref, cfg["columns"]), [p0 * fpitch]])
        err = np.max(np.abs(a - b)) / np.max(np.abs(b))
        say(f"    {name}: adjoint {a}\n    {name}: central differences {b}\n    max err / max = {err:.3e}")
        assert err <= 2e-3
    # The paper's Section 5 finding: the bias columns' resistance barely moves
    # the timing, the readout column's dominates.
    ro = abs(th[0, 0] * gp[0, 0])
    bias = abs(sum(th[1, p] * gp[1, p] for p in range(4)))
    say(f"    peak time log-sensitivity: readout {ro:.3e} s, bias (all quarters) {bias:.3e} s")
    assert bias < ro


def test_gradient_edge_cases(small):
    """No carriers: zero gradient; carriers with track ids outside [0, n_tracks)
    are skipped exactly as by wt_current."""
    cfg = small
    car = rounded_carriers(cfg["carriers"], wt.WT_F32)
    G = torch.as_tensor(_seeded_loss_weights(car["n_tracks"], cfg["spectrum"]["n_time"], 64), device="cuda")
    empty = dict(pos=np.zeros((0, cfg["spectrum"]["n_time"] + 1, 3)), charge=np.zeros(0),
                 track=np.zeros(0, np.int32), n_tracks=car["n_tracks"])
    m0 = ColumnModel(cfg["cell"], cfg["columns"], cfg["spectrum"], empty, precision=wt.WT_F32)
    p0, cur0 = m0.solve(m0.theta0())
    g0, gp0 = m0.gradient(p0, G)
    assert float(cur0.abs().max()) == 0.0 and float(g0.abs().max()) == 0.0 and float(gp0) == 0.0
    # invalid track ids: the same gradient as without those carriers
    bad = dict(car, track=np.where(np.arange(len(car["track"])) % 4 == 0, -1, car["track"]).astype(np.int32))
    bad["track"][1] = car["n_tracks"]
    keep = (bad["track"] >= 0) & (bad["track"] < car["n_tracks"])
    sub = dict(pos=car["pos"][keep], charge=car["charge"][keep], track=bad["track"][keep], n_tracks=car["n_tracks"])
    mb = ColumnModel(cfg["cell"], cfg["columns"], cfg["spectrum"], bad, precision=wt.WT_F32)
    ms = ColumnModel(cfg["cell"], cfg["columns"], cfg["spectrum"], sub, precision=wt.WT_F32)
    pb, _ = mb.solve(mb.theta0())
    psub, _ = ms.solve(ms.theta0())
    gb, gpb = mb.gradient(pb, G)
    gs, gps = ms.gradient(psub, G)
    scale = float(gs.abs().max())
    assert float((gb - gs).abs().max()) <= 1e-5 * scale
    assert abs(float(gpb) - float(gps)) <= 1e-5 * abs(float(gps))
