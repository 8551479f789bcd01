"""The binned Eq. 1 convolution (wt_current with a workspace) through the C ABI.

* On synthetic fields (every node and lag distinct) against the oracle and
  against the unbinned form (no workspace): float64, float32 and float16 H;
  time blocks of 8 and 16 samples staged as 16-byte words, time blocks of
  the LDS Stockham synthesis and unaligned layouts staged value by value;
  ragged last time blocks; N_z not a multiple of the z-tile; polylines that
  leave the cell on every side, stationary and absorbed carriers, invalid
  tracks.
* The workspace's control words: the record count (four per event) against
  a count of events on the host, and the overflow flag: with room for all
  events the binned form runs, with one event less the unbinned form takes
  over (same currents).
* More tracks in one node column than a lane has per-track sums (records of
  the others on the overflow list, and with no room for that list the
  direct form), and more records in one z-tile than one LDS chunk holds
  (several chunks per tile); N_z smaller than a z-tile (nodes wrap).
* No carriers, and carriers that never move.
Bars: float64 1e-12 between the forms and 1e-9 against the oracle; float32
and float16 (exactly representable synthetic field) 1e-5 between the forms
and 1e-4 against the oracle.
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_common import context, current, rel_l2, rounded_carriers, say, solve_h
from paper_2605_13987_amd import layout, workloads, wt

pytestmark = pytest.mark.gpu

TOL_FORMS = {wt.WT_F64: 1e-12, wt.WT_F32: 1e-5}
TOL_ORACLE = {wt.WT_F64: 1e-9, wt.WT_F32: 1e-4}


@pytest.fixture(scope="module")
def ctx():
    c = context()
    yield c
    wt.wt_context_destroy(c)


def _synthetic_run(ctx, cfg, precision, h_format=wt.WT_H_PLAIN, fft_schedule=0, seed=7):
    """A plan and H buffer of cfg, H overwritten by a synthetic field; returns
    (run, the field as the GPU holds it, in float64)."""
    run = solve_h(ctx, cfg, precision, h_format=h_format, fft_schedule=fft_schedule)
    N, nt = cfg["cell"]["N"], cfg["spectrum"]["n_time"]
    f = workloads.synthetic_h_factors(workloads.rng_for(seed), N, nt, scale=1.0)
    Hs = workloads.synthetic_h_full(f)
    tb = run["layout"]["h_time_block"]
    if h_format == wt.WT_H_F16_SCALED:
        Hs = Hs.astype(np.float16).astype(np.float64)
        run["h"].copy_(torch.from_numpy(layout.from_standard(Hs, tb)).to(device="cuda", dtype=torch.float16))
        off = run["layout"]["h_decode_offset"]
        run["hbuf"][off:off + 4].view(torch.float32).fill_(1.0)
    else:
        if precision == wt.WT_F32:
            Hs = Hs.astype(np.float32).astype(np.float64)
        run["h"].copy_(torch.from_numpy(layout.from_standard(Hs, tb)).to(device="cuda", dtype=run["h"].dtype))
    torch.cuda.synchronize()
    return run, Hs


def _random_carriers(cfg, nc, n_tracks, seed, precision):
    rng = np.random.default_rng(seed)
    nt = cfg["spectrum"]["n_time"]
    L = np.asarray(cfg["cell"]["L"])
    pos = np.cumsum(rng.normal(0, 3e-6, size=(nc, nt + 1, 3)), axis=1) + rng.random((nc, 1, 3)) * L
    pos[5:10] = pos[5:10, :1]                                # stationary
    pos[10:15, nt // 2:] = pos[10:15, nt // 2:nt // 2 + 1]   # absorbed half way
    q = rng.choice([-1.0, 1.0], nc) * workloads.E_CHARGE
    track = rng.integers(0, n_tracks, nc).astype(np.int32)
    track[15:18] = -1
    track[18:20] = n_tracks
    return rounded_carriers(dict(pos=pos, charge=q, track=track, n_tracks=n_tracks), precision)


def _oracle(Hs, cfg, car):
    keep = (car["track"] >= 0) & (car["track"] < car["n_tracks"])
    ref = dict(pos=car["pos"][keep], charge=car["charge"][keep], track=car["track"][keep],
               n_tracks=car["n_tracks"])
    return oracle.induced_current(Hs, cfg["cell"], ref)


def _host_event_count(car, precision):
    dt = np.float64 if precision == wt.WT_F64 else np.float32
    P = np.asarray(car["pos"]).astype(dt)
    moving = np.any(P[:, 1:] != P[:, :-1], axis=2)
    mid = 0.5 * (P[:, 1:] + P[:, :-1])
    finite = np.all(np.isfinite(mid), axis=2)
    tr = np.asarray(car["track"])
    valid = (tr >= 0) & (tr < car["n_tracks"])
    return int(np.sum(moving & finite & valid[:, None]))


CASES = [
    # (n_xy, n_z, n_time, precision, h_format, fft_schedule)
    (12, 20, 70, wt.WT_F64, wt.WT_H_PLAIN, 0),      # Stockham time blocks, two z-tiles (one partial)
    (12, 20, 70, wt.WT_F32, wt.WT_H_PLAIN, 0),
    (16, 64, 53, wt.WT_F64, wt.WT_H_PLAIN, 0),      # blocks of 8 (16-byte words), ragged last block
    (16, 64, 53, wt.WT_F32, wt.WT_H_PLAIN, 0),
    (16, 64, 53, wt.WT_F32, wt.WT_H_F16_SCALED, 0),
    (8, 128, 21, wt.WT_F32, wt.WT_H_PLAIN, 1),      # blocks of 16
    (8, 128, 21, wt.WT_F32, wt.WT_H_F16_SCALED, 1),
    (8, 150, 21, wt.WT_F32, wt.WT_H_PLAIN, 0),      # smooth N_z, layout not 16-byte aligned: value by value
    (8, 64, 130, wt.WT_F32, wt.WT_H_PLAIN, 0),      # three wavefronts of output samples
    (10, 6, 33, wt.WT_F32, wt.WT_H_PLAIN, 0),       # N_z below the z-tile: nodes wrap inside one tile
    (10, 6, 33, wt.WT_F64, wt.WT_H_PLAIN, 0),
]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}x{c[1]}-nt{c[2]}-p{c[3]}-f{c[4]}-s{c[5]}" for c in CASES])
def test_binned_matches_oracle_and_unbinned(ctx, case):
    n_xy, n_z, nt, precision, h_format, sched = case
    cfg = workloads.small_pixel(k=71, n_xy=n_xy, n_z=n_z, n_freq=4, n_time=nt, n_pairs=2, n_colloc=6)
    say(f"binned vs unbinned {case}")
    run, Hs = _synthetic_run(ctx, cfg, precision, h_format, sched)
    car = _random_carriers(cfg, 400, 5, 72, precision)
    i_bin = current(ctx, run, car)
    i_dir = current(ctx, run, car, binned=False)
    i_ref = _oracle(Hs, cfg, car)
    e_forms, e_ref = rel_l2(i_bin, i_dir), rel_l2(i_bin, i_ref)
    say(f"  time block {run['layout']['h_time_block']}: binned vs unbinned {e_forms:.2e}, vs oracle {e_ref:.2e}")
    assert e_forms <= TOL_FORMS[precision] and e_ref <= TOL_ORACLE[precision]
    wt.wt_h_plan_destroy(run["plan"])


def _control_words(ws):
    return [int(v) for v in ws[:24].view(torch.int64).cpu()]


def test_event_count_and_overflow_fallback(ctx):
    cfg = workloads.small_pixel(k=73, n_xy=16, n_z=64, n_freq=4, n_time=53, n_pairs=2, n_colloc=6)
    run, Hs = _synthetic_run(ctx, cfg, wt.WT_F32)
    car = _random_carriers(cfg, 300, 4, 74, wt.WT_F32)
    n_ev = _host_event_count(car, wt.WT_F32)
    say(f"  host count of moving steps: {n_ev}")
    d = {k: torch.from_numpy(np.ascontiguousarray(car[k])).to("cuda") for k in ("pos", "charge", "track")}
    d["pos"], d["charge"] = d["pos"].float(), d["charge"].float()
    out = {}
    for cap in (n_ev, n_ev - 1):
        nb = wt.wt_current_workspace(run["plan"], 300, cap)
        ws = torch.full((nb,), 0x33, dtype=torch.uint8, device="cuda")
        o = torch.empty((4, 53), dtype=torch.float32, device="cuda")
        wt.wt_current(ctx, run["plan"], run["h"].data_ptr(), 300, 4, d["pos"].data_ptr(), d["charge"].data_ptr(),
                      d["track"].data_ptr(), o.data_ptr(), ws.data_ptr(), ws.numel())
        torch.cuda.synchronize()
        total, overflow, capacity = _control_words(ws)
        say(f"  capacity {cap}: control words total={total} overflow={overflow} capacity={capacity}")
        assert total == 4 * n_ev and capacity == 4 * cap and overflow == (1 if cap < n_ev else 0)
        out[cap] = o.double().cpu().numpy()
    i_ref = _oracle(Hs, cfg, car)
    for cap, o in out.items():
        assert rel_l2(o, i_ref) <= 1e-4
    assert rel_l2(out[n_ev], out[n_ev - 1]) <= 1e-5
    # smaller than the fixed part: refused
    small = wt.wt_current_workspace(run["plan"], 300, 1) - 1
    ws = torch.empty(small, dtype=torch.uint8, device="cuda")
    o = torch.empty((4, 53), dtype=torch.float32, device="cuda")
    with pytest.raises(wt.WtError) as err:
        wt.wt_current(ctx, run["plan"], run["h"].data_ptr(), 300, 4, d["pos"].data_ptr(), d["charge"].data_ptr(),
                      d["track"].data_ptr(), o.data_ptr(), ws.data_ptr(), ws.numel())
    assert err.value.status == wt.WT_E_WORKSPACE
    wt.wt_h_plan_destroy(run["plan"])


@pytest.mark.parametrize("precision", [wt.WT_F64, wt.WT_F32], ids=["f64", "f32"])
def test_many_tracks_and_crowded_tiles(ctx, precision):
    """200 carriers, each its own track, in one corner of the cell (more
    tracks per block of columns than accumulators), and 300 carriers jittering
    inside one cell (thousands of events in one z-tile)."""
    cfg = workloads.small_pixel(k=75, n_xy=12, n_z=20, n_freq=4, n_time=40, n_pairs=2, n_colloc=6)
    run, Hs = _synthetic_run(ctx, cfg, precision)
    rng = np.random.default_rng(76)
    nt = 40
    h = np.asarray(cfg["cell"]["L"]) / np.asarray(cfg["cell"]["N"])
    a = rng.random((200, 1, 3)) * 2 * h + np.cumsum(rng.normal(0, 0.3e-6, (200, nt + 1, 3)), axis=1)
    b = (np.array([5.5, 6.5, 9.5]) * h + rng.uniform(-0.4, 0.4, (300, nt + 1, 3)) * h)
    pos = np.concatenate([a, b])
    q = rng.choice([-1.0, 1.0], 500) * workloads.E_CHARGE
    track = np.concatenate([np.arange(200), rng.integers(0, 200, 300)]).astype(np.int32)
    car = rounded_carriers(dict(pos=pos, charge=q, track=track, n_tracks=200), precision)
    ctl = []
    # room for three times the steps: the records and the overflow list
    i_bin = current(ctx, run, car, max_events=3 * 500 * nt, control=ctl)
    i_dir = current(ctx, run, car, binned=False)
    i_ref = _oracle(Hs, cfg, car)
    e_forms, e_ref = rel_l2(i_bin, i_dir), rel_l2(i_bin, i_ref)
    say(f"  binned vs unbinned {e_forms:.2e}, vs oracle {e_ref:.2e}; control words {ctl}")
    assert e_forms <= TOL_FORMS[precision] and e_ref <= TOL_ORACLE[precision]
    assert ctl[1] == 0 and ctl[3] > 0                          # binned, with records on the overflow list
    # room for the events only: the overflow list does not fit, the direct form runs
    n_ev = _host_event_count(car, precision)
    ctl = []
    i_tight = current(ctx, run, car, max_events=n_ev, control=ctl)
    say(f"  workspace for {n_ev} events only: control words {ctl}")
    assert ctl[0] == 4 * n_ev and ctl[1] == 1
    assert rel_l2(i_tight, i_dir) <= TOL_FORMS[precision]
    wt.wt_h_plan_destroy(run["plan"])


def test_automatic_form(ctx):
    """The default form: small inputs are not binned (the workspace's control
    words stay as the caller left them), the same inputs with the binned form
    give the same currents."""
    cfg = workloads.small_pixel(k=79, n_xy=12, n_z=20, n_freq=4, n_time=30, n_pairs=2, n_colloc=6)
    run, Hs = _synthetic_run(ctx, cfg, wt.WT_F32)
    car = _random_carriers(cfg, 100, 3, 80, wt.WT_F32)
    d = {k: torch.from_numpy(np.ascontiguousarray(car[k])).to("cuda") for k in ("pos", "charge", "track")}
    d["pos"], d["charge"] = d["pos"].float(), d["charge"].float()
    ws = torch.full((wt.wt_current_workspace(run["plan"], 100),), 0x11, dtype=torch.uint8, device="cuda")
    outs = {}
    for form in (wt.WT_CURRENT_AUTO, wt.WT_CURRENT_BINNED):
        wt.wt_context_set_current_form(ctx, form)
        o = torch.empty((3, 30), dtype=torch.float32, device="cuda")
        wt.wt_current(ctx, run["plan"], run["h"].data_ptr(), 100, 3, d["pos"].data_ptr(), d["charge"].data_ptr(),
                      d["track"].data_ptr(), o.data_ptr(), ws.data_ptr(), ws.numel())
        torch.cuda.synchronize()
        outs[form] = o.double().cpu().numpy()
        if form == wt.WT_CURRENT_AUTO:
            assert bool(torch.all(ws[:24] == 0x11))             # not binned: workspace untouched
    wt.wt_context_set_current_form(ctx, wt.WT_CURRENT_BINNED)
    assert rel_l2(outs[wt.WT_CURRENT_AUTO], outs[wt.WT_CURRENT_BINNED]) <= 1e-5
    assert rel_l2(outs[wt.WT_CURRENT_BINNED], _oracle(Hs, cfg, car)) <= 1e-4
    with pytest.raises(wt.WtError):
        wt.wt_context_set_current_form(ctx, 3)
    wt.wt_h_plan_destroy(run["plan"])


def test_no_carriers_and_no_moving_steps(ctx):
    cfg = workloads.small_pixel(k=77, n_xy=12, n_z=20, n_freq=4, n_time=30, n_pairs=2, n_colloc=6)
    run, _ = _synthetic_run(ctx, cfg, wt.WT_F32)
    rng = np.random.default_rng(78)
    still = np.repeat(rng.random((20, 1, 3)) * 40e-6, 31, axis=1)
    car = rounded_carriers(dict(pos=still, charge=np.full(20, workloads.E_CHARGE),
                                track=np.zeros(20, np.int32), n_tracks=2), wt.WT_F32)
    assert np.all(current(ctx, run, car) == 0.0)
    empty = dict(pos=np.zeros((0, 31, 3)), charge=np.zeros(0), track=np.zeros(0, np.int32), n_tracks=2)
    assert np.all(current(ctx, run, empty) == 0.0)
    wt.wt_h_plan_destroy(run["plan"])
