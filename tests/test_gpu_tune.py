"""The synthesis autotuner (wt_h_plan_tune): it keeps results exact in the
layout it chooses, has nothing to tune where a size has one register-FFT
schedule, and records and reuses its choices through a tuning cache file."""
import numpy as np
import pytest
import torch

import oracle
from gpu_common import context, current, h_standard, rel_l2, rounded_carriers, say
from paper_2605_13987_amd import workloads, wt

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = context()
    yield c
    wt.wt_context_destroy(c)


def _buffers(lay):
    ws = torch.empty(lay["workspace_bytes"], dtype=torch.uint8, device="cuda")
    hbuf = torch.empty(lay["h_bytes"], dtype=torch.uint8, device="cuda")
    return ws, hbuf


@pytest.mark.parametrize("precision", [wt.WT_F64, wt.WT_F32], ids=["f64", "f32"])
def test_tuned_stockham_synthesis_is_exact(ctx, precision):
    cfg = workloads.small_pixel(k=81, n_xy=24, n_z=40, n_freq=8, n_time=45, n_pairs=12, n_colloc=12)
    say(f"test_tuned_stockham_synthesis_is_exact precision={precision}")
    ref = oracle.weighting_field(cfg["cell"], cfg["columns"], cfg["spectrum"])
    plan, lay = wt.wt_h_plan_create(cfg["cell"], cfg["columns"], cfg["spectrum"], precision=precision)
    try:
        ws, hbuf = _buffers(lay)
        rep = wt.wt_h_plan_tune(ctx, plan, ws.data_ptr(), ws.numel(), hbuf.data_ptr(), hbuf.numel())
        say(f"  tune report {rep}")
        assert rep["n_candidates"] > 1 and rep["ms_chosen"] > 0 and rep["ms_default"] > 0
        assert rep["ms_chosen"] <= rep["ms_default"]
        assert rep["threads"] in (256, 512) and rep["h_time_block"] in (1, 2, 4, 8, 16, 32)
        lay2 = wt.wt_h_plan_layout(plan)
        assert lay2["h_time_block"] == rep["h_time_block"]
        assert lay2["h_bytes"] == lay["h_bytes"] and lay2["workspace_bytes"] == lay["workspace_bytes"]
        dt = torch.float64 if precision == wt.WT_F64 else torch.float32
        tol = 1e-9 if precision == wt.WT_F64 else 1e-5
        run = dict(plan=plan, layout=lay2, ws=ws, h=hbuf.view(dt), decode=1.0, precision=precision)
        # H as left by the tuner, then as written by a fresh solve with the tuned plan
        assert rel_l2(h_standard(run, cfg), ref["H"]) <= tol
        st, _ = wt.wt_h_solve(ctx, plan, ws.data_ptr(), ws.numel(), hbuf.data_ptr(), hbuf.numel(), report=True)
        assert st == wt.WT_OK
        assert rel_l2(h_standard(run, cfg), ref["H"]) <= tol
        car = rounded_carriers(cfg["carriers"], precision)
        i_ref = oracle.induced_current(ref["H"], cfg["cell"], car)
        assert rel_l2(current(ctx, run, car), i_ref) <= (1e-9 if precision == wt.WT_F64 else 1e-4)
    finally:
        wt.wt_h_plan_destroy(plan)


def test_register_fft_size_with_one_schedule_has_nothing_to_tune(ctx):
    """N_z = 512 has one register-FFT schedule (blocks of 8)."""
    cfg = workloads.small_pixel(k=82, n_xy=8, n_z=512, n_freq=4, n_time=20, n_pairs=4, n_colloc=8)
    plan, lay = wt.wt_h_plan_create(cfg["cell"], cfg["columns"], cfg["spectrum"], precision=wt.WT_F32)
    try:
        ws, hbuf = _buffers(lay)
        rep = wt.wt_h_plan_tune(ctx, plan, ws.data_ptr(), ws.numel(), hbuf.data_ptr(), hbuf.numel())
        assert rep["n_candidates"] == 1 and rep["ms_chosen"] < 0 and rep["fft_n1"] == 16
        assert wt.wt_h_plan_layout(plan)["h_time_block"] == lay["h_time_block"] == 8
    finally:
        wt.wt_h_plan_destroy(plan)


def _h_of(lay_after, hbuf, cfg):
    run = dict(layout=lay_after, h=hbuf.view(torch.float32), decode=1.0)
    return h_standard(run, cfg)


@pytest.mark.parametrize("n_z", [150, 40], ids=["register-fft", "stockham"])
def test_tuning_cache_file(ctx, tmp_path, n_z):
    """The context's tuning cache: the first tune of a grid times and records
    its choice; a later plan of the same grid (and a context that reads the
    file again) takes it without timing, with H still exact; a malformed file
    is refused and leaves the cache off."""
    cfg = workloads.small_pixel(k=84, n_xy=16, n_z=n_z, n_freq=4, n_time=21, n_pairs=4, n_colloc=8)
    ref = oracle.weighting_field(cfg["cell"], cfg["columns"], cfg["spectrum"])
    path = tmp_path / "tune.txt"
    wt.wt_context_set_tune_cache(ctx, str(path))
    reps = []
    try:
        for k in range(2):
            plan, lay = wt.wt_h_plan_create(cfg["cell"], cfg["columns"], cfg["spectrum"], precision=wt.WT_F32)
            ws, hbuf = _buffers(lay)
            rep = wt.wt_h_plan_tune(ctx, plan, ws.data_ptr(), ws.numel(), hbuf.data_ptr(), hbuf.numel())
            torch.cuda.synchronize()
            say(f"  n_z={n_z} tune {k}: {rep}")
            reps.append(rep)
            lay2 = wt.wt_h_plan_layout(plan)
            assert lay2["h_time_block"] == rep["h_time_block"]
            assert rel_l2(_h_of(lay2, hbuf, cfg), ref["H"]) <= 1e-5
            wt.wt_h_plan_destroy(plan)
        assert reps[0]["from_cache"] == 0 and reps[0]["n_candidates"] > 1
        assert reps[1]["from_cache"] == 1
        for f in ("h_time_block", "threads", "fft_n1"):
            assert reps[1][f] == reps[0][f]
        lines = [l for l in path.read_text().splitlines() if l and not l.startswith("#")]
        assert len(lines) == 1 and len(lines[0].split()) == 14
        # another context reading the same file
        c2 = context()
        try:
            wt.wt_context_set_tune_cache(c2, str(path))
            plan, lay = wt.wt_h_plan_create(cfg["cell"], cfg["columns"], cfg["spectrum"], precision=wt.WT_F32)
            ws, hbuf = _buffers(lay)
            rep = wt.wt_h_plan_tune(c2, plan, ws.data_ptr(), ws.numel(), hbuf.data_ptr(), hbuf.numel())
            assert rep["from_cache"] == 1 and rep["h_time_block"] == reps[0]["h_time_block"]
            wt.wt_h_plan_destroy(plan)
        finally:
            wt.wt_context_destroy(c2)
        # a malformed file is refused; the cache is then off
        path.write_text("not a tuning line\n")
        assert wt.wt_context_set_tune_cache(ctx, str(path), raise_on_error=False) == wt.WT_E_INVALID_ARG
        plan, lay = wt.wt_h_plan_create(cfg["cell"], cfg["columns"], cfg["spectrum"], precision=wt.WT_F32)
        ws, hbuf = _buffers(lay)
        rep = wt.wt_h_plan_tune(ctx, plan, ws.data_ptr(), ws.numel(), hbuf.data_ptr(), hbuf.numel())
        assert rep["from_cache"] == 0
        wt.wt_h_plan_destroy(plan)
    finally:
        wt.wt_context_set_tune_cache(ctx, None)
