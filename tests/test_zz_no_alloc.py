"""wt_h_solve_static (wt_h_solve with the library's static workspace, for
callers that cannot allocate device memory) against wt_h_solve, through the
C ABI: two calls in a row, the second on a smaller grid, each compared with
wt_h_solve of the same plan (same kernels: H and the report must agree
exactly) and the first also with the FP64 oracle (1e-5, the plain path's
bound); plans whose workspace exceeds the static array are rejected."""
import numpy as np
import pytest
import torch

from gpu_common import context, h_standard, rel_l2, say
from paper_2605_13987_amd import workloads, wt

pytestmark = pytest.mark.gpu


def _both(ctx, cfg, precision, h_format=wt.WT_H_PLAIN):
    plan, lay = wt.wt_h_plan_create(cfg["cell"], cfg["columns"], cfg["spectrum"], precision=precision,
                                    h_format=h_format)
    say(f"  {cfg['name']} precision={precision} h_format={h_format}: workspace {lay['workspace_bytes']} B "
        f"(static {wt.WT_STATIC_WORKSPACE_BYTES} B), H {lay['h_bytes']} B")
    assert lay["workspace_bytes"] <= wt.WT_STATIC_WORKSPACE_BYTES
    ws = torch.empty(lay["workspace_bytes"], dtype=torch.uint8, device="cuda")
    h_ref = torch.empty(lay["h_bytes"], dtype=torch.uint8, device="cuda")
    h_st = torch.full((lay["h_bytes"],), 0x7f, dtype=torch.uint8, device="cuda")
    st1, rep1 = wt.wt_h_solve(ctx, plan, ws.data_ptr(), ws.numel(), h_ref.data_ptr(), lay["h_bytes"], report=True)
    say("  wt_h_solve_static")
    st2, rep2 = wt.wt_h_solve_static(ctx, plan, h_st.data_ptr(), lay["h_bytes"], report=True)
    torch.cuda.synchronize()
    assert st1 == wt.WT_OK and st2 == wt.WT_OK
    assert rep1 == rep2, (rep1, rep2)
    # the defined bytes of H: its values, and for float16-scaled H the decode
    # factor after them (the padding between is not written)
    N = cfg["cell"]["N"]
    n_vals = N[0] * N[1] * N[2] * cfg["spectrum"]["n_time"] * 3
    if h_format == wt.WT_H_F16_SCALED:
        off = lay["h_decode_offset"]
        parts = [(0, n_vals * 2), (off, off + 4)]
    else:
        parts = [(0, n_vals * (8 if precision == wt.WT_F64 else 4))]
    same = all(bool(torch.equal(h_ref[a:b], h_st[a:b])) for a, b in parts)
    say(f"  H identical to wt_h_solve: {same}")
    assert same
    return plan, lay, h_st


def test_static_workspace_matches_workspace_solve(px32, px32_oracle):
    ctx = context()
    try:
        plan, lay, h = _both(ctx, px32, wt.WT_F32)
        run = dict(layout=lay, h=h.view(torch.float32), decode=1.0)
        H = h_standard(run, px32)
        err = rel_l2(H, px32_oracle["H"])
        say(f"  H rel L2 vs oracle {err:.2e}")
        assert err <= 1e-5
        wt.wt_h_plan_destroy(plan)
        # second call, smaller grid, double precision and float16-scaled H
        small = workloads.small_pixel(k=23, n_xy=16, n_z=64, n_freq=6, n_time=20, n_pairs=8, n_colloc=12)
        for prec, fmt in ((wt.WT_F64, wt.WT_H_PLAIN), (wt.WT_F32, wt.WT_H_F16_SCALED)):
            plan, _, _ = _both(ctx, small, prec, fmt)
            wt.wt_h_plan_destroy(plan)
    finally:
        wt.wt_context_destroy(ctx)


def test_static_workspace_rejects_large_plans():
    ctx = context()
    try:
        cell = workloads.make_cell(50e-6, 300e-6, 128, 256)
        cols = workloads.uniform_pixel_32x32x64()["columns"]
        spec = dict(n_freq=256, df=workloads.frequency_grid_to_nyquist(256, 10e-12), n_time=200, dt=10e-12)
        plan, lay = wt.wt_h_plan_create(cell, cols, spec, precision=wt.WT_F32)
        assert lay["workspace_bytes"] > wt.WT_STATIC_WORKSPACE_BYTES
        h = torch.full((1024,), 0x55, dtype=torch.uint8, device="cuda")
        st, _ = wt.wt_h_solve_static(ctx, plan, h.data_ptr(), lay["h_bytes"], raise_on_error=False)
        torch.cuda.synchronize()
        msg = wt.LIB.wt_context_last_error(ctx).decode()
        say(f"  status {st}: {msg}")
        assert st == wt.WT_E_WORKSPACE
        assert str(lay["workspace_bytes"]) in msg and str(wt.WT_STATIC_WORKSPACE_BYTES) in msg
        assert bool(torch.all(h == 0x55))           # nothing was enqueued
        wt.wt_h_plan_destroy(plan)
    finally:
        wt.wt_context_destroy(ctx)
