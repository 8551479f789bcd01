"""Parity of the geometry-variant batch: variants of uneven grids (radix 3
and 5 sizes, the largest 160x160x320) solved through the C ABI, with the
plan's default synthesis launch and after wt_h_plan_tune, against the
oracle's direct sums on sampled (x, y) columns (the float32 bar, 1e-5)."""
import pytest
import torch

import oracle
from gpu_common import context, h_columns, intermediates, rel_l2, say
from paper_2605_13987_amd import workloads, wt

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = context()
    yield c
    wt.wt_context_destroy(c)


@pytest.mark.parametrize("k", [0, 22, 37, 9])
def test_variant_field_on_sampled_columns(ctx, k):
    v = workloads.geometry_variant(k, n_pairs=10)
    N = v["cell"]["N"]
    cols = [(0, 0), (N[0] // 2, N[1] // 2), (N[0] // 2 + 3, N[1] // 2 - 2), (N[0] - 1, 5)]
    say(f"variant {k}: grid {N}, {v['spectrum']['n_freq']} frequencies")
    ref = oracle.weighting_field(v["cell"], v["columns"], v["spectrum"], route="columns", cols_ij=cols)
    plan, lay = wt.wt_h_plan_create(v["cell"], v["columns"], v["spectrum"], precision=wt.WT_F32)
    try:
        ws = torch.empty(lay["workspace_bytes"], dtype=torch.uint8, device="cuda")
        hbuf = torch.empty(lay["h_bytes"], dtype=torch.uint8, device="cuda")
        st, rep = wt.wt_h_solve(ctx, plan, ws.data_ptr(), ws.numel(), hbuf.data_ptr(), hbuf.numel(), report=True)
        assert st == wt.WT_OK, rep
        run = dict(plan=plan, layout=lay, ws=ws, h=hbuf.view(torch.float32), decode=1.0, precision=wt.WT_F32)
        im = intermediates(run, v)
        assert rel_l2(im["q"], ref["q"]) <= 1e-9
        err = rel_l2(h_columns(run, v, cols), ref["H_cols"])
        say(f"  default launch (time block {lay['h_time_block']}): H rel L2 {err:.2e}")
        assert err <= 1e-5
        tune = wt.wt_h_plan_tune(ctx, plan, ws.data_ptr(), ws.numel(), hbuf.data_ptr(), hbuf.numel())
        run["layout"] = wt.wt_h_plan_layout(plan)
        err_t = rel_l2(h_columns(run, v, cols), ref["H_cols"])
        say(f"  autotuned {tune}: H rel L2 {err_t:.2e}")
        assert err_t <= 1e-5
    finally:
        wt.wt_h_plan_destroy(plan)
