"""End-to-end parity of the currents at the 128x128x256 workload (256
frequencies, 200 samples, one MIP track of 1e4 e/h pairs = 2e4 carriers):
wt_h_solve then wt_current on the solved H, for every carrier, against the
FP64 oracle's own boundary fit, field (at every node the paths touch) and
Eq. 1.  float32 H within 1e-4 (the plain path's bound), float16-scaled H
within 1e-3 (the mixed path's)."""
import numpy as np
import pytest
import torch

from gpu_common import context, current, oracle_current_on_nodes, rel_l2, rounded_carriers, say, solve_h
from paper_2605_13987_amd import workloads, wt

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def px128():
    return workloads.mip_pixel_128x128x256()


@pytest.fixture(scope="module")
def px128_ref(px128):
    say("oracle: boundary fit, field at the touched nodes, Eq. 1 for all 2e4 carriers")
    return oracle_current_on_nodes(px128, rounded_carriers(px128["carriers"], wt.WT_F32))


@pytest.mark.parametrize("h_format,tol", [(wt.WT_H_PLAIN, 1e-4), (wt.WT_H_F16_SCALED, 1e-3)])
def test_current_on_the_solved_field_128x128x256(px128, px128_ref, h_format, tol):
    ctx = context()
    try:
        run = solve_h(ctx, px128, wt.WT_F32, h_format=h_format)
        assert run["status"] == wt.WT_OK, run["report"]
        got = current(ctx, run, px128["carriers"])
        err = rel_l2(got, px128_ref)
        say(f"  h_format={h_format}: i rel L2 vs oracle {err:.2e} (<= {tol})")
        assert np.all(np.isfinite(got))
        assert err <= tol
        wt.wt_h_plan_destroy(run["plan"])
        del run
        torch.cuda.empty_cache()
    finally:
        wt.wt_context_destroy(ctx)
