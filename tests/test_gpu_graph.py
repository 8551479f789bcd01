"""The whole step (H solve + current) captured once in a HIP graph and
replayed: every replay, with eager work and synchronisations between them,
reproduces the eager result exactly (same kernels, same inputs)."""
import numpy as np
import pytest
import torch

from gpu_common import say
from paper_2605_13987_amd import workloads, wt

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("binned", [False, True], ids=["direct", "binned"])
@pytest.mark.parametrize("h_format", [wt.WT_H_PLAIN, wt.WT_H_F16_SCALED], ids=["f32", "f16"])
def test_captured_step_replays_match_eager(h_format, binned):
    cfg = workloads.small_pixel(k=51, n_xy=32, n_z=128, n_freq=24, n_time=53, n_pairs=200, n_colloc=24)
    say(f"test_captured_step_replays_match_eager h_format={h_format}")
    cell, spec, car = cfg["cell"], cfg["spectrum"], cfg["carriers"]
    stream = torch.cuda.Stream()
    ctx = wt.wt_context_create(0, stream.cuda_stream)
    wt.wt_context_set_current_form(ctx, wt.WT_CURRENT_BINNED if binned else wt.WT_CURRENT_AUTO)
    plan, lay = wt.wt_h_plan_create(cell, cfg["columns"], spec, precision=wt.WT_F32, h_format=h_format)
    ws = torch.zeros(lay["workspace_bytes"], dtype=torch.uint8, device="cuda")
    h = torch.zeros(lay["h_bytes"], dtype=torch.uint8, device="cuda")
    pos = torch.from_numpy(car["pos"]).to("cuda", torch.float32)
    q = torch.from_numpy(car["charge"]).to("cuda", torch.float32)
    tr = torch.from_numpy(car["track"]).to("cuda")
    n_c, n_tr = pos.shape[0], car["n_tracks"]
    out = torch.zeros((n_tr, spec["n_time"]), dtype=torch.float32, device="cuda")
    cws = torch.zeros(wt.wt_current_workspace(plan, n_c) if binned else 0, dtype=torch.uint8, device="cuda")

    def step():
        wt.wt_h_solve(ctx, plan, ws.data_ptr(), ws.numel(), h.data_ptr(), lay["h_bytes"])
        wt.wt_current(ctx, plan, h.data_ptr(), n_c, n_tr, pos.data_ptr(), q.data_ptr(), tr.data_ptr(),
                      out.data_ptr(), cws.data_ptr() if binned else 0, cws.numel())

    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        step()                                     # eager reference (also sets kernel attributes)
    stream.synchronize()
    h_ref, i_ref = h.clone(), out.clone()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=stream):
        step()
    torch.cuda.synchronize()
    for rep in range(4):
        h.zero_()                                  # eager work between replays
        out.fill_(float("nan"))
        cws.fill_(0x5a)
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(h, h_ref), f"replay {rep}: H differs"
        # the current sums over carriers with atomics: equal up to summation order
        err = float((out - i_ref).abs().max() / i_ref.abs().max())
        say(f"  replay {rep}: H equal, current max rel diff {err:.1e}")
        assert err <= 1e-6
    del graph
    wt.wt_h_plan_destroy(plan)
    wt.wt_context_destroy(ctx)
