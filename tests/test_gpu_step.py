"""wt_step (H solve and current in one call, the binning on a second stream
beside the synthesis) against wt_h_solve followed by wt_current: H equal
bit for bit, the current equal up to the order of its atomic sums, the
report equal; two calls in a row on the same buffers with different
carriers; and the captured form replayed against the eager one."""
import pytest
import torch

from gpu_common import say
from paper_2605_13987_amd import workloads, wt

pytestmark = pytest.mark.gpu


def _carriers(cfg, scale=1.0):
    car = cfg["carriers"]
    pos = torch.from_numpy(car["pos"]).to("cuda", torch.float32)
    q = torch.from_numpy(car["charge"]).to("cuda", torch.float32) * scale
    tr = torch.from_numpy(car["track"]).to("cuda")
    return pos, q, tr


def _rel(a, b):
    return float((a - b).abs().max() / b.abs().max())


# n_freq 24 leaves the field table beside the boundary fit, 300 (more
# frequencies than compute units) runs them one after the other
@pytest.mark.parametrize("n_freq", [24, 300])
@pytest.mark.parametrize("form", [1, 2], ids=["binned", "direct"])
@pytest.mark.parametrize("h_format", [wt.WT_H_PLAIN, wt.WT_H_F16_SCALED], ids=["f32", "f16"])
def test_step_matches_solve_then_current(h_format, form, n_freq):
    say(f"test_step_matches_solve_then_current h_format={h_format} form={form} n_freq={n_freq}")
    cfg = workloads.small_pixel(k=61, n_xy=32, n_z=128, n_freq=n_freq, n_time=53, n_pairs=200, n_colloc=24)
    cell, spec = cfg["cell"], cfg["spectrum"]
    stream = torch.cuda.Stream()
    ctx = wt.wt_context_create(0, stream.cuda_stream)
    wt.wt_context_set_current_form(ctx, form)
    plan, lay = wt.wt_h_plan_create(cell, cfg["columns"], spec, precision=wt.WT_F32, h_format=h_format)
    ws = torch.zeros(lay["workspace_bytes"], dtype=torch.uint8, device="cuda")
    h = torch.zeros(lay["h_bytes"], dtype=torch.uint8, device="cuda")
    h_ref = torch.zeros_like(h)
    pos, q, tr = _carriers(cfg)
    n_c, n_tr, nt = pos.shape[0], cfg["carriers"]["n_tracks"], spec["n_time"]
    cws = torch.zeros(wt.wt_current_workspace(plan, n_c), dtype=torch.uint8, device="cuda")
    out = torch.full((n_tr, nt), float("nan"), dtype=torch.float32, device="cuda")
    ref = torch.zeros_like(out)
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        _, rep_ref = wt.wt_h_solve(ctx, plan, ws.data_ptr(), ws.numel(), h_ref.data_ptr(), lay["h_bytes"],
                                   report=True)
        wt.wt_current(ctx, plan, h_ref.data_ptr(), n_c, n_tr, pos.data_ptr(), q.data_ptr(), tr.data_ptr(),
                      ref.data_ptr(), cws.data_ptr(), cws.numel())
    stream.synchronize()
    # two steps in a row: the second with the charges doubled, so that a
    # binning that overtook the first step's accumulation would show
    for rep, scale in enumerate((1.0, 2.0)):
        pos2, q2, tr2 = _carriers(cfg, scale)
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            _, rep_step = wt.wt_step(ctx, plan, ws.data_ptr(), ws.numel(), h.data_ptr(), lay["h_bytes"], n_c, n_tr,
                                     pos2.data_ptr(), q2.data_ptr(), tr2.data_ptr(), out.data_ptr(), cws.data_ptr(),
                                     cws.numel(), report=(rep == 0))
            if rep == 0:
                first = out.clone()
        stream.synchronize()
        assert torch.equal(h, h_ref), "H differs from wt_h_solve's"
        err = _rel(out, scale * ref)
        say(f"  step {rep}: H equal, current max rel diff {err:.1e}")
        assert err <= 1e-6
        if rep == 0:
            assert rep_step == rep_ref
            assert _rel(first, ref) <= 1e-6
    wt.wt_h_plan_destroy(plan)
    wt.wt_context_destroy(ctx)


def test_step_captured_replays_match_eager():
    say("test_step_captured_replays_match_eager")
    cfg = workloads.small_pixel(k=62, n_xy=32, n_z=128, n_freq=24, n_time=53, n_pairs=200, n_colloc=24)
    cell, spec = cfg["cell"], cfg["spectrum"]
    stream = torch.cuda.Stream()
    ctx = wt.wt_context_create(0, stream.cuda_stream)
    wt.wt_context_set_current_form(ctx, 1)
    plan, lay = wt.wt_h_plan_create(cell, cfg["columns"], spec, precision=wt.WT_F32, h_format=wt.WT_H_F16_SCALED)
    ws = torch.zeros(lay["workspace_bytes"], dtype=torch.uint8, device="cuda")
    h = torch.zeros(lay["h_bytes"], dtype=torch.uint8, device="cuda")
    pos, q, tr = _carriers(cfg)
    n_c, n_tr, nt = pos.shape[0], cfg["carriers"]["n_tracks"], spec["n_time"]
    cws = torch.zeros(wt.wt_current_workspace(plan, n_c), dtype=torch.uint8, device="cuda")
    out = torch.zeros((n_tr, nt), dtype=torch.float32, device="cuda")

    def step():
        wt.wt_step(ctx, plan, ws.data_ptr(), ws.numel(), h.data_ptr(), lay["h_bytes"], n_c, n_tr, pos.data_ptr(),
                   q.data_ptr(), tr.data_ptr(), out.data_ptr(), cws.data_ptr(), cws.numel())

    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        step()
    stream.synchronize()
    h_ref, i_ref = h.clone(), out.clone()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=stream):
        step()
    torch.cuda.synchronize()
    for rep in range(3):
        h.zero_()
        out.fill_(float("nan"))
        cws.fill_(0x5a)
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(h, h_ref), f"replay {rep}: H differs"
        err = _rel(out, i_ref)
        say(f"  replay {rep}: H equal, current max rel diff {err:.1e}")
        assert err <= 1e-6
    del graph
    wt.wt_h_plan_destroy(plan)
    wt.wt_context_destroy(ctx)
