"""wt_batch_run: many geometry variants of uneven size on lanes of streams.

* every item's current equals that of the plain wt_h_solve + wt_current
  sequence for the same plan (up to the atomic summation order of the
  current), for 1, 2 and 3 lanes;
* per-item status: an item whose plan does not fit the lane buffers, and one
  with no output, are skipped with their own status, the others run;
* the batched call captured in a HIP graph: replays, with eager work and
  synchronisations between them, match the eager result.
"""
import numpy as np
import pytest
import torch

from gpu_common import say
from paper_2605_13987_amd import workloads, wt

pytestmark = pytest.mark.gpu

SHAPES = [(16, 32, 6, 21), (24, 72, 5, 30), (8, 128, 4, 17), (20, 40, 7, 25), (16, 150, 5, 21)]


def _items(precision=wt.WT_F32):
    dt = torch.float64 if precision == wt.WT_F64 else torch.float32
    out = []
    for k, (n_xy, n_z, nf, nt) in enumerate(SHAPES):
        cfg = workloads.small_pixel(k=120 + k, n_xy=n_xy, n_z=n_z, n_freq=nf, n_time=nt, n_pairs=40, n_colloc=10)
        plan, lay = wt.wt_h_plan_create(cfg["cell"], cfg["columns"], cfg["spectrum"], precision=precision)
        car = cfg["carriers"]
        it = dict(plan=plan, lay=lay, pos=torch.from_numpy(car["pos"]).to("cuda", dt),
                  q=torch.from_numpy(car["charge"]).to("cuda", dt), tr=torch.from_numpy(car["track"]).to("cuda"),
                  n_tracks=car["n_tracks"], out=torch.full((car["n_tracks"], nt), float("nan"), dtype=dt,
                                                           device="cuda"))
        out.append(it)
    return out


def _arg(it):
    return dict(plan=it["plan"], n_carriers=it["pos"].shape[0], n_tracks=it["n_tracks"], d_pos=it["pos"].data_ptr(),
                d_charge=it["q"].data_ptr(), d_track=it["tr"].data_ptr(), d_current=it["out"].data_ptr())


def _sequential(ctx, items):
    ref = []
    for it in items:
        lay = it["lay"]
        ws = torch.empty(lay["workspace_bytes"], dtype=torch.uint8, device="cuda")
        h = torch.empty(lay["h_bytes"], dtype=torch.uint8, device="cuda")
        wt.wt_h_solve(ctx, it["plan"], ws.data_ptr(), ws.numel(), h.data_ptr(), h.numel())
        out = torch.empty_like(it["out"])
        wt.wt_current(ctx, it["plan"], h.data_ptr(), it["pos"].shape[0], it["n_tracks"], it["pos"].data_ptr(),
                      it["q"].data_ptr(), it["tr"].data_ptr(), out.data_ptr())
        torch.cuda.synchronize()
        ref.append(out.clone())
    return ref


def _lane_buffers(items, n_lanes, extra=1.0):
    ws_b = max(it["lay"]["workspace_bytes"] for it in items)
    h_b = int(max(it["lay"]["h_bytes"] for it in items) * extra)
    ws = [torch.empty(ws_b, dtype=torch.uint8, device="cuda") for _ in range(n_lanes)]
    hs = [torch.empty(h_b, dtype=torch.uint8, device="cuda") for _ in range(n_lanes)]
    return ws, ws_b, hs, h_b


def _rel(a, b):
    return float((a - b).abs().max() / b.abs().max())


@pytest.mark.parametrize("precision", [wt.WT_F64, wt.WT_F32], ids=["f64", "f32"])
@pytest.mark.parametrize("n_lanes", [1, 2, 3])
def test_batch_matches_sequential(n_lanes, precision):
    say(f"test_batch_matches_sequential lanes={n_lanes} precision={precision}")
    ctx = wt.wt_context_create(0, torch.cuda.current_stream().cuda_stream)
    items = _items(precision)
    ref = _sequential(ctx, items)
    ws, ws_b, hs, h_b = _lane_buffers(items, n_lanes)
    st, per = wt.wt_batch_run(ctx, [_arg(it) for it in items], [w.data_ptr() for w in ws], ws_b,
                              [h.data_ptr() for h in hs], h_b)
    torch.cuda.synchronize()
    assert st == wt.WT_OK and per == [wt.WT_OK] * len(items)
    tol = 1e-12 if precision == wt.WT_F64 else 1e-5
    for k, (it, r) in enumerate(zip(items, ref)):
        err = _rel(it["out"], r)
        say(f"  item {k} {SHAPES[k]}: max rel diff {err:.1e}")
        assert err <= tol
    for it in items:
        wt.wt_h_plan_destroy(it["plan"])
    wt.wt_context_destroy(ctx)


def test_batch_item_status():
    ctx = wt.wt_context_create(0, torch.cuda.current_stream().cuda_stream)
    items = _items()
    small = sorted(range(len(items)), key=lambda i: items[i]["lay"]["h_bytes"])
    # lane buffers sized for all but the largest item's H
    h_b = items[small[-2]]["lay"]["h_bytes"]
    ws_b = max(it["lay"]["workspace_bytes"] for it in items)
    ws = [torch.empty(ws_b, dtype=torch.uint8, device="cuda") for _ in range(2)]
    hs = [torch.empty(h_b, dtype=torch.uint8, device="cuda") for _ in range(2)]
    args = [_arg(it) for it in items]
    args[small[0]]["d_current"] = 0                           # no output: invalid
    st, per = wt.wt_batch_run(ctx, args, [w.data_ptr() for w in ws], ws_b, [h.data_ptr() for h in hs], h_b,
                              raise_on_error=False)
    torch.cuda.synchronize()
    want = [wt.WT_OK] * len(items)
    want[small[-1]] = wt.WT_E_WORKSPACE
    want[small[0]] = wt.WT_E_INVALID_ARG
    assert per == want
    assert st == want[min(small[0], small[-1])]               # the first skipped item's status
    ref = _sequential(ctx, items)
    for k, it in enumerate(items):
        if want[k] == wt.WT_OK:
            assert _rel(it["out"], ref[k]) <= 1e-5
        else:
            assert torch.isnan(it["out"]).all()                   # skipped: untouched
    # bad arguments: nothing runs
    assert wt.wt_batch_run(ctx, args, [], ws_b, [], h_b, raise_on_error=False)[0] == wt.WT_E_INVALID_ARG
    nine = [ws[0].data_ptr()] * 9
    assert wt.wt_batch_run(ctx, args, nine, ws_b, nine, h_b, raise_on_error=False)[0] == wt.WT_E_INVALID_ARG
    for it in items:
        wt.wt_h_plan_destroy(it["plan"])
    wt.wt_context_destroy(ctx)


def test_batch_graph_replays_match_eager():
    say("test_batch_graph_replays_match_eager")
    stream = torch.cuda.Stream()
    ctx = wt.wt_context_create(0, stream.cuda_stream)
    items = _items()
    ws, ws_b, hs, h_b = _lane_buffers(items, 3)
    args = [_arg(it) for it in items]

    def run():
        wt.wt_batch_run(ctx, args, [w.data_ptr() for w in ws], ws_b, [h.data_ptr() for h in hs], h_b)

    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        run()                                                 # eager: makes the lanes, sets kernel attributes
    stream.synchronize()
    ref = [it["out"].clone() for it in items]
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=stream):
        run()
    torch.cuda.synchronize()
    for rep in range(3):
        for it in items:
            it["out"].fill_(float("nan"))                     # eager work between replays
        for h in hs:
            h.zero_()
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            graph.replay()
        torch.cuda.synchronize()
        err = max(_rel(it["out"], r) for it, r in zip(items, ref))
        say(f"  replay {rep}: max rel diff {err:.1e}")
        assert err <= 1e-5
    del graph
    for it in items:
        wt.wt_h_plan_destroy(it["plan"])
    wt.wt_context_destroy(ctx)


def _oracle_refs(keys):
    """The FP64 oracle's H (whole grid) and currents for the items SHAPES[k]."""
    import oracle

    refs = {}
    for k in keys:
        n_xy, n_z, nf, nt = SHAPES[k]
        cfg = workloads.small_pixel(k=120 + k, n_xy=n_xy, n_z=n_z, n_freq=nf, n_time=nt, n_pairs=40, n_colloc=10)
        ref = oracle.weighting_field(cfg["cell"], cfg["columns"], cfg["spectrum"])
        car = dict(cfg["carriers"])
        car["pos"] = np.asarray(car["pos"]).astype(np.float32).astype(np.float64)
        car["charge"] = np.asarray(car["charge"]).astype(np.float32).astype(np.float64)
        refs[k] = dict(cfg=cfg, H=ref["H"], i=oracle.induced_current(ref["H"], cfg["cell"], car))
    return refs


def _check_items_against_oracle(items, keys, hs, refs, label):
    from gpu_common import h_standard, rel_l2

    # two items on two lanes: the larger H goes first, to lane 0 (longest
    # first, each to the lane with the least work)
    order = sorted(range(len(keys)), key=lambda j: -items[j]["lay"]["h_bytes"])
    for lane, j in enumerate(order):
        k, it = keys[j], items[j]
        r = refs[k]
        N, nt = r["cfg"]["cell"]["N"], r["cfg"]["spectrum"]["n_time"]
        n_vals = N[0] * N[1] * N[2] * nt * 3
        run = dict(layout=it["lay"], h=hs[lane].view(torch.float32)[:n_vals], decode=1.0)
        e_h = rel_l2(h_standard(run, r["cfg"]), r["H"])
        e_i = rel_l2(it["out"].double().cpu().numpy(), r["i"])
        say(f"  {label} item {k} {SHAPES[k]} (lane {lane}): H rel L2 {e_h:.2e}, i rel L2 {e_i:.2e}")
        assert e_h <= 1e-5 and e_i <= 1e-4


def test_batch_items_against_the_oracle():
    """Two variants of uneven grids through wt_batch_run on two lanes, eager
    and as replays of a captured graph: each lane's H (whole grid) and each
    item's currents against the FP64 oracle (float32 H 1e-5, i 1e-4)."""
    keys = [1, 4]
    say("oracle: two variants, whole-grid H and currents")
    refs = _oracle_refs(keys)
    stream = torch.cuda.Stream()
    ctx = wt.wt_context_create(0, stream.cuda_stream)
    wt.wt_context_set_current_form(ctx, wt.WT_CURRENT_BINNED)    # the lanes' currents binned
    all_items = _items()
    items = [all_items[k] for k in keys]
    ws, ws_b, hs, h_b = _lane_buffers(items, 2)
    args = [_arg(it) for it in items]

    def run():
        wt.wt_batch_run(ctx, args, [w.data_ptr() for w in ws], ws_b, [h.data_ptr() for h in hs], h_b)

    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        run()
    stream.synchronize()
    _check_items_against_oracle(items, keys, hs, refs, "eager")
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=stream):
        run()
    torch.cuda.synchronize()
    for rep in range(2):
        for it in items:
            it["out"].fill_(float("nan"))
        for h in hs:
            h.zero_()
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            graph.replay()
        torch.cuda.synchronize()
        _check_items_against_oracle(items, keys, hs, refs, f"replay {rep}")
    del graph
    for it in all_items:
        wt.wt_h_plan_destroy(it["plan"])
    wt.wt_context_destroy(ctx)
