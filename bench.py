#!/usr/bin/env python3
"""Benchmark of the weighting-field path on one MI355X.

One step = the whole hot path on one batch of synthetic input: Green's tables,
collocation solves for all frequencies, time transform, in-plane field table,
synthesis of H(x, y, z, t) on the whole grid, and the Eq. 1 current of all
carriers.  Workload: periodic 50x50x300 um pixel on a 128x128x256 grid, five
seeded column resistivities, 256 frequencies up to 50 GHz, 200 samples of
10 ps, one minimum-ionising track along z with 1e4 electron/hole pairs
(2e4 carriers).  H and the current are computed in float32, the boundary fit
and time transform in float64.  Inputs are resident on the GPU before timing.

Prints one JSON line.  value = grid points x frequencies per second of the
whole step; tracks/s and carriers/s of the current stage are extra fields.
The same step with H stored as scaled float16 (the mixed-precision path) is
timed after it and reported under "mixed", with its errors against the FP64
oracle (H) and the float32 path (the current).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "H(x,t) grid·freq pts/s + carrier tracks/s, mixed vs plain FP64 at stated rel err"
HBM_PEAK_GBS = 8000.0

# HBM bytes per launch of k_synthesis_pipe on this workload (float32, float16 and float64
# H): rocprofv3 FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0 (the factors a 1 GiB
# device-to-device copy gives for the same counters), in
# profiles/k_synthesis_pipe_128x128x256.md.  Reported only while the kernel's
# sources are the ones they were measured on.
SYNTH_TRAFFIC_BYTES = {"plain": 10170782051, "mixed": 5136826957, "f64": 20341324523}
SYNTH_TRAFFIC_SOURCES_SHA256 = "82f4e289f86c33a2bdf3830c18ebecad6adeffc91c4ddda78acee6d2c20464d3"
SYNTH_SOURCES = ("k_bulk.hip", "synth_pipe.hpp", "fft.hpp", "common.hpp")


def synthesis_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for name in SYNTH_SOURCES:
        with open(os.path.join(ROOT, "paper_2605_13987_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def current_compulsory_bytes_device(pos, cell, n_tracks, nt, elem_bytes, torch, chunk=1 << 17):
    """``current_compulsory_bytes`` for carriers held on the device (torch),
    in chunks of carriers.  Returns (bytes, moving steps)."""
    N, L = cell["N"], cell["L"]
    scale = torch.tensor([N[a] / L[a] for a in range(3)], dtype=torch.float64, device=pos.device)
    nodes, needs = [], []
    n_steps = 0
    for c0 in range(0, pos.shape[0], chunk):
        P = pos[c0:c0 + chunk].double()
        moving = (P[:, 1:] != P[:, :-1]).any(dim=2)
        ci, mi = moving.nonzero(as_tuple=True)
        n_steps += int(ci.numel())
        lo = torch.floor(0.5 * (P[ci, mi] + P[ci, mi + 1]) * scale).long()
        lags = nt - mi
        for ox in (0, 1):
            for oy in (0, 1):
                for oz in (0, 1):
                    x = (lo[:, 0] + ox) % N[0]
                    y = (lo[:, 1] + oy) % N[1]
                    z = (lo[:, 2] + oz) % N[2]
                    nodes.append((x * N[1] + y) * N[2] + z)
                    needs.append(lags)
    node = torch.cat(nodes)
    need = torch.cat(needs)
    uniq, inv = torch.unique(node, return_inverse=True)
    best = torch.zeros(uniq.numel(), dtype=need.dtype, device=need.device).scatter_reduce(0, inv, need, "amax")
    h_bytes = int(best.sum().item()) * 3 * elem_bytes
    return h_bytes + 24 * n_steps + n_tracks * nt * 4, n_steps


def c5_section(torch, wt, np, steps):
    """The 256x256x512 workload (1e6 carriers in 100 tracks, 512 frequencies,
    400 samples): float16-scaled H (80.5 GB) and float32 H (161 GB), one at a
    time, each a whole step (solve + current) timed over ``steps`` steps."""
    from paper_2605_13987_amd import layout, workloads

    cfg = workloads.pixel_256x256x512_tracks(device="cuda", out_dtype=torch.float32)
    cell, spec, car = cfg["cell"], cfg["spectrum"], cfg["carriers"]
    N, nt, n_tr = cell["N"], spec["n_time"], car["n_tracks"]
    n_pts = N[0] * N[1] * N[2]
    n_c = car["pos"].shape[0]
    stream = torch.cuda.current_stream()
    ctx = wt.wt_context_create(0, stream.cuda_stream)
    res = {"workload": (f"{N[0]}x{N[1]}x{N[2]} grid of the 50x50x300 um pixel, {spec['n_freq']} frequencies to "
                        f"50 GHz, {nt} x 10 ps, {n_tr} MIP tracks of 5e3 e/h pairs ({n_c} carriers), drift + "
                        f"0.5 um Gaussian diffusion per step"), "n_carriers": n_c, "n_tracks": n_tr}
    currents, cols_h = {}, {}
    for name, fmt, eb in (("mixed", wt.WT_H_F16_SCALED, 2), ("plain", wt.WT_H_PLAIN, 4)):
        plan, lay = wt.wt_h_plan_create(cell, cfg["columns"], spec, precision=wt.WT_F32, ir_max_iter=2, ir_tol=1e-12,
                                        h_format=fmt)
        ws = torch.empty(lay["workspace_bytes"], dtype=torch.uint8, device="cuda")
        hbuf = torch.empty(lay["h_bytes"], dtype=torch.uint8, device="cuda")
        out = torch.empty((n_tr, nt), dtype=torch.float32, device="cuda")

        def step():
            wt.wt_h_solve(ctx, plan, ws.data_ptr(), ws.numel(), hbuf.data_ptr(), lay["h_bytes"])
            wt.wt_current(ctx, plan, hbuf.data_ptr(), n_c, n_tr, car["pos"].data_ptr(), car["charge"].data_ptr(),
                          car["track"].data_ptr(), out.data_ptr())

        _, rep_s = wt.wt_h_solve(ctx, plan, ws.data_ptr(), ws.numel(), hbuf.data_ptr(), lay["h_bytes"], report=True)
        step()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            step()
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        wt.wt_context_enable_timing(ctx, True)
        wt.wt_h_solve(ctx, plan, ws.data_ptr(), ws.numel(), hbuf.data_ptr(), lay["h_bytes"])
        stage = dict(wt.wt_context_stage_times(ctx))
        wt.wt_current(ctx, plan, hbuf.data_ptr(), n_c, n_tr, car["pos"].data_ptr(), car["charge"].data_ptr(),
                      car["track"].data_ptr(), out.data_ptr())
        stage.update(dict(wt.wt_context_stage_times(ctx)))
        wt.wt_context_enable_timing(ctx, False)
        synth_bytes = n_pts * nt * 3 * eb + N[0] * N[1] * len(cfg["columns"]) * (N[2] // 2) * 3 * 8
        achieved = synth_bytes / (stage["synthesis"] * 1e-3) / 1e9
        cur_bytes, n_steps = current_compulsory_bytes_device(car["pos"], cell, n_tr, nt, eb, torch)
        t_cur = stage["current"] * 1e-3
        res[name] = {"ms_per_step": ms, "value": n_pts * spec["n_freq"] / (ms * 1e-3), "unit": "grid*freq pts/s",
                     "h_bytes": lay["h_bytes"], "h_scale": rep_s["h_scale"],
                     "backward_error_max": rep_s["backward_error_max"],
                     "stage_ms": {k: round(v, 4) for k, v in stage.items()},
                     "tracks_per_s": n_tr / t_cur, "carriers_per_s": n_c / t_cur, "events_per_s": n_steps / t_cur,
                     "synthesis_roofline": {"kernel": "k_synthesis_pipe", "bound": "hbm", "achieved": achieved,
                                            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                                            "bytes_per_launch": synth_bytes},
                     "current_roofline": {"kernel": "k_current", "bound": "hbm", "compulsory_bytes": cur_bytes,
                                          "achieved": cur_bytes / t_cur / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                          "frac": cur_bytes / t_cur / 1e9 / HBM_PEAK_GBS, "moving_steps": n_steps}}
        currents[name] = out.double().cpu().numpy()
        if name == "mixed":
            per = N[2] * nt * 3
            idx = torch.tensor([i * N[1] + j for i, j in C5_COLS], device="cuda")
            h16 = hbuf[:n_pts * nt * 3 * 2].view(torch.float16).view(-1, per)
            vals = h16.index_select(0, idx).double().cpu().numpy() / rep_s["h_scale"]
            cols_h[name] = layout.to_standard(vals, N, nt, lay["h_time_block"])
        print(f"# 256x256x512 {name}: {ms:.2f} ms/step, stages {res[name]['stage_ms']}", file=sys.stderr, flush=True)
        wt.wt_h_plan_destroy(plan)
        del ws, hbuf, out
        torch.cuda.empty_cache()
    wt.wt_context_destroy(ctx)
    a, b = currents["mixed"], currents["plain"]
    res["rel_err"] = {"i_mixed_vs_plain": float(np.linalg.norm(a - b) / np.linalg.norm(b))}
    return res, cfg, cols_h


C5_COLS = [(0, 0), (128, 128), (150, 128), (20, 200)]


def c5_oracle_errors(cfg, cols_h):
    """Errors of the 256x256x512 float16 H on sampled columns against the oracle's direct sums."""
    import numpy as np

    import oracle

    ref = oracle.weighting_field(cfg["cell"], cfg["columns"], cfg["spectrum"], route="columns", cols_ij=C5_COLS)
    out = {}
    for name, h in cols_h.items():
        out[name] = float(np.linalg.norm(h - ref["H_cols"]) / np.linalg.norm(ref["H_cols"]))
    return out


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--variants", type=int, default=64,
                    help="geometry variants in the batched (graph-captured) measurement; 0 skips it")
    ap.add_argument("--cpu-seconds", type=float, default=20.0,
                    help="approximate CPU time of the oracle baseline sample")
    ap.add_argument("--c5-steps", type=int, default=3,
                    help="timed steps of the 256x256x512 workload (1e6 carriers); 0 skips it")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="first copy MIB mebibytes device-to-device 3 times (counter calibration)")
    return ap.parse_args()


def blas_threads():
    try:
        from threadpoolctl import threadpool_info
        n = [p.get("num_threads", 1) for p in threadpool_info()]
        return max(n) if n else 1
    except Exception:
        return os.cpu_count() or 1


def cpu_baseline(cfg, gpu_columns, budget_s):
    """The FP64 oracle on a bounded sample of the same workload.

    Timed parts: the boundary fit for every frequency and the time transform
    (whole-step work), the field on lattices of 256 grid columns added until
    about half the time budget is spent, and Eq. 1 on strided subsets of the
    carriers until about a third of it is.  The whole-step rate is
    extrapolated from them: fit + per-column time x all columns + per-carrier
    time x all carriers.  gpu_columns maps a path name to a function that
    returns the GPU's H on given columns, for the error figures.
    """
    import numpy as np

    from oracle import collocation, convolution, field, green, timegrid
    from paper_2605_13987_amd import workloads

    cell, cols, spec = cfg["cell"], cfg["columns"], cfg["spectrum"]
    N = cell["N"]
    t0 = time.perf_counter()
    sol = collocation.solve_spectrum(cell, cols, spec)
    q_t = timegrid.to_time(sol["q"], spec)
    t_fit = time.perf_counter() - t0
    s, src = green.smoothing_widths(cell, cols), collocation.sources(cols)
    sample, t_cols = [], 0.0
    err_num = {name: 0.0 for name in gpu_columns}
    err_den = 0.0
    for shift in range(64):                       # 16 x 16 lattices off the column axes
        lattice = [((i + 3 + shift) % N[0], (j + 5 + 3 * shift) % N[1])
                   for i in range(0, N[0], N[0] // 16) for j in range(0, N[1], N[1] // 16)]
        seen = set(sample)
        lattice = [c for c in lattice if c not in seen]
        t0 = time.perf_counter()
        ref = field.field_columns(cell, s, src, q_t, lattice)
        t_cols += time.perf_counter() - t0
        for name, fn in gpu_columns.items():
            err_num[name] += float(np.sum((fn(lattice) - ref) ** 2))
        err_den += float(np.sum(ref ** 2))
        sample += lattice
        if t_cols > 0.5 * budget_s:
            break
    err = {name: (v / err_den) ** 0.5 for name, v in err_num.items()}
    # convolution: strided carrier subsets on a synthetic field of the same grid
    car = cfg["carriers"]
    n_car = car["pos"].shape[0]
    f = workloads.synthetic_h_factors(workloads.rng_for(99), N, spec["n_time"])
    h_at = lambda ix, iy, iz: workloads.synthetic_h_values(f, ix, iy, iz)
    stride, n_done, t_conv = 50, 0, 0.0
    for off in range(stride):
        sub = np.arange(off, n_car, stride)
        t0 = time.perf_counter()
        convolution.induced_current(h_at, cell, car["pos"][sub], car["charge"][sub], car["track"][sub],
                                    car["n_tracks"])
        t_conv += time.perf_counter() - t0
        n_done += sub.size
        if t_conv > budget_s / 3:
            break
    n_cols_all = N[0] * N[1]
    t_step = t_fit + t_cols * n_cols_all / len(sample) + t_conv * n_car / n_done
    return dict(value=N[0] * N[1] * N[2] * spec["n_freq"] / t_step, unit="grid*freq pts/s",
                cores=blas_threads(), kind="oracle",
                sample=(f"boundary fit for all {spec['n_freq']} frequencies + time transform ({t_fit:.1f} s), "
                        f"field on {len(sample)} of {n_cols_all} grid columns, all z and t ({t_cols:.1f} s), "
                        f"Eq. 1 on {n_done} of {n_car} carriers ({t_conv:.1f} s); whole step extrapolated "
                        f"from these parts: {t_step:.0f} s"),
                step_s_extrapolated=t_step,
                tracks_per_s=car["n_tracks"] / (t_conv * n_car / n_done),
                carriers_per_s=n_done / t_conv), err


def current_compulsory_bytes(cfg, elem_bytes):
    """Compulsory HBM bytes of the Eq. 1 convolution: every node that is a
    trilinear corner of some moving step, times the lags it is read for (a
    step at m reads lags 0..N_t-1-m), times 3 components, plus 24 B per step
    (midpoint and displacement) and the output.  Returns (bytes, steps)."""
    import numpy as np

    cell, spec, car = cfg["cell"], cfg["spectrum"], cfg["carriers"]
    N, L, nt = cell["N"], cell["L"], spec["n_time"]
    P = np.asarray(car["pos"], dtype=np.float32).astype(np.float64)
    d = P[:, 1:, :] - P[:, :-1, :]
    moving = np.any(d != 0, axis=2)
    c_idx, m_idx = np.nonzero(moving)
    mid = 0.5 * (P[c_idx, m_idx, :] + P[c_idx, m_idx + 1, :]) * (np.asarray(N) / np.asarray(L))
    lo = np.floor(mid).astype(np.int64)
    lags = nt - m_idx
    node = np.empty(0, dtype=np.int64)
    need = np.empty(0, dtype=np.int64)
    for ox in (0, 1):
        for oy in (0, 1):
            for oz in (0, 1):
                x = (lo[:, 0] + ox) % N[0]
                y = (lo[:, 1] + oy) % N[1]
                z = (lo[:, 2] + oz) % N[2]
                node = np.concatenate([node, (x * N[1] + y) * N[2] + z])
                need = np.concatenate([need, lags])
    order = np.lexsort((-need, node))
    node, need = node[order], need[order]
    first = np.ones(node.size, dtype=bool)
    first[1:] = node[1:] != node[:-1]
    h_bytes = int(need[first].sum()) * 3 * elem_bytes
    n_steps = int(c_idx.size)
    return h_bytes + 24 * n_steps + car["n_tracks"] * nt * 4, n_steps


def batched_variants(wt, workloads, torch, n_variants, replays, n_lanes=4):
    """The geometry-variant batch: n_variants seeded cells of uneven grids and
    frequency counts, each a full step (H solve + current of its track), run
    eagerly with the plans' default synthesis launch, then with every plan
    autotuned (wt_h_plan_tune), eagerly and as one captured HIP graph on one
    stream, sharing one workspace and one H buffer sized for the largest
    variant; then the same batch through wt_batch_run over n_lanes lanes of
    streams (a workspace and an H buffer per lane), eager and captured."""
    import numpy as np

    variants = [workloads.geometry_variant(k) for k in range(n_variants)]
    stream = torch.cuda.Stream()
    ctx = wt.wt_context_create(0, stream.cuda_stream)
    items, ws_bytes, h_bytes, pts = [], 0, 0, 0
    for v in variants:
        plan, lay = wt.wt_h_plan_create(v["cell"], v["columns"], v["spectrum"], precision=wt.WT_F32)
        car = v["carriers"]
        N = v["cell"]["N"]
        items.append(dict(plan=plan, lay=lay,
                          pos=torch.from_numpy(car["pos"]).to("cuda", torch.float32),
                          q=torch.from_numpy(car["charge"]).to("cuda", torch.float32),
                          tr=torch.from_numpy(car["track"]).to("cuda"),
                          out=torch.empty((car["n_tracks"], v["spectrum"]["n_time"]), dtype=torch.float32,
                                          device="cuda"),
                          n_tr=car["n_tracks"]))
        ws_bytes = max(ws_bytes, lay["workspace_bytes"])
        h_bytes = max(h_bytes, lay["h_bytes"])
        pts += N[0] * N[1] * N[2] * v["spectrum"]["n_freq"]
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    h = torch.empty(h_bytes, dtype=torch.uint8, device="cuda")

    def batch():
        for it in items:
            wt.wt_h_solve(ctx, it["plan"], ws.data_ptr(), ws.numel(), h.data_ptr(), h.numel())
            wt.wt_current(ctx, it["plan"], h.data_ptr(), it["pos"].shape[0], it["n_tr"], it["pos"].data_ptr(),
                          it["q"].data_ptr(), it["tr"].data_ptr(), it["out"].data_ptr())

    def timed(fn):
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    with torch.cuda.stream(stream):
        batch()                                                   # warm-up, kernel attributes
        t_default = timed(batch)
    t0 = time.perf_counter()
    tuned = [wt.wt_h_plan_tune(ctx, it["plan"], ws.data_ptr(), ws.numel(), h.data_ptr(), h.numel()) for it in items]
    tune_s = time.perf_counter() - t0
    with torch.cuda.stream(stream):
        batch()
        t_eager = timed(batch)
    ref = [it["out"].clone() for it in items]
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=stream):
        batch()
    t_graph = []
    err = 0.0
    for _ in range(replays):
        with torch.cuda.stream(stream):                           # a replay runs on the current stream
            t_graph.append(timed(graph.replay))
        err = max(err, max(float((it["out"] - r).abs().max() / r.abs().max().clamp_min(1e-30))
                           for it, r in zip(items, ref)))
    del graph
    # the same batch on lanes of streams (wt_batch_run: longest item first, to
    # the lane with the least work), eager and as one captured graph
    del ws, h
    lane_ws = [torch.empty(ws_bytes, dtype=torch.uint8, device="cuda") for _ in range(n_lanes)]
    lane_h = [torch.empty(h_bytes, dtype=torch.uint8, device="cuda") for _ in range(n_lanes)]
    args = [dict(plan=it["plan"], n_carriers=it["pos"].shape[0], n_tracks=it["n_tr"], d_pos=it["pos"].data_ptr(),
                 d_charge=it["q"].data_ptr(), d_track=it["tr"].data_ptr(), d_current=it["out"].data_ptr())
            for it in items]

    def lanes():
        wt.wt_batch_run(ctx, args, [w.data_ptr() for w in lane_ws], ws_bytes, [x.data_ptr() for x in lane_h], h_bytes)

    with torch.cuda.stream(stream):
        lanes()
        t_lanes = timed(lanes)
    err_lanes = max(float((it["out"] - r).abs().max() / r.abs().max().clamp_min(1e-30)) for it, r in zip(items, ref))
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=stream):
        lanes()
    t_lanes_graph = []
    for _ in range(replays):
        with torch.cuda.stream(stream):
            t_lanes_graph.append(timed(graph.replay))
        err_lanes = max(err_lanes, max(float((it["out"] - r).abs().max() / r.abs().max().clamp_min(1e-30))
                                       for it, r in zip(items, ref)))
    del graph, lane_ws, lane_h
    for it in items:
        wt.wt_h_plan_destroy(it["plan"])
    wt.wt_context_destroy(ctx)
    n_pipe = sum(1 for r in tuned if r["fft_n1"] > 0)
    n_tuned = sum(1 for r in tuned if r["n_candidates"] > 1)
    return {"n_variants": n_variants, "grid_freq_pts": pts, "ms_eager_default_launch": t_default,
            "autotune_s": tune_s, "variants_autotuned": n_tuned,
            "ms_eager": t_eager, "ms_graph": float(np.median(t_graph)),
            "value_graph": pts / (np.median(t_graph) * 1e-3), "unit": "grid*freq pts/s",
            "replay_vs_eager_current_max_rel_diff": err, "variants_on_register_fft_synthesis": n_pipe,
            "lanes": {"n_lanes": n_lanes, "ms_eager": t_lanes, "ms_graph": float(np.median(t_lanes_graph)),
                      "value_graph": pts / (np.median(t_lanes_graph) * 1e-3),
                      "current_max_rel_diff_vs_one_stream": err_lanes,
                      "note": "wt_batch_run: the items spread over lanes of streams, each lane its own workspace "
                              "and H buffer"},
            "workload": ("seeded geometry variants: pitch 25-100 um, radius 3-10 um, five resistivities "
                         "0.01-1 ohm cm, grids 64..160 x 64..160 x 64..320 (even 2*3*5-smooth), 64-256 frequencies, "
                         "200 x 10 ps, one 1e3-pair MIP track each; float32 H, one shared workspace and H buffer")}


def adjoint_section(cfg, torch, wt, np, reps):
    """Gradient of the peak time and windowed charge of the track's current with
    respect to the 5 resistivities and the radii (adjoint), against the cost of
    the central-difference scan it replaces and against the FP64 adjoint."""
    from paper_2605_13987_amd.grad import ColumnModel, signal_features
    from paper_2605_13987_amd import workloads

    dt = cfg["spectrum"]["dt"]
    rng = workloads.rng_for(63)
    t_c, t_s = rng.uniform(0.5e-9, 1.5e-9), rng.uniform(0.1e-9, 0.4e-9)
    out = {}
    grads = {}
    for prec in (wt.WT_F32, wt.WT_F64):
        model = ColumnModel(cfg["cell"], cfg["columns"], cfg["spectrum"], cfg["carriers"], precision=prec)
        theta = model.theta0()
        plan, cur = model.solve(theta)
        i = cur.detach().requires_grad_(True)
        t_peak, q_w = signal_features(i, dt, t_c, t_s, 2e-9)
        g_tp = torch.autograd.grad(t_peak.sum(), i)[0]
        g_qw = torch.autograd.grad(q_w.sum(), i)[0]
        (tp_th, tp_p), (qw_th, qw_p) = model.gradient(plan, g_tp), model.gradient(plan, g_qw)
        p0 = float(cfg["cell"]["L"][0])
        grads[prec] = (theta.numpy(), np.append(tp_th.numpy().ravel(), p0 * float(tp_p)),
                       np.append(qw_th.numpy().ravel(), p0 * float(qw_p)))
        if prec != wt.WT_F32:
            continue
        s = torch.cuda.current_stream()
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        torch.cuda.synchronize()
        e0.record(s)
        for _ in range(reps):
            plan, cur = model.solve(theta)
        e1.record(s)
        for _ in range(reps):
            model.gradient(plan, g_tp)
        e2.record(s)
        torch.cuda.synchronize()
        fwd, bwd = e0.elapsed_time(e1) / reps, e1.elapsed_time(e2) / reps
        wt.wt_context_enable_timing(model.ctx, True)
        model.gradient(plan, g_tp)
        stages = dict(wt.wt_context_stage_times(model.ctx))
        wt.wt_context_enable_timing(model.ctx, False)
        n_par = sum(len(c["resistivity"]) + 1 for c in cfg["columns"]) + 1
        out.update({"n_params": n_par, "forward_ms": fwd, "backward_ms": bwd,
                    "backward_stage_ms": {k: round(v, 4) for k, v in stages.items()},
                    "central_difference_scan_ms": 2 * n_par * fwd,
                    "note": "backward = wt_h_gradient (event projections, transposed FP64 solves, contraction) for "
                            "5 resistivities, 2 radii and the pitch; the scan it replaces needs 2 forward solves "
                            "per parameter"})
    th, tp32, qw32 = grads[wt.WT_F32]
    _, tp64, qw64 = grads[wt.WT_F64]
    slots = [(w, p) for w, c in enumerate(cfg["columns"]) for p in list(range(len(c["resistivity"]))) + [4]]

    def logd(g):
        # log-derivatives: theta dL/dtheta per live slot, then pitch dL/dpitch
        return np.array([th[w, p] * g[5 * w + p] for w, p in slots] + [g[-1]])

    def rel(a, b):
        return float(np.max(np.abs(logd(a) - logd(b))) / np.max(np.abs(logd(b))))

    out["log_gradient_t_peak_s"] = {"readout_rho": float(logd(tp32)[0]),
                                    "bias_rho_sum": float(sum(logd(tp32)[2:6])),
                                    "readout_radius": float(logd(tp32)[1]), "bias_radius": float(logd(tp32)[6]),
                                    "pitch": float(logd(tp32)[7])}
    out["rel_err_float32_vs_float64_adjoint"] = {"t_peak": rel(tp32, tp64), "q_w": rel(qw32, qw64)}
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              f"(the path's multi-GPU decomposition is described, not built).", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2605_13987_amd import layout, workloads, wt

    if args.copy_probe:
        n = args.copy_probe * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(f"# copy probe: 3 x {args.copy_probe} MiB read + written", file=sys.stderr, flush=True)
        del src, dst

    cfg = workloads.mip_pixel_128x128x256()
    cell, spec, car = cfg["cell"], cfg["spectrum"], cfg["carriers"]
    N = cell["N"]
    n_pts = N[0] * N[1] * N[2]
    per_col = N[2] * spec["n_time"] * 3
    w = len(cfg["columns"])
    stream = torch.cuda.current_stream()
    ctx = wt.wt_context_create(0, stream.cuda_stream)
    pos = torch.from_numpy(car["pos"]).to("cuda", torch.float32)
    q = torch.from_numpy(car["charge"]).to("cuda", torch.float32)
    tr = torch.from_numpy(car["track"]).to("cuda")
    n_c, n_tr = pos.shape[0], car["n_tracks"]

    def run_path(h_format, precision=wt.WT_F32):
        """Time the whole step with H stored in h_format (or the whole path in
        float64); returns the figures and buffers."""
        plan, lay = wt.wt_h_plan_create(cell, cfg["columns"], spec, precision=precision, ir_max_iter=2,
                                        ir_tol=1e-12, h_format=h_format)
        f64 = precision == wt.WT_F64
        dt = torch.float64 if f64 else torch.float32
        ws = torch.empty(lay["workspace_bytes"], dtype=torch.uint8, device="cuda")
        hbuf = torch.empty(lay["h_bytes"], dtype=torch.uint8, device="cuda")
        out = torch.empty((n_tr, spec["n_time"]), dtype=dt, device="cuda")
        pos_p, q_p = (pos.double(), q.double()) if f64 else (pos, q)

        def step():
            wt.wt_h_solve(ctx, plan, ws.data_ptr(), ws.numel(), hbuf.data_ptr(), lay["h_bytes"])
            wt.wt_current(ctx, plan, hbuf.data_ptr(), n_c, n_tr, pos_p.data_ptr(), q_p.data_ptr(), tr.data_ptr(),
                          out.data_ptr())

        st, rep = wt.wt_h_solve(ctx, plan, ws.data_ptr(), ws.numel(), hbuf.data_ptr(), lay["h_bytes"], report=True)
        print(f"# h_format {h_format}: solve report {rep}", file=sys.stderr, flush=True)
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t_wall = time.perf_counter()
        e0.record(stream)
        for _ in range(args.steps):
            step()
        e1.record(stream)
        torch.cuda.synchronize()
        t_wall = time.perf_counter() - t_wall
        ms = e0.elapsed_time(e1) / args.steps
        print(f"# h_format {h_format}: timed {args.steps} steps: {ms:.3f} ms/step "
              f"(wall {1e3 * t_wall / args.steps:.3f} ms)", file=sys.stderr, flush=True)
        # per-stage durations from HIP events recorded by the library on the same stream
        wt.wt_context_enable_timing(ctx, True)
        stage = {}
        reps = max(3, min(args.steps, 10))
        for _ in range(reps):
            wt.wt_h_solve(ctx, plan, ws.data_ptr(), ws.numel(), hbuf.data_ptr(), lay["h_bytes"])
            for name, t in wt.wt_context_stage_times(ctx):
                stage[name] = stage.get(name, 0.0) + t / reps
            wt.wt_current(ctx, plan, hbuf.data_ptr(), n_c, n_tr, pos_p.data_ptr(), q_p.data_ptr(), tr.data_ptr(),
                          out.data_ptr())
            for name, t in wt.wt_context_stage_times(ctx):
                stage[name] = stage.get(name, 0.0) + t / reps
        wt.wt_context_enable_timing(ctx, False)
        torch.cuda.synchronize()
        wt.wt_h_plan_destroy(plan)
        if h_format == wt.WT_H_F16_SCALED:
            h = hbuf[:n_pts * spec["n_time"] * 3 * 2].view(torch.float16)
            off = lay["h_decode_offset"]
            decode = float(hbuf[off:off + 4].view(torch.float32).item())
        else:
            h, decode = hbuf.view(dt), 1.0
        t_h = sum(v for k, v in stage.items() if k != "current") * 1e-3
        t_cur = stage["current"] * 1e-3
        # synthesis kernel: algorithmic bytes = write of H + read of the field table per column
        synth_bytes = h.numel() * h.element_size() + N[0] * N[1] * w * (N[2] // 2) * 3 * (16 if f64 else 8)
        achieved = synth_bytes / (stage["synthesis"] * 1e-3) / 1e9
        return dict(ms=ms, stage=stage, t_h=t_h, t_cur=t_cur, rep=rep, h=h, decode=decode, out=out,
                    synth_bytes=synth_bytes, achieved=achieved, lay=lay)

    def columns_of(r):
        def fn(cols):
            idx = torch.tensor([i * N[1] + j for i, j in cols], device="cuda")
            vals = r["h"].view(-1, per_col).index_select(0, idx).cpu().numpy().astype(np.float64) * r["decode"]
            return layout.to_standard(vals, N, spec["n_time"], r["lay"]["h_time_block"])
        return fn

    plain = run_path(wt.WT_H_PLAIN)
    mixed = run_path(wt.WT_H_F16_SCALED)
    full64 = run_path(wt.WT_H_PLAIN, wt.WT_F64)
    cur_bytes, n_steps = current_compulsory_bytes(cfg, 4)
    cur_bytes16, _ = current_compulsory_bytes(cfg, 2)
    # FP64 boundary fit with M = 256 nodes per column (n = 513) at 512
    # frequencies to 50 GHz: the solve of the 50x50x300 um cell does not depend
    # on the grid (converged Green's function), so a small grid carries it
    m256 = workloads.small_pixel(k=48, n_xy=32, n_z=64, n_freq=512, n_time=16, n_pairs=1, n_colloc=256)
    plan_m, lay_m = wt.wt_h_plan_create(m256["cell"], m256["columns"], m256["spectrum"], precision=wt.WT_F32,
                                        ir_max_iter=2, ir_tol=1e-12)
    ws_m = torch.empty(lay_m["workspace_bytes"], dtype=torch.uint8, device="cuda")
    h_m = torch.empty(lay_m["h_bytes"], dtype=torch.uint8, device="cuda")
    _, rep_m = wt.wt_h_solve(ctx, plan_m, ws_m.data_ptr(), ws_m.numel(), h_m.data_ptr(), lay_m["h_bytes"],
                             report=True, raise_on_error=False)
    wt.wt_context_enable_timing(ctx, True)
    t_m = []
    for _ in range(3):
        wt.wt_h_solve(ctx, plan_m, ws_m.data_ptr(), ws_m.numel(), h_m.data_ptr(), lay_m["h_bytes"])
        t_m.append(dict(wt.wt_context_stage_times(ctx))["collocation_solve"])
    wt.wt_context_enable_timing(ctx, False)
    wt.wt_h_plan_destroy(plan_m)
    del ws_m, h_m
    solve_m256 = {"n_unknowns": lay_m["n_q"] + 1, "n_freq": 512, "ms": float(np.median(t_m)),
                  "backward_error_max": rep_m["backward_error_max"], "ir_iters_max": rep_m["ir_iters_max"]}
    print(f"# M = 256 solve: {solve_m256}", file=sys.stderr, flush=True)

    # readout electronics on the plain path's current: CR-RC front end
    # (tau = 250 ps, 1 kohm), seeded noise, constant fraction 0.5
    g_e = torch.from_numpy(workloads.cr_rc_response(spec["n_time"], spec["dt"])).to("cuda", torch.float32)
    n_e = torch.from_numpy(workloads.noise_samples(31, n_tr, spec["n_time"])).to("cuda", torch.float32)
    v_e = torch.empty((n_tr, spec["n_time"]), dtype=torch.float32, device="cuda")
    f_e = torch.empty((n_tr, 3), dtype=torch.float32, device="cuda")
    sigma_e = 1e-2 * float(plain["out"].abs().max().item()) * 1e3   # 1% of the peak current through 1 kohm

    def elec():
        wt.wt_electronics(ctx, wt.WT_F32, n_tr, spec["n_time"], spec["dt"], plain["out"].data_ptr(), g_e.data_ptr(),
                          n_e.data_ptr(), sigma_e, 0.5, v_e.data_ptr(), f_e.data_ptr())

    elec()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(10):
        elec()
    e1.record(stream)
    torch.cuda.synchronize()
    electronics = {"ms": e0.elapsed_time(e1) / 10, "n_tracks": n_tr,
                   "features_first_track": {"amplitude_V": float(f_e[0, 0]), "t_peak_s": float(f_e[0, 1]),
                                            "t_cfd_s": float(f_e[0, 2])}}

    adjoint = adjoint_section(cfg, torch, wt, np, max(3, min(args.steps, 10)))
    torch.cuda.empty_cache()
    print(f"# adjoint: {adjoint}", file=sys.stderr, flush=True)

    # the whole step captured once as a HIP graph and replayed
    g_stream = torch.cuda.Stream()
    g_ctx = wt.wt_context_create(0, g_stream.cuda_stream)
    g_plan, g_lay = wt.wt_h_plan_create(cell, cfg["columns"], spec, precision=wt.WT_F32, ir_max_iter=2, ir_tol=1e-12)
    g_ws = torch.empty(g_lay["workspace_bytes"], dtype=torch.uint8, device="cuda")
    g_h = torch.empty(g_lay["h_bytes"], dtype=torch.uint8, device="cuda")
    g_out = torch.empty((n_tr, spec["n_time"]), dtype=torch.float32, device="cuda")

    def g_step():
        wt.wt_h_solve(g_ctx, g_plan, g_ws.data_ptr(), g_ws.numel(), g_h.data_ptr(), g_lay["h_bytes"])
        wt.wt_current(g_ctx, g_plan, g_h.data_ptr(), n_c, n_tr, pos.data_ptr(), q.data_ptr(), tr.data_ptr(),
                      g_out.data_ptr())

    with torch.cuda.stream(g_stream):
        g_step()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=g_stream):
        g_step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(g_stream):                             # a replay runs on the current stream
        for _ in range(args.warmup):
            graph.replay()
        e0.record(g_stream)
        for _ in range(args.steps):
            graph.replay()
        e1.record(g_stream)
    torch.cuda.synchronize()
    graph_ms = e0.elapsed_time(e1) / args.steps
    del graph, g_ws, g_h
    wt.wt_h_plan_destroy(g_plan)
    wt.wt_context_destroy(g_ctx)
    torch.cuda.empty_cache()
    print(f"# captured step replayed: {graph_ms:.3f} ms/step", file=sys.stderr, flush=True)
    batch = None
    if args.variants > 0:
        batch = batched_variants(wt, workloads, torch, args.variants, 3)
        print(f"# batch of {args.variants} variants: default launch {batch['ms_eager_default_launch']:.1f} ms, "
              f"autotuned ({batch['autotune_s']:.1f} s) eager {batch['ms_eager']:.1f} ms, graph {batch['ms_graph']:.1f} ms",
              file=sys.stderr, flush=True)
        torch.cuda.empty_cache()

    c5, c5_cfg, c5_cols = None, None, None
    if args.c5_steps > 0:
        c5, c5_cfg, c5_cols = c5_section(torch, wt, np, args.c5_steps)
        torch.cuda.empty_cache()

    i_plain = plain["out"].double().cpu().numpy()
    i_mixed = mixed["out"].double().cpu().numpy()
    i_err_mixed = float(np.linalg.norm(i_mixed - i_plain) / np.linalg.norm(i_plain))
    i_f64 = full64["out"].cpu().numpy()
    i_err_plain_vs_f64 = float(np.linalg.norm(i_plain - i_f64) / np.linalg.norm(i_f64))
    i_err_mixed_vs_f64 = float(np.linalg.norm(i_mixed - i_f64) / np.linalg.norm(i_f64))

    stage, ms = plain["stage"], plain["ms"]
    measured = (list(N) == [128, 128, 256] and spec["n_time"] == 200 and w == 2
                and synthesis_sources_sha256() == SYNTH_TRAFFIC_SOURCES_SHA256)
    traffic = SYNTH_TRAFFIC_BYTES["plain"] if measured else None
    line = {
        "metric": METRIC,
        "value": n_pts * spec["n_freq"] / (ms * 1e-3),
        "unit": "grid*freq pts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": (f"plain path: {N[0]}x{N[1]}x{N[2]} grid of a 50x50x300 um pixel, readout + bias "
                         f"columns (r = 5 um, 5 seeded resistivities), {spec['n_freq']} frequencies to 50 GHz, "
                         f"{spec['n_time']} x 10 ps, one MIP track with {n_c // 2} e/h pairs ({n_c} carriers); "
                         f"f32 field/FFT/convolution and H, f64 boundary fit"),
            "grid": list(N), "n_freq": spec["n_freq"], "n_time": spec["n_time"], "n_carriers": n_c,
            "n_tracks": n_tr, "parallelism": "single GPU",
        },
        "tracks_per_s": n_tr / plain["t_cur"],
        "carriers_per_s": n_c / plain["t_cur"],
        "events_per_s": n_steps / plain["t_cur"],
        "current_roofline": {"kernel": "k_current", "bound": "hbm", "compulsory_bytes": cur_bytes,
                             "achieved": cur_bytes / plain["t_cur"] / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": cur_bytes / plain["t_cur"] / 1e9 / HBM_PEAK_GBS, "moving_steps": n_steps},
        "h_grid_freq_pts_per_s": n_pts * spec["n_freq"] / plain["t_h"],
        "h_grid_time_pts_per_s": n_pts * spec["n_time"] / plain["t_h"],
        "stage_ms": {k: round(v, 4) for k, v in stage.items()},
        "roofline": {"kernel": "k_synthesis_pipe", "bound": "hbm", "achieved": plain["achieved"],
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": plain["achieved"] / HBM_PEAK_GBS,
                     "traffic": traffic, "traffic_unit": "bytes/launch", "bytes_per_launch": plain["synth_bytes"]},
        "solve_report": plain["rep"],
        "solve_m256": solve_m256,
        "electronics": electronics,
        "adjoint": adjoint,
        "graph": {"ms_per_step": graph_ms, "note": "the same step captured once as a HIP graph and replayed"},
        "batched_variants": batch,
        "px256": c5,
        "f64": {
            "path": "the whole path in float64 (H in float64, 20 GB; register-FFT synthesis in blocks of 8 samples)",
            "value": n_pts * spec["n_freq"] / (full64["ms"] * 1e-3),
            "ms_per_step": full64["ms"],
            "tracks_per_s": n_tr / full64["t_cur"],
            "stage_ms": {k: round(v, 4) for k, v in full64["stage"].items()},
            "roofline": {"kernel": "k_synthesis_pipe (float64 H)", "bound": "hbm", "achieved": full64["achieved"],
                         "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": full64["achieved"] / HBM_PEAK_GBS,
                         "traffic": SYNTH_TRAFFIC_BYTES["f64"] if measured else None,
                         "traffic_unit": "bytes/launch", "bytes_per_launch": full64["synth_bytes"]},
            "rel_err": {"i_float32_path_vs_float64_path": i_err_plain_vs_f64,
                        "i_mixed_path_vs_float64_path": i_err_mixed_vs_f64},
        },
        "mixed": {
            "h_storage": "float16 holding H * h_scale (h_scale a power of two), decoded in float32",
            "h_scale": mixed["rep"]["h_scale"],
            "value": n_pts * spec["n_freq"] / (mixed["ms"] * 1e-3),
            "ms_per_step": mixed["ms"],
            "tracks_per_s": n_tr / mixed["t_cur"],
            "events_per_s": n_steps / mixed["t_cur"],
            "current_compulsory_gbs": cur_bytes16 / mixed["t_cur"] / 1e9,
            "h_grid_freq_pts_per_s": n_pts * spec["n_freq"] / mixed["t_h"],
            "stage_ms": {k: round(v, 4) for k, v in mixed["stage"].items()},
            "roofline": {"kernel": "k_synthesis_pipe (float16 H)", "bound": "hbm", "achieved": mixed["achieved"],
                         "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": mixed["achieved"] / HBM_PEAK_GBS,
                         "traffic": SYNTH_TRAFFIC_BYTES["mixed"] if measured else None,
                         "traffic_unit": "bytes/launch", "bytes_per_launch": mixed["synth_bytes"]},
            "rel_err": {"i_vs_float32_path": i_err_mixed},
        },
    }
    if not args.no_cpu_baseline:
        base, err = cpu_baseline(cfg, {"plain": columns_of(plain), "mixed": columns_of(mixed),
                                       "f64": columns_of(full64)}, args.cpu_seconds)
        line["cpu_baseline"] = base
        line["rel_err"] = {"H_sampled_columns_vs_fp64_oracle": err["plain"]}
        line["mixed"]["rel_err"]["H_sampled_columns_vs_fp64_oracle"] = err["mixed"]
        line["f64"]["rel_err"]["H_sampled_columns_vs_fp64_oracle"] = err["f64"]
        if c5 is not None:
            c5["mixed"]["rel_err_H_sampled_columns_vs_fp64_oracle"] = c5_oracle_errors(c5_cfg, c5_cols)["mixed"]
    print(json.dumps(line), flush=True)
    wt.wt_context_destroy(ctx)


if __name__ == "__main__":
    main()
