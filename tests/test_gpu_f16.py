"""GPU parity of the float16-scaled H (the mixed-precision path).

H is stored as float16 values of H * h_scale (a power of two chosen from a
bound on |H|) and decoded in float32.  Bar: 1e-3 relative L2 on H and on the
current against the FP64 oracle; float16 rounding alone is at most 2^-11
relative per value (4.9e-4), and the float32 path underneath is within 1e-5.
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_common import context, current, h_columns, h_standard, rel_l2, rounded_carriers, say, solve_h
from paper_2605_13987_amd import workloads, wt

pytestmark = pytest.mark.gpu

TOL = 1e-3


@pytest.fixture(scope="module")
def ctx():
    c = context()
    yield c
    wt.wt_context_destroy(c)


def _check_scale(run):
    assert run["status"] == wt.WT_OK, run["report"]
    scale = run["report"]["h_scale"]
    assert scale > 0 and run["decode"] == pytest.approx(1.0 / scale, rel=0, abs=0)
    e = np.log2(scale)
    assert e == np.round(e)                                  # a power of two
    hmax = float(run["h"].abs().max().float().item())
    say(f"  h_scale 2^{int(e)}, max stored |H| {hmax:.1f}")
    assert hmax <= 16384.0                                   # the bound holds: no overflow
    assert hmax >= 16384.0 / 2 ** 8                          # and wastes at most 8 bits of range


def test_32x32x64_f16_h_and_current(ctx, px32, px32_oracle):
    say("test_32x32x64_f16_h_and_current")
    run = solve_h(ctx, px32, wt.WT_F32, h_format=wt.WT_H_F16_SCALED)
    _check_scale(run)
    assert run["layout"]["h_bytes"] == run["layout"]["h_decode_offset"] + 256
    H = h_standard(run, px32)
    err_h = rel_l2(H, px32_oracle["H"])
    say(f"  H rel L2 {err_h:.3e}")
    assert err_h <= TOL
    car = rounded_carriers(px32["carriers"], wt.WT_F32)
    i_gpu = current(ctx, run, car)
    i_ref = oracle.induced_current(px32_oracle["H"], px32["cell"], car)
    err_i = rel_l2(i_gpu, i_ref)
    say(f"  i rel L2 {err_i:.3e}")
    assert err_i <= TOL


def test_16x16x128_f16_ragged(ctx):
    cfg = workloads.small_pixel(k=43, n_xy=16, n_z=128, n_freq=6, n_time=37, n_pairs=30, n_colloc=12)
    say("test_16x16x128_f16_ragged")
    ref = oracle.weighting_field(cfg["cell"], cfg["columns"], cfg["spectrum"])
    run = solve_h(ctx, cfg, wt.WT_F32, h_format=wt.WT_H_F16_SCALED)
    _check_scale(run)
    err_h = rel_l2(h_standard(run, cfg), ref["H"])
    say(f"  H rel L2 {err_h:.3e}")
    assert err_h <= TOL
    car = rounded_carriers(cfg["carriers"], wt.WT_F32)
    err_i = rel_l2(current(ctx, run, car), oracle.induced_current(ref["H"], cfg["cell"], car))
    say(f"  i rel L2 {err_i:.3e}")
    assert err_i <= TOL


def test_8x8x512_f16_ragged(ctx):
    cfg = workloads.small_pixel(k=46, n_xy=8, n_z=512, n_freq=5, n_time=21, n_pairs=20, n_colloc=8)
    say("test_8x8x512_f16_ragged")
    ref = oracle.weighting_field(cfg["cell"], cfg["columns"], cfg["spectrum"])
    run = solve_h(ctx, cfg, wt.WT_F32, h_format=wt.WT_H_F16_SCALED)
    assert run["layout"]["h_time_block"] == 8
    _check_scale(run)
    err_h = rel_l2(h_standard(run, cfg), ref["H"])
    say(f"  H rel L2 {err_h:.3e}")
    assert err_h <= TOL
    car = rounded_carriers(cfg["carriers"], wt.WT_F32)
    err_i = rel_l2(current(ctx, run, car), oracle.induced_current(ref["H"], cfg["cell"], car))
    say(f"  i rel L2 {err_i:.3e}")
    assert err_i <= TOL


def test_128x128x256_f16_sampled_columns_and_current_vs_plain(ctx):
    cfg = workloads.mip_pixel_128x128x256()
    say("test_128x128x256_f16_sampled_columns_and_current_vs_plain")
    cols = [(0, 0), (64, 64), (77, 64), (10, 100)]
    run = solve_h(ctx, cfg, wt.WT_F32, h_format=wt.WT_H_F16_SCALED)
    _check_scale(run)
    ref = oracle.weighting_field(cfg["cell"], cfg["columns"], cfg["spectrum"], route="columns", cols_ij=cols)
    err_h = rel_l2(h_columns(run, cfg, cols), ref["H_cols"])
    say(f"  H rel L2 (sampled columns) {err_h:.3e}")
    assert err_h <= TOL
    car = cfg["carriers"]
    i16 = current(ctx, run, car)
    del run
    torch.cuda.empty_cache()
    plain = solve_h(ctx, cfg, wt.WT_F32)
    i32 = current(ctx, plain, car)
    err_i = rel_l2(i16, i32)
    say(f"  i rel L2 vs the float32 path {err_i:.3e}")
    assert err_i <= TOL
