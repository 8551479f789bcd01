"""GPU parity of the register-FFT synthesis for 2,3,5-smooth N_z that are not
powers of two (float path, two columns): H and the current against the FP64
oracle on small grids, float32 H at 1e-5 / 1e-4 and float16-scaled H at 1e-3
(the bars of the power-of-two sizes).

The sizes cover the shapes the kernel distinguishes: N1 > N2 (72 = 9 x 8,
108 = 12 x 9), N1 not dividing N2 (150 = 10 x 15, 180 = 10 x 18, 320 =
10 x 32), an odd N2, so that Z(N_z/2) is not in lane 0 (108, 150, 250 =
10 x 25), N1 dividing N2 (162 = 9 x 18, 200 = 10 x 20), and ragged last
blocks (21 samples: one full block of 16 and an odd tail).  The tuner's
report names the register-FFT factor N1 of the plan, which the test uses to
check that this path, not the Stockham one, ran.  Every compiled schedule of every
register-FFT size, powers of two included (blocks of 8 and 16), is checked
against the oracle through wt_h_options.fft_schedule.
"""
import pytest

import oracle
from gpu_common import context, current, h_standard, rel_l2, rounded_carriers, say, solve_h
from paper_2605_13987_amd import workloads, wt

pytestmark = pytest.mark.gpu

SIZES = [72, 108, 150, 162, 180, 200, 250, 320]


@pytest.fixture(scope="module")
def ctx():
    c = context()
    yield c
    wt.wt_context_destroy(c)


def _register_path(ctx, run):
    """True when the plan's synthesis is the register FFT (the tuner reports
    its factor N1).  Called after H has been checked: tuning rewrites H."""
    ws, hb = run["ws"], run["hbuf"]
    rep = wt.wt_h_plan_tune(ctx, run["plan"], ws.data_ptr(), ws.numel(), hb.data_ptr(), hb.numel())
    return rep["fft_n1"] > 0


@pytest.mark.parametrize("n_z", SIZES)
@pytest.mark.parametrize("h_format", [wt.WT_H_PLAIN, wt.WT_H_F16_SCALED], ids=["f32", "f16"])
def test_smooth_register_synthesis(ctx, n_z, h_format):
    cfg = workloads.small_pixel(k=90 + n_z % 17, n_xy=8, n_z=n_z, n_freq=5, n_time=21, n_pairs=10, n_colloc=8)
    say(f"test_smooth_register_synthesis n_z={n_z} h_format={h_format}")
    ref = oracle.weighting_field(cfg["cell"], cfg["columns"], cfg["spectrum"])
    run = solve_h(ctx, cfg, wt.WT_F32, h_format=h_format)
    assert run["status"] == wt.WT_OK, run["report"]
    assert run["layout"]["h_time_block"] in (8, 16)
    tol_h, tol_i = (1e-5, 1e-4) if h_format == wt.WT_H_PLAIN else (1e-3, 1e-3)
    err_h = rel_l2(h_standard(run, cfg), ref["H"])
    car = rounded_carriers(cfg["carriers"], wt.WT_F32)
    err_i = rel_l2(current(ctx, run, car), oracle.induced_current(ref["H"], cfg["cell"], car))
    say(f"  H rel L2 {err_h:.3e}, i rel L2 {err_i:.3e}")
    assert err_h <= tol_h and err_i <= tol_i
    assert _register_path(ctx, run)


ALL_SIZES = [72, 80, 90, 96, 100, 108, 120, 144, 150, 160, 162, 180, 192, 200, 216, 240, 250, 270, 288, 300, 320]


@pytest.mark.parametrize("n_z", [64, 128, 256, 512] + ALL_SIZES)
def test_every_compiled_schedule(ctx, n_z):
    """Each register-FFT schedule of each size (wt_h_options.fft_schedule),
    float32 H against the oracle; then the tuner's choice rewrites H, checked
    too."""
    cfg = workloads.small_pixel(k=60 + n_z % 23, n_xy=8, n_z=n_z, n_freq=4, n_time=19, n_pairs=4, n_colloc=8)
    ref = oracle.weighting_field(cfg["cell"], cfg["columns"], cfg["spectrum"])
    n = wt.wt_fft_schedule_count(n_z)
    assert n == {64: 2, 128: 2, 256: 2, 512: 1}.get(n_z, 3)
    for k in range(n):
        say(f"test_every_compiled_schedule n_z={n_z} schedule={k}")
        run = solve_h(ctx, cfg, wt.WT_F32, fft_schedule=k)
        assert run["status"] == wt.WT_OK, run["report"]
        err = rel_l2(h_standard(run, cfg), ref["H"])
        say(f"  H rel L2 {err:.2e} (time block {run['layout']['h_time_block']})")
        assert err <= 1e-5
    ws, hb = run["ws"], run["hbuf"]
    rep = wt.wt_h_plan_tune(ctx, run["plan"], ws.data_ptr(), ws.numel(), hb.data_ptr(), hb.numel())
    assert rep["n_candidates"] == n and rep["fft_n1"] > 0 and rep["from_cache"] == 0
    run["layout"] = wt.wt_h_plan_layout(run["plan"])
    assert run["layout"]["h_time_block"] == rep["h_time_block"]
    assert rel_l2(h_standard(run, cfg), ref["H"]) <= 1e-5


def test_smooth_size_in_double_uses_stockham(ctx):
    """The smooth register form is float with two columns only: a double plan
    of the same size keeps the LDS Stockham synthesis, at the FP64 bar."""
    cfg = workloads.small_pixel(k=97, n_xy=8, n_z=150, n_freq=5, n_time=21, n_pairs=10, n_colloc=8)
    ref = oracle.weighting_field(cfg["cell"], cfg["columns"], cfg["spectrum"])
    run = solve_h(ctx, cfg, wt.WT_F64)
    assert run["status"] == wt.WT_OK, run["report"]
    assert rel_l2(h_standard(run, cfg), ref["H"]) <= 1e-9
    assert not _register_path(ctx, run)
