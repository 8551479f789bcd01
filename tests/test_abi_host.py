"""Host-side checks of the C ABI (no GPU work): exported symbols, plan sizes,
argument validation and status codes."""
import copy
import os
import shutil
import subprocess
import sys

import pytest

from paper_2605_13987_amd import workloads, wt

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    declared = wt.declared_symbols()
    assert {"wt_h_plan_create", "wt_h_solve", "wt_current", "wt_context_create"} <= set(declared)
    for name in declared:
        assert hasattr(wt.LIB, name), name
    if shutil.which("nm"):
        out = subprocess.run(["nm", "-D", "--defined-only", wt.LIB_PATH], capture_output=True, text=True).stdout
        exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
        assert set(declared) <= exported


def test_status_strings():
    for code in range(-7, 1):
        assert wt.wt_status_string(code)
    assert wt.wt_status_string(-99) == "unknown status"
    assert wt.wt_stage_name(4) == "synthesis" and wt.wt_stage_name(99) == ""


def _px32():
    c = workloads.uniform_pixel_32x32x64()
    return c["cell"], c["columns"], c["spectrum"]


def test_plan_layout_32_and_128_grids():
    cell, cols, spec = _px32()
    plan, lay = wt.wt_h_plan_create(cell, cols, spec, precision=wt.WT_F64)
    assert lay["n_q"] == 128
    assert lay["h_bytes"] == 32 * 32 * 64 * 64 * 3 * 8
    assert lay["h_time_block"] == 8
    assert lay["workspace_bytes"] > lay["off_ehat"] + 32 * 32 * 32 * 3 * 16 - 1
    assert wt.wt_h_plan_layout(plan) == lay
    wt.wt_h_plan_destroy(plan)
    px128 = workloads.make_cell(50e-6, 300e-6, 128, 256)
    spec2 = dict(n_freq=256, df=workloads.frequency_grid_to_nyquist(256, 10e-12), n_time=200, dt=10e-12)
    plan, lay = wt.wt_h_plan_create(px128, cols, spec2, precision=wt.WT_F32)
    assert lay["h_bytes"] == 128 * 128 * 256 * 200 * 3 * 4
    assert lay["h_time_block"] == 8                   # the default schedule of 256: blocks of 8
    wt.wt_h_plan_destroy(plan)
    plan, lay = wt.wt_h_plan_create(px128, cols, spec2, precision=wt.WT_F32, fft_schedule=1)
    assert lay["h_time_block"] == 16
    wt.wt_h_plan_destroy(plan)
    # in double the register-FFT synthesis stages blocks of 8 samples at N_z = 256
    plan, lay = wt.wt_h_plan_create(px128, cols, spec2, precision=wt.WT_F64)
    assert lay["h_bytes"] == 128 * 128 * 256 * 200 * 3 * 8
    assert lay["h_time_block"] == 8
    wt.wt_h_plan_destroy(plan)


def _status(mutate, precision=wt.WT_F32, **kw):
    cell, cols, spec = _px32()
    cell, cols, spec = copy.deepcopy(cell), copy.deepcopy(cols), copy.deepcopy(spec)
    mutate(cell, cols, spec)
    return wt.wt_h_plan_create_status(cell, cols, spec, precision=precision, **kw)


CASES = [
    ("ok", lambda c, k, s: None, wt.WT_OK),
    ("odd grid", lambda c, k, s: c.update(N=(33, 32, 64)), wt.WT_E_UNSUPPORTED_SIZE),
    ("prime factor 7", lambda c, k, s: c.update(N=(28, 32, 64)), wt.WT_E_UNSUPPORTED_SIZE),
    ("grid too large", lambda c, k, s: c.update(N=(2048, 32, 64)), wt.WT_E_UNSUPPORTED_SIZE),
    ("3-5 smooth sizes", lambda c, k, s: c.update(N=(30, 40, 60)), wt.WT_OK),
    ("zero length", lambda c, k, s: c.update(L=(0.0, 50e-6, 300e-6)), wt.WT_E_INVALID_ARG),
    ("nan eps", lambda c, k, s: c.update(eps_r=float("nan")), wt.WT_E_INVALID_ARG),
    ("conducting bulk", lambda c, k, s: c.update(sigma_bulk=1.0), wt.WT_E_INVALID_ARG),
    ("axis off node", lambda c, k, s: k[0].update(x=25.3e-6), wt.WT_E_GEOMETRY),
    ("axis outside", lambda c, k, s: k[0].update(x=60e-6), wt.WT_E_GEOMETRY),
    ("overlap", lambda c, k, s: k[1].update(x=25e-6 + 6.25e-6, y=25e-6), wt.WT_E_GEOMETRY),
    ("coincident", lambda c, k, s: k[1].update(x=25e-6, y=25e-6), wt.WT_E_GEOMETRY),
    ("radius too big", lambda c, k, s: [col.update(radius=30e-6) for col in k], wt.WT_E_GEOMETRY),
    ("z outside", lambda c, k, s: k[0].update(z_free=400e-6), wt.WT_E_GEOMETRY),
    ("zero span", lambda c, k, s: k[0].update(z_free=0.0), wt.WT_E_GEOMETRY),
    ("one node", lambda c, k, s: k[0].update(n_colloc=1), wt.WT_E_INVALID_ARG),
    ("too many unknowns", lambda c, k, s: [col.update(n_colloc=300) for col in k], wt.WT_E_UNSUPPORTED_SIZE),
    ("zero resistivity", lambda c, k, s: k[0].update(resistivity=[0.0]), wt.WT_E_INVALID_ARG),
    ("five quarters", lambda c, k, s: k[1].update(resistivity=[1e-3] * 5), wt.WT_E_INVALID_ARG),
    ("no frequencies", lambda c, k, s: s.update(n_freq=0), wt.WT_E_INVALID_ARG),
    ("negative dt", lambda c, k, s: s.update(dt=-1e-12), wt.WT_E_INVALID_ARG),
    ("too many samples", lambda c, k, s: s.update(n_time=513), wt.WT_E_UNSUPPORTED_SIZE),
    ("inf df", lambda c, k, s: s.update(df=float("inf")), wt.WT_E_INVALID_ARG),
]


@pytest.mark.parametrize("name,mutate,expect", CASES, ids=[c[0] for c in CASES])
def test_plan_validation(name, mutate, expect):
    assert _status(mutate) == expect


def test_options_validation():
    ok = lambda c, k, s: None
    assert _status(ok, precision=7) == wt.WT_E_INVALID_ARG
    assert _status(ok, ir_max_iter=-1) == wt.WT_E_INVALID_ARG
    assert _status(ok, ir_max_iter=17) == wt.WT_E_INVALID_ARG
    assert _status(ok, ir_tol=float("nan")) == wt.WT_E_INVALID_ARG


def test_null_arguments_are_rejected():
    import ctypes
    lay = wt.wt_h_layout()
    plan = ctypes.c_void_p()
    assert wt.LIB.wt_h_plan_create(None, None, 0, None, None, ctypes.byref(plan), ctypes.byref(lay)) \
        == wt.WT_E_INVALID_ARG
    assert wt.LIB.wt_h_solve(None, None, None, 0, None, 0, None) == wt.WT_E_INVALID_ARG
    assert wt.LIB.wt_current(None, None, None, None, None, 0, None) == wt.WT_E_INVALID_ARG
    assert wt.LIB.wt_h_plan_tune(None, None, None, 0, None, 0, None) == wt.WT_E_INVALID_ARG
    assert wt.LIB.wt_h_plan_destroy(None) == wt.WT_E_INVALID_ARG
    assert wt.LIB.wt_context_destroy(None) == wt.WT_E_INVALID_ARG


def test_context_creation_reports_missing_device():
    import ctypes
    ctx = ctypes.c_void_p()
    st = wt.LIB.wt_context_create(ctypes.byref(ctx), 0, None)
    assert st in (wt.WT_OK, wt.WT_E_HIP)          # WT_OK only where a GPU is present
    if st == wt.WT_OK:
        assert wt.LIB.wt_context_destroy(ctx) == wt.WT_OK
    assert wt.LIB.wt_context_create(ctypes.byref(ctx), 10 ** 6, None) == wt.WT_E_HIP


def test_binding_leaves_one_hip_runtime_in_the_process():
    """Importing the binding alone must not map a second HIP runtime next to
    PyTorch's (two runtimes in one process cannot share the device)."""
    code = ("from paper_2605_13987_amd import wt\n"
            "import torch\n"
            "libs = {l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}\n"
            "print(len(libs))\n")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, cwd=ROOT, timeout=300)
    assert r.returncode == 0, r.stderr
    assert r.stdout.strip().splitlines()[-1] == "1"


def test_f16_scaled_layout_and_validation():
    cfg = workloads.uniform_pixel_32x32x64()
    plan, lay = wt.wt_h_plan_create(cfg["cell"], cfg["columns"], cfg["spectrum"], precision=wt.WT_F32,
                                    h_format=wt.WT_H_F16_SCALED)
    wt.wt_h_plan_destroy(plan)
    n = 32 * 32 * 64 * 64 * 3
    assert lay["h_format"] == wt.WT_H_F16_SCALED
    assert lay["h_decode_offset"] == (n * 2 + 255) // 256 * 256
    assert lay["h_bytes"] == lay["h_decode_offset"] + 256
    plain = wt.wt_h_plan_create(cfg["cell"], cfg["columns"], cfg["spectrum"], precision=wt.WT_F32)
    wt.wt_h_plan_destroy(plain[0])
    assert plain[1]["h_decode_offset"] == 0 and plain[1]["h_bytes"] == n * 4
    # float16 H needs the float path
    assert wt.wt_h_plan_create_status(cfg["cell"], cfg["columns"], cfg["spectrum"], precision=wt.WT_F64,
                                      h_format=wt.WT_H_F16_SCALED) == wt.WT_E_INVALID_ARG
    assert wt.wt_h_plan_create_status(cfg["cell"], cfg["columns"], cfg["spectrum"], precision=wt.WT_F32,
                                      h_format=7) == wt.WT_E_INVALID_ARG
    # and the register-FFT synthesis sizes
    small = workloads.small_pixel(k=41, n_xy=24, n_z=40, n_freq=4, n_time=10, n_pairs=5, n_colloc=8)
    assert wt.wt_h_plan_create_status(small["cell"], small["columns"], small["spectrum"], precision=wt.WT_F32,
                                      h_format=wt.WT_H_F16_SCALED) == wt.WT_E_UNSUPPORTED_SIZE


def test_gradient_workspace_and_validation():
    import ctypes
    cell, cols, spec = _px32()
    plan, lay = wt.wt_h_plan_create(cell, cols, spec, precision=wt.WT_F32)
    try:
        n1 = wt.wt_h_gradient_workspace(plan, 1)
        n100 = wt.wt_h_gradient_workspace(plan, 100)
        nq, nf, nt, nzh = lay["n_q"], spec["n_freq"], spec["n_time"], cell["N"][2] // 2
        # per extra track: two [n_time][n_cols][N_z/2] complex float blocks of event projections
        per = 2 * nt * 2 * nzh * 8
        assert 99 * per <= n100 - n1 <= 99 * per + 1024
        assert n1 >= nq * nq * 8 * 3 + 2 * nf * (nq + 1) * 16
        n = ctypes.c_size_t()
        assert wt.LIB.wt_h_gradient_workspace(plan, 0, ctypes.byref(n)) == wt.WT_E_INVALID_ARG
        assert wt.LIB.wt_h_gradient_workspace(None, 1, ctypes.byref(n)) == wt.WT_E_INVALID_ARG
        car = wt.wt_carriers(1, 1, None, None, None)
        assert wt.LIB.wt_h_gradient(None, plan, None, 0, ctypes.byref(car), None, None, 0, None, None) \
            == wt.WT_E_INVALID_ARG
    finally:
        wt.wt_h_plan_destroy(plan)
    # the transposed solves use the Schur-complement form: at most 128 charges
    big = [dict(c, n_colloc=65) for c in cols]
    plan, _ = wt.wt_h_plan_create(cell, big, spec, precision=wt.WT_F32)
    try:
        n = ctypes.c_size_t()
        assert wt.LIB.wt_h_gradient_workspace(plan, 1, ctypes.byref(n)) == wt.WT_E_UNSUPPORTED_SIZE
    finally:
        wt.wt_h_plan_destroy(plan)



def test_batch_run_rejects_a_null_context():
    st, per = wt.wt_batch_run(None, [], [0], 0, [0], 0, raise_on_error=False)
    assert st == wt.WT_E_INVALID_ARG and per == []


def test_fft_schedules_of_the_smooth_sizes():
    assert [wt.wt_fft_schedule_count(n) for n in (64, 128, 256, 512)] == [2, 2, 2, 1]
    assert wt.wt_fft_schedule_count(40) == 0 and wt.wt_fft_schedule_count(330) == 0
    assert all(wt.wt_fft_schedule_count(n) == 3 for n in (72, 150, 320))
    cfg = workloads.small_pixel(k=5, n_xy=8, n_z=72, n_freq=4, n_time=19, n_pairs=2, n_colloc=8)
    cell, cols, spec = cfg["cell"], cfg["columns"], cfg["spectrum"]
    # the default schedule of 72 is 9 x 8 with blocks of 8 samples; the third, blocks of 16
    blocks = []
    for k in range(3):
        plan, lay = wt.wt_h_plan_create(cell, cols, spec, precision=wt.WT_F32, fft_schedule=k)
        blocks.append(lay["h_time_block"])
        wt.wt_h_plan_destroy(plan)
    assert blocks == [8, 16, 16]
    assert wt.wt_h_plan_create_status(cell, cols, spec, precision=wt.WT_F32, fft_schedule=3) == wt.WT_E_INVALID_ARG
    assert wt.wt_h_plan_create_status(cell, cols, spec, precision=wt.WT_F32, fft_schedule=-1) == wt.WT_E_INVALID_ARG
    # no register-FFT schedule to choose in double plans of a smooth size; powers of two have two
    assert wt.wt_h_plan_create_status(cell, cols, spec, precision=wt.WT_F64, fft_schedule=1) == wt.WT_E_INVALID_ARG
    c64 = workloads.small_pixel(k=5, n_xy=8, n_z=64, n_freq=4, n_time=19, n_pairs=2, n_colloc=8)
    assert wt.wt_h_plan_create_status(c64["cell"], c64["columns"], c64["spectrum"], precision=wt.WT_F32,
                                      fft_schedule=1) == wt.WT_OK
    assert wt.wt_h_plan_create_status(c64["cell"], c64["columns"], c64["spectrum"], precision=wt.WT_F32,
                                      fft_schedule=2) == wt.WT_E_INVALID_ARG
