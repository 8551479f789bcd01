"""ctypes binding of libwt.so, the C ABI declared in include/wt.h.

Argument marshalling only: every step of the computation runs in the HIP
kernels behind the ABI.  Device buffers are passed as integer addresses (for
example ``tensor.data_ptr()`` of torch tensors allocated on the GPU); streams
as integer hipStream_t handles (``torch.cuda.current_stream().cuda_stream``).
Importing this module loads the library and fails loudly if it is missing.
"""
from __future__ import annotations

import ctypes
import os
import re

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libwt.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "wt.h")

c_double, c_int, c_size_t, c_void_p, c_char_p = (ctypes.c_double, ctypes.c_int, ctypes.c_size_t,
                                                   ctypes.c_void_p, ctypes.c_char_p)

WT_OK = 0
WT_E_INVALID_ARG = -1
WT_E_GEOMETRY = -2
WT_E_UNSUPPORTED_SIZE = -3
WT_E_WORKSPACE = -4
WT_E_SINGULAR = -5
WT_E_NOT_CONVERGED = -6
WT_E_HIP = -7
WT_F64 = 0
WT_F32 = 1
WT_H_PLAIN = 0
WT_H_F16_SCALED = 1


class WtError(RuntimeError):
    def __init__(self, status, where, detail=""):
        self.status = status
        msg = f"{where}: {wt_status_string(status)} ({status})"
        if detail:
            msg += f": {detail}"
        super().__init__(msg)


class wt_cell(ctypes.Structure):
    _fields_ = [("Lx", c_double), ("Ly", c_double), ("Lz", c_double),
                ("Nx", c_int), ("Ny", c_int), ("Nz", c_int),
                ("eps_r", c_double), ("sigma_bulk", c_double)]


class wt_column(ctypes.Structure):
    _fields_ = [("x", c_double), ("y", c_double), ("radius", c_double),
                ("z_contact", c_double), ("z_free", c_double),
                ("resistivity", c_double * 4), ("n_resistivity", c_int),
                ("n_colloc", c_int), ("v_applied", c_double)]


class wt_spectrum(ctypes.Structure):
    _fields_ = [("n_freq", c_int), ("df", c_double), ("n_time", c_int), ("dt", c_double)]


class wt_h_options(ctypes.Structure):
    _fields_ = [("precision", c_int), ("ir_max_iter", c_int), ("ir_tol", c_double), ("h_format", c_int),
                ("fft_schedule", c_int)]


class wt_h_report(ctypes.Structure):
    _fields_ = [("backward_error_max", c_double), ("pivot_ratio_max", c_double),
                ("ir_iters_max", c_int), ("singular_count", c_int), ("h_scale", c_double)]


class wt_h_layout(ctypes.Structure):
    _fields_ = [("workspace_bytes", c_size_t), ("h_bytes", c_size_t), ("h_time_block", c_int),
                ("n_q", c_int), ("off_A", c_size_t), ("off_qw", c_size_t), ("off_qt", c_size_t),
                ("off_qhat", c_size_t), ("off_ehat", c_size_t), ("h_format", c_int),
                ("h_decode_offset", c_size_t)]


class wt_tune_report(ctypes.Structure):
    _fields_ = [("n_candidates", c_int), ("h_time_block", c_int), ("threads", c_int),
                ("ms_chosen", c_double), ("ms_default", c_double), ("fft_n1", c_int), ("from_cache", c_int)]


class wt_carriers(ctypes.Structure):
    _fields_ = [("n_carriers", c_int), ("n_tracks", c_int), ("d_pos", c_void_p),
                ("d_charge", c_void_p), ("d_track", c_void_p)]


class wt_batch_item(ctypes.Structure):
    _fields_ = [("plan", c_void_p), ("carriers", wt_carriers), ("d_current", c_void_p)]


WT_MAX_LANES = 8
WT_STATIC_WORKSPACE_BYTES = 32 << 20


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2605_13987_amd.build`")
    # One HIP runtime per process.  The callers' device memory and streams come
    # from PyTorch, whose wheel ships its own HIP runtime; with torch loaded
    # first, libwt.so binds to that runtime.  Loaded the other way round, the
    # process would hold two runtimes and the second cannot use the device.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    sig = {
        "wt_status_string": (c_char_p, [c_int]),
        "wt_stage_name": (c_char_p, [c_int]),
        "wt_context_create": (c_int, [P(c_void_p), c_int, c_void_p]),
        "wt_context_destroy": (c_int, [c_void_p]),
        "wt_context_last_error": (c_char_p, [c_void_p]),
        "wt_context_enable_timing": (c_int, [c_void_p, c_int]),
        "wt_context_stage_times": (c_int, [c_void_p, P(c_double), c_int, P(c_int), P(c_int)]),
        "wt_h_plan_create": (c_int, [P(wt_cell), P(wt_column), c_int, P(wt_spectrum), P(wt_h_options),
                                     P(c_void_p), P(wt_h_layout)]),
        "wt_h_plan_destroy": (c_int, [c_void_p]),
        "wt_h_plan_layout": (c_int, [c_void_p, P(wt_h_layout)]),
        "wt_h_solve": (c_int, [c_void_p, c_void_p, c_void_p, c_size_t, c_void_p, c_size_t, P(wt_h_report)]),
        "wt_h_solve_static": (c_int, [c_void_p, c_void_p, c_void_p, c_size_t, P(wt_h_report)]),
        "wt_current_workspace": (c_int, [c_void_p, c_int, ctypes.c_longlong, P(c_size_t)]),
        "wt_context_set_current_form": (c_int, [c_void_p, c_int]),
        "wt_current": (c_int, [c_void_p, c_void_p, c_void_p, P(wt_carriers), c_void_p, c_size_t, c_void_p]),
        "wt_step": (c_int, [c_void_p, c_void_p, c_void_p, c_size_t, c_void_p, c_size_t, P(wt_carriers), c_void_p,
                            c_size_t, c_void_p, P(wt_h_report)]),
        "wt_electronics": (c_int, [c_void_p, c_int, c_int, c_int, c_double, c_void_p, c_void_p, c_void_p,
                                   c_double, c_double, c_void_p, c_void_p]),
        "wt_h_plan_tune": (c_int, [c_void_p, c_void_p, c_void_p, c_size_t, c_void_p, c_size_t, P(wt_tune_report)]),
        "wt_fft_schedule_count": (c_int, [c_int]),
        "wt_context_set_tune_cache": (c_int, [c_void_p, c_char_p]),
        "wt_batch_run": (c_int, [c_void_p, c_int, P(wt_batch_item), c_int, P(c_void_p), c_size_t, P(c_void_p),
                                 c_size_t, P(c_int)]),
        "wt_h_gradient_workspace": (c_int, [c_void_p, c_int, P(c_size_t)]),
        "wt_h_gradient": (c_int, [c_void_p, c_void_p, c_void_p, c_size_t, P(wt_carriers), c_void_p, c_void_p,
                                  c_size_t, c_void_p, P(wt_h_report)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


LIB = _load()


def declared_symbols():
    """Function names declared in include/wt.h."""
    with open(HEADER) as fh:
        text = fh.read()
    decl = re.findall(r"^\s*(?:const\s+)?[a-z_]+\**\s+\**(wt_[a-z0-9_]+)\s*\(", text, flags=re.M)
    return sorted(set(decl))


def wt_status_string(status: int) -> str:
    return LIB.wt_status_string(int(status)).decode()


def wt_stage_name(stage: int) -> str:
    return LIB.wt_stage_name(int(stage)).decode()


def _check(status, where, ctx=None):
    if status != WT_OK:
        detail = LIB.wt_context_last_error(ctx).decode() if status == WT_E_HIP else ""
        raise WtError(status, where, detail)


# ---------------------------------------------------------------- contexts

def wt_context_create(device: int = 0, stream: int = 0):
    ctx = c_void_p()
    _check(LIB.wt_context_create(ctypes.byref(ctx), int(device), c_void_p(stream or None)), "wt_context_create")
    return ctx


def wt_context_destroy(ctx):
    _check(LIB.wt_context_destroy(ctx), "wt_context_destroy")


def wt_context_enable_timing(ctx, enable: bool = True):
    _check(LIB.wt_context_enable_timing(ctx, int(bool(enable))), "wt_context_enable_timing", ctx)


def wt_context_stage_times(ctx):
    """[(stage name, milliseconds)] of the last call (synchronises)."""
    ms = (c_double * 8)()
    ids = (c_int * 8)()
    n = c_int()
    _check(LIB.wt_context_stage_times(ctx, ms, 8, ids, ctypes.byref(n)), "wt_context_stage_times", ctx)
    return [(wt_stage_name(ids[i]), ms[i]) for i in range(n.value)]


# ---------------------------------------------------------------- plans

def make_cell(cell: dict) -> wt_cell:
    L, N = cell["L"], cell["N"]
    return wt_cell(L[0], L[1], L[2], N[0], N[1], N[2], cell["eps_r"], cell.get("sigma_bulk", 0.0))


def make_columns(columns):
    arr = (wt_column * len(columns))()
    for i, c in enumerate(columns):
        rho = list(c["resistivity"])
        arr[i].x, arr[i].y, arr[i].radius = c["x"], c["y"], c["radius"]
        arr[i].z_contact, arr[i].z_free = c["z_contact"], c["z_free"]
        for k in range(4):
            arr[i].resistivity[k] = rho[k] if k < len(rho) else 0.0
        arr[i].n_resistivity = len(rho)
        arr[i].n_colloc = c["n_colloc"]
        arr[i].v_applied = c["v_applied"]
    return arr


def layout_dict(layout: wt_h_layout) -> dict:
    return {name: getattr(layout, name) for name, _ in wt_h_layout._fields_}


def wt_h_plan_create(cell: dict, columns, spectrum: dict, precision: int = WT_F32,
                     ir_max_iter: int = 2, ir_tol: float = 1e-12, h_format: int = WT_H_PLAIN,
                     fft_schedule: int = 0):
    """Returns (plan handle, layout dict)."""
    plan = c_void_p()
    lay = wt_h_layout()
    sp = wt_spectrum(spectrum["n_freq"], spectrum["df"], spectrum["n_time"], spectrum["dt"])
    opt = wt_h_options(int(precision), int(ir_max_iter), float(ir_tol), int(h_format), int(fft_schedule))
    cols = make_columns(columns)
    _check(LIB.wt_h_plan_create(ctypes.byref(make_cell(cell)), cols, len(columns), ctypes.byref(sp),
                                ctypes.byref(opt), ctypes.byref(plan), ctypes.byref(lay)), "wt_h_plan_create")
    return plan, layout_dict(lay)


def wt_h_plan_create_status(cell: dict, columns, spectrum: dict, precision: int = WT_F32,
                            ir_max_iter: int = 2, ir_tol: float = 1e-12, h_format: int = WT_H_PLAIN,
                            fft_schedule: int = 0) -> int:
    """Status code of plan creation (the plan, if any, is destroyed)."""
    plan = c_void_p()
    lay = wt_h_layout()
    sp = wt_spectrum(spectrum["n_freq"], spectrum["df"], spectrum["n_time"], spectrum["dt"])
    opt = wt_h_options(int(precision), int(ir_max_iter), float(ir_tol), int(h_format), int(fft_schedule))
    cols = make_columns(columns)
    st = LIB.wt_h_plan_create(ctypes.byref(make_cell(cell)), cols, len(columns), ctypes.byref(sp),
                              ctypes.byref(opt), ctypes.byref(plan), ctypes.byref(lay))
    if st == WT_OK:
        LIB.wt_h_plan_destroy(plan)
    return st


def wt_h_plan_destroy(plan):
    _check(LIB.wt_h_plan_destroy(plan), "wt_h_plan_destroy")


def wt_h_plan_layout(plan) -> dict:
    lay = wt_h_layout()
    _check(LIB.wt_h_plan_layout(plan, ctypes.byref(lay)), "wt_h_plan_layout")
    return layout_dict(lay)


def wt_h_plan_tune(ctx, plan, d_workspace: int, workspace_bytes: int, d_h: int, h_bytes: int) -> dict:
    """Autotune the plan's synthesis launch (synchronises; the layout may change)."""
    rep = wt_tune_report()
    _check(LIB.wt_h_plan_tune(ctx, plan, c_void_p(d_workspace), int(workspace_bytes), c_void_p(d_h), int(h_bytes),
                              ctypes.byref(rep)), "wt_h_plan_tune", ctx)
    return {name: getattr(rep, name) for name, _ in wt_tune_report._fields_}


# ---------------------------------------------------------------- solve / current

def wt_h_solve(ctx, plan, d_workspace: int, workspace_bytes: int, d_h: int, h_bytes: int,
               report: bool = False, raise_on_error: bool = True):
    """Enqueue the H solve.  With report=True, synchronises and returns
    (status, report dict); otherwise returns (status, None)."""
    rep = wt_h_report() if report else None
    st = LIB.wt_h_solve(ctx, plan, c_void_p(d_workspace), int(workspace_bytes), c_void_p(d_h), int(h_bytes),
                        ctypes.byref(rep) if report else None)
    if raise_on_error and st != WT_OK:
        _check(st, "wt_h_solve", ctx)
    out = None
    if report:
        out = {name: getattr(rep, name) for name, _ in wt_h_report._fields_}
    return st, out


def wt_h_solve_static(ctx, plan, d_h: int, h_bytes: int, report: bool = False, raise_on_error: bool = True):
    """wt_h_solve with the library's static workspace (no device allocation).
    Returns (status, report dict or None) like wt_h_solve."""
    rep = wt_h_report() if report else None
    st = LIB.wt_h_solve_static(ctx, plan, c_void_p(d_h), int(h_bytes), ctypes.byref(rep) if report else None)
    if raise_on_error and st != WT_OK:
        _check(st, "wt_h_solve_static", ctx)
    out = None
    if report:
        out = {name: getattr(rep, name) for name, _ in wt_h_report._fields_}
    return st, out


WT_CURRENT_AUTO, WT_CURRENT_BINNED, WT_CURRENT_UNBINNED = 0, 1, 2


def wt_context_set_current_form(ctx, form: int):
    """0: bin from 2^24 polyline steps on; 1: bin whenever given a workspace; 2: never bin."""
    _check(LIB.wt_context_set_current_form(ctx, int(form)), "wt_context_set_current_form", ctx)


def wt_current_workspace(plan, n_carriers: int, max_events: int = 0) -> int:
    """Bytes of wt_current's workspace (max_events <= 0: room for every step)."""
    n = c_size_t()
    _check(LIB.wt_current_workspace(plan, int(n_carriers), int(max_events), ctypes.byref(n)), "wt_current_workspace")
    return n.value


def wt_current(ctx, plan, d_h: int, n_carriers: int, n_tracks: int, d_pos: int, d_charge: int,
               d_track: int, d_i_out: int, d_workspace: int = 0, workspace_bytes: int = 0):
    car = wt_carriers(int(n_carriers), int(n_tracks), c_void_p(d_pos), c_void_p(d_charge), c_void_p(d_track))
    _check(LIB.wt_current(ctx, plan, c_void_p(d_h), ctypes.byref(car), c_void_p(d_workspace or None),
                          int(workspace_bytes), c_void_p(d_i_out)), "wt_current", ctx)


def wt_step(ctx, plan, d_workspace: int, workspace_bytes: int, d_h: int, h_bytes: int, n_carriers: int,
            n_tracks: int, d_pos: int, d_charge: int, d_track: int, d_i_out: int, d_cur_workspace: int = 0,
            cur_workspace_bytes: int = 0, report: bool = False, raise_on_error: bool = True):
    """wt_h_solve then wt_current in one call (the binning beside the
    synthesis).  Returns (status, report dict or None) like wt_h_solve."""
    car = wt_carriers(int(n_carriers), int(n_tracks), c_void_p(d_pos), c_void_p(d_charge), c_void_p(d_track))
    rep = wt_h_report() if report else None
    st = LIB.wt_step(ctx, plan, c_void_p(d_workspace), int(workspace_bytes), c_void_p(d_h), int(h_bytes),
                     ctypes.byref(car), c_void_p(d_cur_workspace or None), int(cur_workspace_bytes),
                     c_void_p(d_i_out), ctypes.byref(rep) if report else None)
    if raise_on_error and st != WT_OK:
        _check(st, "wt_step", ctx)
    out = None
    if report:
        out = {name: getattr(rep, name) for name, _ in wt_h_report._fields_}
    return st, out


def wt_context_set_tune_cache(ctx, path, raise_on_error: bool = True) -> int:
    """Use (path) or stop using (None) a tuning cache file for wt_h_plan_tune."""
    st = LIB.wt_context_set_tune_cache(ctx, None if path is None else os.fsencode(path))
    if raise_on_error:
        _check(st, "wt_context_set_tune_cache", ctx)
    return st


def wt_fft_schedule_count(n_z: int) -> int:
    """Register-FFT synthesis schedules compiled for N_z (float, two columns)."""
    return int(LIB.wt_fft_schedule_count(int(n_z)))


def wt_batch_run(ctx, items, d_workspaces, workspace_bytes: int, d_hs, h_bytes: int, raise_on_error: bool = True):
    """Batched wt_h_solve + wt_current over lanes of streams.

    items: list of dicts with plan, n_carriers, n_tracks, d_pos, d_charge,
    d_track, d_current (device pointers as ints); d_workspaces / d_hs: one
    device pointer per lane.  Returns (status, [status per item])."""
    n, lanes = len(items), len(d_workspaces)
    arr = (wt_batch_item * max(n, 1))()
    for i, it in enumerate(items):
        arr[i].plan = it["plan"]
        arr[i].carriers = wt_carriers(int(it["n_carriers"]), int(it["n_tracks"]), c_void_p(it["d_pos"] or None),
                                      c_void_p(it["d_charge"] or None), c_void_p(it["d_track"] or None))
        arr[i].d_current = c_void_p(it["d_current"] or None)
    ws = (c_void_p * max(lanes, 1))(*[c_void_p(x) for x in d_workspaces])
    hs = (c_void_p * max(len(d_hs), 1))(*[c_void_p(x) for x in d_hs])
    status = (c_int * max(n, 1))()
    st = LIB.wt_batch_run(ctx, n, arr, lanes, ws, int(workspace_bytes), hs, int(h_bytes), status)
    per_item = [int(status[i]) for i in range(n)]
    if raise_on_error and st != WT_OK:
        _check(st, "wt_batch_run", ctx)
    return st, per_item


def wt_electronics(ctx, precision: int, n_tracks: int, n_time: int, dt: float, d_current: int, d_response: int,
                   d_noise: int, noise_sigma: float, cfd_fraction: float, d_signal: int, d_features: int,
                   raise_on_error: bool = True) -> int:
    """Front-end response, noise and timing features of the currents (device arrays)."""
    st = LIB.wt_electronics(ctx, int(precision), int(n_tracks), int(n_time), float(dt), c_void_p(d_current),
                            c_void_p(d_response), c_void_p(d_noise or None), float(noise_sigma),
                            float(cfd_fraction), c_void_p(d_signal), c_void_p(d_features))
    if raise_on_error:
        _check(st, "wt_electronics", ctx)
    return st


# ---------------------------------------------------------------- gradient

def wt_h_gradient_workspace(plan, n_tracks: int) -> int:
    """Bytes of the gradient workspace for n_tracks tracks."""
    n = c_size_t()
    _check(LIB.wt_h_gradient_workspace(plan, int(n_tracks), ctypes.byref(n)), "wt_h_gradient_workspace")
    return n.value


def wt_h_gradient(ctx, plan, d_workspace: int, workspace_bytes: int, n_carriers: int, n_tracks: int, d_pos: int,
                  d_charge: int, d_track: int, d_grad_current: int, d_grad_workspace: int,
                  grad_workspace_bytes: int, d_grad_params: int, report: bool = False,
                  raise_on_error: bool = True):
    """Enqueue the adjoint: dL/d(resistivities, radius) per column into
    d_grad_params ([n_cols][5] double).  Returns (status, report dict or None)."""
    car = wt_carriers(int(n_carriers), int(n_tracks), c_void_p(d_pos), c_void_p(d_charge), c_void_p(d_track))
    rep = wt_h_report() if report else None
    st = LIB.wt_h_gradient(ctx, plan, c_void_p(d_workspace), int(workspace_bytes), ctypes.byref(car),
                           c_void_p(d_grad_current), c_void_p(d_grad_workspace), int(grad_workspace_bytes),
                           c_void_p(d_grad_params), ctypes.byref(rep) if report else None)
    if raise_on_error and st != WT_OK:
        _check(st, "wt_h_gradient", ctx)
    out = None
    if report:
        out = {name: getattr(rep, name) for name, _ in wt_h_report._fields_}
    return st, out

