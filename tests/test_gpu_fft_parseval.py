"""The GPU's FFTs in isolation: Parseval and agreement with numpy.fft.

* the in-plane field table (two passes of the library's 2D inverse FFTs over
  the k-space multiplier): for every k_z and component,
  sum_{X,Y} |Ehat|^2 = N_x N_y sum_{k_x,k_y} |M|^2, and Ehat equals
  numpy.fft.ifft2 of the multiplier (computed on the host, in float64, from
  the oracle's multiplier) times N_x N_y;
* the per-column z-synthesis (the register FFTs of the synthesis kernel):
  with the spectrum F(k_z, t) = sum_w Ehat(X - X_w, Y - Y_w, k_z) Qhat_w(k_z, t)
  formed on the host from the GPU's own table and column spectra,
  sum_z H^2 = N_z sum_{all k_z} |F|^2 (Hermitian extension), summed over the
  samples of each sampled column and component, and H equals
  numpy.fft.irfft of F times N_z.
float32 path: 1e-6 relative for Parseval, 1e-5 for the transforms.
"""
import numpy as np
import pytest
import torch

from gpu_common import context, h_columns, rel_l2, say, solve_h, ws_array
from oracle import field as ofield, green
from paper_2605_13987_amd import workloads, wt

pytestmark = pytest.mark.gpu


def _check(cfg, cols_ij):
    cell, cols, spec = cfg["cell"], cfg["columns"], cfg["spectrum"]
    N, nt = cell["N"], spec["n_time"]
    nzh = N[2] // 2
    ctx = context()
    try:
        run = solve_h(ctx, cfg, wt.WT_F32)
        assert run["status"] == wt.WT_OK
        lay = run["layout"]
        E = ws_array(run["ws"], lay["off_ehat"], N[0] * N[1] * nzh * 3, np.complex64)
        E = E.reshape(N[0], N[1], nzh, 3).astype(np.complex128)
        W = len(cols)
        Q = ws_array(run["ws"], lay["off_qhat"], nt * W * nzh, np.complex64).reshape(nt, W, nzh)
        Q = Q.astype(np.complex128)
        # the multiplier on the host (numpy order), k_z >= 0 half
        Mk, _ = ofield._multiplier(cell, green.smoothing_widths(cell, cols))
        worst_p, worst_t = 0.0, 0.0
        for a in range(3):
            M = Mk[a][:, :, :nzh]
            lhs = np.sum(np.abs(E[..., a]) ** 2, axis=(0, 1))
            rhs = N[0] * N[1] * np.sum(np.abs(M) ** 2, axis=(0, 1))
            live = rhs > 1e-12 * rhs.max()
            worst_p = max(worst_p, float(np.max(np.abs(lhs[live] - rhs[live]) / rhs[live])))
            ref = np.fft.ifft2(M, axes=(0, 1)) * (N[0] * N[1])
            worst_t = max(worst_t, rel_l2(E[..., a], ref))
        say(f"  field table: Parseval max rel {worst_p:.2e}, vs numpy ifft2 rel L2 {worst_t:.2e}")
        assert worst_p <= 1e-6 and worst_t <= 1e-5
        # z-synthesis on sampled columns
        h = np.array([cell["L"][a] / N[a] for a in range(2)])
        axes = [(int(round(c["x"] / h[0])) % N[0], int(round(c["y"] / h[1])) % N[1]) for c in cols]
        H = h_columns(run, cfg, cols_ij)                      # (n_cols, Nz, nt, 3)
        energy = np.zeros((len(cols_ij), nt, 3))
        e_z = np.zeros((len(cols_ij), nt, 3))
        ref = np.zeros_like(H)
        for ci, (X, Y) in enumerate(cols_ij):
            for a in range(3):
                F = np.zeros((nzh, nt), dtype=np.complex128)
                for w, (xw, yw) in enumerate(axes):
                    F += E[(X - xw) % N[0], (Y - yw) % N[1], :, a][:, None] * Q[:, w, :].T
                energy[ci, :, a] = N[2] * (np.abs(F[0]) ** 2 + 2 * np.sum(np.abs(F[1:]) ** 2, axis=0))
                e_z[ci, :, a] = np.sum(H[ci, :, :, a] ** 2, axis=0)
                full = np.zeros((N[2] // 2 + 1, nt), dtype=np.complex128)
                full[:nzh] = F
                ref[ci, :, :, a] = np.fft.irfft(full, n=N[2], axis=0) * N[2]
        # energy of every sampled column and component over all samples
        # (components that vanish by symmetry on an axis: relative to the
        # largest); single samples are printed for information, their
        # relative error grows as their energy falls below the column's
        tot_z, tot_f = e_z.sum(axis=1), energy.sum(axis=1)    # (n_cols, 3)
        big = tot_f.max()
        assert big > 0
        live = tot_f > 1e-6 * big
        worst_p = float(np.max(np.abs(tot_z[live] - tot_f[live]) / tot_f[live]))
        worst_dead = float(np.max(np.abs(tot_z[~live] - tot_f[~live]), initial=0.0) / big)
        one = energy > 1e-2 * energy.max()
        worst_one = float(np.max(np.abs(e_z[one] - energy[one]) / energy[one]))
        worst_t = rel_l2(H, ref)
        say(f"  z-synthesis: Parseval max rel {worst_p:.2e} over {int(live.sum())} column components (others "
            f"{worst_dead:.1e} of the largest; single samples above 1% of the largest energy: {worst_one:.1e}), "
            f"vs numpy irfft rel L2 {worst_t:.2e}")
        assert worst_p <= 1e-6 and worst_dead <= 1e-6 and worst_t <= 1e-5
        wt.wt_h_plan_destroy(run["plan"])
    finally:
        wt.wt_context_destroy(ctx)


def test_parseval_32x32x64(px32):
    _check(px32, [(0, 0), (16, 16), (3, 29), (20, 7)])


def test_parseval_128x128x256():
    cfg = workloads.mip_pixel_128x128x256()
    _check(cfg, [(0, 0), (64, 64), (100, 17), (5, 90)])
