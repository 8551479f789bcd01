"""H(x, t) on the grid from the time-domain source charges (FP64).

By linearity the field is the superposition of translated, rescaled copies of
the fundamental solution (Section 3, the V_ext step):

    H(x, t_n) = sum_i q_i(t_n) E_G(x - y_i)               [V m^-1 s^-1 per volt]

and it equals the frequency-to-time quadrature of the per-frequency fields,
because the quadrature and the superposition are both linear.  Three routes
evaluate the same discrete quantity:

* ``field_superposition``: the sum above with the direct E_G (tiny grids);
* ``field_fft``: H = sum_k M(k) rho(k, t) exp(i k.x), M(k) = -i k S(k) /
  (eps |k|^2 V), rho(k, t) = sum_i q_i(t) exp(-i k.y_i), as one full 3D inverse
  FFT per time sample and component;
* ``field_columns``: the same mode sum evaluated directly (no FFT) on selected
  (x, y) grid columns, for every z node; used on grids too large for the FFT
  route in memory.
* ``field_columns_planar_fft``: the same sum on selected columns, with the
  in-plane (k_x, k_y) part of every column at once from 2D inverse FFTs and
  the k_z part by 1D inverse FFTs along z; used where many columns of a large
  grid are needed.
* ``field_nodes_planar_fft``: the same sum at selected grid nodes only, with
  the in-plane part from the same 2D inverse FFTs and the k_z sum taken
  directly at each node; used for the nodes that carrier paths touch on
  large grids.
"""
from __future__ import annotations

import numpy as np

from . import green


def grid_points(cell) -> np.ndarray:
    h = green.spacing(cell)
    N = cell["N"]
    ix, iy, iz = np.meshgrid(*(np.arange(N[a]) * h[a] for a in range(3)), indexing="ij")
    return np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1)


def field_superposition(points, cell, s, src, q_t) -> np.ndarray:
    """H at points (n_p, 3) for source charges q_t (n_time, n_src) -> (n_p, n_time, 3)."""
    n_p = points.shape[0]
    d = (points[:, None, :] - src[None, :, :]).reshape(-1, 3)
    E = green.field(d, cell, s).reshape(n_p, src.shape[0], 3)
    return np.einsum("psa,ts->pta", E, q_t)


def _multiplier(cell, s):
    """M_a(k) on the full FFT grid (numpy ordering), zero at k=0 and Nyquist."""
    L, N = cell["L"], cell["N"]
    m = [np.fft.fftfreq(N[a]) * N[a] for a in range(3)]
    keep = [np.abs(m[a]) < N[a] / 2 for a in range(3)]
    k = [2 * np.pi * m[a] / L[a] for a in range(3)]
    KX, KY, KZ = np.meshgrid(*k, indexing="ij")
    K2 = KX ** 2 + KY ** 2 + KZ ** 2
    mask = keep[0][:, None, None] & keep[1][None, :, None] & keep[2][None, None, :] & (K2 > 0)
    with np.errstate(divide="ignore", invalid="ignore"):
        w = np.where(mask, np.exp(-0.5 * ((KX * s[0]) ** 2 + (KY * s[1]) ** 2 + (KZ * s[2]) ** 2)) / K2, 0.0)
    w = w / (green.permittivity(cell) * float(np.prod(L)))
    return [-1j * Ka * w for Ka in (KX, KY, KZ)], (KX, KY, KZ)


def field_fft(cell, s, src, q_t) -> np.ndarray:
    """H on every grid node by 3D inverse FFTs -> float64 [nx][ny][nz][n_time][3]."""
    N = cell["N"]
    Mk, (KX, KY, KZ) = _multiplier(cell, s)
    n_tot = N[0] * N[1] * N[2]
    kflat = np.stack([KX.ravel(), KY.ravel(), KZ.ravel()], axis=1)
    nt = q_t.shape[0]
    rho = np.empty((n_tot, nt), dtype=np.complex128)
    step = max(1, (1 << 24) // max(1, src.shape[0]))
    for i in range(0, n_tot, step):                   # rho(k,t) = sum_i q_i(t) e^{-ik.y_i}
        rho[i:i + step] = np.exp(-1j * (kflat[i:i + step] @ src.T)) @ q_t.T
    rho = rho.reshape(N[0], N[1], N[2], nt)
    H = np.empty((N[0], N[1], N[2], nt, 3))
    for a in range(3):
        spec = Mk[a][..., None] * rho
        H[..., a] = (np.fft.ifftn(spec, axes=(0, 1, 2)) * n_tot).real
    return H


def field_columns(cell, s, src, q_t, cols_ij) -> np.ndarray:
    """H on grid columns (ix, iy) for all z nodes -> (n_cols, nz, n_time, 3).

    Direct mode sums: the (k_x, k_y) part is summed per source axis position,
    the k_z part per node; no FFT is used.
    """
    L, N = cell["L"], cell["N"]
    h = green.spacing(cell)
    mx, my, mz = (green.axis_modes(N[a]) for a in range(3))
    kx, ky, kz = (2 * np.pi * m / L[a] for a, m in enumerate((mx, my, mz)))
    KX, KY, KZ = np.meshgrid(kx, ky, kz, indexing="ij")
    K2 = KX ** 2 + KY ** 2 + KZ ** 2
    with np.errstate(divide="ignore", invalid="ignore"):
        w = np.where(K2 > 0, np.exp(-0.5 * ((KX * s[0]) ** 2 + (KY * s[1]) ** 2 + (KZ * s[2]) ** 2)) / K2, 0.0)
    w = w / (green.permittivity(cell) * float(np.prod(L)))
    Ma = [(-1j * Ka * w).reshape(kx.size * ky.size, kz.size) for Ka in (KX, KY, KZ)]
    axes = np.unique(src[:, :2], axis=0)
    zk = np.arange(N[2]) * h[2]
    ez = np.exp(1j * np.outer(zk, kz))                                  # (nz, n_kz)
    nt = q_t.shape[0]
    out = np.empty((len(cols_ij), N[2], nt, 3))
    # per axis position: D(kz, t) = sum over its sources of q(t) e^{-i kz z}
    D = []
    for ax in axes:
        sel = np.all(src[:, :2] == ax, axis=1)
        D.append(np.exp(-1j * np.outer(kz, src[sel, 2])) @ q_t[:, sel].T)     # (n_kz, nt)
    for c, (ix, iy) in enumerate(cols_ij):
        X, Y = ix * h[0], iy * h[1]
        acc = [np.zeros((kz.size, nt), dtype=np.complex128) for _ in range(3)]
        for ax, Dw in zip(axes, D):
            ph = np.exp(1j * (np.add.outer(kx * (X - ax[0]), ky * (Y - ax[1])))).ravel()
            for a in range(3):
                B = ph @ Ma[a]                                            # (n_kz,)
                acc[a] += B[:, None] * Dw
        for a in range(3):
            out[c, :, :, a] = (ez @ acc[a]).real
    return out


def field_columns_planar_fft(cell, s, src, q_t, cols_ij, chunk=16) -> np.ndarray:
    """H on grid columns (ix, iy) for all z nodes -> (n_cols, nz, n_time, 3).

    The discrete sum of ``field_columns``, regrouped by source axis w:

        H_a(X, Y, z, t) = Re sum_{k_z} e^{i k_z z} sum_w B_a(X - X_w, Y - Y_w, k_z) D_w(k_z, t),
        B_a(X, Y, k_z)  = sum_{k_x, k_y} M_a(k) e^{i (k_x X + k_y Y)},
        D_w(k_z, t)     = sum_{sources i on axis w} q_i(t) e^{-i k_z z_i}.

    On the grid, B_a is the 2D inverse DFT of M_a over (k_x, k_y), taken for
    every k_z at once (numpy.fft.ifft2 scaled by N_x N_y); the axes lie on grid
    nodes, so the shift by (X_w, Y_w) is an index shift; the k_z sum is a 1D
    inverse DFT along z (numpy.fft.ifft scaled by N_z).  M_a is the multiplier
    of ``field_fft`` (zero at k = 0 and on the Nyquist planes).
    """
    L, N = cell["L"], cell["N"]
    h = np.asarray(green.spacing(cell), dtype=np.float64)
    Mk, (_, _, KZ) = _multiplier(cell, s)
    kz = KZ[0, 0, :]                                                     # numpy order, Nyquist included
    B = [np.fft.ifft2(Mk[a], axes=(0, 1)) * (N[0] * N[1]) for a in range(3)]
    del Mk
    axes = np.unique(src[:, :2], axis=0)
    shift = np.rint(axes / h[None, :2]).astype(np.int64)
    if np.max(np.abs(axes / h[None, :2] - shift)) > 1e-6:
        raise ValueError("source axes must lie on grid nodes")
    D = []
    for ax in axes:
        sel = np.all(src[:, :2] == ax, axis=1)
        D.append(np.exp(-1j * np.outer(kz, src[sel, 2])) @ q_t[:, sel].T)   # (nz, nt)
    nt = q_t.shape[0]
    out = np.empty((len(cols_ij), N[2], nt, 3))
    for c0 in range(0, len(cols_ij), chunk):
        part = cols_ij[c0:c0 + chunk]
        for a in range(3):
            A = np.zeros((len(part), N[2], nt), dtype=np.complex128)
            for (sx, sy), Dw in zip(shift, D):
                bx = np.array([(ix - sx) % N[0] for ix, _ in part])
                by = np.array([(iy - sy) % N[1] for _, iy in part])
                A += B[a][bx, by, :][:, :, None] * Dw[None, :, :]
            out[c0:c0 + len(part), :, :, a] = (np.fft.ifft(A, axis=1) * N[2]).real
    return out


def planar_table(cell, s):
    """B_a(X, Y, k_z) = sum_{k_x, k_y} M_a(k) e^{i (k_x X + k_y Y)} on the grid,
    for every k_z in numpy order: [3] arrays (N_x, N_y, N_z) complex, and k_z."""
    N = cell["N"]
    Mk, (_, _, KZ) = _multiplier(cell, s)
    B = [np.fft.ifft2(Mk[a], axes=(0, 1)) * (N[0] * N[1]) for a in range(3)]
    return B, KZ[0, 0, :].copy()


def field_nodes_planar_fft(cell, s, src, q_t, ix, iy, iz, table=None, chunk=4096) -> np.ndarray:
    """H at grid nodes (ix[i], iy[i], iz[i]) -> (n, n_time, 3).

    The discrete sum of ``field_columns_planar_fft`` taken node by node:

        H_a(X, Y, z, t) = Re sum_{k_z} e^{i k_z z} sum_w B_a(X - X_w, Y - Y_w, k_z) D_w(k_z, t)

    with B_a from ``planar_table`` (2D inverse DFTs of the multiplier) and D_w
    the z-transform of the charges on axis w; the k_z sum is a direct sum at
    each requested node (a product of the per-node row e^{i k_z z} B_a(., k_z)
    with D_w).  ``table`` may hold a precomputed ``planar_table``.
    """
    L, N = cell["L"], cell["N"]
    h = np.asarray(green.spacing(cell), dtype=np.float64)
    B, kz = planar_table(cell, s) if table is None else table
    axes = np.unique(src[:, :2], axis=0)
    shift = np.rint(axes / h[None, :2]).astype(np.int64)
    if np.max(np.abs(axes / h[None, :2] - shift)) > 1e-6:
        raise ValueError("source axes must lie on grid nodes")
    D = []
    for ax in axes:
        sel = np.all(src[:, :2] == ax, axis=1)
        D.append(np.exp(-1j * np.outer(kz, src[sel, 2])) @ q_t[:, sel].T)   # (nz, nt)
    ix, iy, iz = (np.asarray(v, dtype=np.int64) for v in (ix, iy, iz))
    nt = q_t.shape[0]
    out = np.empty((ix.size, nt, 3))
    for i0 in range(0, ix.size, chunk):
        sl = slice(i0, i0 + chunk)
        ez = np.exp(1j * np.outer(iz[sl] * h[2], kz))                        # (n, nz)
        for a in range(3):
            acc = np.zeros((ez.shape[0], nt), dtype=np.complex128)
            for (sx, sy), Dw in zip(shift, D):
                acc += (ez * B[a][(ix[sl] - sx) % N[0], (iy[sl] - sy) % N[1], :]) @ Dw
            out[sl, :, a] = acc.real
    return out
