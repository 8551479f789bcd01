"""Derivatives of the Eq. 1 currents with respect to the column parameters (FP64).

Forward mode, written out step by step on the oracle's own pipeline.  The
parameters are, per column, the resistivity of each of its quarter-columns and
its radius (the quantities the paper varies in its Section 5 results: the
electrode resistance R = 4 rho L / (pi d^2) through resistivity and diameter).

The carrier polylines are inputs and stay fixed: a change of radius moves the
collocation points and widens the boundary-fit sources, not the tracks.  The
bulk field's smoothing widths and source positions do not depend on these
parameters, so the whole dependence enters through the per-frequency system
S(w) [q; c] = b of the boundary fit:

* resistivity rho_{w,p}: the column conductivity is the mean of 1/rho over its
  quarter-columns, so d sigma_w / d rho_{w,p} = -1 / (n_w rho_{w,p}^2), and the
  RC-line block i w R_w(min(m, m')) with R_w(m) = m D_w / (pi r_w^2 (sigma_w +
  i w eps_c)) changes by -i w R_w / (sigma_w + i w eps_c) per unit sigma;
* radius r_w: the RC-line block scales as r_w^-2 (derivative -2 i w R_w / r_w),
  and the collocation matrix changes in the rows of column w (collocation
  points at X_w + r_w) and in the columns of column w (source width r_w / 4).

Then dq(w) = -S(w)^-1 (dS/dtheta) [q; c] at every frequency, and the rest of
the path is linear in the charges: the time quadrature, the bulk field and the
convolution map dq to dH and di exactly as they map q to H and i.

The pitch (a uniform scaling of the in-plane cell size, the column axes and
the carriers' in-plane coordinates, the grid counts held) also changes the
bulk field's mode set and the carrier displacements; its reference here is
the central difference of the whole forward pipeline (``pitch_derivative``),
not a forward-mode derivative.
"""
from __future__ import annotations

import numpy as np

from . import collocation, field, green, pipeline, timegrid


def parameter_names(columns):
    """(column, kind, index) of every parameter: ("rho", p) for p < n_res, ("radius", 0)."""
    out = []
    for w, c in enumerate(columns):
        for p in range(len(c["resistivity"])):
            out.append((w, "rho", p))
        out.append((w, "radius", 0))
    return out


def collocation_matrix_radius_derivative(cell, columns, w_d):
    """dA/dr for the radius of column w_d, as plain mode sums.

    A_ij = G_c(x_i - y_j) with x_i = (X_w + r_w, Y_w, z_i) and G_c the converged
    periodic potential of a Gaussian source of width s_v = r_v / 4 (column v of
    source j).  Per column pair the in-plane mode sum is split from the k_z sum
    as in ``collocation.collocation_matrix``; the two derivatives are
      d/dr_w (rows of w):    sum S(k)/k^2 * (-k_x sin(k_x dx + k_y dy))
      d/dr_v (columns of v): (1/4) sum (-s_v) S(k) cos(k_x dx + k_y dy)
    with S(k) = exp(-k^2 s_v^2 / 2) (d S/k^2 / ds = -s S, the 1/k^2 cancels).
    The mode box is held fixed: its edges sit where the terms are below
    exp(-40) of the leading ones.
    """
    L = cell["L"]
    scale = 1.0 / (green.permittivity(cell) * float(np.prod(L)))
    nodes = [collocation.column_nodes(c) for c in columns]
    sizes = [c["n_colloc"] for c in columns]
    offs = np.concatenate([[0], np.cumsum(sizes)])
    dA = np.zeros((offs[-1], offs[-1]))
    for v, cv in enumerate(columns):
        sc = green.collocation_width(cv)
        mx, my, mz = (green.converged_axis_modes(L[a], sc) for a in range(3))
        kx = 2 * np.pi * mx / L[0]
        ky = 2 * np.pi * my / L[1]
        kz = 2 * np.pi * mz / L[2]
        KX, KY = np.meshgrid(kx, ky, indexing="ij")
        zero_xy = (KX == 0) & (KY == 0)
        for w, cw in enumerate(columns):
            if w != w_d and v != w_d:
                continue
            dx = cw["x"] + cw["radius"] - cv["x"]
            dy = cw["y"] - cv["y"]
            arg = KX * dx + KY * dy
            g = np.zeros(kz.size)
            for iz, kzz in enumerate(kz):
                k2 = KX ** 2 + KY ** 2 + kzz ** 2
                with np.errstate(divide="ignore", invalid="ignore"):
                    sk = np.exp(-0.5 * k2 * sc * sc)
                    term = np.zeros_like(k2)
                    if w == w_d:
                        term = term + sk / k2 * (-KX * np.sin(arg))
                    if v == w_d:
                        term = term + 0.25 * (-sc) * sk * np.cos(arg)
                if kzz == 0.0:
                    term[zero_xy] = 0.0
                g[iz] = term.sum()
            dz = nodes[w][:, None] - nodes[v][None, :]
            dA[offs[w]:offs[w + 1], offs[v]:offs[v + 1]] = scale * np.tensordot(
                np.cos(dz[:, :, None] * kz[None, None, :]), g, axes=([2], [0]))
    return dA


def system_derivative(cell, columns, omega, param, dA_radius=None):
    """dS/dtheta at one angular frequency ((n_q+1) x (n_q+1), complex).

    ``param`` = (w, "rho", p) or (w, "radius", 0); for the radius, ``dA_radius``
    is ``collocation_matrix_radius_derivative`` of that column.
    """
    w_d, kind, p = param
    eps_c = green.permittivity(cell)
    nq = sum(c["n_colloc"] for c in columns)
    dS = np.zeros((nq + 1, nq + 1), dtype=np.complex128)
    if kind == "radius":
        dS[:nq, :nq] = dA_radius
    off = 0
    for w, c in enumerate(columns):
        M = c["n_colloc"]
        if w == w_d:
            R = collocation.cumulative_resistance(c, omega, eps_c)
            mm = np.minimum.outer(np.arange(M), np.arange(M))
            if kind == "rho":
                sigma = collocation.conductivity(c)
                dsig = -1.0 / (len(c["resistivity"]) * c["resistivity"][p] ** 2)
                dR = -R / (sigma + 1j * omega * eps_c) * dsig
            else:
                dR = -2.0 * R / c["radius"]
            dS[off:off + M, off:off + M] += 1j * omega * dR[mm]
        off += M
    return dS


def _solve_equilibrated(S, rhs, nq):
    """S x = rhs with the scaling of ``collocation.solve_frequency`` (q' = a q)."""
    a = np.abs(np.diag(S[:nq, :nq])).max()
    col = np.ones(nq + 1)
    col[:nq] = 1.0 / a
    row = np.ones(nq + 1)
    row[nq] = a
    y = np.linalg.solve((S * col[None, :]) * row[:, None], rhs * row)
    return y * col


def charge_derivatives(cell, columns, sol, param, dA_radius=None):
    """dq(w_j)/dtheta (n_freq, n_q) from the solved spectrum ``sol``."""
    A, q, c, om = sol["A"], sol["q"], sol["c"], sol["omega"]
    nq = A.shape[0]
    eps_c = green.permittivity(cell)
    out = np.empty_like(q)
    for j, w in enumerate(om):
        S, _ = collocation.frequency_system(A, columns, w, eps_c)
        x = np.concatenate([q[j], [c[j]]])
        dS = system_derivative(cell, columns, w, param, dA_radius)
        out[j] = _solve_equilibrated(S, -(dS @ x), nq)[:nq]
    return out


def current_jacobian(cell, columns, spectrum, carriers, params=None):
    """di/dtheta for every parameter: dict param -> (n_tracks, n_time), plus the currents.

    The field goes through the full 3D FFT route (small grids).
    """
    if params is None:
        params = parameter_names(columns)
    s = green.smoothing_widths(cell, columns)
    sol = collocation.solve_spectrum(cell, columns, spectrum)
    src = collocation.sources(columns)
    H = field.field_fft(cell, s, src, timegrid.to_time(sol["q"], spectrum))
    i0 = pipeline.induced_current(H, cell, carriers)
    dA = {}
    jac = {}
    for prm in params:
        w = prm[0]
        if prm[1] == "radius" and w not in dA:
            dA[w] = collocation_matrix_radius_derivative(cell, columns, w)
        dq = charge_derivatives(cell, columns, sol, prm, dA.get(w))
        dH = field.field_fft(cell, s, src, timegrid.to_time(dq, spectrum))
        jac[prm] = pipeline.induced_current(dH, cell, carriers)
    return jac, i0


def perturbed_columns(columns, param, value):
    """Copy of the columns with one parameter set to ``value``."""
    w, kind, p = param
    out = [dict(c, resistivity=list(c["resistivity"])) for c in columns]
    if kind == "rho":
        out[w]["resistivity"][p] = value
    else:
        out[w]["radius"] = value
    return out


def parameter_value(columns, param):
    w, kind, p = param
    return columns[w]["resistivity"][p] if kind == "rho" else columns[w]["radius"]


def scaled_geometry(cell, columns, carriers, scale):
    """The cell, columns and carriers with the in-plane size scaled by ``scale``."""
    L = cell["L"]
    c2 = dict(cell, L=(L[0] * scale, L[1] * scale, L[2]))
    cols = [dict(c, x=c["x"] * scale, y=c["y"] * scale, resistivity=list(c["resistivity"])) for c in columns]
    pos = np.array(carriers["pos"], dtype=np.float64, copy=True)
    pos[..., :2] *= scale
    car = dict(carriers, pos=pos)
    return c2, cols, car


def currents_at_scale(cell, columns, spectrum, carriers, scale):
    """Currents of the whole pipeline (FFT field route) at an in-plane scale."""
    c2, cols, car = scaled_geometry(cell, columns, carriers, scale)
    s = green.smoothing_widths(c2, cols)
    sol = collocation.solve_spectrum(c2, cols, spectrum)
    H = field.field_fft(c2, s, collocation.sources(cols), timegrid.to_time(sol["q"], spectrum))
    return pipeline.induced_current(H, c2, car)


def pitch_derivative(cell, columns, spectrum, carriers, rel_step=1e-4):
    """di/d(pitch) (per metre of L_x) by central differences of the pipeline."""
    ip = currents_at_scale(cell, columns, spectrum, carriers, 1.0 + rel_step)
    im = currents_at_scale(cell, columns, spectrum, carriers, 1.0 - rel_step)
    return (ip - im) / (2.0 * rel_step * cell["L"][0])

