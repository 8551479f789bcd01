"""Fundamental-solution boundary fit, one dense complex solve per frequency (FP64).

Paper, abstract and Section 3: point charges at the electrode boundaries are
adjusted in magnitude so that the boundary conditions hold; the time dependence
of the weighting field comes from the finite resistivity of the graphitised
columns, and the governing equation is the quasi-static (third-order) limit of
Maxwell's equations, which at angular frequency w reads div((sigma + i w eps)
grad psi) = 0.

Model (thin resistive columns):

* column w has its axis at (X_w, Y_w) on a grid node, radius r_w, a contact end
  z^c and a free end z^f, and M_w nodes z_{w,m} = z^c + m (z^f - z^c)/(M_w - 1);
  node spacing D_w;
* source charges q_{w,m} sit on the axis at y_{w,m} = (X_w, Y_w, z_{w,m});
  the potential is matched on the column surface at x_{w,m} = (X_w + r_w, Y_w,
  z_{w,m});
* inside the column, a node's potential drops from the applied contact voltage
  along an RC line: link conductance times length G_w = pi r_w^2 (sigma_w +
  i w eps_c); the axial current through link l is i w times the charge beyond
  it, hence V_{w,m} = V^app_w - i w sum_m' R_w(min(m, m')) q_{w,m'} with the
  cumulative resistance R_w(m) = m D_w / G_w;
* a column made of several quarter-columns in parallel has the mean of their
  conductivities (the four corner bias columns of a pixel meet in one column of
  the periodic cell);
* unknowns: the charges and a gauge constant c; equations:
      sum_j A_ij q_j + i w sum_m' R_w(min(m,m')) q_{w,m'} + c = V^app_w
      sum_j q_j = 0
  with A_ij = G_c(x_i - y_j), the converged periodic fundamental solution of a
  source of width r/4 at the collocation point (``green``), which does not
  depend on the grid that later carries the bulk field.
"""
from __future__ import annotations

import numpy as np

from . import green


def column_nodes(col) -> np.ndarray:
    m = np.arange(col["n_colloc"])
    return col["z_contact"] + m * (col["z_free"] - col["z_contact"]) / (col["n_colloc"] - 1)


def sources(columns) -> np.ndarray:
    """Axis source positions y_{w,m}, columns concatenated in order, (n_q, 3)."""
    out = []
    for c in columns:
        z = column_nodes(c)
        out.append(np.stack([np.full_like(z, c["x"]), np.full_like(z, c["y"]), z], axis=1))
    return np.concatenate(out)


def collocation_points(columns) -> np.ndarray:
    """Surface points x_{w,m} = (X_w + r_w, Y_w, z_{w,m}), (n_q, 3)."""
    out = []
    for c in columns:
        z = column_nodes(c)
        out.append(np.stack([np.full_like(z, c["x"] + c["radius"]),
                             np.full_like(z, c["y"]), z], axis=1))
    return np.concatenate(out)


def conductivity(col) -> float:
    """Conductivity of a column of quarter-columns in parallel (S/m)."""
    return float(np.mean([1.0 / r for r in col["resistivity"]]))


def collocation_matrix(cell, columns) -> np.ndarray:
    """A_ij = G_c(x_i - y_j): converged periodic potential of source j at point i.

    G_c is the Gaussian-charge potential of the converged mode set with the
    source column's width s_c = r/4 (see ``green``).  The mode sum is split as
    (k_x, k_y) then k_z: the in-plane part of the displacement takes one value
    per column pair, so the in-plane sum is done once per pair and k_z, and the
    k_z sum then runs per matrix entry.  Both are plain sums over the modes.
    """
    L = cell["L"]
    scale = 1.0 / (green.permittivity(cell) * float(np.prod(L)))
    nodes = [column_nodes(c) for c in columns]
    sizes = [c["n_colloc"] for c in columns]
    offs = np.concatenate([[0], np.cumsum(sizes)])
    A = np.zeros((offs[-1], offs[-1]))
    for v, cv in enumerate(columns):                      # source column
        sc = green.collocation_width(cv)
        mx, my, mz = (green.converged_axis_modes(L[a], sc) for a in range(3))
        kx = 2 * np.pi * mx / L[0]
        ky = 2 * np.pi * my / L[1]
        kz = 2 * np.pi * mz / L[2]
        KX, KY = np.meshgrid(kx, ky, indexing="ij")
        zero_xy = (KX == 0) & (KY == 0)
        for w, cw in enumerate(columns):                  # collocation column
            dx = cw["x"] + cw["radius"] - cv["x"]
            dy = cw["y"] - cv["y"]
            phase = np.cos(KX * dx + KY * dy)
            g = np.empty(kz.size)
            for iz, kzz in enumerate(kz):
                k2 = KX ** 2 + KY ** 2 + kzz ** 2
                with np.errstate(divide="ignore", invalid="ignore"):
                    term = np.exp(-0.5 * k2 * sc * sc) / k2 * phase
                if kzz == 0.0:
                    term[zero_xy] = 0.0
                g[iz] = term.sum()
            dz = nodes[w][:, None] - nodes[v][None, :]
            A[offs[w]:offs[w + 1], offs[v]:offs[v + 1]] = scale * np.tensordot(
                np.cos(dz[:, :, None] * kz[None, None, :]), g, axes=([2], [0]))
    return A


def collocation_matrix_direct(cell, columns, rows=None, cols=None) -> np.ndarray:
    """Selected entries of A from the direct converged G, entry by entry."""
    x = collocation_points(columns)
    y = sources(columns)
    owner = np.concatenate([[i] * c["n_colloc"] for i, c in enumerate(columns)])
    rows = np.arange(x.shape[0]) if rows is None else np.asarray(rows)
    cols = np.arange(y.shape[0]) if cols is None else np.asarray(cols)
    out = np.empty((rows.size, cols.size))
    for jj, j in enumerate(cols):
        sc = green.collocation_width(columns[owner[j]])
        k = green.converged_mode_set(cell, sc)
        out[:, jj] = green.potential(x[rows] - y[j], cell, sc, k=k)
    return out


def cumulative_resistance(col, omega, eps_c) -> np.ndarray:
    """R_w(m) = sum_{l=1..m} D_w / (pi r^2 (sigma + i w eps_c)), m = 0..M-1."""
    M = col["n_colloc"]
    delta = abs(col["z_free"] - col["z_contact"]) / (M - 1)
    g = np.pi * col["radius"] ** 2 * (conductivity(col) + 1j * omega * eps_c)
    return np.arange(M) * (delta / g)


def frequency_system(A, columns, omega, eps_c):
    """Bordered system S [q; c] = b at one angular frequency."""
    nq = A.shape[0]
    S = np.zeros((nq + 1, nq + 1), dtype=np.complex128)
    S[:nq, :nq] = A
    b = np.zeros(nq + 1, dtype=np.complex128)
    off = 0
    for c in columns:
        M = c["n_colloc"]
        R = cumulative_resistance(c, omega, eps_c)
        mm = np.minimum.outer(np.arange(M), np.arange(M))
        S[off:off + M, off:off + M] += 1j * omega * R[mm]
        b[off:off + M] = c["v_applied"]
        off += M
    S[:nq, nq] = 1.0
    S[nq, :nq] = 1.0
    return S, b


def solve_frequency(A, columns, omega, eps_c):
    """LU with partial pivoting (LAPACK gesv) of the equilibrated system.

    Unknowns are rescaled as q' = a q with a = max |A_ii| and the neutrality row
    is multiplied by a, so every block of the matrix is of order one; the
    solution of the original system is recovered exactly in exact arithmetic.
    Returns (q (n_q,), c).
    """
    nq = A.shape[0]
    S, b = frequency_system(A, columns, omega, eps_c)
    a = np.abs(np.diag(A)).max()
    col = np.ones(nq + 1)
    col[:nq] = 1.0 / a
    row = np.ones(nq + 1)
    row[nq] = a
    Ss = (S * col[None, :]) * row[:, None]
    x = np.linalg.solve(Ss, b * row)
    return x[:nq] / a, x[nq]


def angular_frequencies(spectrum) -> np.ndarray:
    return 2.0 * np.pi * spectrum["df"] * np.arange(spectrum["n_freq"])


def solve_spectrum(cell, columns, spectrum, A=None):
    """Charges q(w_j) (n_freq, n_q) and gauges c(w_j) for every frequency."""
    if A is None:
        A = collocation_matrix(cell, columns)
    eps_c = green.permittivity(cell)
    om = angular_frequencies(spectrum)
    q = np.empty((om.size, A.shape[0]), dtype=np.complex128)
    c = np.empty(om.size, dtype=np.complex128)
    for j, w in enumerate(om):
        q[j], c[j] = solve_frequency(A, columns, w, eps_c)
    return dict(A=A, q=q, c=c, omega=om)
