"""Eq. 1 (introduction): the induced current as a convolution over the carrier path.

    i(t) = -(q / V_w) int_0^t H(x(t'), t - t') . v(t') dt',  V_w = 1 V

Discretised on the time grid t_n = n dt with the carrier polyline P(t_0..t_N):
each step m contributes its displacement dx_m = P(t_{m+1}) - P(t_m) (for
v dt'), taken at the step midpoint xbar_m, with the lag n - m (rectangle rule):

    i_track(t_n) = -(1/V_w) sum_{c in track} q_c sum_{m=0..n} H(xbar_{c,m}, t_{n-m}) . dx_{c,m}

H between grid nodes is the trilinear interpolation of the nodal values with
periodic wrap.  FP64 throughout.
"""
from __future__ import annotations

import numpy as np


def steps(pos):
    """Midpoints and displacements of every polyline step: (n_c, n_t, 3) each."""
    return 0.5 * (pos[:, 1:] + pos[:, :-1]), pos[:, 1:] - pos[:, :-1]


def trilinear_stencil(x, cell):
    """Corner node indices (n, 8, 3) and weights (n, 8) with periodic wrap."""
    L, N = cell["L"], cell["N"]
    h = np.array([L[a] / N[a] for a in range(3)])
    u = x / h
    i0 = np.floor(u)
    f = u - i0
    i0 = i0.astype(np.int64)
    idx = np.empty((x.shape[0], 8, 3), dtype=np.int64)
    wts = np.empty((x.shape[0], 8))
    for c in range(8):
        b = np.array([(c >> 2) & 1, (c >> 1) & 1, c & 1])
        idx[:, c, :] = np.mod(i0 + b[None, :], np.asarray(N)[None, :])
        wts[:, c] = np.prod(np.where(b[None, :] == 1, f, 1.0 - f), axis=1)
    return idx, wts


def induced_current(h_at, cell, pos, charge, track, n_tracks, v_w=1.0):
    """Currents (n_tracks, n_time) in amperes.

    ``h_at(ix, iy, iz)`` returns H at the given nodes as (n, n_time, 3); it may
    index a full array or evaluate a field only where the carriers pass.
    """
    n_time = pos.shape[1] - 1
    xm, dx = steps(pos)
    moving = np.any(dx != 0.0, axis=2)
    cid, mid = np.nonzero(moving)
    xm, dx = xm[cid, mid], dx[cid, mid]
    q = np.asarray(charge, dtype=np.float64)[cid]
    tr = np.asarray(track, dtype=np.int64)[cid]
    out = np.zeros((n_tracks, n_time))
    if cid.size == 0:
        return out
    idx, wts = trilinear_stencil(xm, cell)
    N = cell["N"]
    flat = (idx[..., 0] * N[1] + idx[..., 1]) * N[2] + idx[..., 2]          # (E, 8)
    uniq, inv = np.unique(flat.ravel(), return_inverse=True)
    inv = inv.reshape(flat.shape)
    ux = uniq // (N[1] * N[2])
    uy = (uniq // N[2]) % N[1]
    uz = uniq % N[2]
    Hv = h_at(ux, uy, uz)                                                    # (U, n_time, 3)
    # projection of every corner's lag series on the step: (E, 8, n_time)
    for lag in range(n_time):
        act = mid + lag < n_time
        if not np.any(act):
            break
        e = np.nonzero(act)[0]
        proj = np.einsum("eca,ea->ec", Hv[inv[e], lag, :], dx[e])
        val = q[e] * np.sum(wts[e] * proj, axis=1)
        np.add.at(out, (tr[e], mid[e] + lag), val)
    return -out / v_w
