"""The whole path in the paper's order: boundary fit -> time -> bulk field -> Eq. 1."""
from __future__ import annotations

import numpy as np

from . import collocation, convolution, field, green, timegrid


def weighting_field(cell, columns, spectrum, route="fft", cols_ij=None, points=None):
    """Solve the boundary fit for every frequency, map to time, build H.

    route: "fft" (whole grid), "columns" (selected (ix, iy) columns, all z) or
    "superposition" (arbitrary points, direct sums).  Returns a dict with the
    collocation matrix A, charges q(w) and gauges c(w), time charges q(t),
    source positions and the requested field.
    """
    s = green.smoothing_widths(cell, columns)
    sol = collocation.solve_spectrum(cell, columns, spectrum)
    q_t = timegrid.to_time(sol["q"], spectrum)
    src = collocation.sources(columns)
    out = dict(sol, q_t=q_t, src=src)
    if route == "fft":
        out["H"] = field.field_fft(cell, s, src, q_t)
    elif route == "columns":
        out["H_cols"] = field.field_columns(cell, s, src, q_t, cols_ij)
    elif route == "superposition":
        out["H_pts"] = field.field_superposition(np.asarray(points), cell, s, src, q_t)
    elif route is not None:
        raise ValueError(route)
    return out


def induced_current(H, cell, carriers):
    """Eq. 1 currents (n_tracks, n_time) for a full H array or an H(ix,iy,iz) callable."""
    if callable(H):
        h_at = H
    else:
        def h_at(ix, iy, iz):
            return H[ix, iy, iz]
    return convolution.induced_current(h_at, cell, carriers["pos"], carriers["charge"],
                                       carriers["track"], carriers["n_tracks"])
