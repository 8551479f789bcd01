"""Index helpers for the time-blocked H layout of the library.

H is stored as H[x][y][tb][z][tin][a] with t = tb * TB + tin (the last block
holds the remaining samples).  These helpers convert a flat buffer (numpy
array or torch tensor) to the plain [x][y][z][t][a] order for inspection and
back; they are pure data movement, used by tests and checks.
"""
from __future__ import annotations


def _blocks(n_time, tb):
    t0 = 0
    while t0 < n_time:
        yield t0, min(tb, n_time - t0)
        t0 += tb


def to_standard(h_flat, N, n_time, tb):
    """Flat time-blocked H (any leading column subset of shape (n_cols, Nz*n_time*3)
    or the whole flat buffer) -> [..., Nz, n_time, 3]."""
    nx, ny, nz = N
    per_col = nz * n_time * 3
    h = h_flat.reshape(-1, per_col)
    outs = []
    off = 0
    for t0, ln in _blocks(n_time, tb):
        outs.append(h[:, off:off + nz * ln * 3].reshape(-1, nz, ln, 3))
        off += nz * ln * 3
    mod = type(h_flat).__module__
    if mod.startswith("torch"):
        import torch
        out = torch.cat(outs, dim=2)
    else:
        import numpy as np
        out = np.concatenate(outs, axis=2)
    if h.shape[0] == nx * ny:
        return out.reshape(nx, ny, nz, n_time, 3)
    return out


def from_standard(h_std, tb):
    """[x][y][z][t][a] (numpy or torch) -> flat time-blocked buffer."""
    nx, ny, nz, n_time, _ = h_std.shape
    cols = h_std.reshape(nx * ny, nz, n_time, 3)
    parts = [cols[:, :, t0:t0 + ln, :].reshape(nx * ny, -1) for t0, ln in _blocks(n_time, tb)]
    mod = type(h_std).__module__
    if mod.startswith("torch"):
        import torch
        return torch.cat(parts, dim=1).reshape(-1).contiguous()
    import numpy as np
    return np.ascontiguousarray(np.concatenate(parts, axis=1).reshape(-1))


def element_index(x, y, z, t, a, N, n_time, tb):
    """Flat index of H(x, y, z, t, a); arguments are integers or numpy arrays."""
    import numpy as np
    x, y, z, t, a = (np.asarray(v, dtype=np.int64) for v in (x, y, z, t, a))
    nx, ny, nz = N
    blk = t // tb
    tin = t - blk * tb
    last = (n_time - 1) // tb
    blen = np.where(blk == last, n_time - last * tb, tb)
    return (x * ny + y) * nz * n_time * 3 + blk * tb * nz * 3 + z * blen * 3 + tin * 3 + a
