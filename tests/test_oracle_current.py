"""Pins of the Eq. 1 convolution: brute force, exact interpolation, the
textbook Ramo-Shockley limit and charge conservation."""
import numpy as np

import oracle
from oracle import convolution, field, green
from paper_2605_13987_amd import workloads

UM = 1e-6


def _brute_force(H, cell, pos, q, track, n_tracks):
    """Eq. 1 with plain loops: every carrier, every step, every later sample."""
    L, N = cell["L"], cell["N"]
    nt = pos.shape[1] - 1
    out = np.zeros((n_tracks, nt))
    for c in range(pos.shape[0]):
        for m in range(nt):
            d = pos[c, m + 1] - pos[c, m]
            if not np.any(d != 0):
                continue
            x = 0.5 * (pos[c, m + 1] + pos[c, m])
            u = [x[a] * N[a] / L[a] for a in range(3)]
            i0 = [int(np.floor(u[a])) for a in range(3)]
            f = [u[a] - i0[a] for a in range(3)]
            for n in range(m, nt):
                acc = 0.0
                for bx in (0, 1):
                    for by in (0, 1):
                        for bz in (0, 1):
                            w = ((f[0] if bx else 1 - f[0]) * (f[1] if by else 1 - f[1])
                                 * (f[2] if bz else 1 - f[2]))
                            h = H[(i0[0] + bx) % N[0], (i0[1] + by) % N[1], (i0[2] + bz) % N[2], n - m]
                            acc += w * (h[0] * d[0] + h[1] * d[1] + h[2] * d[2])
                out[track[c], n] -= q[c] * acc
    return out


def test_convolution_matches_brute_force_loops():
    rng = np.random.default_rng(7)
    cell = dict(L=(6e-6, 5e-6, 12e-6), N=(6, 5, 8), eps_r=5.7, sigma_bulk=0.0)
    nt = 10
    H = rng.standard_normal((6, 5, 8, nt, 3))
    nc = 7
    pos = np.cumsum(rng.normal(0, 1.3e-6, size=(nc, nt + 1, 3)), axis=1) + rng.random((nc, 1, 3)) * 5e-6
    pos[2, 4:] = pos[2, 4]                       # absorbed carrier: steps stop
    pos[3] -= 20e-6                              # far outside the cell: periodic wrap
    q = rng.choice([-1.0, 1.0], nc) * 1.6e-19
    track = np.array([0, 1, 1, 0, 2, 2, 1])
    ref = _brute_force(H, cell, pos, q, track, 3)
    got = convolution.induced_current(lambda i, j, k: H[i, j, k], cell, pos, q, track, 3)
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_trilinear_interpolation_is_exact_for_linear_fields():
    """H(x, t) = (g . x + b) u(t) away from the wrap: interpolation is exact,
    so i_n = -q sum_m (g . xbar_m + b) u(t_{n-m}) . dx_m in closed form."""
    rng = np.random.default_rng(8)
    cell = dict(L=(20e-6, 20e-6, 40e-6), N=(10, 10, 20), eps_r=5.7, sigma_bulk=0.0)
    nt = 12
    g = rng.standard_normal((3, 3))              # H_a = sum_b g[a,b] x_b + b_a
    b = rng.standard_normal(3)
    u = rng.standard_normal(nt)
    h = np.array([cell["L"][a] / cell["N"][a] for a in range(3)])
    I = np.stack(np.meshgrid(*(np.arange(cell["N"][a]) * h[a] for a in range(3)), indexing="ij"), axis=-1)
    Hs = I @ g.T + b                             # (nx,ny,nz,3)
    H = Hs[:, :, :, None, :] * u[None, None, None, :, None]
    pos = 6e-6 + np.cumsum(rng.uniform(0, 0.6e-6, size=(3, nt + 1, 3)), axis=1)
    q = np.array([1.6e-19, -1.6e-19, 1.6e-19])
    got = convolution.induced_current(lambda i, j, k: H[i, j, k], cell, pos, q, np.zeros(3, int), 1)
    xm, dx = convolution.steps(pos)
    proj = np.einsum("cma,cma->cm", xm @ g.T + b, dx)           # (c, m)
    ref = np.zeros(nt)
    for n in range(nt):
        for m in range(n + 1):
            ref[n] -= np.sum(q * proj[:, m]) * u[n - m]
    assert np.max(np.abs(got[0] - ref)) <= 1e-12 * np.max(np.abs(ref))


def _perfect_conductor_case(n_freq=33, n_xy=48, n_z=40):
    """Columns of negligible resistivity on a Nyquist frequency grid."""
    cfg = workloads.small_pixel(k=31, n_xy=n_xy, n_z=n_z, n_freq=n_freq,
                                 n_time=2 * (n_freq - 1), n_pairs=12, n_colloc=16,
                                 rho=np.full(5, 1e-25))
    return cfg


def test_textbook_ramo_shockley_limit():
    """With perfectly conducting columns q(w) is the static solution at every
    frequency, the quadrature turns it into q_s delta_{n0}/dt, and Eq. 1
    reduces to i_n = -sum_c q_c H_s(xbar_{c,n}) . dx_{c,n} / dt."""
    cfg = _perfect_conductor_case(n_freq=9, n_xy=24, n_z=40)
    cell, cols, spec, car = cfg["cell"], cfg["columns"], cfg["spectrum"], cfg["carriers"]
    res = oracle.weighting_field(cell, cols, spec)
    q0 = res["q"][0].real
    assert np.max(np.abs(res["q"] - q0[None, :])) <= 1e-12 * np.max(np.abs(q0))
    dt = spec["dt"]
    expect_qt = np.zeros_like(res["q_t"])
    expect_qt[0] = q0 / dt
    assert np.max(np.abs(res["q_t"] - expect_qt)) <= 1e-12 * np.max(np.abs(q0)) / dt
    H = res["H"]
    i = oracle.induced_current(H, cell, car)
    Hs = H[:, :, :, 0, :] * dt                                   # static field
    xm, dx = convolution.steps(car["pos"])
    ref = np.zeros_like(i)
    for c in range(xm.shape[0]):
        idx, w = convolution.trilinear_stencil(xm[c], cell)
        hs = np.einsum("mk,mka->ma", w, Hs[idx[..., 0], idx[..., 1], idx[..., 2]])
        ref[car["track"][c]] -= car["charge"][c] * np.einsum("ma,ma->m", hs, dx[c]) / dt
    assert np.max(np.abs(i - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_charge_conservation_full_traversal():
    """Perfect conductors, every carrier absorbed inside the window: the time
    integral of the current equals q [phi_w(end) - phi_w(start)] with phi_w the
    static weighting potential, up to the midpoint/trilinear quadrature error."""
    cfg = _perfect_conductor_case()
    cell, cols, spec, car = cfg["cell"], cfg["columns"], cfg["spectrum"], cfg["carriers"]
    pos = car["pos"]
    assert np.all(np.linalg.norm(pos[:, -1] - pos[:, -2], axis=1) == 0)      # all absorbed
    res = oracle.weighting_field(cell, cols, spec, route=None)
    s = green.smoothing_widths(cell, cols)
    q0 = res["q"][0].real
    Hs = field.field_fft(cell, s, res["src"], q0[None, :])                    # static field (1 sample)
    # integral of i dt under perfect conductors = -sum_c q_c sum_m H_s(xbar) . dx
    xm, dx = convolution.steps(pos)
    total = np.zeros(car["n_tracks"])
    for c in range(pos.shape[0]):
        idx, w = convolution.trilinear_stencil(xm[c], cell)
        hs = np.einsum("mk,mka->ma", w, Hs[idx[..., 0], idx[..., 1], idx[..., 2], 0])
        total[car["track"][c]] -= car["charge"][c] * np.sum(hs * dx[c])
    # the same integral from the full pipeline (exact discrete identity)
    Hfull = field.field_fft(cell, s, res["src"], res["q_t"])
    cur = oracle.induced_current(Hfull, cell, car)
    assert np.max(np.abs(cur.sum(axis=1) * spec["dt"] - total)) <= 1e-10 * np.max(np.abs(total))
    # physics: potential difference from the bulk Green's function
    src = res["src"]
    phi_end = np.array([green.potential(p - src, cell, s) @ q0 for p in pos[:, -1]])
    phi_start = np.array([green.potential(p - src, cell, s) @ q0 for p in pos[:, 0]])
    expect = np.zeros(car["n_tracks"])
    for c in range(pos.shape[0]):
        expect[car["track"][c]] += car["charge"][c] * (phi_end[c] - phi_start[c])
    scale = np.sum(np.abs(car["charge"] * (phi_end - phi_start)))
    assert np.max(np.abs(total - expect)) <= 2e-3 * scale
