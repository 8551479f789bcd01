"""Pins of the boundary-fit solve: Kirchhoff assembly, QR, static and sum rules, passivity."""
import copy

import numpy as np
import scipy.linalg

import ewald
from oracle import collocation, green


def _kirchhoff_solve(A, columns, omega, eps_c):
    """Same physics assembled from first principles: node potentials V, link
    currents I, Ohm's law per link, charge conservation (KCL) per node, the
    contact node held at the applied voltage, collocation, neutrality."""
    nq = A.shape[0]
    offs = np.concatenate([[0], np.cumsum([c["n_colloc"] for c in columns])])
    nlink = nq - len(columns)
    # unknown layout: q (nq) | V (nq) | I (nlink) | c (1)
    n = 2 * nq + nlink + 1
    S = np.zeros((n, n), dtype=complex)
    b = np.zeros(n, dtype=complex)
    iq, iV, iI, ic = 0, nq, 2 * nq, 2 * nq + nlink
    r = 0
    for i in range(nq):                                  # collocation
        S[r, iq:iq + nq] = A[i]
        S[r, ic] = 1.0
        S[r, iV + i] = -1.0
        r += 1
    link = 0
    for w, col in enumerate(columns):
        M = col["n_colloc"]
        o = offs[w]
        S[r, iV + o] = 1.0                                # contact potential
        b[r] = col["v_applied"]
        r += 1
        delta = abs(col["z_free"] - col["z_contact"]) / (M - 1)
        G = np.pi * col["radius"] ** 2 * (collocation.conductivity(col) + 1j * omega * eps_c)
        first = link
        for l in range(1, M):                             # Ohm: V_{l-1} - V_l = (delta/G) I_l
            S[r, iV + o + l - 1] = 1.0
            S[r, iV + o + l] = -1.0
            S[r, iI + link] = -delta / G
            r += 1
            link += 1
        for m in range(1, M):                             # KCL: i w q_m = I_m - I_{m+1}
            S[r, iq + o + m] = 1j * omega
            S[r, iI + first + m - 1] = -1.0
            if m + 1 < M:
                S[r, iI + first + m] = 1.0
            r += 1
    S[r, iq:iq + nq] = 1.0                                # neutrality
    r += 1
    assert r == n
    x = np.linalg.solve(S, b)
    return x[:nq], x[ic]


def test_compact_rc_line_equals_kirchhoff_assembly(px32, px32_oracle):
    A = px32_oracle["A"]
    eps_c = green.permittivity(px32["cell"])
    for om in (0.0, 2 * np.pi * 1.25e9, 2 * np.pi * 18.75e9, 2 * np.pi * 400e9):
        q, c = collocation.solve_frequency(A, px32["columns"], om, eps_c)
        qk, ck = _kirchhoff_solve(A, px32["columns"], om, eps_c)
        assert np.max(np.abs(q - qk)) <= 1e-9 * np.max(np.abs(qk)), om
        assert abs(c - ck) <= 1e-9 * max(1.0, abs(ck))


def test_lu_agrees_with_qr_and_backward_error(px32, px32_oracle):
    A = px32_oracle["A"]
    eps_c = green.permittivity(px32["cell"])
    nq = A.shape[0]
    for om in px32_oracle["omega"][[0, 5, 15]]:
        S, b = collocation.frequency_system(A, px32["columns"], om, eps_c)
        q, c = collocation.solve_frequency(A, px32["columns"], om, eps_c)
        a = np.abs(np.diag(A)).max()
        colsc = np.r_[np.full(nq, 1 / a), 1.0]
        rowsc = np.r_[np.ones(nq), a]
        Ss = S * colsc[None, :] * rowsc[:, None]
        bs = b * rowsc
        Q, R = scipy.linalg.qr(Ss)
        xq = scipy.linalg.solve_triangular(R, Q.conj().T @ bs)
        x = np.r_[q * a, c]
        kappa = np.linalg.cond(Ss)
        assert np.max(np.abs(x - xq)) <= 1e-15 * kappa * 50 * np.max(np.abs(x))
        berr = np.linalg.norm(Ss @ x - bs, np.inf) / (np.linalg.norm(Ss, np.inf) * np.linalg.norm(x, np.inf))
        assert berr <= 1e-14


def test_static_potentials_on_column_surfaces(px32, px32_oracle):
    """At w = 0 the columns are equipotential: the potential of the fitted
    charges, summed with the Ewald form of the fundamental solution, equals the
    applied voltage minus the gauge at every collocation point."""
    q = px32_oracle["q"][0].real
    c = px32_oracle["c"][0].real
    assert np.max(np.abs(px32_oracle["q"][0].imag)) == 0.0
    x = collocation.collocation_points(px32["columns"])
    y = collocation.sources(px32["columns"])
    widths = np.concatenate([[green.collocation_width(col)] * col["n_colloc"] for col in px32["columns"]])
    vapp = np.concatenate([[col["v_applied"]] * col["n_colloc"] for col in px32["columns"]])
    rng = np.random.default_rng(4)
    for i in rng.choice(x.shape[0], 10, replace=False):
        phi = 0.0
        for wdt in np.unique(widths):
            sel = widths == wdt
            phi += ewald.potential(x[i] - y[sel], px32["cell"]["L"], px32["cell"]["eps_r"], wdt) @ q[sel]
        assert abs(phi + c - vapp[i]) <= 1e-11


def test_electrode_sum_rule(px32, px32_oracle):
    """Unit voltage on every column: no charge moves, the gauge is 1; hence the
    readout and bias responses sum to zero (linearity)."""
    A = px32_oracle["A"]
    eps_c = green.permittivity(px32["cell"])
    cols_all = copy.deepcopy(px32["columns"])
    for col in cols_all:
        col["v_applied"] = 1.0
    cols_bias = copy.deepcopy(px32["columns"])
    cols_bias[0]["v_applied"], cols_bias[1]["v_applied"] = 0.0, 1.0
    qscale = np.max(np.abs(px32_oracle["q"]))
    for j, om in enumerate(px32_oracle["omega"][[0, 3, 15]]):
        q1, c1g = collocation.solve_frequency(A, cols_all, om, eps_c)
        assert np.max(np.abs(q1)) <= 1e-12 * qscale
        assert abs(c1g - 1.0) <= 1e-12
        qb, _ = collocation.solve_frequency(A, cols_bias, om, eps_c)
        qr, _ = collocation.solve_frequency(A, px32["columns"], om, eps_c)
        assert np.max(np.abs(qb + qr)) <= 1e-12 * qscale


def test_readout_admittance_is_passive(px32_oracle):
    """Y(w) = i w Q_readout / V_app of the RC network must have Re Y >= 0
    (with exp(+i w t), a dissipative network absorbs power)."""
    Q = px32_oracle["q"][:, :64].sum(axis=1)
    Y = 1j * px32_oracle["omega"] * Q
    assert np.all(Y.real[1:] > 0)
    # static capacitance is positive and the charge magnitude falls with frequency
    assert Q[0].real > 0 and np.all(np.diff(np.abs(Q)) < 0)


def test_full_height_perfect_conductors_reduce_to_a_2d_line_lattice():
    """Columns spanning the whole periodic height, at zero frequency (perfect
    conductors): the solution is z-invariant, a line charge lambda_w per
    column, and the lambdas solve the 2D problem sum_w' lambda_w' G2(x_w -
    X_w') + c = V_w, sum lambda = 0 with the 2D Ewald lattice sum of Gaussian
    line charges (an independent closed form).  256 nodes per column put the
    aliased k_z = 2 pi n / D terms of the node row below 1e-9; the row of 256
    sources per column is then ill-conditioned (cond ~ 1e8), which bounds the
    z-invariance of the solved charges at ~1e-8."""
    from oracle import collocation, green
    import ewald

    L = (50e-6, 50e-6, 300e-6)
    cell = dict(L=L, N=(32, 32, 64), eps_r=5.7, sigma_bulk=0.0)
    M = 256
    cols = [dict(x=25e-6, y=25e-6, radius=5e-6, z_contact=0.0, z_free=L[2] * (M - 1) / M,
                 resistivity=[1e-3], n_colloc=M, v_applied=1.0),
            dict(x=0.0, y=0.0, radius=5e-6, z_contact=0.0, z_free=L[2] * (M - 1) / M,
                 resistivity=[1e-3], n_colloc=M, v_applied=0.0)]
    A = collocation.collocation_matrix(cell, cols)
    q, c = collocation.solve_frequency(A, cols, 0.0, green.permittivity(cell))
    q = q.real.reshape(2, M)
    # z-invariance
    assert np.max(np.abs(q - q.mean(axis=1, keepdims=True))) <= 1e-7 * np.max(np.abs(q))
    lam = q.mean(axis=1) / (L[2] / M)
    # the 2D system
    s = green.collocation_width(cols[0])
    X = np.array([[c_["x"], c_["y"]] for c_ in cols])
    S = np.zeros((3, 3))
    for i in range(2):
        for j in range(2):
            S[i, j] = ewald.potential_2d((X[i] + [cols[i]["radius"], 0.0]) - X[j], L[:2], 5.7, s)[0]
    S[:2, 2] = 1.0
    S[2, :2] = 1.0
    ref = np.linalg.solve(S, np.array([1.0, 0.0, 0.0]))
    assert np.max(np.abs(lam - ref[:2])) <= 1e-9 * np.max(np.abs(ref[:2]))
    assert abs(c.real - ref[2]) <= 1e-9
    # the 2D lattice sum does not depend on its splitting width
    d = np.array([[3e-6, 1e-6], [20e-6, -7e-6], [0.0, 0.0]])
    g8, g12 = ewald.potential_2d(d, L[:2], 5.7, s, b=8e-6), ewald.potential_2d(d, L[:2], 5.7, s, b=12e-6)
    assert np.max(np.abs(g8 - g12)) <= 1e-12 * np.max(np.abs(g12))

