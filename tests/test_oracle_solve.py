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
