"""The paper's own time-domain scheme (Section 3: iterative forward-Euler
stepping of the boundary charges) applied to the thin-wire RC-line model of
``collocation``, as a cross-check of the frequency-domain solve.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain FP64 numpy.

Column w has conductivity s_w and the geometric resistance factors
rho_w(m) = m D_w / (pi r_w^2), so that the RC-line term of the collocation
system is R_w(m) = rho_w(m) / (s_w + i w eps).  Multiplying node row (w, m)
of  A q + i w R(min) q + c = V  by (s_w + i w eps) gives
    s_w (A q + c - V)  +  i w [ eps (A q + c - V) + P q ] = 0,
P = blockdiag_w rho_w(min(m, m')), which is the frequency form of
    K x' = -G x + g(t),   x = [q; c],
    K = [[eps A + P, eps 1], [1^T, 0]]     (the neutrality row differentiated),
    G = [[diag(s) A, diag(s) 1], [0, 0]],
    g = [diag(s) V(t) + eps V'(t); 0].
A voltage step V(t) = V_app theta(t) puts eps V_app delta(t) into g: the
charges jump to x(0+) = K^-1 [eps V_app; 0] (the high-frequency, purely
capacitive response) and then relax with K x' = -G x + [diag(s) V_app; 0]
towards the DC solution.
"""
import numpy as np

from .collocation import conductivity


def rc_line_system(A, columns, eps_c):
    """K, G, the step drive b_s = [diag(s) V_app; 0] and the jump drive
    b_e = [eps V_app; 0] of the time-domain system."""
    nq = A.shape[0]
    K = np.zeros((nq + 1, nq + 1))
    G = np.zeros((nq + 1, nq + 1))
    b_s = np.zeros(nq + 1)
    b_e = np.zeros(nq + 1)
    K[:nq, :nq] = eps_c * A
    K[:nq, nq] = eps_c
    K[nq, :nq] = 1.0
    off = 0
    for c in columns:
        M = c["n_colloc"]
        delta = abs(c["z_free"] - c["z_contact"]) / (M - 1)
        rho = np.arange(M) * delta / (np.pi * c["radius"] ** 2)
        K[off:off + M, off:off + M] += rho[np.minimum.outer(np.arange(M), np.arange(M))]
        s = conductivity(c)
        G[off:off + M, :nq] = s * A[off:off + M, :]
        G[off:off + M, nq] = s
        b_s[off:off + M] = s * c["v_applied"]
        b_e[off:off + M] = eps_c * c["v_applied"]
        off += M
    return K, G, b_s, b_e


def transfer(K, G, b_s, b_e, omega):
    """[q; c] of a harmonic drive V_app e^{i w t}: (i w K + G) x = b_s + i w b_e,
    with the neutrality row i w sum q = 0 written as sum q = 0 (the same for
    w != 0, and the DC condition at w = 0)."""
    nq = K.shape[0] - 1
    S = 1j * omega * K + G
    S[nq, :] = 0.0
    S[nq, :nq] = 1.0
    return np.linalg.solve(S, b_s + 1j * omega * b_e)


def step_limits(K, G, b_s, b_e):
    """x(0+) (capacitive jump) and x(inf) (DC: G x = b_s with sum q = 0)."""
    nq = K.shape[0] - 1
    x0 = np.linalg.solve(K, b_e)
    Gd = G.copy()
    Gd[nq, :nq] = 1.0                               # neutrality closes the DC system
    x_inf = np.linalg.solve(Gd, b_s)
    return x0, x_inf


def step_response_exact(K, G, b_s, b_e, times):
    """x(t) = x_inf + W exp(L t) W^-1 (x(0+) - x_inf), (L, W) = eig(-K^-1 G)."""
    x0, x_inf = step_limits(K, G, b_s, b_e)
    lam, W = np.linalg.eig(-np.linalg.solve(K, G))
    coef = np.linalg.solve(W, (x0 - x_inf).astype(np.complex128))
    out = np.array([x_inf + (W * np.exp(lam * t)) @ coef for t in np.atleast_1d(times)])
    return out.real, lam


def step_response_euler(K, G, b_s, b_e, dt, n_steps, record_every=1):
    """Forward Euler from x(0+): x_{k+1} = x_k + dt K^-1 (-G x_k + b_s).
    Returns the states at steps 0, record_every, 2 record_every, ..."""
    x, _ = step_limits(K, G, b_s, b_e)
    F = np.linalg.solve(K, -G)                      # K^-1 (-G)
    f = np.linalg.solve(K, b_s)                     # K^-1 b_s
    out = [x.copy()]
    for k in range(1, n_steps + 1):
        x = x + dt * (F @ x + f)
        if k % record_every == 0:
            out.append(x.copy())
    return np.array(out)
