"""Ewald sums for the periodic potential and field of an isotropic Gaussian charge.

Independent closed form used to pin the oracle's mode sums (Ewald 1921).  For a
unit Gaussian charge of width s in a periodic box of volume V with a uniform
neutralising background, splitting with a wider Gaussian of width b gives

  G(d) = sum_n [erf(r_n / (sqrt2 s)) - erf(r_n / (sqrt2 b))] / (4 pi eps r_n)
         - (b^2 - s^2) / (2 eps V)
         + 1/(eps V) sum_{k != 0} exp(-k^2 b^2 / 2) cos(k.d) / k^2

with r_n = |d + n L|: the first sum is the potential of the neutral difference
of the two Gaussians (short range), the constant is that difference's k = 0
term, and the last sum is the smooth wide-Gaussian part in reciprocal space.
"""
import math

import numpy as np
from scipy.special import erf

EPS0 = 8.8541878128e-12


def _wrap(d, L):
    L = np.asarray(L)
    return d - L * np.round(d / L)


def _images(L, b):
    reach = 9.0 * b
    return [np.arange(-int(math.ceil(reach / L[a])) - 1, int(math.ceil(reach / L[a])) + 2) for a in range(3)]


def _recip(L, b):
    kc = math.sqrt(2 * 42.0) / b
    ms = [np.arange(-int(kc * L[a] / (2 * math.pi)) - 1, int(kc * L[a] / (2 * math.pi)) + 2) for a in range(3)]
    g = np.meshgrid(*ms, indexing="ij")
    m = np.stack([x.ravel() for x in g], axis=1)
    m = m[np.any(m != 0, axis=1)]
    return 2 * math.pi * m / np.asarray(L)


def potential(d, L, eps_r, s, b=None):
    eps = eps_r * EPS0
    L = np.asarray(L, dtype=float)
    b = b if b is not None else min(L) / 5.0
    vol = float(np.prod(L))
    d = _wrap(np.atleast_2d(d), L)
    out = np.zeros(d.shape[0])
    ix, iy, iz = _images(L, b)
    for nx in ix:
        for ny in iy:
            for nz in iz:
                r = np.linalg.norm(d + np.array([nx, ny, nz]) * L, axis=1)
                small = r < 1e-300
                rr = np.where(small, 1.0, r)
                val = (erf(rr / (math.sqrt(2) * s)) - erf(rr / (math.sqrt(2) * b))) / (4 * math.pi * eps * rr)
                lim = math.sqrt(2 / math.pi) * (1 / s - 1 / b) / (4 * math.pi * eps)
                out += np.where(small, lim, val)
    out -= (b * b - s * s) / (2 * eps * vol)
    k = _recip(L, b)
    k2 = np.sum(k * k, axis=1)
    w = np.exp(-0.5 * k2 * b * b) / k2
    out += (np.cos(d @ k.T) @ w) / (eps * vol)
    return out


def field(d, L, eps_r, s, b=None):
    """-grad of ``potential`` with respect to d."""
    eps = eps_r * EPS0
    L = np.asarray(L, dtype=float)
    b = b if b is not None else min(L) / 5.0
    vol = float(np.prod(L))
    d = _wrap(np.atleast_2d(d), L)
    out = np.zeros((d.shape[0], 3))
    ix, iy, iz = _images(L, b)
    for nx in ix:
        for ny in iy:
            for nz in iz:
                v = d + np.array([nx, ny, nz]) * L
                r = np.linalg.norm(v, axis=1)
                ok = r > 1e-300
                rr = np.where(ok, r, 1.0)
                f = (erf(rr / (math.sqrt(2) * s)) - erf(rr / (math.sqrt(2) * b)))
                fp = (math.sqrt(2 / math.pi) / s) * np.exp(-rr * rr / (2 * s * s)) \
                    - (math.sqrt(2 / math.pi) / b) * np.exp(-rr * rr / (2 * b * b))
                # d/dr [f/r] = (fp r - f)/r^2 ; E = -(d/dr)(f/(4 pi eps r)) v/r
                dphidr = (fp * rr - f) / (rr * rr) / (4 * math.pi * eps)
                out += np.where(ok[:, None], -dphidr[:, None] * v / rr[:, None], 0.0)
    k = _recip(L, b)
    k2 = np.sum(k * k, axis=1)
    w = np.exp(-0.5 * k2 * b * b) / k2
    out += ((np.sin(d @ k.T) * w) @ k) / (eps * vol)
    return out


def potential_2d(d, L, eps_r, s, b=None):
    """Potential per unit line charge of a 2D periodic lattice of Gaussian line
    charges (width s) in a neutralising background, cell L = (L_x, L_y):

      G2(d) = sum_n [E1(r_n^2 / 2b^2) - E1(r_n^2 / 2s^2)] / (4 pi eps)
              - (b^2 - s^2) / (2 eps A)
              + 1/(eps A) sum_{k != 0} exp(-k^2 b^2 / 2) cos(k.d) / k^2

    (the 2D potential of a Gaussian line charge is -(2 ln r + E1(r^2/2s^2)) /
    (4 pi eps) up to a constant, so the difference of two widths is the short
    sum; the constant is that difference's k = 0 term, A = L_x L_y).
    """
    from scipy.special import exp1

    eps = eps_r * EPS0
    L = np.asarray(L, dtype=float)
    b = b if b is not None else min(L) / 5.0
    area = float(np.prod(L))
    d = _wrap(np.atleast_2d(d), L)
    out = np.zeros(d.shape[0])
    reach = 9.0 * b
    ns = [np.arange(-int(math.ceil(reach / L[a])) - 1, int(math.ceil(reach / L[a])) + 2) for a in range(2)]
    for nx in ns[0]:
        for ny in ns[1]:
            r2 = np.sum((d + np.array([nx, ny]) * L) ** 2, axis=1)
            small = r2 < 1e-300
            rr2 = np.where(small, 1.0, r2)
            val = (exp1(rr2 / (2 * b * b)) - exp1(rr2 / (2 * s * s))) / (4 * math.pi * eps)
            lim = 2.0 * math.log(b / s) / (4 * math.pi * eps)      # E1(x) - E1(y) -> ln(y/x) at r -> 0
            out += np.where(small, lim, val)
    out -= (b * b - s * s) / (2 * eps * area)
    kc = math.sqrt(2 * 42.0) / b
    ms = [np.arange(-int(kc * L[a] / (2 * math.pi)) - 1, int(kc * L[a] / (2 * math.pi)) + 2) for a in range(2)]
    g = np.meshgrid(*ms, indexing="ij")
    m = np.stack([x.ravel() for x in g], axis=1)
    m = m[np.any(m != 0, axis=1)]
    k = 2 * math.pi * m / L
    k2 = np.sum(k * k, axis=1)
    out += (np.cos(d @ k.T) @ (np.exp(-0.5 * k2 * b * b) / k2)) / (eps * area)
    return out

