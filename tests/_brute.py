"""Brute-force integrals that pin the oracle.  Independent of oracle/ code.

tau2d:      the defining double integral of the 1-D table entry (Eq. 8 after
            the p-integral, reduced coordinates), by tensor Gauss-Legendre on
            [0,1]^2 with no reduction to 1-D.
coulomb6d:  the exact <ij|kl> over box planewaves (Eq. 2 with physicist's
            pairing), by reducing the 6-D integral to 3-D (u = xi - xi') and
            integrating 1/|u| over 24 pyramids with apex at the origin, where
            the singularity is removed by the Jacobian.  It does not use the
            Laplace transform, the tables or any quadrature mesh of the method.
"""
import math

import numpy as np


def _gl(n, a=0.0, b=1.0):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (b - a) * x + 0.5 * (b + a), 0.5 * (b - a) * w


def tau2d(beta, m, mp, n=96, panels=4):
    """beta^{-1/2} Int_0^1 Int_0^1 exp(-(xi-xi')^2/beta) e^{2 pi i (m xi + m' xi')} (complex)."""
    xs, ws = [], []
    for p in range(panels):
        x, w = _gl(n, p / panels, (p + 1) / panels)
        xs.append(x)
        ws.append(w)
    x = np.concatenate(xs)
    w = np.concatenate(ws)
    X, Xp = np.meshgrid(x, x, indexing="ij")
    Wt = np.outer(w, w)
    f = np.exp(-(X - Xp) ** 2 / beta) * np.exp(2j * np.pi * (m * X + mp * Xp))
    return (Wt * f).sum() / math.sqrt(beta)


def _overlap(u, m, mp):
    """G(u) = e^{-2 pi i m' u} Int_{max(0,u)}^{min(1,1+u)} e^{2 pi i s xi} d xi, s = m + m'."""
    s = m + mp
    a = np.maximum(0.0, u)
    b = np.minimum(1.0, 1.0 + u)
    if s == 0:
        val = (b - a).astype(complex)
    else:
        val = (np.exp(2j * np.pi * s * b) - np.exp(2j * np.pi * s * a)) / (2j * np.pi * s)
    return np.exp(-2j * np.pi * mp * u) * val


def coulomb6d(ni, nj, nk, nl, L=1.0, n=40):
    """Exact <ij|kl> = Int Int phi_i*(r) phi_j*(r') phi_k(r) phi_l(r') / |r - r'|
    in a box with sides L (a number for a cube, or (Lx, Ly, Lz)).

    With m = n_k - n_i, m' = n_l - n_j and u = xi - xi' (reduced coordinates
    r_d = L_d xi_d) the integral is Int_{[-1,1]^3} prod_d G_d(u_d) /
    sqrt(sum_d L_d^2 u_d^2) d^3u.  Each sign octant of u is split into three
    pyramids (one per coordinate being the largest); with v = r (1, s, t),
    d^3v = r^2 dr ds dt and the distance r sqrt(L_a^2 + L_b^2 s^2 + L_c^2 t^2),
    the integrand is smooth, so plain tensor Gauss-Legendre converges fast.
    """
    m = np.asarray(nk) - np.asarray(ni)
    mp = np.asarray(nl) - np.asarray(nj)
    Ls = np.broadcast_to(np.asarray(L, dtype=np.float64), (3,))
    x, w = _gl(n)
    R, S, T = np.meshgrid(x, x, x, indexing="ij")
    Wt = w[:, None, None] * w[None, :, None] * w[None, None, :]
    total = 0.0 + 0.0j
    for sx in (1.0, -1.0):
        for sy in (1.0, -1.0):
            for sz in (1.0, -1.0):
                sg = (sx, sy, sz)
                for apex in range(3):
                    comp = [None, None, None]
                    comp[apex] = R
                    others = [d for d in range(3) if d != apex]
                    comp[others[0]] = R * S
                    comp[others[1]] = R * T
                    base = Wt * R / np.sqrt(Ls[apex] ** 2 + (Ls[others[0]] * S) ** 2 +
                                            (Ls[others[1]] * T) ** 2)
                    g = np.ones_like(R, dtype=complex)
                    for d in range(3):
                        g = g * _overlap(sg[d] * comp[d], int(m[d]), int(mp[d]))
                    total += (base * g).sum()
    return total
