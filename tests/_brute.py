"""Brute-force integrals that pin the oracle.  Independent of oracle/ code.

tau2d:      the defining double integral of the 1-D table entry (Eq. 8 after
            the p-integral, reduced coordinates), by tensor Gauss-Legendre on
            [0,1]^2 with no reduction to 1-D.
gauss_G2d:  the 1-D factor of the Gaussian basis (Int Int f_u f_v(x)
            exp(-s (x - x')^2) f_u' f_v'(x') dx dx') by tensor Gauss-Legendre
            over a box holding both products.
gauss_exact: <ij|kl> of isotropic s-type Gaussians in closed form (Boys F0).
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


def gauss_G2d(s, a, A, u, v, up, vp, n=160):
    """Int Int f_u(x) f_v(x) exp(-s (x - x')^2) f_up(x') f_vp(x') dx dx' with
    f(x) = (2 a / pi)^{1/4} exp(-a (x - A)^2), by tensor Gauss-Legendre.  For
    s <= 1 over [lo, hi]^2 covering every function to exp(-40); for s > 1 in
    (x, y = sqrt(s) (x' - x)), where the kernel is exp(-y^2) on |y| <= 9 and
    the integral carries s^{-1/2}, so narrow kernels stay resolved."""
    f = lambda k, x: (2 * a[k] / math.pi) ** 0.25 * np.exp(-a[k] * (x - A[k]) ** 2)
    width = max(math.sqrt(40.0 / a[k]) for k in (u, v, up, vp))
    lo = min(A[k] for k in (u, v, up, vp)) - width
    hi = max(A[k] for k in (u, v, up, vp)) + width

    def panels(n_pts, a0, b0, k=8):
        xs, ws = [], []
        for p in range(k):
            x, w = _gl(max(2, n_pts // k * 2), a0 + (b0 - a0) * p / k, a0 + (b0 - a0) * (p + 1) / k)
            xs.append(x)
            ws.append(w)
        return np.concatenate(xs), np.concatenate(ws)
    x, w = panels(n, lo, hi)
    if s <= 1.0:
        X, Xp = np.meshgrid(x, x, indexing="ij")
        F = (f(u, X) * f(v, X)) * np.exp(-s * (X - Xp) ** 2) * (f(up, Xp) * f(vp, Xp))
        return float((np.outer(w, w) * F).sum())
    y, wy = panels(n, -9.0, 9.0)
    X, Y = np.meshgrid(x, y, indexing="ij")
    Xp = X + Y / math.sqrt(s)
    F = (f(u, X) * f(v, X)) * np.exp(-Y * Y) * (f(up, Xp) * f(vp, Xp))
    return float((np.outer(w, wy) * F).sum()) / math.sqrt(s)


def boys0(T):
    """F0(T) = Int_0^1 exp(-T t^2) dt = (1/2) sqrt(pi/T) erf(sqrt(T))."""
    from scipy.special import erf
    T = np.asarray(T, dtype=np.float64)
    small = T < 1e-12
    out = np.empty_like(T)
    out[small] = 1.0 - T[small] / 3.0
    t = T[~small]
    out[~small] = 0.5 * np.sqrt(math.pi / t) * erf(np.sqrt(t))
    return out


def gauss_exact(exps, centers, quads):
    """<ij|kl> = Int Int g_i(r) g_k(r) g_j(r') g_l(r') / |r - r'| for
    isotropic, unit-norm s-type Gaussians g = (2 e / pi)^{3/4}
    exp(-e |r - C|^2), by the textbook closed form: with p = e_i + e_k,
    q = e_j + e_l and product centers P, Q,
      n_i n_j n_k n_l K_ik K_jl 2 pi^{5/2} / (p q sqrt(p + q)) F0(p q |P - Q|^2 / (p + q)),
    K_ik = exp(-(e_i e_k / p) |C_i - C_k|^2).  exps [N], centers [N, 3]."""
    e = np.asarray(exps, dtype=np.float64)
    C = np.asarray(centers, dtype=np.float64)
    q = np.asarray(quads, dtype=np.int64).reshape(-1, 4)
    i, j, k, l = q.T
    nrm = (2 * e / math.pi) ** 0.75
    p = e[i] + e[k]
    qq = e[j] + e[l]
    P = (e[i, None] * C[i] + e[k, None] * C[k]) / p[:, None]
    Q = (e[j, None] * C[j] + e[l, None] * C[l]) / qq[:, None]
    Kik = np.exp(-(e[i] * e[k] / p) * ((C[i] - C[k]) ** 2).sum(1))
    Kjl = np.exp(-(e[j] * e[l] / qq) * ((C[j] - C[l]) ** 2).sum(1))
    T = p * qq / (p + qq) * ((P - Q) ** 2).sum(1)
    return nrm[i] * nrm[j] * nrm[k] * nrm[l] * Kik * Kjl * 2 * math.pi ** 2.5 / \
        (p * qq * np.sqrt(p + qq)) * boys0(T)
