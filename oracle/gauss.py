"""Separable Gaussian basis (oracle side).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Sec. II builds three-dimensional basis functions as products of one-dimensional
ones, g_I(r) = f_l(x) f_m(y) f_n(z), and names products of one-dimensional
Gaussians as the second common case beside planewaves; it works the formulas
out for planewaves only.  This module writes them out for s-type Gaussians.

One-dimensional set: f_u(x) = (2 a_u / pi)^{1/4} exp(-a_u (x - A_u)^2),
u = 0 .. n1-1 (unit norm), the same set along x, y and z.  The basis is every
product: g_I = f_l(x) f_m(y) f_n(z) with I = (l n1 + m) n1 + n, N = n1^3.

Integral (physicist's pairing as for planewaves; the functions are real):
  <ij|kl> = Int Int g_i(r) g_k(r) g_j(r') g_l(r') / |r - r'| d^3r d^3r'.

Pair products (Gaussian product theorem): f_u f_v = c_uv exp(-p (x - P)^2) with
p = a_u + a_v, P = (a_u A_u + a_v A_v) / p and
c_uv = (2 a_u / pi)^{1/4} (2 a_v / pi)^{1/4} exp(-(a_u a_v / p)(A_u - A_v)^2).

Table entry.  Writing 1/r = pi^{-1/2} Int_0^inf s^{-1/2} exp(-s r^2) ds (the
Gaussian form of the Laplace transform of Eqs. 5-6) and s = 1/(beta L^2) for a
reference length L, each direction contributes
  G(s) = Int Int f_u f_v(x) exp(-s (x - x')^2) f_u' f_v'(x') dx dx'
       = c c' pi / sqrt(p q + (p + q) s) exp(-p q s D^2 / (p q + (p + q) s)),
q, c', Q the parameters of the (u', v') product, D = P - Q, and with
tau(beta) = beta^{-1/2} G(1/(beta L^2)):
  tau(beta; (u,v), (u',v')) = c c' pi / sqrt(p q beta + (p + q)/L^2)
                              * exp(-p q D^2 / (p q beta L^2 + p + q)),
  <ij|kl> = (1/(sqrt(pi) L)) Int_0^inf d beta  prod_d tau_d(beta),
the same form as the planewave case (Eq. 14 after quadrature), here with
tau finite at beta = 0 and ~ beta^{-1/2} as beta -> inf.

Screening.  Sec. II counts eta N^{1/3} one-dimensional products because the
product of two well separated Gaussians vanishes; here a pair (u, v) is kept
when exp(-(a_u a_v / p)(A_u - A_v)^2) >= eps, and an integral that needs a
dropped pair in any direction is zero.  Kept pairs u <= v are numbered in
order of u, then v: n_pairs of them, the band of the title.

Pins (tests/test_oracle_pins.py): G(s) against brute-force 2-D quadrature of
its definition, and the reconstructed integrals of isotropic functions
(equal exponents along x, y, z) against the textbook closed form through the
Boys function F0 (tests/_brute.py), which uses neither the tables nor the
Laplace transform.
"""
import math

import numpy as np


def gauss_pairs(a, A, eps=1e-15):
    """Kept one-dimensional pairs: (pairs [P1, 2] with u <= v, pair_map
    [n1, n1] with the pair index of (u, v) and (v, u), or -1 if dropped)."""
    a = np.asarray(a, dtype=np.float64)
    A = np.asarray(A, dtype=np.float64)
    n1 = len(a)
    pmap = -np.ones((n1, n1), dtype=np.int64)
    pairs = []
    for u in range(n1):
        for v in range(u, n1):
            p = a[u] + a[v]
            if math.exp(-(a[u] * a[v] / p) * (A[u] - A[v]) ** 2) >= eps:
                pmap[u, v] = pmap[v, u] = len(pairs)
                pairs.append((u, v))
    return np.array(pairs, dtype=np.int64).reshape(-1, 2), pmap


def pair_params(a, A, pairs):
    """(c, p, P) of each kept pair's product Gaussian."""
    a = np.asarray(a, dtype=np.float64)
    A = np.asarray(A, dtype=np.float64)
    u, v = pairs[:, 0], pairs[:, 1]
    p = a[u] + a[v]
    P = (a[u] * A[u] + a[v] * A[v]) / p
    c = (2 * a[u] / math.pi) ** 0.25 * (2 * a[v] / math.pi) ** 0.25 * \
        np.exp(-(a[u] * a[v] / p) * (A[u] - A[v]) ** 2)
    return c, p, P


def gauss_G(s, cp, p, P, cq, q, Q):
    """G(s) of the module docstring for one pair of products (closed form)."""
    den = p * q + (p + q) * s
    return cp * cq * math.pi / math.sqrt(den) * math.exp(-p * q * s * (P - Q) ** 2 / den)


def gauss_tau(beta, a, A, pairs, L=1.0):
    """tau_q(pair, pair') for every node and kept pair: float64 [Q, P1, P1]."""
    beta = np.atleast_1d(np.asarray(beta, dtype=np.float64))
    c, p, P = pair_params(a, A, pairs)
    n = len(pairs)
    out = np.empty((beta.size, n, n))
    # every (x, y) entry by the formula, elementwise over the pair grid
    pq = p[:, None] * p[None, :]
    ps = p[:, None] + p[None, :]
    cc = c[:, None] * c[None, :]
    d2 = (P[:, None] - P[None, :]) ** 2
    for iq, b in enumerate(beta):
        den = pq * b + ps / (L * L)
        out[iq] = cc * math.pi / np.sqrt(den) * np.exp(-pq * d2 / (pq * b * L * L + ps))
    return out


def gauss_decode(quads, n1):
    """1-D indices (l_x, l_y, l_z) of each of the four functions: [n, 4, 3]."""
    q = np.asarray(quads, dtype=np.int64).reshape(-1, 4)
    if q.size and (q.min() < 0 or q.max() >= n1 ** 3):
        raise IndexError("quadruple index out of range")
    return np.stack([q // (n1 * n1), (q // n1) % n1, q % n1], axis=-1)


def gauss_reconstruct(tau, W, pmap, n1, quads, L=1.0):
    """<ij|kl> for each row (i, j, k, l) by the node sum of Eq. 14 over the
    three direction factors; zero where a pair is dropped in any direction."""
    W = np.asarray(W, dtype=np.float64)
    l = gauss_decode(quads, n1)
    n = l.shape[0]
    prod = np.broadcast_to(W[:, None], (len(W), n)).copy()
    keep = np.ones(n, dtype=bool)
    for d in range(3):
        pr = pmap[l[:, 0, d], l[:, 2, d]]      # (i, k) at r
        pc = pmap[l[:, 1, d], l[:, 3, d]]      # (j, l) at r'
        keep &= (pr >= 0) & (pc >= 0)
        prod *= tau[:, np.maximum(pr, 0), np.maximum(pc, 0)]
    out = prod.sum(axis=0) / (math.sqrt(math.pi) * L)
    out[~keep] = 0.0
    return out
