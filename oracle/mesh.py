"""Quadrature meshes on the Laplace variable (oracle side).

Variable.  Eqs. 5-8 integrate over alpha with the kernel exp(-alpha p^2).  The
oracle works with the dimensionless beta = 4 alpha / L^2, so that each 1-D
factor becomes a function of beta alone (see tables.py).  The split point
alpha_c of Eq. 7 becomes beta_c = 4 alpha_c / L^2; the default beta_c = 1 is
the reading of the paper's "alpha_c = 1" that reproduces Table I.

Interval 1, [0, beta_c]: Gauss-Legendre in beta (Eq. 12, first sum).

Tail, [beta_c, inf): the substitution t = beta^{-1/2} of Eq. 11 maps it onto
t in (0, beta_c^{-1/2}], where the integrand is a polynomial-like function of
t (Eq. 10 power series).  Gauss-Legendre in t; each node goes back to
beta = 1/t^2 with weight 2 w / t^3 from d beta = -2 t^{-3} dt (the
back-transformation of Eq. 13, whose printed weight is garbled).

Mesh 1 (Sec. III, Table I left): Q points on interval 1 and Q on the tail.
Mesh 2 (Sec. III, Table I right): interval 1 cut at beta_c * 5^{-7}, ...,
beta_c * 5^{-1}, q points on each of the 8 pieces, plus q_tail tail points
(the tail count is not printed; 8 is the default).

Mesh 3 (not in the paper's tables; built on its suggestions in Sec. II after
Eq. 14 that the nodes can be cut by matching the rule to the integrand's
functional form and that a rule made for polynomials in x^2 is twice as
efficient): interval 1 is cut into the same geometric pieces, but each piece
is integrated by Gauss-Legendre in s = beta^{1/2}, beta = s^2 with weight
2 s w (near beta = 0 the integrand is a power series in beta^{1/2}: each
factor tends to sqrt(pi) - sqrt(beta) + ..., so in s it is polynomial-like);
the tail uses the q_tail-point rule in t exact for polynomials in t^2 (the
tail integrand of Eq. 11 is a series in t^2), i.e. the q_tail positive nodes
of the 2 q_tail-point Gauss-Legendre rule on [-t_c, t_c].

Gauss-Legendre rules are the roots of P_q and the weights 2/((1-x^2) P_q'^2),
evaluated in 34-digit arithmetic (mpmath; numpy's eigenvalue nodes serve only
as starting points of the Newton polish) and rounded to FP64 once, after the
map to the interval -- and for the tail after beta = 1/t^2 and W = 2 w / t^3.
numpy's own weights are not used: at q >= 90 they carry relative errors up to
1e-11, above the 1e-12 parity bar.
"""
import functools

import mpmath as mp
import numpy as np

_DPS = 34


@functools.lru_cache(maxsize=None)
def _gl_unit(q: int):
    """Nodes and weights on [-1, 1] as 34-digit mpf tuples, ascending."""
    with mp.workdps(_DPS):
        xs, ws = [], []
        for g in np.polynomial.legendre.leggauss(q)[0]:
            z = mp.mpf(float(g))
            for _ in range(5):
                p, pm = mp.legendre(q, z), mp.legendre(q - 1, z)
                dp = q * (z * p - pm) / (z * z - 1)     # (z^2 - 1) P' = q (z P_q - P_{q-1})
                z -= p / dp
            p, pm = mp.legendre(q, z), mp.legendre(q - 1, z)
            dp = q * (z * p - pm) / (z * z - 1)
            xs.append(z)
            ws.append(2 / ((1 - z * z) * dp * dp))
        return tuple(xs), tuple(ws)


def _gl_mp(q: int, a, b):
    xs, ws = _gl_unit(q)
    with mp.workdps(_DPS):
        a, b = mp.mpf(a), mp.mpf(b)
        half, mid = (b - a) / 2, (b + a) / 2
        return [mid + half * x for x in xs], [half * w for w in ws]


def gauss_legendre(q: int, a: float, b: float):
    """q-point Gauss-Legendre nodes and weights on [a, b] (FP64, correctly rounded)."""
    if q < 1:
        raise ValueError("q must be >= 1")
    x, w = _gl_mp(q, a, b)
    return np.array([float(v) for v in x]), np.array([float(v) for v in w])


def _tail(q_tail: int, beta_c: float):
    """Tail nodes: GL in t on (0, beta_c^{-1/2}], beta = 1/t^2, W = 2 w / t^3."""
    with mp.workdps(_DPS):
        t, w = _gl_mp(q_tail, 0, 1 / mp.sqrt(mp.mpf(beta_c)))
        beta = [1 / (x * x) for x in t]
        W = [2 * y / (x * x * x) for x, y in zip(t, w)]
    return np.array([float(v) for v in beta]), np.array([float(v) for v in W])


def mesh1(q: int, beta_c: float = 1.0):
    """Mesh 1: q GL points on [0, beta_c] and q on the t-mapped tail (2q nodes).

    Returns (beta, W, n_interval1): node positions, weights, and how many of
    the leading nodes belong to interval 1.
    """
    b1, w1 = gauss_legendre(q, 0.0, beta_c)
    b2, w2 = _tail(q, beta_c)
    return np.concatenate([b1, b2]), np.concatenate([w1, w2]), q


def mesh2(q_sub: int, q_tail: int = 8, n_sub: int = 8, ratio: float = 5.0,
          beta_c: float = 1.0):
    """Mesh 2: n_sub geometric pieces of [0, beta_c] times q_sub points, plus tail.

    Piece edges are 0, beta_c * ratio^{-(n_sub-1)}, ..., beta_c * ratio^{-1},
    beta_c (for the paper's 8 pieces and ratio 5: [0,5^-7], [5^-7,5^-6], ...,
    [5^-1, 1]).  Returns (beta, W, n_interval1).
    """
    edges = [0.0] + [beta_c * ratio ** (-(n_sub - 1 - k)) for k in range(n_sub)]
    bs, ws = [], []
    for k in range(n_sub):
        b, w = gauss_legendre(q_sub, edges[k], edges[k + 1])
        bs.append(b)
        ws.append(w)
    b2, w2 = _tail(q_tail, beta_c)
    bs.append(b2)
    ws.append(w2)
    return np.concatenate(bs), np.concatenate(ws), n_sub * q_sub


def default_mesh(n_nodes: int, beta_c: float = 1.0):
    """The default mapping of a node count Q to Mesh 2: Q = 8 q + 8.

    8 geometric pieces with q = (Q - 8)/8 points each and an 8-point tail.
    """
    if n_nodes < 16 or n_nodes % 8:
        raise ValueError("default mesh needs Q >= 16 and Q % 8 == 0")
    return mesh2((n_nodes - 8) // 8, 8, 8, 5.0, beta_c)


def _tail_even(q_tail: int, beta_c: float):
    """Tail nodes of the rule in t exact for polynomials in t^2, degree
    <= 4 q_tail - 2, on (0, beta_c^{-1/2}]: an even integrand's integral over
    [-t_c, t_c] is twice that over [0, t_c], and the 2 q_tail-point
    Gauss-Legendre rule on [-t_c, t_c] is symmetric, so its q_tail positive
    nodes with their weights integrate [0, t_c].  Then beta = 1/t^2,
    W = 2 w / t^3 as for the plain tail."""
    with mp.workdps(_DPS):
        xs, ws = _gl_unit(2 * q_tail)
        tc = 1 / mp.sqrt(mp.mpf(beta_c))
        pos = [(x, w) for x, w in zip(xs, ws) if x > 0]
        t = [tc * x for x, _ in pos]
        w = [tc * y for _, y in pos]
        beta = [1 / (x * x) for x in t]
        W = [2 * y / (x * x * x) for x, y in zip(t, w)]
    return np.array([float(v) for v in beta]), np.array([float(v) for v in W])


def mesh3(q_sub: int, q_tail: int = 4, n_sub: int = 4, ratio: float = 7.0,
          beta_c: float = 1.0):
    """Mesh 3: the geometric pieces of Mesh 2 (edges 0, beta_c ratio^{-(n_sub-1)},
    ..., beta_c), each with q_sub Gauss-Legendre points in s = sqrt(beta)
    (node beta = s^2, weight 2 s w), plus q_tail tail points of the rule exact
    for polynomials in t^2 (see the module docstring).
    Returns (beta, W, n_interval1)."""
    edges = [0.0] + [beta_c * ratio ** (-(n_sub - 1 - k)) for k in range(n_sub)]
    bs, ws = [], []
    with mp.workdps(_DPS):
        for k in range(n_sub):
            s, w = _gl_mp(q_sub, mp.sqrt(mp.mpf(edges[k])), mp.sqrt(mp.mpf(edges[k + 1])))
            bs.append(np.array([float(x * x) for x in s]))
            ws.append(np.array([float(2 * x * y) for x, y in zip(s, w)]))
    b2, w2 = _tail_even(q_tail, beta_c)
    bs.append(b2)
    ws.append(w2)
    return np.concatenate(bs), np.concatenate(ws), n_sub * q_sub
