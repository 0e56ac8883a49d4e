"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: values the
paper prints (Table I, the shell closings), closed forms (the unit-cube
Coulomb constant, tau(beta; 0, 0)), brute-force integration of the defining
integrals (tests/_brute.py), high-precision arithmetic (mpmath), exactness
properties of Gauss quadrature, and invariants of the Coulomb integrals.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import workloads
from tests import _brute

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as fh:
        return json.load(fh)


# ---------------------------------------------------------------- basis ----

def test_shell_closings_match_paper():
    g = _gold("shell_closings.json")
    counts = oracle.shell_counts(169)
    assert [int(counts[r2]) for r2 in g["R2"]] == g["M"]


def test_basis_sizes_and_order():
    # independent count: per x, count (y, z) in the disk y^2 + z^2 <= r2 - x^2
    def count(r2):
        r = math.isqrt(r2)
        return sum(1 for x in range(-r, r + 1) for y in range(-r, r + 1)
                   for z in range(-r, r + 1) if x * x + y * y + z * z <= r2)
    for r2, n in [(2, 19), (9, 123), (40, 1045), (169, 9171)]:
        assert count(r2) == n
        assert len(oracle.enumerate_basis(r2)) == n
    b = oracle.enumerate_basis(40)
    n2 = (b * b).sum(1)
    assert np.all(np.diff(n2) >= 0)
    assert len({tuple(v) for v in b}) == len(b)
    assert tuple(b[0]) == (0, 0, 0)
    # occupied sphere is an index prefix
    assert np.array_equal(oracle.enumerate_basis(9), b[:123])


# ----------------------------------------------------------------- mesh ----

@pytest.mark.parametrize("degree", [2, 3, 4, 5, 6])
def test_gauss_legendre_against_mpmath_quadrature_class_and_exactness(degree):
    """mpmath's own Gauss-Legendre rule (3 * 2^(degree-1) points, computed by
    its quadrature module) against the oracle's, and polynomial exactness."""
    import mpmath as mp
    from mpmath.calculus.quadrature import GaussLegendre
    with mp.workdps(34):
        ref = sorted(GaussLegendre(mp.mp).calc_nodes(degree, mp.mp.prec), key=lambda t: t[0])
    xr = np.array([float(a) for a, _ in ref])
    wr = np.array([float(b) for _, b in ref])
    q = len(ref)
    x, w = oracle.gauss_legendre(q, -1.0, 1.0)
    assert np.max(np.abs(x - xr)) <= 2.3e-16
    assert np.max(np.abs(w - wr) / wr) <= 4.5e-16
    a, b = 0.3, 2.7
    x, w = oracle.gauss_legendre(q, a, b)
    for k in range(min(2 * q, 60)):
        exact = (b ** (k + 1) - a ** (k + 1)) / (k + 1)
        # rounding of x**k grows like k ulps
        tol = (1e-15 + 4e-16 * k) * (w * np.abs(x) ** k).sum()
        assert abs((w * x ** k).sum() - exact) <= tol


def test_gauss_legendre_high_order_tail_nodes_are_correctly_rounded():
    """Mesh 1 of Table I reaches 180 points; its smallest tail nodes t ~ 1e-4
    must be exact to rounding (W = 2 w / t^3 amplifies their error)."""
    beta, W, n1 = oracle.mesh1(180)
    tb, tw = beta[n1:], W[n1:]
    # exactness of the tail rule on t^(2n) <-> beta^(-(n + 3/2)) for high n
    for n in (0, 5, 40, 100, 179):
        exact = 1.0 / (n + 0.5)
        assert abs((tw * tb ** (-(n + 1.5))).sum() - exact) < 1e-14 * exact


@pytest.mark.parametrize("beta_c", [1.0, 0.37, 2.5])
def test_mesh2_interval_and_tail_exactness(beta_c):
    q, qt = 6, 8
    beta, W, n1 = oracle.mesh2(q, qt, beta_c=beta_c)
    assert len(beta) == 8 * q + qt and n1 == 8 * q
    b1, w1 = beta[:n1], W[:n1]
    assert np.all((b1 > 0) & (b1 < beta_c))
    # geometric pieces: each piece integrates polynomials of degree <= 2q-1
    assert abs(w1.sum() - beta_c) < 1e-15
    for k in range(1, 2 * q):
        exact = beta_c ** (k + 1) / (k + 1)
        assert abs((w1 * b1 ** k).sum() - exact) < 1e-14 * max(1.0, exact)
    # tail: Int_{beta_c}^inf beta^{-(n + 3/2)} d beta = beta_c^{-(n+1/2)} / (n + 1/2)
    b2, w2 = beta[n1:], W[n1:]
    assert np.all(b2 > beta_c)
    for n in range(qt):
        exact = beta_c ** (-(n + 0.5)) / (n + 0.5)
        assert abs((w2 * b2 ** (-(n + 1.5))).sum() - exact) < 1e-13 * exact


def test_mesh1_and_default_mesh_shapes():
    beta, W, n1 = oracle.mesh1(90)
    assert len(beta) == 180 and n1 == 90
    beta, W, n1 = oracle.default_mesh(96)
    assert len(beta) == 96 and n1 == 88
    with pytest.raises(ValueError):
        oracle.default_mesh(50)


@pytest.mark.parametrize("beta_c", [1.0, 0.37, 2.5])
def test_mesh3_piece_and_tail_exactness(beta_c):
    """Mesh 3: each geometric piece integrates beta^(k/2) exactly for
    k <= 2q - 2 (Gauss-Legendre in s = sqrt(beta): s^k * 2 s is a polynomial
    of degree <= 2q - 1); the tail rule integrates t^(2n), i.e.
    beta^-(n + 3/2), exactly for n <= 2 q_tail - 1 -- twice the range of the
    plain Gauss-Legendre tail with as many points, which fails at n = q_tail."""
    q, qt = 6, 4
    beta, W, n1 = oracle.mesh3(q, qt, n_sub=5, ratio=6.0, beta_c=beta_c)
    assert len(beta) == 5 * q + qt and n1 == 5 * q
    b1, w1 = beta[:n1], W[:n1]
    assert np.all((b1 > 0) & (b1 < beta_c)) and np.all(np.diff(b1) > 0)
    for k in range(2 * q - 1):
        exact = beta_c ** (k / 2 + 1) / (k / 2 + 1)
        assert abs((w1 * b1 ** (k / 2)).sum() - exact) < 1e-14 * max(1.0, exact), k
    b2, w2 = beta[n1:], W[n1:]
    assert np.all(b2 > beta_c)
    tail = lambda bb, ww, n: (ww * bb ** (-(n + 1.5))).sum()
    for n in range(2 * qt):
        exact = beta_c ** (-(n + 0.5)) / (n + 0.5)
        assert abs(tail(b2, w2, n) - exact) < 1e-13 * exact, n
    n = 2 * qt
    exact = beta_c ** (-(n + 0.5)) / (n + 0.5)
    assert abs(tail(b2, w2, n) - exact) > 1e-9 * exact
    bg, wg, n1g = oracle.mesh2(q, qt, beta_c=beta_c)
    exact = beta_c ** (-(qt + 0.5)) / (qt + 0.5)
    assert abs(tail(bg[n1g:], wg[n1g:], qt) - exact) > 1e-6 * exact


@pytest.mark.parametrize("q", [1, 2, 4, 7, 12])
def test_tail_rule_in_t_squared_is_gauss_jacobi(q):
    """With x = t^2 the even rule on [0, 1] is the Gauss rule for the weight
    x^(-1/2) on [0, 1], i.e. Gauss-Jacobi (alpha, beta) = (0, -1/2) mapped by
    x = (1 + y)/2: t_k = sqrt((1 + y_k)/2), w_k = (sqrt(2)/4) w_k^J
    (SciPy's roots_jacobi, an independent routine)."""
    from scipy.special import roots_jacobi
    y, wj = roots_jacobi(q, 0.0, -0.5)
    t_ref = np.sqrt((1 + y) / 2)
    w_ref = math.sqrt(2.0) / 4 * wj
    beta, W, n1 = oracle.mesh3(1, q, n_sub=1, ratio=2.0, beta_c=1.0)
    t = beta[n1:] ** -0.5
    w = W[n1:] * t ** 3 / 2
    order = np.argsort(t)
    assert np.max(np.abs(t[order] - np.sort(t_ref))) < 1e-14
    assert np.max(np.abs(w[order] - w_ref[np.argsort(t_ref)]) / w_ref) < 1e-13


def test_mesh3_reaches_the_converged_integrals_with_fewer_nodes():
    """Mesh 3 with 36 nodes (4 pieces of 8, ratio 7, 4 tail points) against
    the converged Mesh 2 (8 x 21 + 8 = 176 nodes) on the 9171-planewave basis:
    within 1e-9 on random quadruples, and <00|00> within 1e-9 of the
    unit-cube closed form (3e-10 measured); Mesh 2 with 88 nodes is further
    off."""
    b = oracle.enumerate_basis(169)
    quads = workloads.lookup_stream(len(b), 925, 3000, seed=17)
    quads[0] = 0
    bref, wref, _ = oracle.mesh2(21, 8)
    ref = oracle.reconstruct(oracle.tau_table(bref, 26), wref, b, quads)
    beta, W, _ = oracle.mesh3(8, 4, n_sub=4, ratio=7.0)
    got = oracle.reconstruct(oracle.tau_table(beta, 26), W, b, quads)
    assert np.max(np.abs(got - ref)) < 1e-9
    assert abs(got[0] - oracle.k_cube()) < 1e-9
    b2, w2, _ = oracle.default_mesh(88)
    old = oracle.reconstruct(oracle.tau_table(b2, 26), w2, b, quads)
    assert np.max(np.abs(old - ref)) > np.max(np.abs(got - ref))


@pytest.mark.slow
def test_mesh3_reproduces_table_one_converged_ratio():
    """Sec. III, Table I: the converged E_x/E_KS = 0.965431 at M = 9171
    (Mesh 2, 8 x 10 and 8 x 15 points) within the printed precision, from
    Mesh 3 with 36 and 44 nodes."""
    g = _gold("table1.json")
    b = oracle.enumerate_basis(g["n2occ"])
    h, R = oracle.diff_histogram(b)
    eks = oracle.e_ks(g["M"])
    conv = g["mesh2"]["10"][1]
    for q in (8, 10):
        beta, W, _ = oracle.mesh3(q, 4, n_sub=4, ratio=7.0)
        ex = oracle.exchange_from_histogram(h, R, oracle.tau_diag(beta, 2 * R), W)
        assert abs(ex / eks - conv) < 1.5e-6, (q, ex / eks)


# --------------------------------------------------------------- tables ----

def test_tau00_closed_form():
    beta = np.array([1e-8, 6e-7, 1e-4, 0.03, 1.0, 7.5, 3e3, 4e7])
    t = oracle.tau_table(beta, 0)[:, 0, 0]
    ref = oracle.tau00_closed_form(beta)
    assert np.max(np.abs(t - ref) / ref) < 1e-15


@pytest.mark.parametrize("beta", [0.08, 0.5, 1.2, 10.0, 300.0])
def test_tau_against_bruteforce_double_integral(beta):
    K = 4
    tab = oracle.tau_table([beta], K)[0]
    scale = np.abs(tab).max()
    for m in range(-3, 4):
        for mp in range(-3, 4):
            ref = _brute.tau2d(beta, m, mp)
            assert abs(ref.imag) < 1e-15 * scale
            assert abs(tab[m + K, mp + K] - ref.real) < 2e-15 * scale, (m, mp)


def test_tau_against_mpmath_small_and_large_beta():
    import mpmath as mp
    mp.mp.dps = 40

    def mp_tau(beta, m, mp_):
        beta = mp.mpf(beta)
        b = min(mp.mpf(1), 30 * mp.sqrt(beta))
        pts = mp.linspace(0, b, 4 * (abs(m) + abs(mp_)) + 4)
        s = m + mp_
        if s == 0:
            d = mp.quad(lambda u: (1 - u) * mp.exp(-u * u / beta) * mp.cos(2 * mp.pi * m * u), pts)
            return 2 * d / mp.sqrt(beta)
        S = lambda k: mp.quad(lambda u: mp.exp(-u * u / beta) * mp.sin(2 * mp.pi * k * u), pts)
        return -(S(m) + S(mp_)) / (mp.pi * s * mp.sqrt(beta))

    K = 26
    for beta in (2e-7, 1e-3, 1e4):
        tab = oracle.tau_table([beta], K)[0]
        scale = np.abs(tab).max()
        for m, mp_ in [(0, 0), (13, -13), (26, -26), (1, 2), (-7, 20), (25, 26), (-26, 3)]:
            ref = float(mp_tau(beta, m, mp_))
            assert abs(tab[m + K, mp_ + K] - ref) < 1e-15 * scale, (beta, m, mp_)


def test_tau_limits():
    K = 3
    small = oracle.tau_table([1e-9], K)[0]
    for m in range(-K, K + 1):
        assert abs(small[m + K, -m + K] - math.sqrt(math.pi)) < 1e-3
    off = small.copy()
    for m in range(-K, K + 1):
        off[m + K, -m + K] = 0.0
    assert np.abs(off).max() < 1e-3
    big = 1e8
    large = oracle.tau_table([big], K)[0] * math.sqrt(big)
    assert abs(large[K, K] - 1.0) < 1e-8
    large[K, K] = 0.0
    assert np.abs(large).max() < 1e-8


def test_tau_symmetries():
    K = 6
    tab = oracle.tau_table([0.02, 1.0, 50.0], K)
    assert np.allclose(tab, tab.transpose(0, 2, 1), rtol=0, atol=1e-16)
    assert np.allclose(tab, tab[:, ::-1, ::-1], rtol=0, atol=1e-16)
    # but not under (m, m') -> (-m, m')
    assert np.abs(tab - tab[:, ::-1, :]).max() > 1e-3


# --------------------------------------------------------- integrals --------

@pytest.fixture(scope="module")
def fine():
    """Basis |n|^2 <= 2 (19 PW) with a fine Mesh 2 (8 x 14 + 16 nodes)."""
    b = oracle.enumerate_basis(2)
    beta, W, _ = oracle.mesh2(14, 16)
    tau = oracle.tau_table(beta, 2)
    return b, beta, W, tau


def test_unit_cube_coulomb_constant(fine):
    b, beta, W, tau = fine
    c = oracle.reconstruct(tau, W, b, np.array([[0, 0, 0, 0], [3, 5, 3, 5]]))
    assert abs(c[0] - oracle.k_cube()) < 2e-11 * oracle.k_cube()
    assert c[0] == c[1]
    # 1/L scaling with the beta-mesh (tables do not depend on L)
    c2 = oracle.reconstruct(tau, W, b, np.array([[0, 0, 0, 0]]), L=2.5)
    assert abs(c2[0] * 2.5 - c[0]) < 1e-15 * c[0]


@pytest.mark.slow
def test_integrals_against_bruteforce_6d(fine):
    b, beta, W, tau = fine
    quads = [(0, 0, 0, 0), (1, 2, 3, 4), (5, 1, 0, 7), (3, 3, 12, 18), (0, 6, 1, 2),
             (7, 9, 11, 13), (18, 2, 4, 16)]
    got = oracle.reconstruct(tau, W, b, np.array(quads))
    for q, c in zip(quads, got):
        ref = _brute.coulomb6d(*[b[x] for x in q], n=40)
        assert abs(ref.imag) < 1e-14
        assert abs(c - ref.real) < 1e-10 * max(abs(ref.real), 1e-3), (q, c, ref)


def test_split_point_independence():
    """The exact integral does not depend on where the Laplace range is split."""
    b = oracle.enumerate_basis(2)
    quads = np.array([[0, 0, 0, 0], [1, 2, 3, 4], [5, 1, 0, 7]])
    vals = []
    for bc in (0.5, 1.0, 2.0):
        beta, W, _ = oracle.mesh2(14, 16, beta_c=bc)
        vals.append(oracle.reconstruct(oracle.tau_table(beta, 2), W, b, quads))
    vals = np.array(vals)
    assert np.max(np.abs(vals - vals[1])) < 1e-10


def test_convergence_in_node_count():
    b = oracle.enumerate_basis(2)
    quads = np.array([[0, 0, 0, 0], [1, 2, 3, 4], [5, 1, 0, 7], [7, 9, 11, 13]])
    beta, W, _ = oracle.default_mesh(176)
    ref = oracle.reconstruct(oracle.tau_table(beta, 2), W, b, quads)
    errs = []
    for Q in (32, 48, 64, 96, 128):
        beta, W, _ = oracle.default_mesh(Q)
        errs.append(np.abs(oracle.reconstruct(oracle.tau_table(beta, 2), W, b, quads) - ref).max())
    assert all(errs[k + 1] < errs[k] for k in range(len(errs) - 1)), errs
    assert errs[-1] < 1e-10


def test_integral_symmetries_and_schwarz():
    b = oracle.enumerate_basis(9)
    N = len(b)
    beta, W, _ = oracle.default_mesh(48)
    tau = oracle.tau_table(beta, 6)
    qs = workloads.uniform_quads(N, 400, seed=11)
    i, j, k, l = qs.T
    f = lambda a, b_, c, d: oracle.reconstruct(tau, W, b, np.stack([a, b_, c, d], 1))
    v = f(i, j, k, l)
    assert np.array_equal(v, f(j, i, l, k))
    assert np.array_equal(v, f(k, l, i, j))
    assert np.array_equal(v, f(l, k, j, i))
    # i <-> k alone is not a symmetry
    assert np.abs(v - f(k, j, i, l)).max() > 1e-4
    # Schwarz: |<ij|kl>| <= sqrt(<ik|ki> <lj|jl>), exchange integrals positive
    a, c = f(i, k, k, i), f(l, j, j, l)
    assert np.all(a > 0) and np.all(c > 0)
    assert np.all(np.abs(v) <= np.sqrt(a * c) * (1 + 1e-14))
    # axis permutation and axis reflection of all four wavevectors
    index = {tuple(x): n for n, x in enumerate(b)}
    for tr in (lambda x: x[[1, 2, 0]], lambda x: x * np.array([1, -1, 1])):
        mapped = np.array([[index[tuple(tr(b[x]))] for x in row] for row in qs[:100]])
        w2 = oracle.reconstruct(tau, W, b, mapped)
        assert np.max(np.abs(w2 - v[:100])) < 1e-15 * np.abs(v).max()


def test_out_of_range_index_raises():
    b = oracle.enumerate_basis(2)
    beta, W, _ = oracle.default_mesh(16)
    tau = oracle.tau_table(beta, 2)
    with pytest.raises(IndexError):
        oracle.reconstruct(tau, W, b, np.array([[0, 0, 0, 19]]))


# -------------------------------------------------------------- energies ----

def test_exchange_direct_equals_histogram_and_hartree_closed_form():
    b = oracle.enumerate_basis(9)
    occ = np.arange(123, dtype=np.int32)
    beta, W, _ = oracle.default_mesh(48)
    K = 6
    tau = oracle.tau_table(beta, K)
    diag = oracle.tau_diag(beta, K)
    assert np.array_equal(diag, np.array([[tau[q, m + K, -m + K] for m in range(-K, K + 1)]
                                           for q in range(len(beta))]))
    for f in (None, workloads.occupations(123, seed=3)):
        eh, ex = oracle.energies(tau, W, b, occ, f)
        h, R = oracle.diff_histogram(b[occ], f)
        ex2 = oracle.exchange_from_histogram(h, R, diag, W)
        assert abs(ex - ex2) < 1e-13 * abs(ex)
        fs = 123.0 if f is None else f.sum()
        c0 = oracle.reconstruct(tau, W, b, np.array([[0, 0, 0, 0]]))[0]
        assert abs(eh - 0.5 * fs * fs * c0) < 1e-13 * eh
        assert ex < 0 and eh > 0
    # dropping the i = j terms changes the energy visibly (they are included)
    eh, ex = oracle.energies(tau, W, b, occ)
    c0 = oracle.reconstruct(tau, W, b, np.array([[0, 0, 0, 0]]))[0]
    assert abs((ex + 0.5 * 123 * c0) - ex) / abs(ex) > 0.02


@pytest.mark.slow
def test_table_one_reproduced():
    """Sec. III, Table I: E_x / E_KS at M = 9171 for Mesh 1 and Mesh 2."""
    g = _gold("table1.json")
    b = oracle.enumerate_basis(g["n2occ"])
    assert len(b) == g["M"]
    h, R = oracle.diff_histogram(b)
    eks = oracle.e_ks(g["M"])
    tol = 1.5e-6
    for q, (i1, tot) in g["mesh2"].items():
        beta, W, n1 = oracle.mesh2(int(q), 8)
        c = oracle.exchange_from_histogram(h, R, oracle.tau_diag(beta, 2 * R), W, per_node=True)
        assert abs(c[:n1].sum() / eks - i1) < tol and abs(c.sum() / eks - tot) < tol
    for Q, (i1, tot) in g["mesh1"].items():
        beta, W, n1 = oracle.mesh1(int(Q))
        c = oracle.exchange_from_histogram(h, R, oracle.tau_diag(beta, 2 * R), W, per_node=True)
        assert abs(c[:n1].sum() / eks - i1) < tol and abs(c.sum() / eks - tot) < tol


@pytest.mark.slow
def test_exchange_ratio_tends_to_one_with_shell_size():
    """Fig. 1 / Sec. III: E_x/E_KS rises with M and extrapolates linearly toward 1."""
    g = _gold("shell_closings.json")
    b = oracle.enumerate_basis(169)
    beta, W, _ = oracle.mesh2(10, 8)
    diag = oracle.tau_diag(beta, 26)
    ratios = []
    for M in g["M"]:
        h, R = oracle.diff_histogram(b[:M])
        ratios.append(oracle.exchange_from_histogram(h, R, diag, W) / oracle.e_ks(M))
    ratios = np.array(ratios)
    assert np.all(np.diff(ratios) > 0)
    x = np.array(g["M"], dtype=float) ** (-1.0 / 3.0)
    slope, icpt = np.polyfit(x[-5:], ratios[-5:], 1)
    assert 0.99 < icpt < 1.0 and slope < 0


# ------------------------------------------------------ rectangular boxes ----
# Each direction of a box with sides (Lx, Ly, Lz) uses the cube's table
# function at the node scaled by (L_d / L0)^-2, L0 = (Lx Ly Lz)^(1/3).

BOXES = [(1.0, 1.3, 0.8), (2.0, 1.0, 0.5)]


@pytest.mark.parametrize("sides", BOXES)
def test_box_integrals_against_bruteforce_6d(sides):
    b = oracle.enumerate_basis(2)
    beta, W, _ = oracle.mesh2(21, 24)     # aspect ratios up to 4 need a finer mesh
    L0, rho, taus = oracle.box_tables(beta, 2, sides)
    assert abs(np.prod(rho) - 1.0) < 1e-15
    quads = [(0, 0, 0, 0), (1, 2, 3, 4), (5, 1, 0, 7), (3, 3, 12, 18), (7, 9, 11, 13), (18, 2, 4, 16)]
    got = oracle.reconstruct(taus, W, b, np.array(quads), L=L0)
    for q, c in zip(quads, got):
        ref = _brute.coulomb6d(*[b[x] for x in q], L=sides, n=40)
        assert abs(ref.imag) < 1e-14
        assert abs(c - ref.real) < 1e-10 * max(abs(ref.real), 1e-3), (sides, q, c, ref)


def test_box_axis_permutation_and_scaling():
    """Swapping two sides and the same two components of every basis vector
    leaves each integral unchanged; scaling all sides by s divides it by s;
    equal sides give the cube's tables exactly."""
    b = oracle.enumerate_basis(9)
    beta, W, _ = oracle.default_mesh(48)
    quads = workloads.uniform_quads(len(b), 400, seed=21)
    L0, _, t1 = oracle.box_tables(beta, 6, (1.0, 1.4, 0.7))
    v1 = oracle.reconstruct(t1, W, b, quads, L=L0)
    L0s, _, t2 = oracle.box_tables(beta, 6, (1.4, 1.0, 0.7))
    v2 = oracle.reconstruct(t2, W, b[:, [1, 0, 2]], quads, L=L0s)
    scale = np.abs(v1).max()
    assert np.max(np.abs(v1 - v2)) < 1e-15 * scale
    L0d, _, t3 = oracle.box_tables(beta, 6, (2.0, 2.8, 1.4))
    v3 = oracle.reconstruct(t3, W, b, quads, L=L0d)
    assert np.max(np.abs(2.0 * v3 - v1)) < 1e-15 * scale
    _, _, tc = oracle.box_tables(beta, 6, (1.0, 1.0, 1.0))
    assert np.array_equal(tc[0], oracle.tau_table(beta, 6)) and np.array_equal(tc[1], tc[2])
    # Hartree: every <ij|ij> is <00|00>
    occ = np.arange(19)
    eh, ex = oracle.energies(t1, W, b, occ, L=L0)
    c00 = oracle.reconstruct(t1, W, b, np.zeros((1, 4), dtype=np.int32), L=L0)[0]
    assert abs(eh - 0.5 * 19 ** 2 * c00) < 1e-13 * eh and ex < 0


# ------------------------------------------------------ Gaussian basis ----

def _gauss_setup():
    a, A = workloads.gaussian_set(workloads.GAUSS_SMALL)
    pairs, pmap = oracle.gauss_pairs(a, A, 1e-15)
    return a, A, pairs, pmap


def test_gauss_factor_against_bruteforce_2d():
    """The 1-D factor G(s) in closed form (Gaussian product theorem, then
    two Gaussian integrals) against tensor Gauss-Legendre of its defining
    double integral, for pairs at several separations and kernel widths."""
    a, A, pairs, pmap = _gauss_setup()
    c, p, P = oracle.pair_params(a, A, pairs)
    for (u, v, up, vp) in [(0, 0, 0, 0), (0, 3, 5, 6), (1, 2, 9, 11), (4, 4, 10, 7), (2, 8, 3, 3)]:
        x, y = pmap[u, v], pmap[up, vp]
        assert x >= 0 and y >= 0
        for s in (1e-3, 0.05, 0.7, 4.0, 60.0):
            ref = _brute.gauss_G2d(s, a, A, u, v, up, vp, n=320)
            got = oracle.gauss_G(s, c[x], p[x], P[x], c[y], p[y], P[y])
            assert abs(got - ref) <= 2e-12 * abs(ref) + 1e-300, (u, v, up, vp, s, got, ref)


def test_gauss_integrals_against_boys_closed_form():
    """Isotropic s-type Gaussians (one exponent in all three directions): the
    scheme's integrals (pair tables on a 46-node Mesh 3, reference length 8
    bohr, about the extent of the centers) against the closed form through
    the Boys function; the screened integrals are zero and their exact values
    below 1e-16."""
    a, A, pairs, pmap = _gauss_setup()
    n1 = len(a)
    ne = len(workloads.GAUSS_SMALL.exponents)
    iso = np.array([(l * n1 + m) * n1 + n for l in range(n1) for m in range(n1) for n in range(n1)
                    if l % ne == m % ne == n % ne])
    quads = iso[workloads.rng(3).integers(0, len(iso), (3000, 4))]
    lidx = oracle.gauss_decode(quads, n1)
    ex = np.array([_brute.gauss_exact(a[lidx[r, :, 0]], A[lidx[r]], np.array([[0, 1, 2, 3]]))[0]
                   for r in range(len(quads))])
    beta, W, _ = oracle.mesh3(10, 6, n_sub=4, ratio=7.0)
    L = 8.0
    got = oracle.gauss_reconstruct(oracle.gauss_tau(beta, a, A, pairs, L=L), W, pmap, n1, quads, L=L)
    kept = got != 0
    assert kept.sum() > 2000
    assert np.max(np.abs(got - ex)) < 1e-12
    assert np.max(np.abs(got - ex)[kept] / np.abs(ex[kept])) < 1e-9
    assert np.max(np.abs(ex[~kept])) < 1e-16


@pytest.mark.slow
def test_gauss_anisotropic_integrals_by_laplace_quadrature():
    """Functions whose exponents differ between directions (no closed form):
    pi^{-1/2} Int_0^inf s^{-1/2} prod_d G_d(s) ds with each G_d by brute-force
    2-D quadrature and the s-integral by adaptive QUADPACK (the split at
    s = 1 and the map s -> 1/s above it keep both ends finite), against the
    scheme on its mesh."""
    from scipy.integrate import quad
    a, A, pairs, pmap = _gauss_setup()
    n1 = len(a)
    quads = np.array([[(0 * n1 + 3) * n1 + 5, (1 * n1 + 2) * n1 + 4, (2 * n1 + 1) * n1 + 7,
                       (0 * n1 + 0) * n1 + 6],
                      [(5 * n1 + 8) * n1 + 1, (9 * n1 + 9) * n1 + 2, (4 * n1 + 11) * n1 + 0,
                       (6 * n1 + 7) * n1 + 3]])
    lidx = oracle.gauss_decode(quads, n1)
    beta, W, _ = oracle.mesh3(10, 6, n_sub=4, ratio=7.0)
    L = 8.0
    got = oracle.gauss_reconstruct(oracle.gauss_tau(beta, a, A, pairs, L=L), W, pmap, n1, quads, L=L)
    for r in range(len(quads)):
        l = lidx[r]

        def integrand(s):
            g = 1.0
            for d in range(3):
                g *= _brute.gauss_G2d(s, a, A, l[0, d], l[2, d], l[1, d], l[3, d], n=96)
            return g / math.sqrt(s)
        lo = quad(lambda t: integrand(t * t) * 2 * t, 0.0, 1.0, epsabs=1e-15, epsrel=1e-12, limit=200)[0]
        hi = quad(lambda t: integrand(1.0 / t) / (t * t), 1e-12, 1.0, epsabs=1e-15, epsrel=1e-12,
                  limit=200)[0]
        ref = (lo + hi) / math.sqrt(math.pi)
        assert abs(got[r] - ref) < 1e-9 * abs(ref), (r, got[r], ref)


def test_gauss_integral_symmetries():
    """Real functions: <ij|kl> = <kj|il> = <il|kj> = <jk|li>... the eight
    permutations that keep i, k at r and j, l at r' or swap the two sides,
    exactly; the screening is exact in the pair band."""
    a, A, pairs, pmap = _gauss_setup()
    n1 = len(a)
    beta, W, _ = oracle.mesh3(8, 4)
    tau = oracle.gauss_tau(beta, a, A, pairs, L=8.0)
    q = workloads.uniform_quads(n1 ** 3, 2000, seed=4)
    i, j, k, l = q.T
    f = lambda *c: oracle.gauss_reconstruct(tau, W, pmap, n1, np.stack(c, 1), L=8.0)
    v = f(i, j, k, l)
    for perm in ((k, j, i, l), (i, l, k, j), (k, l, i, j), (j, i, l, k), (l, k, j, i)):
        assert np.array_equal(v, f(*perm))
    assert (v == 0).sum() > 0 and (v != 0).sum() > 0
    with pytest.raises(IndexError):
        oracle.gauss_reconstruct(tau, W, pmap, n1, np.array([[0, 0, 0, n1 ** 3]]))
