"""Per-node 1-D Coulomb tables for planewaves (oracle side).

Eq. 8 for one Cartesian direction with box planewaves f_n(x) = L^{-1/2}
exp(2 pi i n x / L): the bra functions are conjugated, i and k share the
coordinate x, j and l share x' (physicist's <ij|kl>), so the x-integrand
carries exp(2 pi i (m x + m' x') / L) with m = k - i and m' = l - j.  Doing the
p_x integral gives the Gaussian kernel of Eq. 9; in reduced coordinates
x = L xi and with beta = 4 alpha / L^2 the 1-D factor times beta^{-1/2} is

    tau(beta; m, m') = beta^{-1/2} Int_0^1 Int_0^1 exp(-(xi - xi')^2 / beta)
                                         exp(2 pi i (m xi + m' xi')) dxi dxi'

and the integral becomes <ij|kl> = (1/(sqrt(pi) L)) Int_0^inf d beta
prod_{x,y,z} tau(beta; m_d, m'_d) (from 1/r = (2 sqrt(pi))^{-1}
Int alpha^{-3/2} exp(-r^2/4 alpha) d alpha).  tau is real and symmetric under
(m, m') -> (m', m) and (m, m') -> (-m, -m').

Reduction to 1-D integrals (substitute u = xi - xi'; the xi-integral over the
strip is elementary):

    s = m + m' = 0:  tau = 2 beta^{-1/2} D(m),
                     D(m) = Int_0^1 (1 - u) exp(-u^2/beta) cos(2 pi m u) du
    s != 0:          tau = -(S(m) + S(m')) / (pi s sqrt(beta)),
                     S(m) = Int_0^1 exp(-u^2/beta) sin(2 pi m u) du

The paper only says these 1-D integrals are obtainable "without significant
difficulty" (Sec. II); this reduction is checked in the tests against a
brute-force 2-D quadrature of the defining double integral.

S and D are computed with SciPy's QUADPACK (adaptive Gauss-Kronrod; the
oscillatory QAWO rule for m != 0) on [0, min(1, 12 sqrt(beta))]; beyond that
point exp(-u^2/beta) < 1e-62.  D is integrated directly rather than through
the integration-by-parts identity, which cancels badly for large beta.
"""
import math
import warnings

import numpy as np
from scipy.integrate import IntegrationWarning, quad

_EPSABS = 1e-17
_EPSREL = 1e-15
_LIMIT = 200
_CUT = 12.0


def _upper(beta: float) -> float:
    return min(1.0, _CUT * math.sqrt(beta))


def primitives(beta: float, mmax: int, need_s: bool = True):
    """S(m) and D(m) for m = 0..mmax at one beta (see module docstring)."""
    b = _upper(beta)
    S = np.zeros(mmax + 1)
    D = np.zeros(mmax + 1)
    gauss = lambda u: math.exp(-u * u / beta)
    ramp = lambda u: (1.0 - u) * math.exp(-u * u / beta)
    kw = dict(epsabs=_EPSABS, epsrel=_EPSREL, limit=_LIMIT)
    with warnings.catch_warnings():
        # QUADPACK flags "roundoff prevents the requested tolerance" at these
        # tight settings; the achieved accuracy is pinned against mpmath in
        # the tests.
        warnings.simplefilter("ignore", IntegrationWarning)
        D[0] = quad(ramp, 0.0, b, **kw)[0]
        for m in range(1, mmax + 1):
            w = 2.0 * math.pi * m
            D[m] = quad(ramp, 0.0, b, weight="cos", wvar=w, **kw)[0]
            if need_s:
                S[m] = quad(gauss, 0.0, b, weight="sin", wvar=w, **kw)[0]
    return S, D


def tau_table(beta, K: int) -> np.ndarray:
    """tau_q(m, m') for every node and m, m' in [-K, K].

    Returns float64 [Q, 2K+1, 2K+1]; entry [q, m+K, m'+K].
    """
    beta = np.atleast_1d(np.asarray(beta, dtype=np.float64))
    nd = 2 * K + 1
    out = np.empty((beta.size, nd, nd))
    mm = np.arange(-K, K + 1)
    M, MP = np.meshgrid(mm, mm, indexing="ij")
    s = M + MP
    for q, bq in enumerate(beta):
        S, D = primitives(float(bq), K)
        Sfull = np.sign(mm) * S[np.abs(mm)]           # S is odd in m
        rb = math.sqrt(bq)
        with np.errstate(divide="ignore", invalid="ignore"):
            off = -(Sfull[M + K] + Sfull[MP + K]) / (math.pi * s * rb)
        diag = 2.0 / rb * D[np.abs(M)]
        out[q] = np.where(s == 0, diag, off)
    return out


def box_tables(beta, K: int, sides):
    """Direction tables of a rectangular box with sides (Lx, Ly, Lz).

    Writing 1/r as a Gaussian integral, each direction d of a box factorises
    as in a cube of side L_d, with its Gaussian exponent scaled by the side:
    on the reference mesh beta = 1/(t L0^2) direction d sees
    beta_d = beta / rho_d^2, rho_d = L_d / L0, and the node sum of Eq. 14
    becomes (sqrt(pi) L0 rho_x rho_y rho_z)^{-1} sum_q W_q prod_d
    tau(beta_q / rho_d^2; m_d, m'_d).  With L0 the geometric mean of the
    sides the rho product is 1 and the prefactor keeps its cube form.

    Returns (L0, rho [3], tau [3, Q, 2K+1, 2K+1]).
    """
    sides = np.asarray(sides, dtype=np.float64)
    L0 = float(np.prod(sides) ** (1.0 / 3.0))
    rho = sides / L0
    beta = np.atleast_1d(np.asarray(beta, dtype=np.float64))
    tau = np.stack([tau_table(beta / (r * r), K) for r in rho])
    return L0, rho, tau


def tau_diag(beta, K: int) -> np.ndarray:
    """Diagonal entries tau_q(m, -m) for m in [-K, K]: float64 [Q, 2K+1].

    These are the only entries exchange integrals <ij|ji> read.
    """
    beta = np.atleast_1d(np.asarray(beta, dtype=np.float64))
    mm = np.abs(np.arange(-K, K + 1))
    out = np.empty((beta.size, 2 * K + 1))
    for q, bq in enumerate(beta):
        _, D = primitives(float(bq), K, need_s=False)
        out[q] = 2.0 / math.sqrt(bq) * D[mm]
    return out


def tau00_closed_form(beta) -> np.ndarray:
    """tau(beta; 0, 0) in closed form: sqrt(pi) erf(beta^{-1/2}) - sqrt(beta)(1 - e^{-1/beta}).

    Follows from the s = 0 reduction with m = 0 (both integrals elementary).
    Used as a pin, not by the oracle's own table path.
    """
    from scipy.special import erf
    beta = np.asarray(beta, dtype=np.float64)
    return math.sqrt(math.pi) * erf(beta ** -0.5) + np.sqrt(beta) * np.expm1(-1.0 / beta)
