"""Closed-form reference quantities (oracle side)."""
import math


def e_ks(M: float, L: float = 1.0) -> float:
    """Kohn-Sham (LDA) exchange energy of M same-spin electrons in a cube of side L.

    Sec. III: E_KS = -(3/4) (6/pi)^{1/3} M^{4/3} / L, the large-M limit of the
    exact exchange energy; per spin channel.
    """
    return -0.75 * (6.0 / math.pi) ** (1.0 / 3.0) * M ** (4.0 / 3.0) / L


def k_cube() -> float:
    """Mean inverse distance between two uniform points of the unit cube.

    Int_{[0,1]^6} d^3r d^3r' / |r - r'|
      = 2 [ (1 + sqrt2 - 2 sqrt3)/5 - pi/3 + ln((1 + sqrt2)(2 + sqrt3)) ]
      = 1.88231264438966...
    For planewaves every m = m' = 0 integral <ij|ij> equals k_cube()/L, which
    pins the Laplace-transform prefactor and the free-space boundary
    condition of Eqs. 3-7.
    """
    s2, s3 = math.sqrt(2.0), math.sqrt(3.0)
    return 2.0 * ((1.0 + s2 - 2.0 * s3) / 5.0 - math.pi / 3.0
                  + math.log((1.0 + s2) * (2.0 + s3)))
