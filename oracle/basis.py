"""Planewave basis enumeration (oracle side).

Sec. II: a planewave basis keeps every product function whose wavevector is
below a cutoff, (2 pi / L)|I| < k_c.  On the integer lattice that is the ball
|n|^2 <= n2max.  Sec. III lists the occupied-sphere sizes at shell closings
(M = 7, 33, 123, ...), which are lattice-point counts of such balls.

The paper does not fix an order.  This oracle (and the library) use the
canonical order (|n|^2, n_x, n_y, n_z) ascending, so every ball |n|^2 <= r2
is an index prefix of any larger one.
"""
import math

import numpy as np


def enumerate_basis(n2max: int) -> np.ndarray:
    """All n in Z^3 with |n|^2 <= n2max, sorted by (|n|^2, n_x, n_y, n_z).

    Returns an int64 array of shape [N, 3].  Written as a plain triple loop so
    it can be checked by eye; n2max up to a few hundred takes well under a
    second.
    """
    if n2max < 0:
        raise ValueError("n2max must be >= 0")
    r = math.isqrt(n2max)
    pts = []
    for x in range(-r, r + 1):
        for y in range(-r, r + 1):
            for z in range(-r, r + 1):
                n2 = x * x + y * y + z * z
                if n2 <= n2max:
                    pts.append((n2, x, y, z))
    pts.sort()
    return np.array([p[1:] for p in pts], dtype=np.int64).reshape(-1, 3)


def shell_counts(n2max: int) -> np.ndarray:
    """Number of basis vectors with |n|^2 <= r2 for r2 = 0..n2max."""
    b = enumerate_basis(n2max)
    n2 = (b * b).sum(axis=1)
    return np.array([(n2 <= r2).sum() for r2 in range(n2max + 1)], dtype=np.int64)
