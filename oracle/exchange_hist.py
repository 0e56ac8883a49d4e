"""Exchange energy through the histogram of wavevector differences (oracle side).

An independent route to the Sec. III exchange energy, used to cross-check the
literal pair loop of sums.c and to reach M = 9171 (Table I) on a CPU.

For planewave orbitals <ij|ji> depends only on Delta = n_j - n_i (Sec. III:
the product of two planewaves is a planewave), through the diagonal entries
tau_q(Delta_d, -Delta_d).  Hence

  E_x = -1/(2 sqrt(pi) L) sum_Delta h(Delta) sum_q W_q
            tau_q(Dx,-Dx) tau_q(Dy,-Dy) tau_q(Dz,-Dz),
  h(Delta) = sum_{i,j : n_j - n_i = Delta} f_i f_j .

h is counted pair by pair (no FFT), so for unit occupations it is exact.
"""
import math

import numpy as np


def diff_histogram(vecs, f=None, chunk=256):
    """h(Delta) over all ordered pairs of the given integer vectors.

    Returns (h, R) with h of shape [4R+1]^3 indexed by Delta + 2R, where
    R = max |component| of the vectors.
    """
    v = np.asarray(vecs, dtype=np.int64).reshape(-1, 3)
    M = v.shape[0]
    R = int(np.abs(v).max()) if M else 0
    nd = 4 * R + 1
    w = np.ones(M) if f is None else np.asarray(f, dtype=np.float64).reshape(-1)
    h = np.zeros(nd ** 3)
    for i0 in range(0, M, chunk):
        vi = v[i0:i0 + chunk]
        d = v[None, :, :] - vi[:, None, :] + 2 * R          # n_j - n_i, shifted
        flat = (d[..., 0] * nd + d[..., 1]) * nd + d[..., 2]
        wij = w[i0:i0 + chunk, None] * w[None, :]
        h += np.bincount(flat.ravel(), weights=wij.ravel(), minlength=nd ** 3)
    return h.reshape(nd, nd, nd), R


def exchange_from_histogram(h, R, diag, W, L=1.0, per_node=False):
    """E_x from a difference histogram and diagonal tables.

    diag: [Q, 2K+1] with diag[q, m + K] = tau_q(m, -m), K >= 2R.
    Returns E_x, or the per-node contributions [Q] when per_node is set
    (their sum is E_x; a subset gives e.g. the interval-1 part of Table I).
    """
    diag = np.asarray(diag, dtype=np.float64)
    W = np.asarray(W, dtype=np.float64)
    Q, nd_t = diag.shape
    K = (nd_t - 1) // 2
    if K < 2 * R:
        raise ValueError("diagonal table too small for these differences")
    sel = np.arange(-2 * R, 2 * R + 1) + K
    D = diag[:, sel]                                      # [Q, 4R+1]
    nz = np.nonzero(h)
    hv = h[nz]
    contrib = np.empty(Q)
    for q in range(Q):
        kq = D[q, nz[0]] * D[q, nz[1]] * D[q, nz[2]]
        contrib[q] = W[q] * math.fsum(hv * kq)
    contrib *= -1.0 / (2.0 * math.sqrt(math.pi) * L)
    if per_node:
        return contrib
    return math.fsum(contrib)
