"""Shared helpers of the GPU parity tests: oracle set-ups and the error metric.

Integral parity is condition-aware: |C - C_ref| <= tol * scale with
scale = sum_q |W_q X_q Y_q Z_q| / (sqrt(pi) L), the sum of the magnitudes of
the node terms of Eq. 14.  Many integrals of a random quadruple stream are
small near-cancelling sums, so plain relative error would measure the
cancellation, not the arithmetic.  Energies use plain relative error (their
node terms are all positive).
"""
import functools
import math

import numpy as np

import oracle

TOL_FP64 = 1e-12          # condition-aware, FP64 path
TOL_MIXED = 1e-12         # condition-aware, split-FP32 path (float-float)
# condition-aware, single-FP32 path: each entry W^(1/3) tau rounded once to
# FP32 (3 roundings per node term) and at most 4 in the pairwise sum of a
# four-node word (the first product; the second product and the fused
# multiply-add that adds it to its pair; the sum of the two pairs), each at
# most 2^-24 relative: 7 * 2^-24 = 4.2e-7 of the sum of the node terms'
# magnitudes; the FP64 accumulation adds ~1e-16.
TOL_FP32 = 4.2e-7
TOL_E_FP64 = 1e-12        # relative, energies
TOL_E_MIXED = 1e-12
TOL_TABLE = 1e-14         # tables: relative to each node's largest |tau|


@functools.lru_cache(maxsize=None)
def setup(n2max, n_nodes=0, mesh=None, beta_c=1.0):
    """Oracle basis, mesh and tables.  mesh: None (default Mesh 2 for n_nodes),
    ("geometric", q_sub, q_tail), ("root", q_sub, q_tail, n_sub, ratio) (Mesh 3)
    or ("two_interval", q)."""
    b = oracle.enumerate_basis(n2max)
    nmax = math.isqrt(n2max)
    if mesh is None:
        beta, W, n1 = oracle.default_mesh(n_nodes, beta_c)
    elif mesh[0] == "geometric":
        beta, W, n1 = oracle.mesh2(mesh[1], mesh[2], beta_c=beta_c)
    elif mesh[0] == "root":
        beta, W, n1 = oracle.mesh3(mesh[1], mesh[2], n_sub=mesh[3], ratio=mesh[4], beta_c=beta_c)
    else:
        beta, W, n1 = oracle.mesh1(mesh[1], beta_c=beta_c)
    tau = oracle.tau_table(beta, 2 * nmax)
    return dict(basis=b, beta=beta, W=W, n1=n1, tau=tau, K=2 * nmax)


def cond_scale(tau, W, basis, quads, L=1.0):
    """tau: [Q, nd, nd] for a cube, [3, Q, nd, nd] (one table per direction)
    for a box, whose L is the reference length."""
    K = (tau.shape[-1] - 1) // 2
    q = np.asarray(quads, dtype=np.int64)
    m = basis[q[:, 2]] - basis[q[:, 0]] + K
    mp = basis[q[:, 3]] - basis[q[:, 1]] + K
    prod = np.abs(W)[:, None] * np.ones((1, len(q)))
    for d in range(3):
        td = tau[d] if tau.ndim == 4 else tau
        prod = prod * np.abs(td[:, m[:, d], mp[:, d]])
    return prod.sum(axis=0) / (math.sqrt(math.pi) * L)


def worst_cond_err(got, ref, scale):
    return float(np.max(np.abs(np.asarray(got) - ref) / scale)) if len(ref) else 0.0
