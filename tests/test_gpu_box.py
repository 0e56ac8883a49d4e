"""Rectangular boxes on the GPU: direction tables, reconstruction on both
paths and pair sums against the oracle (oracle.box_tables)."""
import math
import sys

import numpy as np
import pytest

import oracle
import workloads
from tests import _parity as P

pytestmark = pytest.mark.gpu
DIRECT_DEFAULT = 1 << 19


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def pw():
    import torch
    import paper_1502_08043_amd as pw
    assert torch.cuda.is_available()
    return pw


def _dev(a, dtype):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def _oracle_box(n2max, Q, sides):
    b = oracle.enumerate_basis(n2max)
    beta, W, _ = oracle.default_mesh(Q)
    L0, rho, taus = oracle.box_tables(beta, 2 * math.isqrt(n2max), sides)
    return dict(basis=b, beta=beta, W=W, L0=L0, taus=taus)


def _cond_scale(o, quads):
    taus, W, b = o["taus"], o["W"], o["basis"]
    K = (taus.shape[-1] - 1) // 2
    q = np.asarray(quads, dtype=np.int64)
    m = b[q[:, 2]] - b[q[:, 0]] + K
    mp = b[q[:, 3]] - b[q[:, 1]] + K
    prod = np.abs(W)[:, None] * np.ones((1, len(q)))
    for d in range(3):
        prod = prod * np.abs(taus[d][:, m[:, d], mp[:, d]])
    return prod.sum(axis=0) / (math.sqrt(math.pi) * o["L0"])


CASES = [(9, 48, (1.0, 1.3, 0.8)), (40, 64, (2.0, 1.0, 0.5)), (169, 96, (1.0, 1.5, 0.75))]


@pytest.mark.parametrize("n2max,Q,sides", CASES)
def test_box_tables_and_reconstruction(pw, n2max, Q, sides):
    import torch
    o = _oracle_box(n2max, Q, sides)
    with pw.Table.box(*sides, n2max, Q) as t:
        assert t.ndir == 3 and t.sides == sides and abs(t.L - o["L0"]) < 1e-15 * o["L0"]
        tab = t.copy_tables().cpu().numpy()
        scale = np.abs(o["taus"]).max(axis=(2, 3), keepdims=True)
        assert np.max(np.abs(tab - o["taus"]) / scale) < P.TOL_TABLE
        n = 30001 if n2max < 169 else 600_001
        quads = workloads.uniform_quads(len(o["basis"]), n, seed=n2max)
        rows = workloads.sample_rows(n, min(n, 20000), seed=1)
        ref = oracle.reconstruct(o["taus"], o["W"], o["basis"], quads[rows], L=o["L0"])
        cs = _cond_scale(o, quads[rows])
        dq = _dev(quads, torch.int32)
        rr = torch.from_numpy(rows).cuda()
        outs = {}
        tols = {pw.FP64: P.TOL_FP64, pw.MIXED: P.TOL_MIXED, pw.FP32: P.TOL_FP32}
        # the direct kernel, the default layouts and the one-lane layout (fused
        # when its slab and the basis maps fit in LDS, else refused)
        for path, dm, lay in (("direct", DIRECT_DEFAULT, None), ("passes", 0, None), ("one-lane", 0, (1, 8))):
            t.set_direct_max(dm)
            if lay:
                try:
                    t.set_layout(*lay)
                except pw.PwcError as e:   # the slab does not fit in LDS
                    assert e.status == pw.ERR_RANGE
                    continue
            for prec in (pw.FP64, pw.MIXED, pw.FP32):
                out = t.reconstruct(dq, precision=prec)
                t.sync()
                err = P.worst_cond_err(out[rr].cpu().numpy(), ref, cs)
                say(f"[box] {sides} n2max={n2max} Q={Q} {path} prec={prec} fused={t.fused(prec)}: {err:.2e}")
                assert err < tols[prec]
                outs[path, prec] = out
            if lay:
                t.set_layout(0, 0)
        for prec in (pw.FP64, pw.MIXED, pw.FP32):
            for path in ("passes", "one-lane"):
                if (path, prec) not in outs:
                    continue
                a, b = outs["direct", prec], outs[path, prec]
                tol = 1e-6 if prec == pw.FP32 else 1e-12
                assert (a - b).abs().max().item() <= tol * b.abs().max().item()


@pytest.mark.parametrize("n2max,Q,sides", CASES)
def test_box_energies(pw, n2max, Q, sides):
    import torch
    o = _oracle_box(n2max, Q, sides)
    occ = np.arange(min(len(o["basis"]), 123 if n2max < 169 else 257))
    f = workloads.rng(7).uniform(0.25, 1.0, len(occ))
    ref = oracle.energies(o["taus"], o["W"], o["basis"], occ, f=f, L=o["L0"])
    with pw.Table.box(*sides, n2max, Q) as t:
        for algo in (pw.PAIR_NODESUM, pw.PAIR_KTABLE):
            for prec in (pw.FP64, pw.MIXED):
                eh, ex = t.energies(_dev(occ, torch.int32), _dev(f, torch.float64),
                                    precision=prec, algo=algo)
                say(f"[box] energies {sides} algo={algo} prec={prec}: "
                    f"{abs(eh - ref[0]) / abs(ref[0]):.1e} {abs(ex - ref[1]) / abs(ref[1]):.1e}")
                assert abs(eh - ref[0]) < P.TOL_E_FP64 * abs(ref[0])
                assert abs(ex - ref[1]) < P.TOL_E_FP64 * abs(ref[1])


def test_box_with_equal_sides_is_the_cube(pw):
    import torch
    with pw.Table.box(1.25, 1.25, 1.25, 40, 64) as b, pw.Table(1.25, 40, 64) as c:
        assert b.ndir == 1 and torch.equal(b.copy_tables(), c.copy_tables())
        q = _dev(workloads.uniform_quads(b.N, 700_001, seed=2), torch.int32)
        for prec in (pw.FP64, pw.MIXED):
            assert torch.equal(b.reconstruct(q, precision=prec), c.reconstruct(q, precision=prec))
        b.sync()
        c.sync()


def test_box_axis_permutation(pw):
    """Box (a, b, c) and box (b, a, c) with the x and y components of every
    basis vector swapped give the same integrals."""
    import torch
    with pw.Table.box(1.0, 1.4, 0.7, 40, 64) as t1, pw.Table.box(1.4, 1.0, 0.7, 40, 64) as t2:
        b = t1.basis()
        index = {tuple(v): i for i, v in enumerate(b)}
        perm = np.array([index[(v[1], v[0], v[2])] for v in b], dtype=np.int64)
        quads = workloads.uniform_quads(len(b), 200_000, seed=9)
        for dm in (DIRECT_DEFAULT, 0):
            t1.set_direct_max(dm)
            t2.set_direct_max(dm)
            a = t1.reconstruct(_dev(quads, torch.int32))
            c = t2.reconstruct(_dev(perm[quads], torch.int32))
            assert (a - c).abs().max().item() <= 1e-13 * a.abs().max().item()
        t1.sync()
        t2.sync()


def test_box_save_load(pw, tmp_path):
    import torch
    path = tmp_path / "box.tab"
    q = _dev(workloads.uniform_quads(1045, 50_000, seed=5), torch.int32)
    with pw.Table.box(2.0, 1.0, 0.5, 40, 64) as t:
        t.save(path)
        ref = t.reconstruct(q)
        tab = t.copy_tables()
        t.sync()
    with pw.Table.load(path) as u:
        assert u.sides == (2.0, 1.0, 0.5) and u.ndir == 3
        assert torch.equal(u.copy_tables(), tab)
        assert torch.equal(u.reconstruct(q), ref)
        u.sync()
