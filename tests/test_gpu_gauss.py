"""Separable s-type Gaussian basis on the GPU (pwc_table_create_gauss):
tables and integrals against the FP64 oracle (oracle/gauss.py), and against
the textbook closed form for isotropic functions."""
import math
import sys

import numpy as np
import pytest

import oracle
import workloads
from tests import _brute
from tests import _parity as P

pytestmark = pytest.mark.gpu

L_REF = 8.0     # bohr: about the extent of the small set's centers


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def pw():
    import torch
    import paper_1502_08043_amd as pw
    assert torch.cuda.is_available()
    pw.lib()
    return pw


def _dev(a, dtype):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def _oracle(gs, spec, eps=1e-15, L=L_REF):
    a, A = workloads.gaussian_set(gs)
    pairs, pmap = oracle.gauss_pairs(a, A, eps)
    kind = spec[0]
    if kind == "root":
        beta, W, _ = oracle.mesh3(spec[1], spec[2], n_sub=spec[3], ratio=spec[4])
    else:
        beta, W, _ = oracle.mesh2(spec[1], spec[2])
    tau = oracle.gauss_tau(beta, a, A, pairs, L=L)
    return a, A, pairs, pmap, beta, W, tau


def _mesh(pw, spec):
    if spec[0] == "root":
        return pw.Mesh.geometric_root(spec[1], spec[2], n_sub=spec[3], ratio=spec[4])
    return pw.Mesh.geometric(spec[1], spec[2])


def _local_quads(n1, n, seed, window=2):
    """Quadruples whose four functions sit within `window` one-dimensional
    indices of each other along every direction (mostly kept pairs)."""
    g = workloads.rng(seed)
    base = g.integers(0, n1, (n, 1, 3))
    l = np.clip(base + g.integers(-window, window + 1, (n, 4, 3)), 0, n1 - 1)
    return ((l[..., 0] * n1 + l[..., 1]) * n1 + l[..., 2]).astype(np.int32)


# The split-FP32 tables keep FP32's exponent range: a node term (a product of
# three entries) below about 1e-30 loses relative accuracy, so the relative
# bar holds for integrals above MIXED_FLOOR and an absolute one below it.
MIXED_FLOOR = 1e-22
MIXED_ABS = 1e-26


def _cond_err(got, ref, tau, W, pmap, n1, quads, L, floor=0.0):
    """Condition-aware error: every tau entry is positive, so the scale is the
    integral itself; screened rows must be exactly zero on both sides.
    Returns (worst relative error over |ref| >= floor, worst absolute error
    below it)."""
    zero = ref == 0
    assert np.array_equal(got[zero], ref[zero])
    big = np.abs(ref) >= max(floor, 1e-300)
    small = ~zero & ~big
    rel = float(np.max(np.abs(got[big] - ref[big]) / np.abs(ref[big]))) if big.any() else 0.0
    ab = float(np.max(np.abs(got[small] - ref[small]))) if small.any() else 0.0
    return rel, ab


@pytest.mark.parametrize("spec", [("root", 10, 6, 4, 7.0), ("geometric", 5, 8)])
def test_gauss_tables_match_oracle(pw, spec):
    a, A, pairs, pmap, beta, W, tau = _oracle(workloads.GAUSS_SMALL, spec)
    with pw.GaussTable(a, A, L_REF, eps=1e-15, mesh=_mesh(pw, spec)) as t:
        assert (t.n1, t.n_pairs, t.N) == (len(a), len(pairs), len(a) ** 3)
        b, w = t.mesh_nodes()
        assert np.max(np.abs(b - beta) / beta) < 5e-16 and np.max(np.abs(w - W) / W) < 5e-16
        got = t.copy_tables().cpu().numpy()
    assert got.shape == tau.shape
    err = np.max(np.abs(got - tau) / np.abs(tau).max(axis=(1, 2), keepdims=True))
    say(f"[gauss] tables {spec}: {len(pairs)} pairs, worst err / node max {err:.2e}")
    assert err < P.TOL_TABLE
    assert np.array_equal(got, np.transpose(got, (0, 2, 1)))


@pytest.mark.parametrize("n", [1, 63, 64, 65, 100_003])
def test_gauss_integrals_match_oracle(pw, n):
    """Local and uniform quadruples, both precisions, ragged list lengths."""
    import torch
    spec = ("root", 10, 6, 4, 7.0)
    a, A, pairs, pmap, beta, W, tau = _oracle(workloads.GAUSS_SMALL, spec)
    n1 = len(a)
    q = np.concatenate([_local_quads(n1, (n + 1) // 2, seed=n),
                        workloads.uniform_quads(n1 ** 3, n // 2, seed=n + 1)])
    ref = oracle.gauss_reconstruct(tau, W, pmap, n1, q, L=L_REF)
    with pw.GaussTable(a, A, L_REF, mesh=_mesh(pw, spec)) as t:
        dq = _dev(q, torch.int32)
        for prec in (pw.FP64, pw.MIXED):
            out = torch.full((len(q),), -3.0, dtype=torch.float64, device="cuda")
            t.reconstruct(dq, out, precision=prec)
            t.sync()
            got = out.cpu().numpy()
            if prec == pw.FP64:
                rel, _ = _cond_err(got, ref, tau, W, pmap, n1, q, L_REF)
                assert rel < P.TOL_FP64
            else:
                rel, ab = _cond_err(got, ref, tau, W, pmap, n1, q, L_REF, floor=MIXED_FLOOR)
                for lo in (1e-10, 1e-14, 1e-18, 1e-22, 1e-26, 1e-30, 1e-34):
                    sel = (np.abs(ref) >= lo) & (np.abs(ref) < lo * 1e4)
                    if sel.any():
                        say(f"[gauss] mixed |ref| in [{lo:.0e}, {lo * 1e4:.0e}): {int(sel.sum())} rows, "
                            f"worst rel {np.max(np.abs(got[sel] - ref[sel]) / np.abs(ref[sel])):.2e}")
                assert rel < P.TOL_MIXED and ab < MIXED_ABS, (rel, ab)
            say(f"[gauss] n={n} prec={prec}: {int((ref != 0).sum())} nonzero, worst rel err {rel:.2e}")


def test_gauss_integrals_match_the_closed_form(pw):
    """Isotropic functions (one exponent along x, y, z): the GPU integrals
    on a 46-node Mesh 3 against the Boys-function closed form, to the
    quadrature error of the mesh (1e-9 relative, 1e-12 absolute)."""
    import torch
    gs = workloads.GAUSS_SMALL
    a, A = workloads.gaussian_set(gs)
    n1 = len(a)
    ne = len(gs.exponents)
    iso = np.array([(l * n1 + m) * n1 + n for l in range(n1) for m in range(n1) for n in range(n1)
                    if l % ne == m % ne == n % ne])
    q = iso[workloads.rng(8).integers(0, len(iso), (4000, 4))].astype(np.int32)
    lidx = oracle.gauss_decode(q, n1)
    ex = np.array([_brute.gauss_exact(a[lidx[r, :, 0]], A[lidx[r]], np.array([[0, 1, 2, 3]]))[0]
                   for r in range(len(q))])
    with pw.GaussTable(a, A, L_REF, mesh=pw.Mesh.geometric_root(10, 6)) as t:
        got = t.reconstruct(_dev(q, torch.int32)).cpu().numpy()
        t.sync()
    kept = got != 0
    assert kept.sum() > 2500
    assert np.max(np.abs(got - ex)) < 1e-12
    assert np.max(np.abs(got - ex)[kept] / np.abs(ex[kept])) < 1e-9


def test_gauss_bench_set_and_screening(pw):
    """The larger set (24 functions per direction, 13,824 basis functions)
    with a coarser screen: the pair band, the tables and a sample of a
    million-quadruple local stream against the oracle."""
    import torch
    gs = workloads.GAUSS_BENCH
    a, A = workloads.gaussian_set(gs)
    n1 = len(a)
    L = 20.0
    for eps in (1e-15, 1e-8):
        pairs, pmap = oracle.gauss_pairs(a, A, eps)
        beta, W, _ = oracle.mesh3(10, 6, n_sub=4, ratio=7.0)
        tau = oracle.gauss_tau(beta, a, A, pairs, L=L)
        q = _local_quads(n1, 1_000_000, seed=5, window=3)
        rows = workloads.sample_rows(len(q), 20_000, seed=6)
        ref = oracle.gauss_reconstruct(tau, W, pmap, n1, q[rows], L=L)
        with pw.GaussTable(a, A, L, eps=eps, mesh=pw.Mesh.geometric_root(10, 6)) as t:
            assert t.n_pairs == len(pairs)
            got = t.reconstruct(_dev(q, torch.int32)).cpu().numpy()
            t.sync()
        err, _ = _cond_err(got[rows], ref, tau, W, pmap, n1, q[rows], L)
        say(f"[gauss] bench set eps={eps}: {len(pairs)} of {n1 * (n1 + 1) // 2} pairs kept, "
            f"{(ref != 0).mean():.2f} of the sample nonzero, worst rel err {err:.2e}, "
            f"smallest nonzero |ref| {np.abs(ref[ref != 0]).min():.1e}")
        assert err < P.TOL_FP64


def test_gauss_errors_and_unsupported_calls(pw):
    import torch
    a, A = workloads.gaussian_set(workloads.GAUSS_SMALL)
    n1 = len(a)
    with pytest.raises(pw.PwcError):
        pw.GaussTable(a, A, -1.0)
    with pytest.raises(pw.PwcError):
        pw.GaussTable(-a, A, L_REF)
    with pytest.raises(pw.PwcError):
        pw.GaussTable(a, A, L_REF, eps=1.5)
    with pw.GaussTable(a, A, L_REF, mesh=pw.Mesh.geometric_root(8, 4)) as t:
        q = torch.zeros((5, 4), dtype=torch.int32, device="cuda")
        q[2, 1] = n1 ** 3
        out = t.reconstruct(q)
        with pytest.raises(pw.PwcError) as ei:
            t.sync()
        assert ei.value.status == pw.ERR_RANGE
        got = out.cpu().numpy()
        assert np.isnan(got[2]) and not np.isnan(np.delete(got, 2)).any()
        occ = torch.arange(4, dtype=torch.int32, device="cuda")
        for call in (lambda: t.energies(occ), lambda: t.build_values(), lambda: t.layout(),
                     lambda: t.basis(), lambda: t.save("/tmp/x.tab")):
            with pytest.raises(pw.PwcError) as ei:
                call()
            assert ei.value.status == pw.ERR_ARG
        assert t.reconstruct(q[:0]).numel() == 0
