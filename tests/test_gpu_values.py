"""The value table (pwc_table_build_values): every distinct integral evaluated
once, then one read per quadruple.  Checked against the FP64 oracle and
against the node-sum paths of the same table."""
import math
import sys

import numpy as np
import pytest

import oracle
import workloads
from tests import _parity as P

pytestmark = pytest.mark.gpu


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


def _entries(n2max):
    # orbits of the (m, m') plane, nd = 4 nmax + 1, under the four-element
    # fold group (Burnside: (nd^2 + 2 nd + 1) / 4 = (2 nmax + 1)^2)
    return (2 * math.isqrt(n2max) + 1) ** 2


@pytest.mark.parametrize("n2max,Q,n", [(9, 48, 60001), (40, 64, 200003), (169, 96, 2_000_001)])
def test_values_match_oracle_and_node_sums(pw, n2max, Q, n):
    import torch
    o = P.setup(n2max, Q)
    E = _entries(n2max)
    with pw.Table(1.0, n2max, Q) as t:
        built, nbytes = t.values_info()
        assert not built and nbytes == 8 * E * (E + 1) * (E + 2) // 6
        base = t.device_bytes
        quads = workloads.lookup_stream(len(o["basis"]), min(len(o["basis"]), 925), n, seed=n2max)
        dq = _dev(quads, torch.int32)
        t.set_direct_max(0)
        passes = t.reconstruct(dq)
        t.set_direct_max(1 << 19)
        direct = t.reconstruct(dq[:100_000])
        t.build_values()
        assert t.values_info() == (True, nbytes) and t.device_bytes == base + nbytes
        got = t.reconstruct(dq)
        mixed = t.reconstruct(dq, precision=pw.MIXED)    # node sums, not the values
        t.sync()
        rows = workloads.sample_rows(n, min(n, 20000), seed=3)
        ref = oracle.reconstruct(o["tau"], o["W"], o["basis"], quads[rows])
        cs = P.cond_scale(o["tau"], o["W"], o["basis"], quads[rows])
        err = P.worst_cond_err(got.cpu().numpy()[rows], ref, cs)
        say(f"[values] n2max={n2max} Q={Q} E={E}: {nbytes / 2**20:.1f} MiB, n={n}, "
            f"oracle err {err:.2e} (condition-aware)")
        assert err < P.TOL_FP64
        assert P.worst_cond_err(mixed.cpu().numpy()[rows], ref, cs) < P.TOL_MIXED
        # every output against the node passes and the direct kernel
        top = passes.abs().max().item()
        assert (got - passes).abs().max().item() <= 1e-13 * top
        assert (got[:100_000] - direct).abs().max().item() <= 1e-13 * top


def test_values_rebuild_is_bitwise_and_free_falls_back(pw):
    import torch
    quads = workloads.uniform_quads(1045, 300_000, seed=9)
    dq = _dev(quads, torch.int32)
    with pw.Table(1.0, 40, 64) as t:
        t.build_values()
        t.build_values()                      # no-op
        a = t.reconstruct(dq)
        t.free_values()
        assert t.values_info()[0] is False
        b = t.reconstruct(dq)                 # node sums again
        t.build_values()
        c = t.reconstruct(dq)
        t.sync()
    assert torch.equal(a, c)
    assert (a - b).abs().max().item() <= 1e-13 * b.abs().max().item()


@pytest.mark.parametrize("n", [0, 1, 1023, 1025, 2048, 2049, 4097])
def test_values_ragged_lengths(pw, n):
    import torch
    o = P.setup(9, 48)
    quads = workloads.uniform_quads(123, max(n, 1), seed=n)[:n]
    with pw.Table(1.0, 9, 48) as t:
        t.build_values()
        out = torch.full((n + 3,), -7.0, dtype=torch.float64, device="cuda")
        if n:
            t.reconstruct(_dev(quads, torch.int32), out=out[:n])
        else:
            t.reconstruct(torch.empty((0, 4), dtype=torch.int32, device="cuda"), out=out[:0])
        t.sync()
        got = out.cpu().numpy()
    assert np.all(got[n:] == -7.0)            # nothing written past the end
    if n:
        ref = oracle.reconstruct(o["tau"], o["W"], o["basis"], quads)
        cs = P.cond_scale(o["tau"], o["W"], o["basis"], quads)
        assert P.worst_cond_err(got[:n], ref, cs) < P.TOL_FP64


def test_values_out_of_range_index(pw):
    import torch
    quads = workloads.uniform_quads(123, 5000, seed=2)
    bad = quads.copy()
    bad[17, 2] = 123
    bad[4000, 0] = -1
    with pw.Table(1.0, 9, 48) as t:
        t.build_values()
        ref = t.reconstruct(_dev(quads, torch.int32))
        t.sync()
        got = t.reconstruct(_dev(bad, torch.int32))
        with pytest.raises(pw.PwcError) as ei:
            t.sync()
        assert ei.value.status == pw.ERR_RANGE
        t.sync()                               # the error word was cleared
    g = got.cpu().numpy()
    assert np.isnan(g[17]) and np.isnan(g[4000])
    keep = np.ones(5000, bool)
    keep[[17, 4000]] = False
    assert np.array_equal(g[keep], ref.cpu().numpy()[keep])


@pytest.mark.parametrize("n2max,Q,sides", [(9, 48, (1.0, 1.3, 0.8)), (40, 64, (2.0, 1.0, 0.5))])
def test_values_box(pw, n2max, Q, sides):
    import torch
    b = oracle.enumerate_basis(n2max)
    beta, W, _ = oracle.default_mesh(Q)
    L0, rho, taus = oracle.box_tables(beta, 2 * math.isqrt(n2max), sides)
    E1 = _entries(n2max)
    quads = workloads.uniform_quads(len(b), 100_001, seed=5)
    with pw.Table.box(*sides, n2max, Q) as t:
        assert t.values_info()[1] == 8 * E1 ** 3
        t.set_direct_max(0)
        passes = t.reconstruct(_dev(quads, torch.int32))
        t.build_values()
        got = t.reconstruct(_dev(quads, torch.int32))
        t.sync()
    rows = workloads.sample_rows(len(quads), 20000, seed=4)
    ref = oracle.reconstruct(taus, W, b, quads[rows], L=L0)
    K = 2 * math.isqrt(n2max)
    q = quads[rows].astype(np.int64)
    m, mp = b[q[:, 2]] - b[q[:, 0]] + K, b[q[:, 3]] - b[q[:, 1]] + K
    prod = np.abs(W)[:, None] * np.ones((1, len(q)))
    for d in range(3):
        prod = prod * np.abs(taus[d][:, m[:, d], mp[:, d]])
    cs = prod.sum(axis=0) / (math.sqrt(math.pi) * L0)
    err = P.worst_cond_err(got.cpu().numpy()[rows], ref, cs)
    say(f"[values] box {sides} n2max={n2max}: oracle err {err:.2e}")
    assert err < P.TOL_FP64
    assert (got - passes).abs().max().item() <= 1e-13 * passes.abs().max().item()


def test_values_full_size_lookup_stream(pw):
    """The 1e8-quadruple stream on the 9171-planewave table: sampled outputs
    against the oracle, every output against the node passes."""
    import torch
    w = workloads.C4_STREAM
    o = P.setup(w.n2max, w.n_nodes)
    N = len(o["basis"])
    M = int(((o["basis"].astype(np.int64) ** 2).sum(1) <= w.n2occ).sum())
    assert (N, M) == (9171, 925)
    quads = workloads.lookup_stream(N, M, w.n_quads, w.seed)
    dq = _dev(quads, torch.int32)
    with pw.Table(w.L, w.n2max, w.n_nodes) as t:
        passes = t.reconstruct(dq)
        t.build_values()
        got = t.reconstruct(dq)
        t.sync()
    rows = workloads.sample_rows(w.n_quads, 20000, seed=11)
    ref = oracle.reconstruct(o["tau"], o["W"], o["basis"], quads[rows], L=w.L)
    cs = P.cond_scale(o["tau"], o["W"], o["basis"], quads[rows], L=w.L)
    err = P.worst_cond_err(got[torch.from_numpy(rows).cuda()].cpu().numpy(), ref, cs)
    dev = (got - passes).abs().max().item() / passes.abs().max().item()
    say(f"[values] C4 1e8: oracle err {err:.2e}, max |values - passes| / max {dev:.1e}")
    assert err < P.TOL_FP64 and dev <= 1e-13


def test_cached_blocks_are_reused_safely(pw):
    """Freed tables leave their device blocks to later tables; a table built
    into a reused block gives bitwise the same results."""
    import torch
    quads = _dev(workloads.lookup_stream(9171, 925, 500_000, seed=21), torch.int32)
    with pw.Table(1.0, 169, 96) as t:
        t.build_values()
        first = t.reconstruct(quads)
        t.sync()
    with pw.Table(1.0, 40, 64) as s:           # another table in between
        s.build_values()
        s.reconstruct(quads[:1000] % 1045)
        s.sync()
    with pw.Table(2.0, 169, 96) as t:          # same sizes: reuses the blocks
        t.build_values()
        half = t.reconstruct(quads)
        t.sync()
    with pw.Table(1.0, 169, 96) as t:
        t.build_values()
        again = t.reconstruct(quads)
        t.sync()
    pw.release_cached_memory()                 # blocks, staging buffers, build block lists
    with pw.Table(1.0, 169, 96) as t:          # everything formed again
        t.build_values()
        fresh = t.reconstruct(quads)
        t.sync()
    assert torch.equal(first, again) and torch.equal(first, fresh)
    assert (2.0 * half - first).abs().max().item() <= 1e-15 * first.abs().max().item()


def test_values_largest_cutoff_wide_indices_and_global_maps(pw):
    """n2max = 624 (65,117 PW, E = 2401): 2.3e9 values (18.5 GB) indexed past
    2^31, and a basis too large for LDS, so the decode reads its maps from
    global memory.  Quadruples with (m, m') = (48, 48) in x read the table's
    last entries."""
    import torch
    o = P.setup(624, 16)
    b = o["basis"]
    where = {tuple(v): i for i, v in enumerate(b.tolist())}
    far = [where[(-24, 0, 0)], where[(24, 0, 0)], where[(0, 0, 0)], where[(0, 7, 0)]]
    # n_k - n_i = (48, 0, 0) and n_l - n_j = (48, 0, 0): the last orbit in x
    crafted = np.array([[far[0], far[0], far[1], far[1]],
                        [far[0], far[2], far[1], far[3]],
                        [far[2], far[0], far[3], far[1]]], dtype=np.int32)
    quads = np.concatenate([workloads.uniform_quads(len(b), 200_000, seed=77), crafted])
    E = _entries(624)
    dq = _dev(quads, torch.int32)
    with pw.Table(1.0, 624, 16) as t:
        nvals = t.values_info()[1] // 8
        assert nvals == E * (E + 1) * (E + 2) // 6 and nvals > 2 ** 31
        t.set_direct_max(0)
        passes = t.reconstruct(dq)
        t.build_values()
        got = t.reconstruct(dq)
        t.sync()
    rows = np.concatenate([workloads.sample_rows(200_000, 5000, seed=5), np.arange(200_000, 200_003)])
    ref = oracle.reconstruct(o["tau"], o["W"], b, quads[rows])
    cs = P.cond_scale(o["tau"], o["W"], b, quads[rows])
    g = got.cpu().numpy()
    err = P.worst_cond_err(g[rows], ref, cs)
    say(f"[values] n2max=624 Q=16 E={E}: {nvals} values, oracle err {err:.2e}")
    assert err < P.TOL_FP64
    assert (got - passes).abs().max().item() <= 1e-13 * passes.abs().max().item()


def test_values_full_size_box(pw):
    """A 9171-planewave box: all 729^3 direction triples (3.1 GB)."""
    import torch
    sides = (1.0, 1.5, 0.75)
    b = oracle.enumerate_basis(169)
    beta, W, _ = oracle.default_mesh(96)
    L0, rho, taus = oracle.box_tables(beta, 26, sides)
    quads = workloads.lookup_stream(9171, 925, 1_000_000, seed=6)
    dq = _dev(quads, torch.int32)
    with pw.Table.box(*sides, 169, 96) as t:
        assert t.values_info()[1] == 8 * 729 ** 3
        t.set_direct_max(0)
        passes = t.reconstruct(dq)
        t.build_values()
        got = t.reconstruct(dq)
        t.sync()
    rows = workloads.sample_rows(len(quads), 10000, seed=8)
    ref = oracle.reconstruct(taus, W, b, quads[rows], L=L0)
    q = quads[rows].astype(np.int64)
    m, mp = b[q[:, 2]] - b[q[:, 0]] + 26, b[q[:, 3]] - b[q[:, 1]] + 26
    prod = np.abs(W)[:, None] * np.ones((1, len(q)))
    for d in range(3):
        prod = prod * np.abs(taus[d][:, m[:, d], mp[:, d]])
    cs = prod.sum(axis=0) / (math.sqrt(math.pi) * L0)
    err = P.worst_cond_err(got.cpu().numpy()[rows], ref, cs)
    say(f"[values] box {sides} 9171 PW: oracle err {err:.2e}")
    assert err < P.TOL_FP64
    assert (got - passes).abs().max().item() <= 1e-13 * passes.abs().max().item()


def test_values_build_is_stream_ordered(pw):
    """The build is asynchronous on its stream: a reconstruction queued after
    it on the same stream, or on another stream that waits for it, reads the
    finished values."""
    import torch
    quads = _dev(workloads.lookup_stream(1045, 123, 200_000, seed=31), torch.int32)
    with pw.Table(1.0, 40, 64) as t:
        ref = t.reconstruct(quads)                # node sums
        t.sync()
        side = torch.cuda.Stream()
        with torch.cuda.stream(side):
            t.build_values(stream=side)
            same = t.reconstruct(quads, stream=side)
        torch.cuda.current_stream().wait_stream(side)
        other = t.reconstruct(quads)
        t.sync()
        torch.cuda.synchronize()
    tol = 1e-14 * ref.abs().max().item()
    assert (same - ref).abs().max().item() <= tol
    assert torch.equal(same, other)


def _oracle_tables(sides, n2max, Q):
    """Oracle basis, weights, tables and reference length for a cube (sides
    of length 1) or a box on the default mesh."""
    o = P.setup(n2max, Q)
    if len(sides) == 1:
        return o["basis"], o["W"], o["tau"], sides[0]
    L0, _, tau = oracle.box_tables(o["beta"], o["K"], sides)
    return o["basis"], o["W"], tau, L0


@pytest.mark.parametrize("sides,n2max,Q", [((1.0,), 169, 96), ((1.0,), 40, 64), ((1.0, 1.3, 0.8), 40, 64)])
def test_values_at_the_edge_of_the_reachable_set(pw, monkeypatch, sides, n2max, Q):
    """The build skips values no quadruple can reach (orbit sizes summing past
    8 n2max).  Quadruples on the outer shells, many of them antipodal
    (k = -i, l = -j: |m|^2 + |m'|^2 = 8 n2max on the outermost shell), read the
    values nearest that edge; each must equal the node passes of the table,
    and a sample the oracle.  The value block is filled with NaN before the
    build (a test-only switch of the library), so a value the build missed
    cannot pass for one left in a recycled block by an earlier table."""
    import torch
    monkeypatch.setenv("PWC_TEST_POISON_VALUES", "1")
    make = (lambda: pw.Table(sides[0], n2max, Q)) if len(sides) == 1 else \
        (lambda: pw.Table.box(*sides, n2max, Q))
    with make() as t:
        b = t.basis().astype(np.int64)
        where = {tuple(v): k for k, v in enumerate(b)}
        neg = np.array([where[tuple(-v)] for v in b])
        r2 = (b * b).sum(1)
        outer = np.flatnonzero(r2 >= max(1, n2max - 12))
        g = workloads.rng(7)
        n = 600_000
        i = outer[g.integers(0, len(outer), n)]
        j = outer[g.integers(0, len(outer), n)]
        k = outer[g.integers(0, len(outer), n)]
        l = outer[g.integers(0, len(outer), n)]
        anti = np.arange(n) % 3 == 0                 # k = -i, l = -j
        k[anti], l[anti] = neg[i[anti]], neg[j[anti]]
        half = np.arange(n) % 3 == 1                 # k = -i only
        k[half] = neg[i[half]]
        q = _dev(np.stack([i, j, k, l], 1).astype(np.int32), torch.int32)
        m = b[k] - b[i]
        mp = b[l] - b[j]
        edge = int(((m * m).sum(1) + (mp * mp).sum(1)).max())
        t.set_direct_max(0)
        ref = t.reconstruct(q)
        t.build_values()
        got = t.reconstruct(q)
        t.sync()
    top = ref.abs().max().item()
    err = (got - ref).abs().max().item()
    assert not torch.isnan(got).any().item()
    # the oracle on every antipodal row of the first 9000 and 3000 others
    ob, oW, otau, L0 = _oracle_tables(sides, n2max, Q)
    qh = np.stack([i, j, k, l], 1).astype(np.int32)
    rows = np.concatenate([np.arange(0, 9000, 3), np.arange(1, 9000, 3)])
    oref = oracle.reconstruct(otau, oW, ob, qh[rows], L=L0)
    oerr = P.worst_cond_err(got.cpu().numpy()[rows], oref, P.cond_scale(otau, oW, ob, qh[rows], L=L0))
    say(f"[values] edge n2max={n2max} sides={sides}: max |m|^2+|m'|^2 = {edge} "
        f"(bound {8 * n2max}), max diff {err:.2e} of {top:.3g}, oracle {oerr:.2e}")
    assert edge == 8 * n2max
    assert err <= 1e-13 * top
    assert oerr < P.TOL_FP64


@pytest.mark.parametrize("n2max", [1, 2, 3, 5, 8, 12, 17, 26, 37, 50, 72, 101])
def test_values_every_cutoff_against_node_passes(pw, monkeypatch, n2max):
    """The build's block list (per pair tile, the c tiles up to its reach)
    for many cutoffs, on a cube and a box: every value a quadruple reads,
    outer shells included, equals the node passes of the same table, and a
    sample of 3000 the oracle.  The value block starts as NaN (test-only
    switch), so nothing the build skipped can be read unnoticed."""
    import torch
    monkeypatch.setenv("PWC_TEST_POISON_VALUES", "1")
    for sides in ((1.0,), (1.0, 1.2, 0.9)):
        make = (lambda: pw.Table(1.0, n2max, 32)) if len(sides) == 1 else \
            (lambda: pw.Table.box(*sides, n2max, 32))
        with make() as t:
            b = t.basis().astype(np.int64)
            r2 = (b * b).sum(1)
            g = workloads.rng(n2max)
            outer = np.flatnonzero(r2 >= max(0, r2.max() - 3))
            n = 100_000
            pick = lambda: np.where(g.uniform(size=n) < 0.5, outer[g.integers(0, len(outer), n)],
                                    g.integers(0, t.N, n))
            qh = np.stack([pick(), pick(), pick(), pick()], 1).astype(np.int32)
            q = _dev(qh, torch.int32)
            t.set_direct_max(0)
            ref = t.reconstruct(q)
            t.build_values()
            got = t.reconstruct(q)
            t.sync()
        top = ref.abs().max().item()
        assert not torch.isnan(got).any().item()
        assert (got - ref).abs().max().item() <= 1e-13 * top
        ob, oW, otau, L0 = _oracle_tables(sides, n2max, 32)
        rows = np.arange(3000)
        oref = oracle.reconstruct(otau, oW, ob, qh[rows], L=L0)
        oerr = P.worst_cond_err(got.cpu().numpy()[rows], oref, P.cond_scale(otau, oW, ob, qh[rows], L=L0))
        assert oerr < P.TOL_FP64, (sides, oerr)
