"""GPU tests of the continuous-batching server (pwc_server_*)."""
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
    return pw


def _requests(pw, keys, count, seed):
    """A seeded mix of reconstruct and energies requests over the given keys."""
    import torch
    g = workloads.rng(seed)
    reqs = []
    basis_n = {}
    for k in keys:
        with pw.Table(*k) as t:
            b = t.basis().astype(np.int64)
            basis_n[k] = (t.N, (b * b).sum(1))
    for r in range(count):
        k = keys[int(g.integers(0, len(keys)))]
        N, n2 = basis_n[k]
        prec = int(g.integers(0, 2))
        if g.uniform() < 0.7:
            n = int(np.exp(g.uniform(np.log(1e3), np.log(2e5))))
            q = torch.from_numpy(workloads.uniform_quads(N, n, seed=seed * 1000 + r)).cuda()
            reqs.append(("rec", k, prec, q, None))
        else:
            M = int((n2 <= int(g.integers(1, 10))).sum())
            occ = torch.arange(M, dtype=torch.int32, device="cuda")
            reqs.append(("ene", k, prec, occ, int(g.integers(0, 3))))
    return reqs


def _run(pw, srv, reqs, together):
    import torch
    outs, tickets = [], []
    for kind, k, prec, x, algo in reqs:
        L, n2max, Q = k
        if kind == "rec":
            out = torch.full((x.shape[0],), -1.0, dtype=torch.float64, device="cuda")
            t = srv.submit_reconstruct(L, n2max, x, out, precision=prec, n_nodes=Q)
        else:
            out = torch.full((2,), -1.0, dtype=torch.float64, device="cuda")
            t = srv.submit_energies(L, n2max, x, out, precision=prec, algo=algo, n_nodes=Q)
        outs.append(out)
        if together:
            tickets.append(t)
        else:
            res = srv.wait(t)
            assert res.status == pw.OK, res.status
    for t in tickets:
        res = srv.wait(t)
        assert res.status == pw.OK, res.status
    return [o.cpu().numpy() for o in outs]


def test_each_result_is_identical_alone_and_in_the_mix(pw):
    import torch
    keys = [(1.0, 40, 64), (2.0, 25, 48), (0.7, 64, 32), (1.4, 36, 96)]
    reqs = _requests(pw, keys, 40, seed=11)
    with pw.Server(8 << 30, max_inflight=6) as srv:
        alone = _run(pw, srv, reqs, together=False)
        srv.reset_stats()
        mixed = _run(pw, srv, reqs, together=True)
        st = srv.stats()
    say(f"[server] mix of {len(reqs)}: p50 {st['p50_ms']:.3f} ms p99 {st['p99_ms']:.3f} ms, "
        f"{st['integrals_per_s']:.3g} integrals/s, builds {st['table_builds']}, "
        f"launches {st['launches']}, batched {st['batched']}")
    assert st["batched"] > 0 and st["launches"] + st["batched"] == len(reqs)
    for a, b in zip(alone, mixed):
        assert np.array_equal(a, b)
    # and identical to the library called directly
    for (kind, k, prec, x, algo), a in list(zip(reqs, alone))[:12]:
        with pw.Table(*k) as t:
            if kind == "rec":
                d = t.reconstruct(x, precision=prec).cpu().numpy()
            else:
                d = t.energies_async(x, precision=prec, algo=algo).cpu().numpy()
            t.sync()
        assert np.array_equal(a, d)
    assert st["completed"] == len(reqs) and st["failed"] == 0
    assert st["p99_ms"] >= st["p50_ms"] > 0


def test_small_budget_queues_and_evicts_but_never_fails(pw):
    import torch
    keys = [(L, 400, 128) for L in (0.5, 0.6, 0.7, 0.85, 1.0, 1.2, 1.4, 1.7)]
    with pw.Table(*keys[0]) as t:
        tb = t.device_bytes
    budget = 3 * tb + (4 << 20)                     # three tables and the largest scratch
    assert 2 * tb < budget < len(keys) * tb        # forces eviction
    reqs = _requests(pw, keys, 18, seed=5)
    with pw.Server(8 << 30, max_inflight=4) as big:
        ref = _run(pw, big, reqs, together=False)
    with pw.Server(budget, max_inflight=4) as srv:
        got = _run(pw, srv, reqs, together=True)
        st = srv.stats()
    say(f"[server] budget {budget / 2**20:.1f} MiB, table {tb / 2**20:.1f} MiB: builds {st['table_builds']}, "
        f"evictions {st['evictions']}, resident {st['resident_bytes'] / 2**20:.1f} MiB")
    assert st["failed"] == 0 and st["completed"] == len(reqs)
    assert st["evictions"] > 0 and st["resident_bytes"] <= budget
    for a, b in zip(ref, got):
        assert np.array_equal(a, b)


def test_bad_request_inside_a_batch_fails_alone(pw):
    """One slot busy with a long request while three small ones queue: they
    share one direct launch, and the bad one fails without touching the
    others."""
    import torch
    good = torch.from_numpy(workloads.uniform_quads(123, 3000, seed=4)).cuda()
    bad = good.clone()
    bad[1234, 3] = 10 ** 6
    # long enough (about 1 ms) that the three small requests queue behind it
    big = torch.from_numpy(workloads.uniform_quads(9171, 16_000_000, seed=5)).cuda()
    big_out = torch.empty(big.shape[0], dtype=torch.float64, device="cuda")
    outs = [torch.empty(3000, dtype=torch.float64, device="cuda") for _ in range(3)]
    with pw.Server(1 << 30, max_inflight=1) as srv:
        t0 = srv.submit_reconstruct(1.0, 9, good, torch.empty_like(outs[0]), n_nodes=48)
        srv.wait(t0)                                     # the 123-PW table is resident
        tb = srv.submit_reconstruct(1.0, 169, big, big_out, n_nodes=96)   # build + 1.6e7 quads
        ts = [srv.submit_reconstruct(1.0, 9, q, o, n_nodes=48) for q, o in zip((good, bad, good), outs)]
        sts = [srv.wait(x).status for x in ts]
        assert srv.wait(tb).status == pw.OK
        st = srv.stats()
    say(f"[server] batch: launches {st['launches']}, batched {st['batched']}")
    assert sts == [pw.OK, pw.ERR_RANGE, pw.OK]
    assert st["batched"] >= 2
    with pw.Table(1.0, 9, 48) as tab:
        ref = tab.reconstruct(good).cpu().numpy()
    assert np.array_equal(outs[0].cpu().numpy(), ref) and np.array_equal(outs[2].cpu().numpy(), ref)
    got = outs[1].cpu().numpy()
    assert np.isnan(got[1234])
    keep = np.arange(3000) != 1234
    assert np.array_equal(got[keep], ref[keep])


def test_server_errors(pw):
    import torch
    q = torch.zeros((10, 4), dtype=torch.int32, device="cuda")
    out = torch.empty(10, dtype=torch.float64, device="cuda")
    with pw.Server(1 << 20, max_inflight=2) as srv:       # smaller than any 9171-PW table
        t = srv.submit_reconstruct(1.0, 169, q, out, n_nodes=96)
        assert srv.wait(t).status == pw.ERR_NOMEM
        with pytest.raises(pw.PwcError) as ei:
            srv.submit_reconstruct(1.0, 169, q, out, n_nodes=50)   # bad node count
        assert ei.value.status == pw.ERR_ARG
        with pytest.raises(pw.PwcError) as ei:
            srv.wait(987654)
        assert ei.value.status == pw.ERR_STATE
    with pw.Server(1 << 30, max_inflight=2) as srv:
        bad = torch.tensor([[0, 0, 0, 10 ** 6]], dtype=torch.int32, device="cuda")
        o1 = torch.empty(1, dtype=torch.float64, device="cuda")
        t = srv.submit_reconstruct(1.0, 9, bad, o1, n_nodes=48)
        assert srv.wait(t).status == pw.ERR_RANGE
        assert np.isnan(o1.cpu().numpy()[0])
        occ = torch.arange(7, dtype=torch.int32, device="cuda")
        e = torch.empty(2, dtype=torch.float64, device="cuda")
        t = srv.submit_energies(1.0, 600, occ, e, algo=pw.PAIR_KTABLE, n_nodes=16)
        assert srv.wait(t).status == pw.ERR_ARG


def test_box_requests_match_the_library(pw):
    """Requests on rectangular boxes (L = (Lx, Ly, Lz)) share the queue with
    cubes, get their own cached tables and give the library's results."""
    import torch
    box, cube = (1.0, 1.3, 0.8), 1.0
    q = torch.from_numpy(workloads.uniform_quads(1045, 40_000, seed=12)).cuda()
    outs = {k: torch.empty(40_000, dtype=torch.float64, device="cuda") for k in ("box", "cube")}
    occ = torch.arange(123, dtype=torch.int32, device="cuda")
    e_box = torch.empty(2, dtype=torch.float64, device="cuda")
    with pw.Server(1 << 30, max_inflight=2) as srv:
        ts = [srv.submit_reconstruct(box, 40, q, outs["box"], n_nodes=64),
              srv.submit_reconstruct(cube, 40, q, outs["cube"], n_nodes=64),
              srv.submit_energies(box, 40, occ, e_box, n_nodes=64)]
        assert all(srv.wait(t).status == pw.OK for t in ts)
        assert srv.stats()["table_builds"] == 2
    with pw.Table.box(*box, 40, 64) as tb, pw.Table(cube, 40, 64) as tc:
        assert torch.equal(outs["box"], tb.reconstruct(q))
        assert torch.equal(outs["cube"], tc.reconstruct(q))
        assert np.array_equal(e_box.cpu().numpy(), np.array(tb.energies(occ)))
        assert not torch.equal(outs["box"], outs["cube"])


def test_bad_request_beside_a_good_one_on_the_same_table(pw):
    """Two node-pass requests (above the largest direct-kernel size) on one
    table run in two slots at once; the one with a bad index fails and the
    other does not, as each slot raises its own error word.  The fused node
    sums pair a wave's 512 quadruples of a chunk together, so the bad one
    moves the others of its wave to other lanes: those may differ from the
    good request's by the rounding of their node terms' order, the rest not
    at all."""
    import torch
    n = 1_100_000
    good_h = workloads.uniform_quads(1045, n, seed=21)
    good = torch.from_numpy(good_h).cuda()
    bad = good.clone()
    bad[n // 2, 0] = -5
    outs = [torch.empty(n, dtype=torch.float64, device="cuda") for _ in range(4)]
    occ = torch.arange(123, dtype=torch.int32, device="cuda")
    occ_bad = occ.clone()
    occ_bad[7] = 5000
    e_good = torch.empty(2, dtype=torch.float64, device="cuda")
    e_bad = torch.empty(2, dtype=torch.float64, device="cuda")
    with pw.Server(1 << 30, max_inflight=4) as srv:
        ts = [srv.submit_reconstruct(1.0, 40, q, o, n_nodes=64)
              for q, o in zip((bad, good, bad, good), outs)]
        te = [srv.submit_energies(1.0, 40, x, e, n_nodes=64, algo=pw.PAIR_NODESUM)
              for x, e in ((occ_bad, e_bad), (occ, e_good))]
        sts = [srv.wait(x).status for x in ts]
        ste = [srv.wait(x).status for x in te]
    assert sts == [pw.ERR_RANGE, pw.OK, pw.ERR_RANGE, pw.OK]
    assert ste == [pw.ERR_RANGE, pw.OK]
    with pw.Table(1.0, 40, 64) as tab:
        ref = tab.reconstruct(good).cpu().numpy()
        e_ref = np.array(tab.energies(occ, algo=pw.PAIR_NODESUM))
    assert np.array_equal(outs[1].cpu().numpy(), ref) and np.array_equal(outs[3].cpu().numpy(), ref)
    got = outs[0].cpu().numpy()
    assert np.isnan(got[n // 2])
    moved = np.nonzero((got != ref) & (np.arange(n) != n // 2))[0]
    assert len(moved) < 512
    o = P.setup(40, 64)
    scale = P.cond_scale(o["tau"], o["W"], o["basis"], good_h[moved])
    assert np.all(np.abs(got[moved] - ref[moved]) <= 1e-14 * scale)
    assert np.array_equal(e_good.cpu().numpy(), e_ref)


def test_two_waiters_on_one_ticket(pw):
    """A ticket is collected once; a second thread waiting on it returns
    ERR_STATE instead of waiting forever."""
    import threading
    import torch
    q = torch.from_numpy(workloads.uniform_quads(123, 1000, seed=3)).cuda()
    out = torch.empty(1000, dtype=torch.float64, device="cuda")
    got = []
    with pw.Server(1 << 30, max_inflight=1) as srv:
        t = srv.submit_reconstruct(1.0, 9, q, out, n_nodes=48)

        def waiter():
            try:
                got.append(srv.wait(t).status)
            except pw.PwcError as e:
                got.append(e.status)

        th = [threading.Thread(target=waiter) for _ in range(2)]
        for x in th:
            x.start()
        for x in th:
            x.join(timeout=60)
        assert not any(x.is_alive() for x in th)
    assert sorted(got) == sorted([pw.OK, pw.ERR_STATE])


def _oracle_key(key):
    """Oracle basis, weights, tables and reference length of a serving key
    (sides, n2max, mesh spec): a cube or a box, the default beta-mesh or a
    literal alpha_c (beta_c = 4 alpha_c / L0^2)."""
    sides, n2max, spec = key
    b = oracle.enumerate_basis(n2max)
    K = 2 * math.isqrt(n2max)
    L0 = float(np.prod(sides) ** (1.0 / 3.0)) if len(sides) == 3 else sides[0]
    kind, q, qt, alpha_c = spec
    beta_c = 4.0 * alpha_c / (L0 * L0) if alpha_c > 0 else 1.0
    if kind == "geometric":
        beta, W, _ = oracle.mesh2(q, qt, beta_c=beta_c)
    else:
        beta, W, _ = oracle.mesh1(q, beta_c=beta_c)
    if len(sides) == 3:
        L0, _, tau = oracle.box_tables(beta, K, sides)
    else:
        tau = oracle.tau_table(beta, K)
    return b, W, tau, L0


def test_served_outputs_match_the_oracle(pw):
    """What the server returns, against the FP64 oracle: reconstructions on
    the direct kernel (batched) and on the node passes, and energies with
    every pair algorithm, in both precisions, on a cube with the default
    mesh, a cube with a literal alpha_c, a box and a two-interval mesh, all
    submitted together so that they share slots and launches."""
    import torch
    keys = [((1.0,), 40, ("geometric", 7, 8, 0.0)),
            ((1.3,), 25, ("geometric", 5, 8, 0.25)),
            ((1.0, 1.3, 0.8), 25, ("geometric", 5, 8, 0.0)),
            ((0.8,), 16, ("two_interval", 24, 24, 0.0))]
    jobs = []
    g = workloads.rng(2015)
    for key in keys:
        sides, n2max, (kind, q, qt, alpha_c) = key
        mesh = (pw.Mesh.geometric(q, qt, alpha_c=alpha_c) if kind == "geometric"
                else pw.Mesh.two_interval(q, qt, alpha_c=alpha_c))
        b, W, tau, L0 = _oracle_key(key)
        N = len(b)
        L = sides if len(sides) == 3 else sides[0]
        r2 = (b.astype(np.int64) ** 2).sum(1)
        M = int((r2 <= 4).sum())
        f = g.uniform(0.25, 1.0, M)
        for prec in (pw.FP64, pw.MIXED, pw.FP32):
            for n in (3001, 40_000, 1_100_000):            # two direct sizes, one above any
                quads = workloads.lookup_stream(N, M, n, seed=int(g.integers(1 << 30)))
                jobs.append(("rec", key, L, mesh, prec, quads, None))
            if prec == pw.FP32:
                continue                                   # reconstruction only
            for algo in (pw.PAIR_AUTO, pw.PAIR_NODESUM):
                jobs.append(("ene", key, L, mesh, prec, np.arange(M, dtype=np.int32), (algo, f)))
    # Inputs staged first, so that the requests go in back to back and queue.
    staged = []
    for kind, key, L, mesh, prec, x, extra in jobs:
        dx = torch.from_numpy(x).cuda()
        fd = torch.from_numpy(extra[1]).cuda() if kind == "ene" else None
        out = torch.full((len(x) if kind == "rec" else 2,), -1.0, dtype=torch.float64, device="cuda")
        staged.append((dx, fd, out))
    torch.cuda.synchronize()
    outs = [o for _, _, o in staged]
    tickets = []
    with pw.Server(2 << 30, max_inflight=6) as srv:
        # Every table resident first: queued small reconstructions then join
        # the direct launch of the one at the head of the queue.
        warm = {}
        for (kind, key, L, mesh, prec, x, extra), (dx, _, _) in zip(jobs, staged):
            if kind == "rec" and key not in warm:
                warm[key] = srv.submit_reconstruct(L, key[1], dx[:64].clone(),
                                                   torch.empty(64, dtype=torch.float64, device="cuda"),
                                                   mesh=mesh)
        assert all(srv.wait(t).status == pw.OK for t in warm.values())
        for (kind, key, L, mesh, prec, x, extra), (dx, fd, out) in zip(jobs, staged):
            if kind == "rec":
                tickets.append(srv.submit_reconstruct(L, key[1], dx, out, precision=prec, mesh=mesh))
            else:
                tickets.append(srv.submit_energies(L, key[1], dx, out, f=fd, precision=prec,
                                                   algo=extra[0], mesh=mesh))
        results = [srv.wait(t) for t in tickets]
        st = srv.stats()
    assert all(r.status == pw.OK for r in results)
    assert st["batched"] > 0
    worst = {}
    for (kind, key, L, mesh, prec, x, extra), out, res in zip(jobs, outs, results):
        b, W, tau, L0 = _oracle_key(key)
        got = out.cpu().numpy()
        if kind == "rec":
            rows = np.arange(0, len(x), 1 if len(x) <= 40_000 else 7)   # every 7th of the long ones
            ref = oracle.reconstruct(tau, W, b, x[rows], L=L0)
            err = P.worst_cond_err(got[rows], ref, P.cond_scale(tau, W, b, x[rows], L=L0))
            tol = {pw.FP64: P.TOL_FP64, pw.MIXED: P.TOL_MIXED, pw.FP32: P.TOL_FP32}[prec]
            assert err < tol, (key, prec, len(x), err)
        else:
            eh, ex = oracle.energies(tau, W, b, x, f=extra[1], L=L0)
            err = max(abs(got[0] - eh) / abs(eh), abs(got[1] - ex) / abs(ex))
            assert err < (P.TOL_E_FP64 if prec == pw.FP64 else P.TOL_E_MIXED), (key, prec, err)
            assert res.e_h == got[0] and res.e_x == got[1]
        k = (kind, str(key[0]), prec)
        worst[k] = max(worst.get(k, 0.0), err)
    say("[server] served vs oracle: " + ", ".join(f"{k}: {v:.1e}" for k, v in sorted(worst.items())))


def test_scratch_is_priced_by_the_path_taken(pw):
    """Admission prices each request's device scratch from the kernels it
    will run on its table: the node-sum pair partials grow as (M/32)^2
    (1.3 MB at M = 9171), the kernel-table ones stay small, the direct
    kernel and the fused node sums of the cube need none, and the node passes of a box (2187 folded rows: no fused schedule)
    need the decoded stream, 8 bytes per quadruple.  With a budget of the table plus 0.6 MB,
    what cannot fit beside the table fails with ERR_NOMEM at once and the
    rest runs; with more it all runs, and the results are the library's."""
    import torch
    pw.release_cached_memory()                 # no recycled (larger) blocks
    key = (1.0, 169, 64)                      # FP64 node sums: fused
    with pw.Table(*key) as t:
        tb = t.device_bytes
        occ = torch.arange(t.N, dtype=torch.int32, device="cuda")
        e_node = np.array(t.energies(occ, algo=pw.PAIR_NODESUM))
        e_kt = np.array(t.energies(occ, algo=pw.PAIR_KTABLE))
        small = torch.from_numpy(workloads.uniform_quads(t.N, 10_000, seed=8)).cuda()
        big = torch.from_numpy(workloads.uniform_quads(t.N, 1_000_000, seed=9)).cuda()
        r_small = t.reconstruct(small)
        t.set_direct_max(0)
        r_big = t.reconstruct(big)
        t.sync()

    def run(budget):
        outs = {k: torch.full((2,), -1.0, dtype=torch.float64, device="cuda") for k in ("node", "kt")}
        o_small = torch.empty(10_000, dtype=torch.float64, device="cuda")
        o_big = torch.empty(1_000_000, dtype=torch.float64, device="cuda")
        with pw.Server(budget, max_inflight=2) as srv:
            ts = {"kt": srv.submit_energies(*key[:2], occ, outs["kt"], algo=pw.PAIR_KTABLE, n_nodes=key[2]),
                  "node": srv.submit_energies(*key[:2], occ, outs["node"], algo=pw.PAIR_NODESUM,
                                              n_nodes=key[2]),
                  "small": srv.submit_reconstruct(*key[:2], small, o_small, n_nodes=key[2]),
                  "big": srv.submit_reconstruct(*key[:2], big, o_big, n_nodes=key[2])}
            st = {k: srv.wait(v).status for k, v in ts.items()}
        return st, outs, o_small, o_big

    st, outs, o_small, o_big = run(tb + 600_000)
    say(f"[server] table {tb} B + 0.6 MB: {st}")
    assert st == {"kt": pw.OK, "node": pw.ERR_NOMEM, "small": pw.OK, "big": pw.OK}
    assert np.array_equal(outs["kt"].cpu().numpy(), e_kt)
    assert torch.equal(o_small, r_small) and torch.equal(o_big, r_big)
    st, outs, o_small, o_big = run(tb + 6_000_000)
    assert all(v == pw.OK for v in st.values()), st
    assert np.array_equal(outs["node"].cpu().numpy(), e_node)
    assert np.array_equal(outs["kt"].cpu().numpy(), e_kt)
    assert torch.equal(o_big, r_big) and torch.equal(o_small, r_small)

    # The box's node passes keep the decoded stream: 8.8 MB for 1.1e6
    # quadruples (above the largest direct-kernel size).
    sides = (1.0, 1.3, 0.8)
    pw.release_cached_memory()
    with pw.Table.box(*sides, 169, 64) as t:
        tbb = t.device_bytes
        big_box = torch.from_numpy(workloads.uniform_quads(t.N, 1_100_000, seed=10)).cuda()
        r_box = t.reconstruct(big_box)
        t.sync()
    for budget, status in ((tbb + 600_000, pw.ERR_NOMEM), (tbb + 12_000_000, pw.OK)):
        o_box = torch.full((1_100_000,), -1.0, dtype=torch.float64, device="cuda")
        with pw.Server(budget, max_inflight=2) as srv:
            got = srv.wait(srv.submit_reconstruct(sides, 169, big_box, o_box, n_nodes=64)).status
        say(f"[server] box table {tbb} B + {budget - tbb} B: {got}")
        assert got == status
        if status == pw.OK:
            assert torch.equal(o_box, r_box)


def test_eviction_does_not_wait_for_other_tables(pw):
    """A table released while a long reconstruction on another table is in
    flight returns without waiting for it (its blocks wait for their own
    streams' events instead), and a new table reuses the released block only
    once the work that read it is done: results stay bitwise those of a
    quiet device."""
    import time
    import torch
    pw.release_cached_memory()
    gen = torch.Generator(device="cuda").manual_seed(5)
    big = torch.randint(0, 9171, (60_000_000, 4), dtype=torch.int32, device="cuda", generator=gen)
    q = torch.from_numpy(workloads.uniform_quads(1045, 200_000, seed=6)).cuda()
    with pw.Table(1.0, 169, 96) as slow, pw.Table(1.0, 40, 64) as ref_t:
        ref_t.set_direct_max(0)
        ref = ref_t.reconstruct(q)
        slow.set_direct_max(0)
        torch.cuda.synchronize()
        side = torch.cuda.Stream()
        with torch.cuda.stream(side):
            out_big = slow.reconstruct(big, precision=pw.MIXED)   # a few ms of node passes
        t = pw.Table(1.0, 40, 64)
        t.set_direct_max(0)
        got = t.reconstruct(q)
        t0 = time.perf_counter()
        t.close()                                   # releases its block behind the default stream
        dt = time.perf_counter() - t0
        busy = not side.query()
        u = pw.Table(1.0, 40, 64)                   # same size: may take the released block
        u.set_direct_max(0)
        again = u.reconstruct(q)
        u.sync()
        torch.cuda.synchronize()
        u.close()
        slow.sync(side)
    say(f"[server] release took {dt * 1e3:.3f} ms with the side stream busy={busy}")
    assert torch.equal(got, ref) and torch.equal(again, ref)
    assert not torch.isnan(out_big).any().item()
    if busy:
        assert dt < 2e-3
