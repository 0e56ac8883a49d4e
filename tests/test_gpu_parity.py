"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle."""
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


@pytest.fixture(scope="module")
def tables(pw):
    made = {}

    def get(n2max, n_nodes, L=1.0):
        key = (n2max, n_nodes, L)
        if key not in made:
            say(f"[parity] table n2max={n2max} Q={n_nodes} L={L}")
            made[key] = pw.Table(L, n2max, n_nodes)
        return made[key]
    yield get
    for t in made.values():
        t.close()


# ---------------------------------------------------------------- tables ----

@pytest.mark.parametrize("n2max,Q", [(2, 16), (9, 48), (40, 64), (169, 96), (400, 128)])
def test_tables_basis_mesh_match_oracle(pw, tables, n2max, Q):
    t = tables(n2max, Q)
    o = P.setup(n2max, Q)
    assert np.array_equal(t.basis(), o["basis"])
    beta, W = t.mesh_nodes()
    # both sides round an extended-precision rule once: agreement to an ulp or two
    assert np.max(np.abs(beta - o["beta"]) / o["beta"]) < 5e-16
    assert np.max(np.abs(W - o["W"]) / o["W"]) < 5e-16
    tau = t.copy_tables().cpu().numpy()
    assert tau.shape == o["tau"].shape
    scale = np.abs(o["tau"]).max(axis=(1, 2))
    err = (np.abs(tau - o["tau"]).max(axis=(1, 2)) / scale).max()
    say(f"[parity] tables n2max={n2max} Q={Q}: worst err / node max = {err:.2e}")
    assert err < P.TOL_TABLE


@pytest.mark.parametrize("kind", ["two_interval", "fixed_alpha"])
def test_tables_other_meshes(pw, kind):
    if kind == "two_interval":
        m = pw.Mesh.two_interval(20)
        o = P.setup(9, mesh=("two_interval", 20))
        L = 1.0
    else:
        L = 2.0
        m = pw.Mesh.geometric(5, 8, alpha_c=0.25)       # beta_c = 4 alpha_c / L^2 = 0.25
        o = P.setup(9, mesh=("geometric", 5, 8), beta_c=0.25)
    with pw.Table(L, 9, 0, mesh=m) as t:
        beta, W = t.mesh_nodes()
        assert np.max(np.abs(beta - o["beta"]) / o["beta"]) < 5e-16
        assert np.max(np.abs(W - o["W"]) / o["W"]) < 5e-16
        tau = t.copy_tables().cpu().numpy()
        scale = np.abs(o["tau"]).max(axis=(1, 2))
        assert (np.abs(tau - o["tau"]).max(axis=(1, 2)) / scale).max() < P.TOL_TABLE


@pytest.mark.parametrize("n2max,spec", [(169, (8, 4, 4, 7.0)), (40, (5, 3, 6, 5.0)), (9, (3, 2, 3, 10.0))])
def test_root_mesh_tables_integrals_energies(pw, n2max, spec):
    """Mesh 3 (GEOMETRIC_ROOT): mesh, tables, integrals on every path (direct
    kernel, node passes, value table; both precisions) and energies (both pair
    algorithms and precisions) against the oracle on the same mesh."""
    import torch
    q, qt, n_sub, ratio = spec
    o = P.setup(n2max, mesh=("root", q, qt, n_sub, ratio))
    m = pw.Mesh.geometric_root(q, qt, n_sub=n_sub, ratio=ratio)
    N = len(o["basis"])
    M = int(((o["basis"].astype(np.int64) ** 2).sum(1) <= min(n2max, 36)).sum())
    with pw.Table(1.0, n2max, 0, mesh=m) as t:
        beta, W = t.mesh_nodes()
        assert np.max(np.abs(beta - o["beta"]) / o["beta"]) < 5e-16
        assert np.max(np.abs(W - o["W"]) / o["W"]) < 5e-16
        tau = t.copy_tables().cpu().numpy()
        scale = np.abs(o["tau"]).max(axis=(1, 2))
        assert (np.abs(tau - o["tau"]).max(axis=(1, 2)) / scale).max() < P.TOL_TABLE
        quads = workloads.lookup_stream(N, M, 700_001, seed=n2max)
        rows = workloads.sample_rows(len(quads), 20_000, seed=2)
        t.set_direct_max(0)
        _check_reconstruct(pw, t, o, quads[rows], label=f"root mesh passes {n2max}")
        t.set_direct_max(1 << 19)
        _check_reconstruct(pw, t, o, quads[rows], label=f"root mesh direct {n2max}")
        t.build_values()
        got = t.reconstruct(_dev(quads, torch.int32)).cpu().numpy()[rows]
        t.sync()
        ref = oracle.reconstruct(o["tau"], o["W"], o["basis"], quads[rows])
        err = P.worst_cond_err(got, ref, P.cond_scale(o["tau"], o["W"], o["basis"], quads[rows]))
        assert err < P.TOL_FP64, err
        occ = np.arange(M, dtype=np.int32)
        f = workloads.occupations(M, seed=5)
        eh, ex = oracle.energies(o["tau"], o["W"], o["basis"], occ, f)
        for prec in (pw.FP64, pw.MIXED):
            for algo in (pw.PAIR_KTABLE, pw.PAIR_NODESUM):
                gh, gx = t.energies(_dev(occ, torch.int32), _dev(f, torch.float64), precision=prec, algo=algo)
                assert abs(gh - eh) < P.TOL_E_FP64 * eh and abs(gx - ex) < P.TOL_E_FP64 * abs(ex)


def test_root_mesh_table_one_converged_ratio(pw):
    """Sec. III, Table I: E_x/E_KS at M = 9171 from a 36-node Mesh 3 on the
    GPU, within the printed precision of the converged 0.965431 and within
    1e-12 of the oracle's histogram route on the same mesh."""
    import json
    import os
    import torch
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "table1.json")))
    b = oracle.enumerate_basis(169)
    h, R = oracle.diff_histogram(b)
    beta, W, _ = oracle.mesh3(8, 4, n_sub=4, ratio=7.0)
    ref = oracle.exchange_from_histogram(h, R, oracle.tau_diag(beta, 2 * R), W)
    occ = torch.arange(len(b), dtype=torch.int32, device="cuda")
    with pw.Table(1.0, 169, 0, mesh=pw.Mesh.geometric_root(8, 4, n_sub=4, ratio=7.0)) as t:
        for prec in (pw.FP64, pw.MIXED):
            for algo in (pw.PAIR_KTABLE, pw.PAIR_NODESUM):
                _, ex = t.energies(occ, precision=prec, algo=algo)
                assert abs(ex - ref) < 1e-12 * abs(ref)
                assert abs(ex / oracle.e_ks(len(b)) - g["mesh2"]["10"][1]) < 1.5e-6


# ------------------------------------------------------------ integrals ----

def _check_reconstruct(pw, t, o, quads, L=1.0, label=""):
    import torch
    dq = _dev(quads, torch.int32)
    ref = oracle.reconstruct(o["tau"], o["W"], o["basis"], quads, L=L)
    scale = P.cond_scale(o["tau"], o["W"], o["basis"], quads, L=L)
    errs = {}
    for prec, tol in ((pw.FP64, P.TOL_FP64), (pw.MIXED, P.TOL_MIXED), (pw.FP32, P.TOL_FP32)):
        out = t.reconstruct(dq, precision=prec)
        t.sync()
        got = out.cpu().numpy()
        errs[prec] = P.worst_cond_err(got, ref, scale)
        assert errs[prec] < tol, (label, prec, errs[prec])
    say(f"[parity] reconstruct {label}: n={len(quads)} fp64 {errs[pw.FP64]:.2e} "
        f"mixed {errs[pw.MIXED]:.2e} fp32 {errs[pw.FP32]:.2e} (condition-aware)")
    return errs


@pytest.mark.parametrize("path", ["direct", "passes"])
def test_reconstruct_plain_all_occupied_quadruples(pw, tables, path):
    w = workloads.C1_PLAIN
    t = tables(w.n2max, w.n_nodes)
    o = P.setup(w.n2max, w.n_nodes)
    M = int((np.asarray(o["basis"]) ** 2).sum(1).__le__(w.n2occ).sum())
    assert M == 19
    t.set_direct_max(DIRECT_DEFAULT if path == "direct" else 0)
    try:
        _check_reconstruct(pw, t, o, workloads.all_quads(M), label=f"19^4 (123 PW, Q=48) {path}")
    finally:
        t.set_direct_max(DIRECT_DEFAULT)


DIRECT_DEFAULT = 1 << 19

# The two schedules of the node sums against each other, condition-aware:
# the fused launch deals a chunk's quadruples to lanes wave-wide when it has
# several node ranges, the separate launches slot by slot.  A lane's
# position sets the order in which it adds a range's words, and the high
# lane of a pair reads the quadruple's rows in reverse order, which
# reassociates each node's triple product (two roundings on either side)
# and the word sums that follow.  FP64: a few units of 2^-53 of the sum of
# the terms' magnitudes (1e-14 leaves room); float-float: of 2^-48;
# single FP32: products and the pairwise word sum, at most 4 roundings of
# 2^-24 on either side, 8 * 2^-24 = 4.8e-7.  With one range the dealing is
# the same, and so are the bits.
SCHEDULE_TOL = {"fp64": 1e-14, "fp32": 4.8e-7, "mixed": 2e-13}


def _same_sums(a, b, o, quads, name, ranges, L=1.0):
    import torch
    if ranges == 1:
        assert torch.equal(a, b), name
        return
    scale = P.cond_scale(o["tau"], o["W"], o["basis"], quads, L=L)
    d = (a - b).abs().cpu().numpy()
    assert np.all(d <= SCHEDULE_TOL[name] * scale), (name, float((d / scale).max()))


@pytest.mark.parametrize("path", ["direct", "passes"])
@pytest.mark.parametrize("n", [1, 2, 255, 1023, 1024, 1025, 2047, 2048, 2049, 4097, 30001])
def test_reconstruct_ragged_sizes(pw, tables, n, path):
    """Sizes around the tiles of both reconstruction paths (one lane per
    quadruple in one launch; node passes over the padded stream)."""
    w = workloads.C2_SPLIT
    t = tables(w.n2max, w.n_nodes)
    o = P.setup(w.n2max, w.n_nodes)
    t.set_direct_max(DIRECT_DEFAULT if path == "direct" else 0)
    try:
        _check_reconstruct(pw, t, o, workloads.uniform_quads(len(o["basis"]), n, seed=n),
                           label=f"ragged n={n} {path}")
    finally:
        t.set_direct_max(DIRECT_DEFAULT)


@pytest.mark.parametrize("n2max,Q", [(9, 48), (40, 64), (169, 96), (400, 128)])
def test_direct_and_node_passes_agree(pw, n2max, Q):
    """The direct kernel (small lists) and the node passes on the same
    quadruples, both against the oracle and against each other."""
    import torch
    o = P.setup(n2max, Q)
    with pw.Table(1.0, n2max, Q) as t:
        quads = workloads.uniform_quads(len(o["basis"]), 20000, seed=Q)
        dq = _dev(quads, torch.int32)
        out = {}
        for path, m in (("direct", DIRECT_DEFAULT), ("passes", 0)):
            t.set_direct_max(m)
            _check_reconstruct(pw, t, o, quads, label=f"n2max={n2max} Q={Q} {path}")
            for prec in (pw.FP64, pw.MIXED, pw.FP32):
                out[path, prec] = t.reconstruct(dq, precision=prec)
        t.sync()
        for prec, tol in ((pw.FP64, 1e-13), (pw.MIXED, 1e-12), (pw.FP32, 1e-6)):
            a, b = out["direct", prec], out["passes", prec]
            assert (a - b).abs().max().item() <= tol * b.abs().max().item()
        with pytest.raises(pw.PwcError):
            t.set_direct_max((1 << 20) + 1)


def test_reconstruct_profile_matches_and_times_every_launch(pw, tables):
    import torch
    t = tables(169, 96)
    q = _dev(workloads.lookup_stream(9171, 925, 300000, 3), torch.int32)
    t.set_direct_max(0)                 # the profile entry point always runs the node passes
    try:
        ref = t.reconstruct(q)
    finally:
        t.set_direct_max(DIRECT_DEFAULT)
    out, ms = t.reconstruct_profile(q)
    lay = t.layout()
    _same_sums(out, ref, P.setup(169, 96), q.cpu().numpy(), "fp64", lay["passes"])
    assert lay["passes"] == -(-96 // lay["nodes_per_pass"])
    assert len(ms) == 1 + lay["passes"] and np.all(ms > 0)


ALL_LAYOUTS = [(16, 1), (8, 2), (8, 1), (4, 2), (2, 4), (1, 8), (4, 1)]
C16 = [(8, 1), (4, 2), (2, 4), (1, 8)]             # 16 nodes per pass
# (n2max, Q, default (lanes, words) for FP64 and for split-FP32, bytes per
#  decoded quadruple, layouts whose slab fits)
LAYOUTS = [
    (40, 64, (1, 8), (1, 8), 4, ALL_LAYOUTS),
    (169, 96, (1, 8), (1, 8), 4, C16 + [(4, 1)]),
    (256, 32, (1, 8), (2, 4), 8, C16 + [(4, 1)]),
    (400, 128, (4, 1), (4, 1), 8, [(4, 1)]),
]


@pytest.mark.parametrize("n2max,Q,d64,dmx,eb,fits", LAYOUTS)
def test_reconstruct_every_lane_layout(pw, n2max, Q, d64, dmx, eb, fits):
    """Every lane layout and both packed-entry widths against the oracle, on
    a ragged uniform stream, and the layouts against each other."""
    import torch
    o = P.setup(n2max, Q)

    def lanes_words(t, prec):
        lay = t.layout(prec)
        return lay["lanes"], lay["words"]
    with pw.Table(1.0, n2max, Q) as t:
        t.set_direct_max(0)                             # node passes at every size
        assert (lanes_words(t, pw.FP64), lanes_words(t, pw.MIXED)) == (d64, dmx)
        assert t.layout(pw.FP64)["entry_bytes"] == t.layout(pw.MIXED)["entry_bytes"] == eb
        quads = workloads.uniform_quads(len(o["basis"]), 50001, seed=n2max)
        dq = _dev(quads, torch.int32)
        base = {}
        for G, W in fits:
            t.set_layout(G, W)
            for prec, npw in ((pw.FP64, 2), (pw.MIXED, 2), (pw.FP32, 4)):
                lay = t.layout(prec)
                if prec == pw.FP32 and -(-Q // (npw * G * W)) * npw * G * W > -(-Q // 32) * 32:
                    continue   # its passes would run past the padded rows: FP32 keeps its default
                assert (lay["lanes"], lay["words"]) == (G, W)
                assert lay["nodes_per_pass"] == npw * G * W
                assert lay["passes"] == -(-Q // (npw * G * W))
            for prec in (pw.FP64, pw.MIXED, pw.FP32):
                lay = t.layout(prec)
                assert not t.fused(prec) or (lay["lanes"], lay["words"]) == (1, 8)
            _check_reconstruct(pw, t, o, quads, label=f"n2max={n2max} Q={Q} layout={G}x{W}")
            for prec in (pw.FP64, pw.MIXED, pw.FP32):
                out = t.reconstruct(dq, precision=prec)
                t.sync()
                if prec in base:   # layouts differ only in rounding order
                    tol = {pw.FP64: 1e-13, pw.MIXED: 1e-12, pw.FP32: 1e-6}[prec]
                    assert (out - base[prec]).abs().max().item() <= tol * base[prec].abs().max().item()
                else:
                    base[prec] = out
        for G, W in set(ALL_LAYOUTS) - set(fits):
            with pytest.raises(pw.PwcError) as ei:
                t.set_layout(G, W)
            assert ei.value.status == pw.ERR_RANGE
        with pytest.raises(pw.PwcError) as ei:
            t.set_layout(16, 2)
        assert ei.value.status == pw.ERR_ARG
        t.set_layout(0, 0)
        assert (lanes_words(t, pw.FP64), lanes_words(t, pw.MIXED)) == (d64, dmx)
        # the 9171-planewave table (729 folded rows) runs every precision
        # fused; tables with more than 1024 rows never do
        if n2max == 169:
            assert all(t.fused(p) for p in (pw.FP64, pw.MIXED, pw.FP32))
        if t.layout(pw.FP64)["entry_bytes"] == 8:
            assert not any(t.fused(p) for p in (pw.FP64, pw.MIXED, pw.FP32))


# Meshes whose last node range is short in the fused one-lane schedule:
# (mesh spec, Q, {precision: (fused, words of the last range)}).  FP64 and
# split FP32 take 16 nodes a range, single FP32 32.
SHORT_RANGES = [
    (("root", 16, 4, 4, 7.0), 68, {"fp64": (True, 2), "fp32": (True, 1)}),
    (("root", 16, 2, 4, 7.0), 66, {"fp64": (True, 1), "fp32": (True, 1)}),
    (("geometric", 8, 8), 72, {"fp64": (True, 4), "fp32": (True, 2)}),
    (("root", 1, 4, 4, 7.0), 8, {"fp64": (True, 4), "fp32": (True, 2)}),
    (("root", 24, 4, 4, 7.0), 100, {"fp64": (True, 2), "fp32": (True, 1)}),
]


@pytest.mark.parametrize("mesh,Q,expect", SHORT_RANGES)
def test_fused_short_last_range(pw, mesh, Q, expect):
    """The fused schedule reads only the real words of a short last node
    range (1, 2 or 4 of 8): the separate launches' sums (which read the zero
    padding too) to the rounding of the word order, bit for bit with one
    range, and within the bar of the oracle, in all three
    arithmetics, on a ragged stream."""
    import torch
    n2max = 25
    o = P.setup(n2max, mesh=mesh)
    assert len(o["W"]) == Q
    kind, args = mesh[0], mesh[1:]
    m = pw.Mesh.geometric_root(*args) if kind == "root" else pw.Mesh.geometric(*args)
    quads = workloads.uniform_quads(len(o["basis"]), 30001, seed=Q)
    dq = _dev(quads, torch.int32)
    with pw.Table(1.0, n2max, mesh=m) as t:
        assert t.Q == Q
        t.set_direct_max(0)
        t.set_layout(1, 8)
        for name, prec in (("fp64", pw.FP64), ("mixed", pw.MIXED), ("fp32", pw.FP32)):
            fused, _ = expect["fp64" if name == "mixed" else name]
            assert t.fused(prec) == fused, (name, t.layout(prec))
            a = t.reconstruct(dq, precision=prec)
            b, _ = t.reconstruct_profile(dq, precision=prec)
            t.sync()
            _same_sums(a, b, o, quads, name, t.layout(prec)["passes"])
        _check_reconstruct(pw, t, o, quads, label=f"Q={Q} short last range")
        t.set_layout(0, 0)


# A table whose fused slab takes 8 staged words per lane: 841 folded rows at
# n2max = 200, the decode maps still beside them in LDS.  One range and
# several, full and short last ranges, in the three arithmetics:
# Q: {precision: (node ranges, words of the last range)}.
EIGHT_WORD = {
    16: {"fp64": (1, 8), "fp32": (1, 4)},
    72: {"fp64": (5, 4), "fp32": (3, 2)},
    96: {"fp64": (6, 8), "fp32": (3, 8)},
}


@pytest.mark.parametrize("Q", sorted(EIGHT_WORD))
def test_fused_eight_word_slab(pw, Q):
    """The fused kernels that stage 8 slab words per lane (and hold 6
    quadruples per lane, not 8): the separate launches' sums to the rounding
    of the word order (bit for bit with one range), and within the bar of
    the oracle, on a ragged stream."""
    import torch
    n2max = 200
    o = P.setup(n2max, Q)
    quads = workloads.uniform_quads(len(o["basis"]), 30001, seed=Q + 200)
    dq = _dev(quads, torch.int32)
    with pw.Table(1.0, n2max, Q) as t:
        t.set_direct_max(0)
        t.set_layout(1, 8)
        for name, prec in (("fp64", pw.FP64), ("mixed", pw.MIXED), ("fp32", pw.FP32)):
            ranges, words = EIGHT_WORD[Q]["fp64" if name == "mixed" else name]
            lay = t.layout(prec)
            assert t.fused(prec) and lay["passes"] == ranges, (name, lay)
            npw = 4 if name == "fp32" else 2   # nodes per 16-byte word
            last = Q - (ranges - 1) * 8 * npw
            assert min(w for w in (1, 2, 4, 8) if w * npw >= last) == words
            a = t.reconstruct(dq, precision=prec)
            b, _ = t.reconstruct_profile(dq, precision=prec)
            t.sync()
            _same_sums(a, b, o, quads, name, ranges)
        _check_reconstruct(pw, t, o, quads, label=f"n2max=200 Q={Q} eight-word slab")
        t.set_layout(0, 0)


@pytest.mark.parametrize("kind", ["diagonal", "half_diagonal", "one_quadruple"])
def test_fused_pairing_with_skewed_classes(pw, tables, kind):
    """Streams whose classes cannot be paired: every (i, i, i, i) reads the
    folded row of m = m' = 0 three times, so all its quadruples share one
    parity class; half the stream such; one quadruple repeated.  The fused
    node sums then deal many or all of a chunk's quadruples as left over,
    and each result must still be its own quadruple's: against the oracle,
    and against the separate launches within the rounding of the order of
    the node terms, in all three arithmetics, on a ragged stream."""
    import torch
    t = tables(169, 96)
    o = P.setup(169, 96)
    n = 30001
    draw = workloads.uniform_quads(t.N, n, seed=61)
    if kind == "diagonal":
        quads = np.repeat(draw[:, :1], 4, axis=1)
    elif kind == "half_diagonal":
        quads = draw.copy()
        quads[: n // 2] = np.repeat(draw[: n // 2, :1], 4, axis=1)
    else:
        quads = np.repeat(draw[:1], n, axis=0)
    quads = np.ascontiguousarray(quads, dtype=np.int32)
    dq = _dev(quads, torch.int32)
    t.set_direct_max(0)
    try:
        for name, prec in (("fp64", pw.FP64), ("mixed", pw.MIXED), ("fp32", pw.FP32)):
            assert t.fused(prec) and t.layout(prec)["passes"] > 1
            a = t.reconstruct(dq, precision=prec)
            b, _ = t.reconstruct_profile(dq, precision=prec)
            t.sync()
            _same_sums(a, b, o, quads, name, t.layout(prec)["passes"])
        _check_reconstruct(pw, t, o, quads, label=f"skewed classes: {kind}")
    finally:
        t.set_direct_max(DIRECT_DEFAULT)


def test_reconstruct_offset_views_leave_neighbours(pw, tables):
    """Quadruples and outputs handed over as views into larger buffers (a
    ragged last chunk in the fused schedule, whose loads and stores are
    bounded by the chunk): the results are those of contiguous copies bit
    for bit, and no word outside the output view is written."""
    import torch
    t = tables(169, 96)
    n = 20001
    quads = workloads.uniform_quads(t.N, n + 3, seed=77)
    dq = _dev(quads, torch.int32)
    t.set_direct_max(0)
    try:
        for prec in (pw.FP64, pw.MIXED, pw.FP32):
            assert t.fused(prec)
            ref = t.reconstruct(dq[3:].clone(), precision=prec)
            big = torch.full((n + 4101,), 7.25, dtype=torch.float64, device="cuda")
            got = t.reconstruct(dq[3:], big[5:5 + n], precision=prec)
            t.sync()
            assert torch.equal(got, ref)
            assert bool((big[:5] == 7.25).all()) and bool((big[5 + n:] == 7.25).all())
        o = P.setup(169, 96)
        _check_reconstruct(pw, t, o, quads[3:3 + 2000], label="offset views")
    finally:
        t.set_direct_max(DIRECT_DEFAULT)


def test_reconstruct_empty(pw, tables):
    import torch
    t = tables(9, 48)
    out = t.reconstruct(torch.empty((0, 4), dtype=torch.int32, device="cuda"))
    t.sync()
    assert out.numel() == 0


def _sampled_stream_check(pw, t, o, quads_host, sample, label):
    import torch
    dq = _dev(quads_host, torch.int32)
    rows = workloads.sample_rows(len(quads_host), sample, seed=99)
    q = quads_host[rows]
    ref = oracle.reconstruct(o["tau"], o["W"], o["basis"], q)
    scale = P.cond_scale(o["tau"], o["W"], o["basis"], q)
    outs = {}
    for prec, tol in ((pw.FP64, P.TOL_FP64), (pw.MIXED, P.TOL_MIXED), (pw.FP32, P.TOL_FP32)):
        out = t.reconstruct(dq, precision=prec)
        t.sync()
        got = out[torch.from_numpy(rows).cuda()].cpu().numpy()
        err = P.worst_cond_err(got, ref, scale)
        say(f"[parity] {label} prec={prec}: sampled {len(rows)} worst {err:.2e}")
        assert err < tol
        assert bool(torch.isfinite(out).all())
        outs[prec] = out
    return outs


def test_reconstruct_uniform_stream_1045pw(pw, tables):
    w = workloads.C2_SPLIT
    t = tables(w.n2max, w.n_nodes)
    o = P.setup(w.n2max, w.n_nodes)
    quads = workloads.uniform_quads(len(o["basis"]), w.n_quads, w.seed)
    _sampled_stream_check(pw, t, o, quads, 20000, "1e7 uniform, 1045 PW, Q=64")


def test_reconstruct_lookup_stream_full_size(pw, tables):
    """1e8 quadruples over the 9171-PW basis at Q = 96, the launch the benchmark times."""
    import torch
    w = workloads.C4_STREAM
    t = tables(w.n2max, w.n_nodes)
    o = P.setup(w.n2max, w.n_nodes)
    N = len(o["basis"])
    M = int(((o["basis"] ** 2).sum(1) <= w.n2occ).sum())
    assert (N, M) == (9171, 925)
    quads = workloads.lookup_stream(N, M, w.n_quads, w.seed)
    outs = _sampled_stream_check(pw, t, o, quads, 20000, "1e8 lookup stream, 9171 PW, Q=96")
    # every output: split-FP32 against FP64, relative to the largest |value|
    d = (outs[pw.MIXED] - outs[pw.FP64]).abs().max().item()
    say(f"[parity] lookup stream: max |mixed - fp64| = {d:.2e}")
    assert d < 1e-10


# -------------------------------------------------------------- energies ----

@pytest.mark.parametrize("wl", ["plain_fp64_123pw", "split_fp32_1045pw", "paper_scale_9171pw"])
@pytest.mark.parametrize("weights", [False, True])
@pytest.mark.parametrize("algo", ["nodesum", "ktable"])
def test_energies_match_oracle(pw, tables, wl, weights, algo):
    import torch
    w = workloads.ALL[wl]
    t = tables(w.n2max, w.n_nodes)
    o = P.setup(w.n2max, w.n_nodes)
    M = int(((o["basis"] ** 2).sum(1) <= w.n2occ).sum())
    occ = np.arange(M, dtype=np.int32)
    f = workloads.occupations(M, seed=5) if weights else None
    eh_ref, ex_ref = oracle.energies(o["tau"], o["W"], o["basis"], occ, f)
    docc = _dev(occ, torch.int32)
    df = _dev(f, torch.float64) if weights else None
    a = pw.PAIR_NODESUM if algo == "nodesum" else pw.PAIR_KTABLE
    for prec, tol in ((pw.FP64, P.TOL_E_FP64), (pw.MIXED, P.TOL_E_MIXED)):
        eh, ex = t.energies(docc, df, precision=prec, algo=a)
        rh, rx = abs(eh - eh_ref) / eh_ref, abs(ex - ex_ref) / abs(ex_ref)
        say(f"[parity] energies {wl} M={M} f={weights} {algo} prec={prec}: "
            f"E_H rel {rh:.2e}, E_x rel {rx:.2e}")
        assert rh < tol and rx < tol


def test_kernel_table_only_when_it_fits(pw):
    import torch
    occ = torch.arange(7, dtype=torch.int32, device="cuda")
    with pw.Table(1.0, 600, 16) as t:            # nmax = 24: C(99, 3) entries exceed LDS
        with pytest.raises(pw.PwcError) as ei:
            t.energies_async(occ, algo=pw.PAIR_KTABLE)
        assert ei.value.status == pw.ERR_ARG
        a = t.energies(occ, algo=pw.PAIR_NODESUM)
        b = t.energies(occ)                        # AUTO falls back to node sums
        assert a == b


def test_energies_permuted_occupied_list(pw, tables):
    """Any list of basis indices may be occupied; order does not matter."""
    import torch
    t = tables(40, 64)
    o = P.setup(40, 64)
    occ = workloads.rng(4).permutation(len(o["basis"]))[:200].astype(np.int32)
    eh_ref, ex_ref = oracle.energies(o["tau"], o["W"], o["basis"], occ)
    eh, ex = t.energies(_dev(occ, torch.int32))
    assert abs(ex - ex_ref) < 1e-12 * abs(ex_ref) and abs(eh - eh_ref) < 1e-12 * eh_ref


def test_energies_empty_and_deterministic(pw, tables):
    import torch
    t = tables(40, 64)
    assert t.energies(torch.empty(0, dtype=torch.int32, device="cuda")) == (0.0, 0.0)
    occ = torch.arange(123, dtype=torch.int32, device="cuda")
    a = t.energies(occ)
    b = t.energies(occ)
    assert a == b


def test_table_one_mesh2_on_gpu(pw):
    """Sec. III, Table I at M = 9171 (Mesh 2, 8 x 10 + 8 tail): E_x / E_KS = 0.965431."""
    import torch
    with pw.Table(1.0, 169, 0, mesh=pw.Mesh.geometric(10, 8)) as t:
        occ = torch.arange(9171, dtype=torch.int32, device="cuda")
        eh, ex = t.energies(occ)
        ratio = ex / oracle.e_ks(9171)
        o = P.setup(169, mesh=("geometric", 10, 8))
        h, R = oracle.diff_histogram(o["basis"])
        diag = o["tau"][:, np.arange(-26, 27) + 26, -np.arange(-26, 27) + 26]
        ex_ref = oracle.exchange_from_histogram(h, R, diag, o["W"])
        say(f"[parity] Table I on GPU: ratio {ratio:.7f}, rel err vs oracle "
            f"{abs(ex - ex_ref) / abs(ex_ref):.2e}")
        assert abs(ratio - 0.965431) < 1.5e-6
        assert abs(ex - ex_ref) < 1e-12 * abs(ex_ref)


# ------------------------------------------------------ errors, invariants ----

def test_out_of_range_index_reports_and_poisons_only_its_row(pw, tables):
    import torch
    t = tables(9, 48)
    o = P.setup(9, 48)
    N = len(o["basis"])
    quads = workloads.uniform_quads(N, 5000, seed=8)
    bad = quads.copy()
    bad[17, 2] = N
    bad[4000, 0] = -3
    for prec, direct_max in ((pw.FP64, DIRECT_DEFAULT), (pw.MIXED, DIRECT_DEFAULT),
                             (pw.FP64, 0), (pw.MIXED, 0)):
        t.set_direct_max(direct_max)
        out = t.reconstruct(_dev(bad, torch.int32), precision=prec)
        t.set_direct_max(DIRECT_DEFAULT)
        with pytest.raises(pw.PwcError) as ei:
            t.sync()
        assert ei.value.status == pw.ERR_RANGE
        got = out.cpu().numpy()
        assert np.isnan(got[17]) and np.isnan(got[4000])
        keep = np.ones(len(got), bool)
        keep[[17, 4000]] = False
        ref = oracle.reconstruct(o["tau"], o["W"], o["basis"], quads[keep])
        scale = P.cond_scale(o["tau"], o["W"], o["basis"], quads[keep])
        assert P.worst_cond_err(got[keep], ref, scale) < P.TOL_MIXED
        t.sync()   # the error word was cleared
    occ = torch.tensor([0, 1, N], dtype=torch.int32, device="cuda")
    for algo in (pw.PAIR_NODESUM, pw.PAIR_KTABLE):
        out = t.energies_async(occ, algo=algo)
        with pytest.raises(pw.PwcError) as ei:
            t.sync()
        assert ei.value.status == pw.ERR_RANGE
        assert np.isnan(out.cpu().numpy()[1])


def test_bad_occupied_index_in_a_long_list_poisons_the_energies(pw, tables):
    """A bad index far into the occupied list lands in full tiles above the
    diagonal, which the kernel-table exchange sums on a shorter path; those
    tiles still see the NaN weight, for unit and given occupations."""
    import torch
    t = tables(169, 96)
    occ = torch.arange(4000, dtype=torch.int32, device="cuda")
    occ[3001] = t.N + 7
    f = torch.linspace(0.5, 1.5, 4000, dtype=torch.float64, device="cuda")
    for ff in (None, f):
        out = t.energies_async(occ, ff, algo=pw.PAIR_KTABLE)
        with pytest.raises(pw.PwcError) as ei:
            t.sync()
        assert ei.value.status == pw.ERR_RANGE
        e = out.cpu().numpy()
        assert np.isnan(e[0]) and np.isnan(e[1])


def test_one_over_L_scaling(pw, tables):
    import torch
    q = _dev(workloads.uniform_quads(123, 3000, seed=2), torch.int32)
    a = tables(9, 48, 1.0).reconstruct(q)
    b = tables(9, 48, 2.5).reconstruct(q)
    assert torch.allclose(a, b * 2.5, rtol=1e-15, atol=0)


def test_concurrent_streams_share_one_table(pw, tables):
    import torch
    t = tables(40, 64)
    q = _dev(workloads.uniform_quads(1045, 200000, seed=3), torch.int32)
    ref = t.reconstruct(q)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(s1):
        a = t.reconstruct(q, stream=s1)
    with torch.cuda.stream(s2):
        b = t.reconstruct(q, precision=pw.MIXED, stream=s2)
        c = t.reconstruct(q, stream=s2)
    torch.cuda.synchronize()
    assert torch.equal(a, ref) and torch.equal(c, ref)
    assert (b - ref).abs().max().item() < 1e-12


def test_table_built_on_one_stream_is_used_at_once_on_others(pw, tables):
    """pwc_table_create returns once its kernels are queued; each later call
    makes its own stream wait for them, so a table created on a side stream
    gives the same results on other streams with no synchronization between."""
    import torch
    ref_t = tables(169, 96)
    q = _dev(workloads.lookup_stream(9171, 925, 1_000_000, seed=13), torch.int32)
    occ = torch.arange(925, dtype=torch.int32, device="cuda")
    ref = ref_t.reconstruct(q)
    e_ref = np.array(ref_t.energies(occ))
    torch.cuda.synchronize()
    side, other = torch.cuda.Stream(), torch.cuda.Stream()
    for values in (False, True):
        with torch.cuda.stream(side):
            t = pw.Table(1.0, 169, 96, stream=side)
        with torch.cuda.stream(other):
            if values:
                t.build_values(stream=other)
            a = t.reconstruct(q, stream=other)
            e = torch.empty(2, dtype=torch.float64, device="cuda")
            t.energies_async(occ, out=e, stream=other)
        if values:                                 # the value build is ordered on `other` only
            torch.cuda.current_stream().wait_stream(other)
        b = t.reconstruct(q)                       # the default stream
        torch.cuda.synchronize()
        t.sync()
        tol = 0.0 if not values else 1e-14 * ref.abs().max().item()
        assert (a - ref).abs().max().item() <= tol and torch.equal(a, b)
        assert np.array_equal(e.cpu().numpy(), e_ref)
        t.close()


@pytest.mark.parametrize("n2max,mesh", [(169, ("geometric", 11, 8)), (25, ("two_interval", 20))])
def test_table_save_load_round_trip(pw, tmp_path, n2max, mesh):
    """A saved and reloaded table has the same mesh and FP64 tables and gives
    bitwise the same integrals (value table, direct kernel and node passes;
    both precisions) and energies; a damaged file is refused."""
    import torch
    m = pw.Mesh.geometric(mesh[1], mesh[2]) if mesh[0] == "geometric" else pw.Mesh.two_interval(mesh[1])
    path = tmp_path / "t.tab"
    with pw.Table(1.0, n2max, 0, mesh=m) as t:
        t.save(path)
        quads = _dev(workloads.uniform_quads(t.N, 700_001, seed=3), torch.int32)
        occ = torch.arange(min(t.N, 123), dtype=torch.int32, device="cuda")
        ref = {}
        for dm in (DIRECT_DEFAULT, 0):
            t.set_direct_max(dm)
            for prec in (pw.FP64, pw.MIXED):
                ref[dm, prec] = t.reconstruct(quads[:200_000] if dm else quads, precision=prec)
        t.set_direct_max(DIRECT_DEFAULT)
        e_ref = t.energies(occ)
        tau_ref, mesh_ref = t.copy_tables(), t.mesh_nodes()
        t.build_values()
        v_ref = t.reconstruct(quads)
        t.sync()
    with pw.Table.load(path) as u:
        assert (u.L, u.n2max, u.Q) == (1.0, n2max, sum(1 for _ in mesh_ref[0]))
        assert torch.equal(u.copy_tables(), tau_ref)
        for a, b in zip(u.mesh_nodes(), mesh_ref):
            assert np.array_equal(a, b)
        for dm in (DIRECT_DEFAULT, 0):
            u.set_direct_max(dm)
            for prec in (pw.FP64, pw.MIXED):
                got = u.reconstruct(quads[:200_000] if dm else quads, precision=prec)
                assert torch.equal(got, ref[dm, prec])
        u.set_direct_max(DIRECT_DEFAULT)
        assert np.array_equal(u.energies(occ), e_ref)
        u.build_values()                       # values are derived, not stored
        assert torch.equal(u.reconstruct(quads), v_ref)
        u.sync()
    # the file holds one value per orbit of the fold (about a quarter of the
    # nd^2 entries per node), the mesh and the orbit representatives
    nmax = math.isqrt(n2max)
    nd, E1, Q = 4 * nmax + 1, (2 * nmax + 1) ** 2, len(mesh_ref[0])
    size = path.stat().st_size
    assert size == 112 + 8 * (2 * Q + Q * E1) + 2 * E1
    assert size < 0.3 * 8 * Q * nd * nd
    raw = bytearray(path.read_bytes())
    raw[200] ^= 1
    (tmp_path / "flip.tab").write_bytes(bytes(raw))
    with pytest.raises(pw.PwcError) as ei:
        pw.Table.load(tmp_path / "flip.tab")
    assert ei.value.status == pw.ERR_IO


def test_tables_created_from_many_threads_at_once(pw):
    """Table creation from several host threads at once (the upload staging
    buffers are shared by the process) gives every thread the same tables."""
    import threading
    import torch
    with pw.Table(1.0, 40, 64) as ref_t:
        ref = ref_t.copy_tables().cpu().numpy()
    got, errors = [], []

    def work():
        try:
            for _ in range(6):
                s = torch.cuda.Stream()
                with torch.cuda.stream(s):
                    t = pw.Table(1.0, 40, 64, stream=s)
                    tab = t.copy_tables(stream=s)
                s.synchronize()
                got.append(tab.cpu().numpy())
                t.close()
        except Exception as e:          # noqa: BLE001 - reported below
            errors.append(e)

    th = [threading.Thread(target=work) for _ in range(6)]
    for x in th:
        x.start()
    for x in th:
        x.join(timeout=120)
    assert not errors and not any(x.is_alive() for x in th)
    assert len(got) == 36 and all(np.array_equal(g, ref) for g in got)
