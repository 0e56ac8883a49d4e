"""pwc_reconstruct_noalloc: the node passes with the library's fixed device
scratch (tables whose passes run fused need none), against pwc_reconstruct
(the same kernels, with a per-call allocation where they keep a decoded
stream) and the FP64 oracle, on two calls in a row, the second smaller."""
import ctypes
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


def _noalloc(pw, t, q, out, prec):
    """Straight through the C ABI."""
    import torch
    return pw.lib().pwc_reconstruct_noalloc(t.handle, ctypes.c_void_p(q.data_ptr()), q.shape[0],
                                            ctypes.c_void_p(out.data_ptr()), int(prec),
                                            ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))


@pytest.mark.parametrize("sides,n2max,Q", [((1.0,), 169, 96), ((1.0, 1.3, 0.8), 169, 64),
                                          ((1.0,), 40, 64)])
def test_noalloc_matches_the_allocating_call(pw, sides, n2max, Q):
    """Two calls in a row (the second with a smaller input, so stale scratch
    from the first would show), both precisions: bitwise equal to
    pwc_reconstruct on the node passes, and within the parity bar of the
    oracle on a sample.  The 9171-planewave box has 2187 folded rows: its
    passes keep a decoded stream of 8 bytes per quadruple in the fixed
    scratch.  The cubes' one-lane layout runs fused and keeps none (their
    other layouts keep 4 bytes per quadruple)."""
    import torch
    o = P.setup(n2max, Q)
    if len(sides) == 3:
        L0, _, tau = oracle.box_tables(o["beta"], o["K"], sides)
        make = lambda: pw.Table.box(*sides, n2max, Q)
    else:
        L0, tau = sides[0], o["tau"]
        make = lambda: pw.Table(sides[0], n2max, Q)
    N = len(o["basis"])
    with make() as t:
        t.set_direct_max(0)
        for n, seed in ((pw.NOALLOC_MAX_QUADS - 1000, 1), (300_001, 2)):
            qh = workloads.lookup_stream(N, min(N, 925), n, seed=seed)
            q = torch.from_numpy(qh).cuda()
            for prec in (pw.FP64, pw.MIXED, pw.FP32):
                out = torch.full((n,), -7.0, dtype=torch.float64, device="cuda")
                say(f"[noalloc] sides={sides} n2max={n2max} Q={Q} n={n} prec={prec}")
                assert _noalloc(pw, t, q, out, prec) == pw.OK
                ref = t.reconstruct(q, precision=prec)
                t.sync()
                assert torch.equal(out, ref)
                rows = workloads.sample_rows(n, 4000, seed=seed)
                oref = oracle.reconstruct(tau, o["W"], o["basis"], qh[rows], L=L0)
                err = P.worst_cond_err(out.cpu().numpy()[rows], oref,
                                       P.cond_scale(tau, o["W"], o["basis"], qh[rows], L=L0))
                assert err < {pw.FP64: P.TOL_FP64, pw.MIXED: P.TOL_MIXED, pw.FP32: P.TOL_FP32}[prec], err


def test_noalloc_limits_and_errors(pw):
    import torch
    with pw.Table(1.0, 9, 48) as t:
        q = torch.zeros((8, 4), dtype=torch.int32, device="cuda")
        out = torch.empty(8, dtype=torch.float64, device="cuda")
        # past the fixed scratch: refused, nothing enqueued
        assert pw.lib().pwc_reconstruct_noalloc(t.handle, ctypes.c_void_p(q.data_ptr()),
                                                pw.NOALLOC_MAX_QUADS + 1,
                                                ctypes.c_void_p(out.data_ptr()), 0, None) == pw.ERR_LIMIT
        assert _noalloc(pw, t, q[:0], out[:0], pw.FP64) == pw.OK          # n = 0
        bad = q.clone()
        bad[3, 2] = 10 ** 6
        out.fill_(0.0)
        assert _noalloc(pw, t, bad, out, pw.FP64) == pw.OK
        with pytest.raises(pw.PwcError) as ei:
            t.sync()
        assert ei.value.status == pw.ERR_RANGE
        got = out.cpu().numpy()
        assert np.isnan(got[3]) and not np.isnan(np.delete(got, 3)).any()
        # a value table does not change the path: still the node passes
        t.build_values()
        qq = torch.from_numpy(workloads.uniform_quads(123, 5000, seed=4)).cuda()
        o1 = torch.empty(5000, dtype=torch.float64, device="cuda")
        assert _noalloc(pw, t, qq, o1, pw.FP64) == pw.OK
        t.set_direct_max(0)
        t.free_values()
        assert torch.equal(o1, t.reconstruct(qq))
        t.sync()
