"""Benchmark of the separable planewave Coulomb hot path on one MI355X.

Workload (default): the 9171-planewave basis (|n|^2 <= 169) in a unit cube at
Q = 96 nodes (default geometric mesh, 8 x 11 + 8), a seeded stream of 1e8
quadruples (half uniform over the basis, half over the 925-orbital occupied
sphere |n|^2 <= 36) and the Hartree + exchange energies of that sphere.

One step = one pass of the whole path: table construction (basis, mesh, 1-D
primitives, table layouts, exchange kernel table), the value table (every
distinct integral by Eq. 14 over all nodes), reconstruction of the 1e8
integrals by one value read each, and the pair sums with their final
reductions.  Inputs are resident in HBM before the timed region; every step
builds its table and value table afresh.  `value` is that FP64 step.  Two more
legs run the same step without a value table: FP64 node sums
(`fp64_node_sums`) and split-FP32 node sums (`mixed`).

The JSON line also carries
  roofline      -- the dominant kernel of the step (the value-table read,
                   k_rec_values) against the MI355X HBM peak, its launch time
                   taken live with HIP events; value_build and
                   node_pass_roofline give the FP64 rates of the value-table
                   build and of the steady node pass;
  cpu_baseline  -- the FP64 CPU oracle on a sample of the same stream;
  legs          -- per-leg step and kernel times, pair-sum rates;
  serving       -- p50/p99 latency of a Poisson request stream over many
                   boxes, cutoffs and node counts.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
                    [--serve-requests R | --no-serve]
    python bench.py --pmc-workload     # the short run the counter profiles use
"""
import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads  # noqa: E402

FP64_PEAK_TFLOPS = 78.6                     # MI355X FP64 vector, dense
FP32_PEAK_TFLOPS = 157.3                    # MI355X FP32 vector, dense
HBM_PEAK_GBPS = 8000.0
CSRC = os.path.join(ROOT, "paper_1502_08043_amd", "csrc")
# kernel source -> committed counter summary of its kernel on the lookup stream
SOURCES = {"values": (os.path.join(CSRC, "value_kernels.hip"),
                      os.path.join(ROOT, "profiles", "k_rec_values_lookup_stream_9171pw_traffic.txt")),
           "passes": (os.path.join(CSRC, "reconstruct_kernels.hip"),
                      os.path.join(ROOT, "profiles", "k_rec_pass_lookup_stream_9171pw_traffic.txt"))}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--kernel-reps", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--quads", type=int, default=workloads.C4_STREAM.n_quads)
    ap.add_argument("--serve-requests", type=int, default=400)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--pmc-workload", action="store_true")
    ap.add_argument("--kernel-hash", action="store_true",
                    help="print the code hash the recorded counter traffic is keyed on")
    return ap.parse_args()


def kernel_hash(which="values"):
    """First 16 hex digits of sha256 of a kernel file's code, with // comments
    and blank lines removed (a comment edit keeps the hash)."""
    with open(SOURCES[which][0]) as fh:
        code = [re.sub(r"\s*//.*$", "", line).rstrip() for line in fh]
    text = "\n".join(line for line in code if line.strip())
    return hashlib.sha256(text.encode()).hexdigest()[:16]


def recorded_traffic(which="values"):
    """HBM bytes per launch of a kernel from its committed counter summary, or
    None if the summary is missing or was taken on another kernel source."""
    try:
        text = open(SOURCES[which][1]).read()
    except OSError:
        return None
    m_hash = re.search(r"kernel_source_sha256_16:\s*([0-9a-f]+)", text)
    m_bytes = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not m_hash or not m_bytes or m_hash.group(1) != kernel_hash(which):
        return None
    return float(m_bytes.group(1))


def reachable_values(n2max):
    """Sorted orbit triples (a <= b <= c) of a cube that a quadruple of the
    basis |n|^2 <= n2max can read: with m = n_k - n_i and m' = n_l - n_j,
    |m|^2 + |m'|^2 <= 8 n2max, and that is the sum over the three directions
    of each orbit's m^2 + m'^2.  This is the work the value-table build
    does (it skips tiles with no such value); the algorithmic count."""
    K = 2 * math.isqrt(n2max)
    m, mp = np.meshgrid(np.arange(-K, K + 1), np.arange(-K, K + 1), indexing="ij")
    m, mp = m.ravel(), mp.ravel()
    # one representative per orbit of (m, m') -> (m', m), (-m, -m')
    keys = np.stack([np.minimum.reduce([m * 1000 + mp, mp * 1000 + m, -m * 1000 - mp, -mp * 1000 - m])])
    _, first = np.unique(keys, return_index=True)
    s = np.sort(m[first] ** 2 + mp[first] ** 2)
    T = 8 * n2max
    total = 0
    for c in range(len(s)):
        b = np.arange(c + 1)
        room = T - s[b] - s[c]
        na = np.minimum(b + 1, np.searchsorted(s, room, side="right"))
        total += int(na[room >= 0].sum())
    return total


def pmc_workload():
    """A plain copy of known size, three FP64 node-sum reconstructions of the
    stream, then the value table and three reconstructions that read it."""
    import torch
    import paper_1502_08043_amd as pw
    w = workloads.C4_STREAM
    a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")      # 1 GiB
    b = torch.empty_like(a)
    torch.mul(a, 1.0, out=b)                                            # reads 1 GiB, writes 1 GiB
    t = pw.Table(w.L, w.n2max, w.n_nodes)
    M = int(((t.basis().astype(np.int64) ** 2).sum(1) <= w.n2occ).sum())
    q = torch.from_numpy(workloads.lookup_stream(t.N, M, w.n_quads, w.seed)).cuda()
    out = torch.empty(w.n_quads, dtype=torch.float64, device="cuda")
    for _ in range(3):
        t.reconstruct(q, out, pw.FP64)
    t.build_values()
    for _ in range(3):
        t.reconstruct(q, out, pw.FP64)
    torch.cuda.synchronize()
    t.sync()
    print(f"pmc workload done; kernel_source_sha256_16: values {kernel_hash('values')} "
          f"passes {kernel_hash('passes')}", flush=True)


def fixed_error_leg(pw, w, quads, n, steps, warmup, target=1e-9):
    """Throughput at equal total error: the smallest default-mesh Q whose
    integrals are within `target` (absolute, L = 1) of the converged mesh
    (Q = 176, 8 x 21 + 8 nodes) on a sample of the stream, then both
    precisions timed at that Q.  Rounding (about 1e-13 on either path) is far
    below the target, so the quadrature error decides Q."""
    import torch
    half = n // 2
    rows = torch.cat([torch.arange(500_000), half + torch.arange(500_000)]).cuda()
    sample = quads[rows].contiguous()
    with pw.Table(w.L, w.n2max, 176) as t:
        t.build_values()
        ref = t.reconstruct(sample)
        t.sync()
    errs = {}
    q_star = None
    for Q in (48, 56, 64, 72, 80, 88, 96, 112, 128):
        with pw.Table(w.L, w.n2max, Q) as t:
            t.build_values()
            got = t.reconstruct(sample)
            t.sync()
        errs[Q] = (got - ref).abs().max().item()
        if q_star is None and errs[Q] <= target:
            q_star = Q
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    occ = torch.arange(925, dtype=torch.int32, device="cuda")
    eout = torch.empty(2, dtype=torch.float64, device="cuda")
    rates = {}
    for name, prec, values in (("fp64", pw.FP64, True), ("mixed", pw.MIXED, False)):
        def step():
            t = pw.Table(w.L, w.n2max, q_star)
            if values:
                t.build_values()
            t.reconstruct(quads, out, precision=prec)
            t.energies_async(occ, None, prec, eout)
            t.sync()
            t.close()
        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        rates[name] = n * steps / (time.perf_counter() - t0)
    return {"target_abs_error": target, "reference_Q": 176,
            "sample": "1e6 quadruples of the stream (first 5e5 of each half)",
            "max_abs_error_vs_Q176": {str(k): v for k, v in errs.items()}, "Q": q_star,
            "fp64_value_table_integrals_per_s": rates["fp64"],
            "mixed_node_sums_integrals_per_s": rates["mixed"],
            "mixed_vs_fp64": rates["mixed"] / rates["fp64"]}


def serving_leg(pw, n_requests):
    """Poisson request stream over (L, cutoff, Q) keys; p50/p99 at 80% load."""
    import torch
    mix = workloads.ServingMix(n_requests=n_requests)
    reqs = workloads.serving_stream(mix)
    probe = pw.Table(1.0, 100, 16)
    n2 = (probe.basis().astype(np.int64) ** 2).sum(1)
    probe.close()
    pool = torch.randint(0, 1 << 30, (mix.n_range[1], 4), dtype=torch.int32, device="cuda")
    nbasis = {}
    inputs = []
    for r in reqs:
        if r.n2max not in nbasis:
            with pw.Table(1.0, r.n2max, 16) as small:   # basis size of this cutoff
                nbasis[r.n2max] = small.N
        if r.kind == 0:
            q = (pool[:r.n_quads] % nbasis[r.n2max]).contiguous()
            inputs.append((q, torch.empty(r.n_quads, dtype=torch.float64, device="cuda")))
        else:
            M = int((n2 <= r.n2occ).sum())
            inputs.append((torch.arange(M, dtype=torch.int32, device="cuda"),
                           torch.empty(2, dtype=torch.float64, device="cuda")))
    torch.cuda.synchronize()

    def mesh(Q):
        return pw.Mesh.geometric((Q - 8) // 8, 8, alpha_c=0.25)

    def submit(srv, r, x):
        if r.kind == 0:
            return srv.submit_reconstruct(r.L, r.n2max, x[0], x[1], mesh=mesh(r.n_nodes))
        return srv.submit_energies(r.L, r.n2max, x[0], x[1], mesh=mesh(r.n_nodes))

    with pw.Server(16 << 30, max_inflight=8) as srv:
        # serial pass: builds every table and measures the service time
        t0 = time.perf_counter()
        for r, x in zip(reqs, inputs):
            res = srv.wait(submit(srv, r, x))
            assert res.status == pw.OK
        serial_s = time.perf_counter() - t0
        st_serial = srv.stats()
        srv.reset_stats()
        t0 = time.perf_counter()
        for r, x in zip(reqs, inputs):
            srv.wait(submit(srv, r, x))
        warm_serial_s = time.perf_counter() - t0
        srv.reset_stats()
        # Poisson replay at 80% of the warm single-stream capacity
        rate = 0.8 * len(reqs) / warm_serial_s
        gaps = workloads.rng(mix.seed + 1).exponential(1.0 / rate, size=len(reqs))
        arrivals = np.cumsum(gaps)
        tickets = []
        t0 = time.perf_counter()
        for a, r, x in zip(arrivals, reqs, inputs):
            while time.perf_counter() - t0 < a:
                pass
            tickets.append(submit(srv, r, x))
        for tk in tickets:
            srv.wait(tk)
        st = srv.stats()
    return {"requests": len(reqs), "offered_load": 0.8, "offered_rate_hz": rate,
            "distinct_tables": int(st_serial["table_builds"]),
            "cold_serial_s": serial_s, "warm_serial_s": warm_serial_s,
            "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"], "max_ms": st["max_ms"],
            "integrals_per_s": st["integrals_per_s"], "completed": int(st["completed"]),
            "failed": int(st["failed"]), "slots": 8,
            "mix": "80% reconstruct (n log-uniform 1e4..1e6), 20% energies; L in 8 values "
                   "[0.5, 4], n2max = R^2 (R 5..20), Q in {32,48,64,96,128}, alpha_c = 0.25; "
                   "Zipf(1.1) key popularity"}


def main():
    args = parse()
    if args.kernel_hash:
        print(f"values {kernel_hash('values')} passes {kernel_hash('passes')}")
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the path shards by "
              "quadruple ranges and pair rows with replicated tables, but no multi-GPU "
              "figure is measured here.", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1502_08043_amd as pw

    torch.cuda.set_device(0)
    if args.pmc_workload:
        pmc_workload()
        return
    w = workloads.C4_STREAM
    stream = torch.cuda.current_stream()

    probe = pw.Table(w.L, w.n2max, w.n_nodes)
    basis = probe.basis().astype(np.int64)
    N, Q, table_bytes = probe.N, probe.Q, probe.device_bytes
    probe.close()
    M = int(((basis ** 2).sum(1) <= w.n2occ).sum())
    n = args.quads
    log(f"[bench] N={N} M={M} Q={Q} quads={n}: generating inputs")
    quads_h = workloads.lookup_stream(N, M, n, w.seed)
    quads = torch.from_numpy(quads_h).cuda()
    occ = torch.arange(M, dtype=torch.int32, device="cuda")
    occ_all = torch.arange(N, dtype=torch.int32, device="cuda")
    LEGS = (("fp64", pw.FP64, True), ("fp64_node_sums", pw.FP64, False), ("mixed", pw.MIXED, False))
    out = {name: torch.empty(n, dtype=torch.float64, device="cuda") for name, _, _ in LEGS}
    eout = torch.empty(2, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()

    def step(prec, values, o):
        t = pw.Table(w.L, w.n2max, w.n_nodes)            # basis, mesh, primitives, layouts
        if values:
            t.build_values()                             # every distinct integral, Eq. 14
        t.reconstruct(quads, o, precision=prec)          # value reads, or decode + node passes
        t.energies_async(occ, None, prec, eout)          # pair sums + reductions
        t.sync()                                         # surfaces kernel errors
        t.close()

    legs = {}
    for name, prec, values in LEGS:
        for _ in range(args.warmup):
            step(prec, values, out[name])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step(prec, values, out[name])
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        legs[name] = {"ms_per_step": dt * 1e3, "integrals_per_s": n / dt}
        log(f"[bench] {name}: {dt * 1e3:.3f} ms/step, {n / dt:.4g} integrals/s")

    def timed(fn, reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    t = pw.Table(w.L, w.n2max, w.n_nodes)
    # the value table: its build (one launch) and the reads
    vb = []
    for _ in range(args.kernel_reps):
        t.free_values()
        vb.append(timed(t.build_values, 1))
    nvalues = t.values_info()[1] // 8
    legs["fp64"]["value_build_ms"] = float(np.mean(vb))
    legs["fp64"]["value_table_bytes"] = nvalues * 8
    t.reconstruct(quads, out["fp64"])
    legs["fp64"]["reconstruct_ms"] = timed(lambda: t.reconstruct(quads, out["fp64"]), args.kernel_reps)
    log(f"[bench] fp64 values: build {legs['fp64']['value_build_ms']:.3f} ms "
        f"({nvalues} values), reads {legs['fp64']['reconstruct_ms']:.3f} ms")
    t.free_values()
    for name, prec, values in LEGS[1:]:
        t.reconstruct(quads, out[name], precision=prec)
        legs[name]["reconstruct_ms"] = timed(lambda: t.reconstruct(quads, out[name], precision=prec),
                                             args.kernel_reps)
        # per launch: decode, then the node passes
        stages = np.array([t.reconstruct_profile(quads, out[name], precision=prec)[1]
                           for _ in range(args.kernel_reps)]).mean(axis=0)
        legs[name]["decode_ms"] = float(stages[0])
        legs[name]["pass_ms"] = [float(v) for v in stages[1:]]
        legs[name]["layout"] = t.layout(prec)
        for MM, o, key in ((M, occ, "exchange_M925"), (N, occ_all, "exchange_M9171")):
            for algo, an in ((pw.PAIR_KTABLE, "ktable"), (pw.PAIR_NODESUM, "nodesum")):
                t.energies_async(o, None, prec, eout, algo=algo)
                reps = 20 if (MM == M or algo == pw.PAIR_KTABLE) else 3
                ms = timed(lambda: t.energies_async(o, None, prec, eout, algo=algo), reps)
                legs[name][f"{key}_{an}_ms"] = ms
                legs[name][f"{key}_{an}_pairs_per_s"] = MM * MM / (ms * 1e-3)
        t.sync()
        log(f"[bench] {name}: reconstruct {legs[name]['reconstruct_ms']:.3f} ms "
            f"(decode {stages[0]:.3f} + passes {', '.join(f'{v:.3f}' for v in stages[1:])}); "
            f"exchange M={M} {legs[name]['exchange_M925_ktable_ms'] * 1e3:.1f} us, "
            f"M={N} {legs[name]['exchange_M9171_ktable_ms'] * 1e3:.1f} us (kernel table), "
            f"{legs[name]['exchange_M9171_nodesum_ms']:.3f} ms (node sums)")
    tb0 = time.perf_counter()
    for _ in range(5):
        pw.Table(w.L, w.n2max, w.n_nodes).close()
    table_ms = (time.perf_counter() - tb0) / 5 * 1e3
    e_fp64 = t.energies(occ)
    t.close()

    # Roofline of the step's dominant kernel, the value-table read: per
    # quadruple 16 bytes of indices in, one 8-byte value read, 8 bytes out,
    # one launch per call.
    gather_ms = legs["fp64"]["reconstruct_ms"]
    achieved = 32.0 * n / (gather_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBPS, "traffic": recorded_traffic("values"),
                "kernel": "k_rec_values (decode, one value read per quadruple)",
                "launches_per_call": 1, "algorithmic_bytes_per_launch": 32.0 * n,
                "avg_launch_ms": gather_ms, "kernel_source_sha256_16": kernel_hash("values")}
    # The value-table build is a contraction, V[p][c] = sum_q P_q(p) T_q(c): its
    # algorithmic work is one multiply-add (2 flops) per node and value that a
    # quadruple can read (the build skips the rest); the pair products P,
    # shared by every c, are not counted.  Eq. 14 evaluated per value would
    # take 4 flops per node term ("eq14_equivalent").
    vb_ms = legs["fp64"]["value_build_ms"]
    nreach = reachable_values(w.n2max)
    vb_tf = 2.0 * Q * nreach / (vb_ms * 1e-3) / 1e12
    value_build = {"kernel": "k_values_build", "values": nvalues, "values_reachable": nreach,
                   "avg_launch_ms": vb_ms,
                   "achieved": vb_tf, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                   "frac": vb_tf / FP64_PEAK_TFLOPS, "bound": "mfma",
                   "algorithmic_flops_per_launch": 2.0 * Q * nreach,
                   "eq14_equivalent_TFLOPs": 2.0 * vb_tf}
    # The steady FP64 node pass (node sums without a value table).  Algorithmic
    # work of Eq. 14: 4 flops per node term, c nodes per pass and integral.
    lay = legs["fp64_node_sums"]["layout"]
    c = lay["nodes_per_pass"]
    P = len(legs["fp64_node_sums"]["pass_ms"])
    steady = legs["fp64_node_sums"]["pass_ms"][1:] or legs["fp64_node_sums"]["pass_ms"]
    pass_ms = float(np.mean(steady))
    flops = 4.0 * c * n
    np_tf = flops / (pass_ms * 1e-3) / 1e12
    node_pass_roofline = {
        "bound": "alu", "achieved": np_tf, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
        "frac": np_tf / FP64_PEAK_TFLOPS, "traffic": recorded_traffic("passes"),
        "kernel": f"k_rec_pass<F64, G={lay['lanes']}, W={lay['words']}> steady node pass",
        "launches_per_call": P, "nodes_per_launch": c,
        "algorithmic_flops_per_launch": flops, "avg_launch_ms": pass_ms,
        "first_pass_with_decode_ms": legs["fp64_node_sums"]["pass_ms"][0],
        "lds_read_TBps": 3 * 8 * c * n / (pass_ms * 1e-3) / 1e12,
        "hbm_algorithmic_GBps": 20.0 * n / (pass_ms * 1e-3) / 1e9,
        "whole_call_TFLOPs": 4.0 * Q * n / (legs["fp64_node_sums"]["reconstruct_ms"] * 1e-3) / 1e12,
        "kernel_source_sha256_16": kernel_hash("passes")}
    # The split-FP32 steady pass, counted the same way (4 algorithmic flops per
    # node term) against the FP32 vector peak; a float-float node term takes
    # about 16 FP32 instructions.
    mlay = legs["mixed"]["layout"]
    msteady = legs["mixed"]["pass_ms"][1:] or legs["mixed"]["pass_ms"]
    mpass_ms = float(np.mean(msteady))
    mflops = 4.0 * mlay["nodes_per_pass"] * n
    m_tf = mflops / (mpass_ms * 1e-3) / 1e12
    mixed_pass = {"kernel": f"k_rec_pass<FF, G={mlay['lanes']}, W={mlay['words']}> steady node pass",
                  "achieved": m_tf, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                  "frac": m_tf / FP32_PEAK_TFLOPS, "avg_launch_ms": mpass_ms,
                  "lds_read_TBps": 3 * 8 * mlay["nodes_per_pass"] * n / (mpass_ms * 1e-3) / 1e12}

    fixed_error = fixed_error_leg(pw, w, quads, n, args.steps, args.warmup)
    log(f"[bench] fixed error 1e-9: Q = {fixed_error['Q']}, FP64 value table "
        f"{fixed_error['fp64_value_table_integrals_per_s']:.4g}/s, mixed "
        f"{fixed_error['mixed_node_sums_integrals_per_s']:.4g}/s; errors {fixed_error['max_abs_error_vs_Q176']}")

    serving = None
    if not args.no_serve:
        log(f"[bench] serving leg: {args.serve_requests} requests")
        serving = serving_leg(pw, args.serve_requests)
        log(f"[bench] serving: p50 {serving['p50_ms']:.3f} ms, p99 {serving['p99_ms']:.3f} ms at "
            f"{serving['offered_rate_hz']:.0f} req/s")

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
        basis64 = oracle.enumerate_basis(w.n2max)
        beta, W, _ = oracle.default_mesh(w.n_nodes)
        t0 = time.perf_counter()
        tau = oracle.tau_table(beta, 2 * int(math.isqrt(w.n2max)))
        t_tab = time.perf_counter() - t0
        sample = min(n, 100_000_000)      # the whole stream: about 1-2 s on 16 host threads
        rows = np.concatenate([np.arange(sample // 2), n // 2 + np.arange(sample - sample // 2)])
        qs = quads_h[rows]
        t0 = time.perf_counter()
        ref = oracle.reconstruct(tau, W, basis64, qs, nthreads=threads)
        t_rec = time.perf_counter() - t0
        # condition-aware error: |C - C_ref| / sum_q |W_q X Y Z| / (sqrt(pi) L)
        sub = rows[::100]
        K = (tau.shape[1] - 1) // 2
        qq = quads_h[sub].astype(np.int64)
        m = basis64[qq[:, 2]] - basis64[qq[:, 0]] + K
        mp = basis64[qq[:, 3]] - basis64[qq[:, 1]] + K
        scale = np.abs(W)[:, None] * np.ones((1, len(qq)))
        for d in range(3):
            scale = scale * np.abs(tau[:, m[:, d], mp[:, d]])
        scale = scale.sum(0) / math.sqrt(math.pi)
        errs = {}
        for k in ("fp64", "fp64_node_sums", "mixed"):
            got = out[k][torch.from_numpy(rows).cuda()].cpu().numpy()
            errs[k] = {"max_abs": float(np.max(np.abs(got - ref))),
                       "max_condition_aware": float(np.max(np.abs(got[::100] - ref[::100]) / scale))}
        # quadrature error of the timed mesh: the oracle on the converged mesh
        # (Q = 176) for a subsample, against the FP64 result
        sub2 = rows[:: max(1, len(rows) // 20000)]
        beta_c, W_c, _ = oracle.default_mesh(176)
        tau_c = oracle.tau_table(beta_c, 2 * int(math.isqrt(w.n2max)))
        ref_c = oracle.reconstruct(tau_c, W_c, basis64, quads_h[sub2], nthreads=threads)
        got_c = out["fp64"][torch.from_numpy(sub2).cuda()].cpu().numpy()
        errs["fp64_vs_converged_Q176"] = {"max_abs": float(np.max(np.abs(got_c - ref_c))),
                                          "sample": len(sub2)}
        cpu = {"value": sample / t_rec, "unit": "integrals/s", "cores": threads, "kind": "oracle",
               "sample": (f"the whole stream, {sample} quadruples" if sample == n else
                          f"{sample} quadruples of the stream (first {sample // 2} of each half)"),
               "table_build_s": t_tab, "gpu_error_vs_oracle": errs}
        log(f"[bench] oracle: {sample / t_rec:.4g} integrals/s on {threads} threads; errors {errs}")

    res = {
        "metric": "integrals/s and pair-sum/s at 9.2k-PW basis, mixed vs FP64 at fixed err; p99 ms",
        "value": legs["fp64"]["integrals_per_s"],
        "unit": "integrals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": legs["fp64"]["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "L": w.L, "n2max": w.n2max, "basis_N": N,
                   "occupied_M": M, "n_nodes": Q, "mesh": "geometric 8x11 + 8 tail",
                   "n_quads": n, "seed": w.seed, "table_device_bytes": table_bytes,
                   "step": "table build + value table + reconstruct all quads + E_H/E_x at M=925"},
        "pair_sums_per_s": {
            "M925_ktable": legs["fp64_node_sums"]["exchange_M925_ktable_pairs_per_s"],
            "M9171_ktable": legs["fp64_node_sums"]["exchange_M9171_ktable_pairs_per_s"],
            "M9171_nodesum": legs["fp64_node_sums"]["exchange_M9171_nodesum_pairs_per_s"]},
        "mixed_vs_fp64": {"integrals_per_s_ratio_node_sums": legs["mixed"]["integrals_per_s"] /
                          legs["fp64_node_sums"]["integrals_per_s"],
                          "integrals_per_s_ratio_vs_value_table": legs["mixed"]["integrals_per_s"] /
                          legs["fp64"]["integrals_per_s"]},
        "p99_ms": serving["p99_ms"] if serving else None,
        "legs": legs,
        "table_build_ms": table_ms,
        "energies_fp64_M925": {"E_H": e_fp64[0], "E_x": e_fp64[1]},
        "serving": serving,
        "roofline": roofline,
        "value_build": value_build,
        "node_pass_roofline": node_pass_roofline,
        "mixed_pass": mixed_pass,
        "fixed_error": fixed_error,
        "cpu_baseline": cpu,
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
