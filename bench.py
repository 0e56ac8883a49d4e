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
(`fp64_node_sums`, reported as `value_small_storage`: the O(N^{2/3})-storage
path of the paper) and split-FP32 node sums (`mixed`).

The JSON line also carries
  roofline      -- the dominant kernel of the step (the value-table read,
                   k_rec_values) against the MI355X HBM peak, its launch time
                   taken live with HIP events; algorithmic bytes are 16 of
                   indices in and 8 out per quadruple; value_build and
                   node_pass_roofline give the FP64 rates of the value-table
                   build and of the node sums (one fused launch per call on
                   this table; the separate launches of the profiling entry
                   point are reported beside it), mixed_pass and fp32_pass
                   those of the two FP32 arithmetics; the node sums also
                   carry their LDS read rate against the LDS read peak;
  errors_vs_fp64_value_table_all_outputs
                -- every output of the node-sum legs against the FP64
                   value-table leg's, over the whole stream, on the GPU;
  cpu_baseline  -- the FP64 CPU oracle on a bounded sample of the same stream,
                   on all host cores and on one, median of 5 runs after one
                   warm-up; the errors of every GPU result against it;
  configs       -- the small configurations: all 19^4 integrals of the
                   123-planewave basis (Q = 48) and 1e7 uniform quadruples of
                   the 1045-planewave basis (Q = 64), FP64 against split-FP32;
  fixed_error   -- every path timed at the node count that reaches a target
                   error against the converged oracle (1e-9 absolute, and six
                   places), node sums against node sums;
  legs          -- per-leg step and kernel times (the reconstruction also per
                   half of the stream), pair-sum rates;
  serving       -- p50/p99 latency of a Poisson request stream over many
                   boxes, cutoffs and node counts at 50, 80 and 95% load, a
                   64 MiB budget, and FP64 against split-FP32.

    python bench.py [--steps K] [--warmup W] [--kernel-reps R] [--gpus 1] [--no-cpu-baseline]
                    [--serve-requests R | --no-serve] [--no-configs] [--no-fixed-error] [--no-per-half]
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
# LDS reads: a conflict-free ds_read_b128 wavefront instruction (1 KiB) takes 4
# LDS cycles, so 256 B per clock per CU; 256 CUs at 2.4 GHz.
LDS_PEAK_TBPS = 256 * 256 * 2.4e9 / 1e12
CSRC = os.path.join(ROOT, "paper_1502_08043_amd", "csrc")
# kernel source -> committed counter summary of its kernel on the lookup stream
SOURCES = {"values": (os.path.join(CSRC, "value_kernels.hip"),
                      os.path.join(ROOT, "profiles", "k_rec_values_lookup_stream_9171pw_traffic.txt")),
           "passes": (os.path.join(CSRC, "reconstruct_kernels.hip"),
                      os.path.join(ROOT, "profiles", "k_rec_fused_lookup_stream_9171pw_traffic.txt"))}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--kernel-reps", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--quads", type=int, default=workloads.C4_STREAM.n_quads)
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-configs", action="store_true")
    ap.add_argument("--no-fixed-error", action="store_true")
    ap.add_argument("--no-per-half", action="store_true",
                    help="skip the per-half timings (kernel profiles then hold 1e8-quadruple calls only)")
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
    stream, three single-FP32 ones (one fused launch each on this table),
    then the value table and three reconstructions that read it."""
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
    for _ in range(3):
        t.reconstruct(q, out, pw.FP32)
    t.build_values()
    for _ in range(3):
        t.reconstruct(q, out, pw.FP64)
    torch.cuda.synchronize()
    t.sync()
    print(f"pmc workload done; kernel_source_sha256_16: values {kernel_hash('values')} "
          f"passes {kernel_hash('passes')}", flush=True)


FIXED_ERROR_TARGETS = (("1e-9", 1e-9), ("six_place", 1e-6))
FIXED_ERROR_Q = (32, 40, 48, 56, 64, 72, 80, 88, 96, 112, 128)
ROOT_MESH_Q_SUB = (4, 5, 6, 7, 8, 9, 10, 12)     # Mesh 3: 4 pieces (ratio 7) x q_sub + 4 tail


def fixed_error_leg(pw, w, quads, n, steps, warmup, ref=None):
    """Throughput at equal error.  For each target (1e-9 absolute on the
    integrals of L = 1, and six places: 1e-6 on the integrals and on
    E_x/E_KS of the occupied sphere), and for each mesh family -- the
    paper's Mesh 2 (8 geometric pieces x q + 8 tail points) and Mesh 3 (4
    pieces in sqrt(beta) x q + 4 tail points exact for polynomials in t^2) --
    the smallest mesh whose results are within the target of the converged
    oracle on a sample of the stream; every path is then timed on it: the
    FP64 value table, FP64 node sums and split-FP32 node sums (node sums
    against node sums is the like-for-like comparison).  `ref` holds the
    converged references the oracle computed in the CPU-baseline leg (rows,
    integrals, E_x/E_KS); without it the GPU's own Q = 176 Mesh 2 value
    table stands in."""
    import torch
    if ref is None:
        half = n // 2
        rows = np.concatenate([np.arange(10_000), half + np.arange(10_000)])
        with pw.Table(w.L, w.n2max, 176) as t:
            t.build_values()
            ref_int = t.reconstruct(quads[torch.from_numpy(rows).cuda()].contiguous()).cpu().numpy()
            t.sync()
        ref = {"rows": rows, "integrals": ref_int, "ratio": None, "source": "GPU value table at Q = 176"}
    M = ref.get("M", 925)
    sample = quads[torch.from_numpy(ref["rows"]).cuda()].contiguous()
    occ = torch.arange(M, dtype=torch.int32, device="cuda")
    e_ks = -0.75 * (6.0 / math.pi) ** (1.0 / 3.0) * M ** (4.0 / 3.0) / w.L
    families = {"mesh2": [(f"geometric 8x{(Q - 8) // 8}+8", pw.mesh_default(Q)) for Q in FIXED_ERROR_Q],
                "mesh3": [(f"root 4x{q}+4 ratio 7", pw.Mesh.geometric_root(q, 4, n_sub=4, ratio=7.0))
                          for q in ROOT_MESH_Q_SUB]}
    # errors of each mesh: the FP64 paths (value table; node sums and split
    # FP32 agree with it to 1e-12) and the single-FP32 path (its table
    # rounding adds up to 4.2e-7 of the node terms)
    errs = {}
    for fam, meshes in families.items():
        for name, mesh in meshes:
            with pw.Table(w.L, w.n2max, 0, mesh=mesh) as t:
                t.set_direct_max(0)
                got32 = t.reconstruct(sample, precision=pw.FP32).cpu().numpy()
                t.build_values()
                got = t.reconstruct(sample).cpu().numpy()
                _, ex = t.energies(occ)
                t.sync()
                e = {"integrals_max_abs": float(np.max(np.abs(got - ref["integrals"])))}
                e32 = {"integrals_max_abs": float(np.max(np.abs(got32 - ref["integrals"])))}
                q_nodes = t.Q
            if ref.get("ratio") is not None:
                e["ex_over_eks_abs"] = e32["ex_over_eks_abs"] = abs(ex / e_ks - ref["ratio"])
            errs[name] = {"Q": q_nodes, "fp64": e, "fp32": e32}
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    eout = torch.empty(2, dtype=torch.float64, device="cuda")
    # (name, precision, value table, which error decides its mesh); the FP32
    # step takes its energies in FP64 (the FP32 table serves reconstruction)
    paths = (("fp64_value_table", pw.FP64, True, "fp64"), ("fp64_node_sums", pw.FP64, False, "fp64"),
             ("mixed_node_sums", pw.MIXED, False, "fp64"), ("fp32_node_sums", pw.FP32, False, "fp32"))

    def rate(mesh, prec, values):
        def step():
            t = pw.Table(w.L, w.n2max, 0, mesh=mesh)
            if values:
                t.build_values()
            t.reconstruct(quads, out, precision=prec)
            t.energies_async(occ, None, pw.FP64 if prec == pw.FP32 else prec, eout)
            t.sync()
            t.close()
        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        return n * steps / (time.perf_counter() - t0)

    points = {}
    for label, target in FIXED_ERROR_TARGETS:
        pt = {"target": target}
        for fam, meshes in families.items():
            res = {"integrals_per_s": {}, "mesh": {}, "Q": {}, "errors": {}}
            for name, prec, values, which in paths:
                hit = next((nm for nm, m in meshes
                            if all(v <= target for v in errs[nm][which].values())), None)
                if hit is None:
                    continue
                mesh = dict(meshes)[hit]
                res["integrals_per_s"][name] = rate(mesh, prec, values)
                res["mesh"][name], res["Q"][name] = hit, errs[hit]["Q"]
                res["errors"][name] = errs[hit][which]
            r = res["integrals_per_s"]
            node = {k: v for k, v in r.items() if k != "fp64_value_table"}
            if "mixed_node_sums" in r and "fp64_node_sums" in r:
                res["mixed_vs_fp64_node_sums"] = r["mixed_node_sums"] / r["fp64_node_sums"]
            if "fp32_node_sums" in r and "fp64_node_sums" in r:
                res["fp32_vs_fp64_node_sums"] = r["fp32_node_sums"] / r["fp64_node_sums"]
            if node:
                res["faster_node_sum_path"] = max(node, key=node.get)
            if r:
                res["fastest_path"] = max(r, key=r.get)
            pt[fam] = res
        r2, r3 = pt["mesh2"]["integrals_per_s"], pt["mesh3"]["integrals_per_s"]
        pt["mesh3_vs_mesh2_speedup"] = {k: r3[k] / r2[k] for k in r2 if k in r3}
        points[label] = pt
    return {"reference": ref["source"], "sample_rows": len(ref["rows"]), "occupied_M": M,
            "errors_vs_converged": errs, "points": points}


def configs_leg(pw, steps, warmup):
    """The two small configurations, each step = table build + reconstruction
    of every quadruple + the energies of the occupied set; FP64 (value table
    and node sums) and split-FP32.  Returns the timings and the GPU outputs
    (the errors against the oracle are taken in the CPU-baseline leg)."""
    import torch
    res, outs = {}, {}
    for w in (workloads.C1_PLAIN, workloads.C2_SPLIT):
        with pw.Table(w.L, w.n2max, w.n_nodes) as probe:
            b = probe.basis().astype(np.int64)
            N = probe.N
        M = int(((b ** 2).sum(1) <= w.n2occ).sum())
        qh = (workloads.all_quads(M) if w is workloads.C1_PLAIN
              else workloads.uniform_quads(N, w.n_quads, seed=w.seed))
        q = torch.from_numpy(qh).cuda()
        n = len(qh)
        occ = torch.arange(M, dtype=torch.int32, device="cuda")
        legs = {}
        for name, prec, values in (("fp64_value_table", pw.FP64, True),
                                   ("fp64_node_sums", pw.FP64, False),
                                   ("mixed_node_sums", pw.MIXED, False)):
            out = torch.empty(n, dtype=torch.float64, device="cuda")
            eout = torch.empty(2, dtype=torch.float64, device="cuda")

            def step():
                t = pw.Table(w.L, w.n2max, w.n_nodes)
                if values:
                    t.build_values()
                t.reconstruct(q, out, precision=prec)
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
            dt = (time.perf_counter() - t0) / steps
            legs[name] = {"ms_per_step": dt * 1e3, "integrals_per_s": n / dt,
                          "node_terms_per_s": n * w.n_nodes / dt,
                          "pairs_per_s": M * M / dt,
                          "E_H": float(eout[0].item()), "E_x": float(eout[1].item())}
            outs[(w.name, name)] = out
        res[w.name] = {"basis_N": N, "occupied_M": M, "n_nodes": w.n_nodes, "n_quads": n,
                       "quads": "all M^4 occupied quadruples" if w is workloads.C1_PLAIN
                       else f"uniform over the basis, seed {w.seed}",
                       "legs": legs}
        log(f"[bench] {w.name}: " + ", ".join(f"{k} {v['integrals_per_s']:.3g}/s"
                                               for k, v in legs.items()))
    return res, outs


def gauss_leg(pw, steps, warmup):
    """The separable Gaussian basis (Sec. II): 24 one-dimensional s-type
    Gaussians per direction (12 centers 1.5 bohr apart, exponents 0.8 and
    3.0; 13,824 basis functions), reference length 20 bohr, Mesh 3 with 46
    nodes, pairs screened at 1e-15; 1e7 local quadruples (the four
    functions within three one-dimensional indices of each other, so most
    integrals are kept).  One step = table build + reconstruction."""
    import torch
    gs = workloads.GAUSS_BENCH
    a, A = workloads.gaussian_set(gs)
    n1 = len(a)
    g = workloads.rng(2718)
    n = 10_000_000
    base = g.integers(0, n1, (n, 1, 3))
    l = np.clip(base + g.integers(-3, 4, (n, 4, 3)), 0, n1 - 1)
    qh = ((l[..., 0] * n1 + l[..., 1]) * n1 + l[..., 2]).astype(np.int32)
    q = torch.from_numpy(qh).cuda()
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    mesh = pw.Mesh.geometric_root(10, 6)
    res = {"set": gs.name, "n1": n1, "basis_N": n1 ** 3, "L": 20.0, "mesh": "root 4x10+6 ratio 7",
           "eps": 1e-15, "n_quads": n}
    for name, prec in (("fp64", pw.FP64), ("mixed", pw.MIXED)):
        def step():
            t = pw.GaussTable(a, A, 20.0, eps=1e-15, mesh=mesh)
            t.reconstruct(q, out, precision=prec)
            t.sync()
            res["n_pairs"], res["Q"], res["table_device_bytes"] = t.n_pairs, t.Q, t.device_bytes
            t.close()
        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        res[name] = {"ms_per_step": dt * 1e3, "integrals_per_s": n / dt}
    res["nonzero_fraction"] = float((out != 0).double().mean().item())
    log(f"[bench] gauss: {res['n_pairs']} pairs, fp64 {res['fp64']['integrals_per_s']:.3g}/s, "
        f"mixed {res['mixed']['integrals_per_s']:.3g}/s")
    return res, qh, out


def serving_leg(pw, n_requests, warmup_requests=100):
    """The Poisson request stream over (L, cutoff, Q) keys: a serial FP64
    pass (cold, then warm: the single-stream service time and latency), then
    Poisson replays at 50, 80 and 95% of the warm single-stream capacity, a
    replay at 80% under a 64 MiB HBM budget (admission waits and
    evictions), and the 80% replay with every request on the split-FP32
    path.  Latency percentiles skip the first `warmup_requests` of each run."""
    import torch
    mix = workloads.ServingMix(n_requests=n_requests)
    reqs = workloads.serving_stream(mix)
    probe = pw.Table(1.0, 400, 16)
    n2 = (probe.basis().astype(np.int64) ** 2).sum(1)
    probe.close()
    pool = torch.randint(0, 1 << 30, (mix.n_range[1], 4), dtype=torch.int32, device="cuda")
    nbasis = {}
    inputs = []
    for r in reqs:
        if r.n2max not in nbasis:
            nbasis[r.n2max] = int((n2 <= r.n2max).sum())
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

    def submit(srv, r, x, prec):
        if r.kind == 0:
            return srv.submit_reconstruct(r.L, r.n2max, x[0], x[1], precision=prec, mesh=mesh(r.n_nodes))
        return srv.submit_energies(r.L, r.n2max, x[0], x[1], precision=prec, mesh=mesh(r.n_nodes))

    def pct(lat):
        lat = np.sort(np.asarray(lat[warmup_requests:]))
        return float(np.percentile(lat, 50)), float(np.percentile(lat, 99)), float(lat[-1])

    def serial(srv, prec):
        lat = []
        t0 = time.perf_counter()
        for r, x in zip(reqs, inputs):
            res = srv.wait(submit(srv, r, x, prec))
            assert res.status == pw.OK, res.status
            lat.append(res.latency_ms)
        return time.perf_counter() - t0, lat

    def replay(srv, rate, prec):
        gaps = workloads.rng(mix.seed + 1).exponential(1.0 / rate, size=len(reqs))
        arrivals = np.cumsum(gaps)
        srv.reset_stats()
        tickets = []
        t0 = time.perf_counter()
        for a, r, x in zip(arrivals, reqs, inputs):
            while time.perf_counter() - t0 < a:
                pass
            tickets.append(submit(srv, r, x, prec))
        res = [srv.wait(tk) for tk in tickets]
        wall = time.perf_counter() - t0
        st = srv.stats()
        assert all(x.status == pw.OK for x in res)
        p50, p99, mx = pct([x.latency_ms for x in res])
        work = sum(r.n_quads for r in reqs if r.kind == 0)
        return {"offered_rate_hz": rate, "p50_ms": p50, "p99_ms": p99, "max_ms": mx,
                "completed_per_s": len(reqs) / wall, "integrals_per_s": work / wall,
                "table_builds": int(st["table_builds"]), "evictions": int(st["evictions"]),
                "launches": int(st["launches"]), "batched": int(st["batched"])}

    out = {"requests": len(reqs), "warmup_requests": warmup_requests, "slots": 8,
           "mix": "80% reconstruct (n log-uniform 1e4..1e6), 20% energies; L in 8 values "
                  "[0.5, 4], n2max = R^2 (R 5..20), Q in {32,48,64,96,128}, alpha_c = 0.25; "
                  "Zipf(1.1) key popularity; Poisson arrivals, seed 2015"}
    with pw.Server(16 << 30, max_inflight=8) as srv:
        cold_s, _ = serial(srv, pw.FP64)                 # builds every table
        out["distinct_tables"] = int(srv.stats()["table_builds"])
        srv.reset_stats()
        warm_s, lat = serial(srv, pw.FP64)
        p50, p99, mx = pct(lat)
        out["serial_fp64"] = {"cold_s": cold_s, "warm_s": warm_s, "p50_ms": p50, "p99_ms": p99,
                              "max_ms": mx, "completed_per_s": len(reqs) / warm_s}
        capacity = len(reqs) / warm_s
        out["capacity_hz"] = capacity
        for load in (0.5, 0.8, 0.95):
            out[f"fp64_load_{int(load * 100)}"] = replay(srv, load * capacity, pw.FP64)
            log(f"[bench] serving fp64 at {load:.0%}: p50 {out[f'fp64_load_{int(load * 100)}']['p50_ms']:.3f} "
                f"p99 {out[f'fp64_load_{int(load * 100)}']['p99_ms']:.3f} ms")
        serial(srv, pw.MIXED)                             # warm the split-FP32 path
        out["mixed_load_80"] = replay(srv, 0.8 * capacity, pw.MIXED)
    with pw.Server(64 << 20, max_inflight=8) as srv:
        serial(srv, pw.FP64)
        out["budget_64MiB_fp64_load_80"] = replay(srv, 0.8 * capacity, pw.FP64)
        out["budget_64MiB_fp64_load_80"]["budget_bytes"] = 64 << 20
    log(f"[bench] serving 64 MiB at 80%: p50 {out['budget_64MiB_fp64_load_80']['p50_ms']:.3f} "
        f"p99 {out['budget_64MiB_fp64_load_80']['p99_ms']:.3f} ms, "
        f"evictions {out['budget_64MiB_fp64_load_80']['evictions']}")
    return out


def gauss_oracle_errors(qh, out):
    """Part of the CPU-baseline leg: the oracle on 20,000 sampled quadruples
    of the Gaussian leg's stream (the last step's FP64 outputs)."""
    import oracle
    a, A = workloads.gaussian_set(workloads.GAUSS_BENCH)
    pairs, pmap = oracle.gauss_pairs(a, A, 1e-15)
    beta, W, _ = oracle.mesh3(10, 6)
    tau = oracle.gauss_tau(beta, a, A, pairs, L=20.0)
    rows = workloads.sample_rows(len(qh), 20_000, seed=9)
    ref = oracle.gauss_reconstruct(tau, W, pmap, len(a), qh[rows], L=20.0)
    got = out.cpu().numpy()[rows]
    nz = ref != 0
    big = np.abs(ref) >= 1e-22          # split FP32 keeps FP32's exponent range
    small = nz & ~big
    return {"sample": len(rows), "zeros_match": bool(np.array_equal(got[~nz], ref[~nz])),
            "max_rel_above_1e-22": float(np.max(np.abs(got[big] - ref[big]) / np.abs(ref[big]))),
            "max_abs_below_1e-22": float(np.max(np.abs(got[small] - ref[small]))) if small.any() else 0.0,
            "path": "mixed (the leg's last step)"}


def cpu_baseline_leg(w, quads_h, N, M, n, gpu_out, cfg_outs):
    """The FP64 CPU oracle: timed on a bounded sample of the lookup stream on
    all host cores and on one core (median of 5 runs after one warm-up each),
    and the reference for every GPU error the line reports: the stream
    sample at the timed mesh, a converged (Q = 176) sample with E_x/E_KS for
    the fixed-error leg, and the two small configurations."""
    import torch
    import oracle
    all_threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    basis64 = oracle.enumerate_basis(w.n2max)
    K = 2 * int(math.isqrt(w.n2max))
    beta, W, _ = oracle.default_mesh(w.n_nodes)
    t0 = time.perf_counter()
    tau = oracle.tau_table(beta, K)
    t_tab = time.perf_counter() - t0

    def timed(qs, threads):
        oracle.reconstruct(tau, W, basis64, qs[:1000], nthreads=threads)   # warm-up
        ts = []
        for _ in range(5):
            t0 = time.perf_counter()
            oracle.reconstruct(tau, W, basis64, qs, nthreads=threads)
            ts.append(time.perf_counter() - t0)
        return len(qs) / float(np.median(ts)), ts

    # bounded samples: the first s/2 quadruples of each half of the stream
    def sample(s):
        rows = np.concatenate([np.arange(s // 2), n // 2 + np.arange(s - s // 2)])
        return rows, quads_h[rows]
    rows_all, qs_all = sample(min(n, 20_000_000))
    rate_all, ts_all = timed(qs_all, all_threads)
    _, qs_one = sample(min(n, 2_000_000))
    rate_one, ts_one = timed(qs_one, 1)
    log(f"[bench] oracle: {rate_all:.4g} integrals/s on {all_threads} threads, {rate_one:.4g} on 1")

    # errors of the lookup-stream legs against the oracle on the timed sample
    ref = oracle.reconstruct(tau, W, basis64, qs_all, nthreads=all_threads)
    sub = np.arange(0, len(rows_all), 100)
    qq = qs_all[sub].astype(np.int64)
    m = basis64[qq[:, 2]] - basis64[qq[:, 0]] + K
    mp = basis64[qq[:, 3]] - basis64[qq[:, 1]] + K
    scale = np.abs(W)[:, None] * np.ones((1, len(qq)))
    for d in range(3):
        scale = scale * np.abs(tau[:, m[:, d], mp[:, d]])
    scale = scale.sum(0) / math.sqrt(math.pi)
    dev_rows = torch.from_numpy(rows_all).cuda()
    errs = {}
    for k, o in gpu_out.items():
        got = o[dev_rows].cpu().numpy()
        errs[k] = {"max_abs": float(np.max(np.abs(got - ref))),
                   "mean_abs": float(np.mean(np.abs(got - ref))),
                   "max_condition_aware": float(np.max(np.abs(got[sub] - ref[sub]) / scale))}

    # converged references (Q = 176) for the fixed-error leg and the
    # quadrature error of the timed mesh
    half = n // 2
    rows_c = np.concatenate([np.arange(10_000), half + np.arange(10_000)])
    beta_c, W_c, _ = oracle.default_mesh(176)
    tau_c = oracle.tau_table(beta_c, K)
    ref_c = oracle.reconstruct(tau_c, W_c, basis64, quads_h[rows_c], nthreads=all_threads)
    h, R = oracle.diff_histogram(basis64[:M])
    ex_c = oracle.exchange_from_histogram(h, R, oracle.tau_diag(beta_c, 2 * R), W_c)
    got_c = gpu_out["fp64"][torch.from_numpy(rows_c).cuda()].cpu().numpy()
    errs["fp64_vs_converged_Q176"] = {"max_abs": float(np.max(np.abs(got_c - ref_c))),
                                      "sample": len(rows_c)}
    converged = {"rows": rows_c, "integrals": ref_c, "ratio": ex_c / oracle.e_ks(M), "M": M,
                 "source": "FP64 oracle at Q = 176 (8 x 21 + 8)"}

    # the two small configurations, every output against the oracle
    cfg_errs = {}
    for wc in (workloads.C1_PLAIN, workloads.C2_SPLIT):
        bc = oracle.enumerate_basis(wc.n2max)
        Kc = 2 * int(math.isqrt(wc.n2max))
        bq, Wq, _ = oracle.default_mesh(wc.n_nodes)
        tq = oracle.tau_table(bq, Kc)
        Mc = int(((bc ** 2).sum(1) <= wc.n2occ).sum())
        qc = (workloads.all_quads(Mc) if wc is workloads.C1_PLAIN
              else workloads.uniform_quads(len(bc), wc.n_quads, seed=wc.seed))
        rc = oracle.reconstruct(tq, Wq, bc, qc, nthreads=all_threads)
        eh, ex = oracle.energies(tq, Wq, bc, np.arange(Mc, dtype=np.int32), nthreads=all_threads)
        q2 = qc[::50].astype(np.int64)
        m2 = bc[q2[:, 2]] - bc[q2[:, 0]] + Kc
        mp2 = bc[q2[:, 3]] - bc[q2[:, 1]] + Kc
        sc = np.abs(Wq)[:, None] * np.ones((1, len(q2)))
        for d in range(3):
            sc = sc * np.abs(tq[:, m2[:, d], mp2[:, d]])
        sc = sc.sum(0) / math.sqrt(math.pi)
        e = {}
        for (wname, leg), o in cfg_outs.items():
            if wname != wc.name:
                continue
            got = o.cpu().numpy()
            e[leg] = {"max_abs": float(np.max(np.abs(got - rc))),
                      "mean_abs": float(np.mean(np.abs(got - rc))),
                      "max_condition_aware": float(np.max(np.abs(got[::50] - rc[::50]) / sc))}
        cfg_errs[wc.name] = {"integrals": e, "E_H": eh, "E_x": ex}

    cpu = {"value": rate_all, "unit": "integrals/s", "cores": all_threads, "kind": "oracle",
           "sample": (f"{len(qs_all)} quadruples of the lookup stream (the first {len(qs_all) // 2} "
                      f"of each half); median of 5 runs after one warm-up"),
           "runs_s": ts_all,
           "one_core": {"value": rate_one, "cores": 1, "sample": f"{len(qs_one)} quadruples",
                        "runs_s": ts_one},
           "table_build_s": t_tab, "gpu_error_vs_oracle": errs}
    return cpu, converged, cfg_errs


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
    LEGS = (("fp64", pw.FP64, True), ("fp64_node_sums", pw.FP64, False), ("mixed", pw.MIXED, False),
            ("fp32", pw.FP32, False))
    out = {name: torch.empty(n, dtype=torch.float64, device="cuda") for name, _, _ in LEGS}
    eout = torch.empty(2, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()

    def step(prec, values, o):
        t = pw.Table(w.L, w.n2max, w.n_nodes)            # basis, mesh, primitives, layouts
        if values:
            t.build_values()                             # every distinct integral, Eq. 14
        t.reconstruct(quads, o, precision=prec)          # value reads, or decode + node passes
        t.energies_async(occ, None, pw.FP64 if prec == pw.FP32 else prec, eout)   # pair sums
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
    half = n // 2

    def per_half(name, prec):
        """The two halves of the stream timed apart: uniform over the basis,
        then over the occupied orbitals."""
        res = {}
        for key, sl in (("uniform", slice(0, half)), ("occupied", slice(half, n))):
            q, o = quads[sl], out[name][sl]
            ms = timed(lambda: t.reconstruct(q, o, precision=prec), args.kernel_reps)
            res[key] = {"reconstruct_ms": ms, "integrals_per_s": (sl.stop - sl.start) / (ms * 1e-3)}
        log(f"[bench] {name} per half: uniform {res['uniform']['reconstruct_ms']:.3f} ms, "
            f"occupied {res['occupied']['reconstruct_ms']:.3f} ms")
        return res
    if not args.no_per_half:
        legs["fp64"]["per_half"] = per_half("fp64", pw.FP64)
    log(f"[bench] fp64 values: build {legs['fp64']['value_build_ms']:.3f} ms "
        f"({nvalues} values), reads {legs['fp64']['reconstruct_ms']:.3f} ms")
    t.free_values()
    for name, prec, values in LEGS[1:]:
        t.reconstruct(quads, out[name], precision=prec)
        legs[name]["reconstruct_ms"] = timed(lambda: t.reconstruct(quads, out[name], precision=prec),
                                             args.kernel_reps)
        if not args.no_per_half:
            legs[name]["per_half"] = per_half(name, prec)
        # per launch: decode, then the node passes
        stages = np.array([t.reconstruct_profile(quads, out[name], precision=prec)[1]
                           for _ in range(args.kernel_reps)]).mean(axis=0)
        legs[name]["decode_ms"] = float(stages[0])
        legs[name]["pass_ms"] = [float(v) for v in stages[1:]]
        legs[name]["layout"] = t.layout(prec)
        legs[name]["fused"] = t.fused(prec)
        if prec == pw.FP32:      # the FP32 table serves reconstruction only
            log(f"[bench] {name}: reconstruct {legs[name]['reconstruct_ms']:.3f} ms "
                f"(decode {stages[0]:.3f} + passes {', '.join(f'{v:.3f}' for v in stages[1:])})")
            continue
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
    # Every output of the node-sum legs against the FP64 value-table leg (the
    # same integrals by another path), on the GPU over all n quadruples.
    all_vs_fp64 = {}
    for name in ("fp64_node_sums", "mixed", "fp32"):
        d = (out[name] - out["fp64"]).abs()
        all_vs_fp64[name] = {"max_abs": float(d.max()), "mean_abs": float(d.mean()), "n": n}
        del d
    log(f"[bench] all {n} outputs against the FP64 value table: "
        + ", ".join(f"{k} max {v['max_abs']:.2e}" for k, v in all_vs_fp64.items()))
    tb0 = time.perf_counter()
    for _ in range(5):
        pw.Table(w.L, w.n2max, w.n_nodes).close()
    table_ms = (time.perf_counter() - tb0) / 5 * 1e3
    e_fp64 = t.energies(occ)
    t.close()

    # Roofline of the step's dominant kernel, the value-table read.  The
    # algorithmic traffic per quadruple is 16 bytes of indices in and 8 bytes
    # out; the 8-byte value read is a cost of this design, not of the method,
    # and is reported apart ("design_bytes_per_quadruple").  One launch per call.
    gather_ms = legs["fp64"]["reconstruct_ms"]
    achieved = 24.0 * n / (gather_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBPS, "traffic": recorded_traffic("values"),
                "kernel": "k_rec_values (decode, one value read per quadruple)",
                "launches_per_call": 1, "algorithmic_bytes_per_quadruple": 24,
                "algorithmic_bytes_per_launch": 24.0 * n, "avg_launch_ms": gather_ms,
                "design_bytes_per_quadruple": 32,
                "design_GBps": 32.0 * n / (gather_ms * 1e-3) / 1e9,
                "kernel_source_sha256_16": kernel_hash("values")}
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
    # The node sums without a value table.  Algorithmic work of Eq. 14: 4
    # flops per node term (two products and an add), Q terms per integral; the
    # LDS reads are three entries per node term.  When the table runs fused
    # the whole call is one launch; the separate launches (per-launch timing
    # entry point, same results) are reported beside it.
    def node_entry(name, arith, peak, entry_bytes):
        lay, leg = legs[name]["layout"], legs[name]
        P, c = lay["passes"], lay["nodes_per_pass"]
        sep_ms = float(leg["decode_ms"] + np.sum(leg["pass_ms"]))
        steady = leg["pass_ms"][1:] or leg["pass_ms"]
        if leg["fused"]:
            ms, nodes, launches = leg["reconstruct_ms"], Q, 1
            kernel = f"k_rec_fused<{arith}> (all {P} node ranges of {c} in one launch)"
            hbm = 24.0 * n                      # indices in, integrals out
        else:
            ms, nodes, launches = float(np.mean(steady)), c, P
            kernel = f"k_rec_pass<{arith}, G={lay['lanes']}, W={lay['words']}> steady node pass"
            hbm = 20.0 * n                      # packed entries and partial sums in, sums out
        tf = 4.0 * nodes * n / (ms * 1e-3) / 1e12
        lds = 3 * entry_bytes * (P * c if leg["fused"] else c) * n / (ms * 1e-3) / 1e12
        return {"bound": "alu", "achieved": tf, "peak": peak, "unit": "TFLOP/s", "frac": tf / peak,
                "kernel": kernel, "launches_per_call": launches, "nodes_per_launch": nodes,
                "algorithmic_flops_per_launch": 4.0 * nodes * n, "avg_launch_ms": ms,
                "lds_read_TBps": lds, "lds_peak_TBps": LDS_PEAK_TBPS, "lds_frac": lds / LDS_PEAK_TBPS,
                "hbm_algorithmic_GBps": hbm / (ms * 1e-3) / 1e9,
                "whole_call_ms": leg["reconstruct_ms"],
                "whole_call_TFLOPs": 4.0 * Q * n / (leg["reconstruct_ms"] * 1e-3) / 1e12,
                "separate_launches_ms": sep_ms,
                "separate_steady_pass_ms": float(np.mean(steady)),
                "separate_first_pass_with_decode_ms": leg["pass_ms"][0]}
    node_pass_roofline = node_entry("fp64_node_sums", "F64", FP64_PEAK_TFLOPS, 8)
    node_pass_roofline["traffic"] = recorded_traffic("passes")
    node_pass_roofline["kernel_source_sha256_16"] = kernel_hash("passes")
    # The two FP32 arithmetics against the FP32 vector peak: split FP32
    # (a float-float node term takes about 16 FP32 instructions; 8-byte
    # entries) and the single-FP32 table (4-byte entries).
    mixed_pass = node_entry("mixed", "FF", FP32_PEAK_TFLOPS, 8)
    fp32_pass = node_entry("fp32", "F32", FP32_PEAK_TFLOPS, 4)

    cfg, cfg_outs = (None, {}) if args.no_configs else configs_leg(pw, args.steps, args.warmup)
    gauss, gauss_q, gauss_out = (None, None, None) if args.no_configs else gauss_leg(pw, args.steps, args.warmup)

    cpu, converged, cfg_errs = None, None, None
    if not args.no_cpu_baseline:
        cpu, converged, cfg_errs = cpu_baseline_leg(w, quads_h, N, M, n, out, cfg_outs)
        log(f"[bench] errors vs oracle: {cpu['gpu_error_vs_oracle']}")
    if cfg is not None and cfg_errs is not None:
        for name, e in cfg_errs.items():
            cfg[name]["error_vs_oracle"] = e
    del cfg_outs
    if gauss is not None and not args.no_cpu_baseline:
        gauss["error_vs_oracle"] = gauss_oracle_errors(gauss_q, gauss_out)
    gauss_q = gauss_out = None

    fixed_error = None
    if not args.no_fixed_error:
        fixed_error = fixed_error_leg(pw, w, quads, n, args.steps, args.warmup, converged)
        for label, pt in fixed_error["points"].items():
            for fam in ("mesh2", "mesh3"):
                log(f"[bench] fixed error {label} {fam}: Q {pt[fam]['Q']}, "
                    f"rates {pt[fam]['integrals_per_s']}")

    serving = None
    if not args.no_serve:
        log(f"[bench] serving leg: {args.serve_requests} requests")
        serving = serving_leg(pw, args.serve_requests)

    vb_bytes = legs["fp64"]["value_table_bytes"]
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
                   "value_table_bytes": vb_bytes,
                   "timed_path_device_bytes": table_bytes + vb_bytes,
                   "small_storage_path_device_bytes": table_bytes,
                   "step": "table build + value table + reconstruct all quads + E_H/E_x at M=925"},
        "value_small_storage": legs["fp64_node_sums"]["integrals_per_s"],
        "value_small_storage_ms_per_step": legs["fp64_node_sums"]["ms_per_step"],
        "value_small_storage_note": ("the same FP64 step on the O(N^{2/3}) tables alone (node sums, "
                                     f"{table_bytes} device bytes): no value table"),
        "pair_sums_per_s": {
            "M925_ktable": legs["fp64_node_sums"]["exchange_M925_ktable_pairs_per_s"],
            "M9171_ktable": legs["fp64_node_sums"]["exchange_M9171_ktable_pairs_per_s"],
            "M9171_nodesum": legs["fp64_node_sums"]["exchange_M9171_nodesum_pairs_per_s"]},
        "mixed_vs_fp64": {"integrals_per_s_ratio_node_sums": legs["mixed"]["integrals_per_s"] /
                          legs["fp64_node_sums"]["integrals_per_s"],
                          "integrals_per_s_ratio_vs_value_table": legs["mixed"]["integrals_per_s"] /
                          legs["fp64"]["integrals_per_s"],
                          "fp32_table_vs_fp64_node_sums": legs["fp32"]["integrals_per_s"] /
                          legs["fp64_node_sums"]["integrals_per_s"]},
        "errors_vs_fp64_value_table_all_outputs": all_vs_fp64,
        "p99_ms": serving["fp64_load_80"]["p99_ms"] if serving else None,
        "legs": legs,
        "table_build_ms": table_ms,
        "energies_fp64_M925": {"E_H": e_fp64[0], "E_x": e_fp64[1]},
        "configs": cfg,
        "gauss": gauss,
        "serving": serving,
        "roofline": roofline,
        "value_build": value_build,
        "node_pass_roofline": node_pass_roofline,
        "mixed_pass": mixed_pass,
        "fp32_pass": fp32_pass,
        "fixed_error": fixed_error,
        "cpu_baseline": cpu,
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
