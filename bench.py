#!/usr/bin/env python3
"""PiPNN build throughput on one MI355X.

One step is one pass of the whole hot path over the workload, with the
points already resident in HBM: sketches and norms, randomized ball carving,
the leaf pick + HashPrune on every leaf, and the final RobustPrune (Alg. 4).
The default workload is 1,000,000 x 128 integer-valued points (a seeded
1,000-cluster mixture stored as float32, BigANN-shaped), FP32 leaf GEMM,
C_max 2048, two leaves per point, k 16, l_max 64, R 32, alpha 1.2.

After the timed steps the graph of the last build is searched with 10,000
queries from the same mixture for recall@10 against exact brute force
(FP64), and the smallest beam width reaching 0.95 is reported.

`--prec` / `--rescore-mult` / `--rescore-extra` choose the leaf-GEMM form of
the measured build (default FP32). `variants` lists other forms (by default
bf16 exact, bf16 with FP32 rescoring of the top-2k and of the top k + 4, fp8
with rescoring of the top-2k, FP32 with two replicas of the partition, and
FP32 with the All-to-All Prune leaf picker) built, timed and searched the
same way on the same points after the main measurement.

Printed: one JSON line. `rooflines` holds every main kernel of the build
(leaf pick, partition, binning, merge, RobustPrune) against the roofline
that bounds it, each from its algorithmic work and its time per build from
HIP events recorded around it on its own stream during the timed steps;
`roofline` is the entry of the kernel that takes the most time (the fused
leaf distance + selection kernel on the default workload). `precision` is
the 1M x 96 vMF workload built with the float32, bf16 + rescore (top-2k
and top k + 4) and fp8 + rescore leaf GEMMs, with each form's error against
the FP64 oracle on sampled leaves. `cpu_baseline` is the FP64 oracle timed on a bounded sample
of the same build (each phase on a sample of its units, scaled by the unit
counts of the GPU build; phase times from the oracle's own steady clock),
plus the oracle's whole pipeline on the 10,000-point workload on one thread
and on all threads, and the host's CPU model.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# published dense MFMA peaks of one MI355X, TFLOP/s, by operand precision
PEAK_MFMA_TFLOPS = {"fp32": 157.3, "bf16": 2500.0, "fp16": 2500.0, "fp8": 5000.0}
PREC_CODES = {"fp32": 0, "bf16": 1, "fp8": 2, "fp16": 3}
RECALL_LS = [10, 12, 16, 20, 24, 32, 40, 48, 64, 80, 96, 128, 160, 192, 256, 384, 512]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", type=int, default=2)
    ap.add_argument("--n", type=int, default=None, help="override the point count")
    ap.add_argument("--queries", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-recall", action="store_true")
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the insert/query serving stage")
    ap.add_argument("--serve-requests", type=int, default=1000,
                    help="requests of the serving stage per load (80%% queries, 20%% insertions)")
    ap.add_argument("--serve-rates", default="0.25,0.5,0.75,1.0",
                    help="offered loads of the serving stage, as fractions of its closed-loop "
                         "capacity")
    ap.add_argument("--serve-recall-queries", type=int, default=1000,
                    help="queries per load whose recall@10 is checked against exact ground "
                         "truth at their epoch")
    ap.add_argument("--cpu-budget", type=float, default=4.0,
                    help="target seconds of oracle work per sampled phase")
    ap.add_argument("--prec", default=None, choices=sorted(PREC_CODES),
                    help="operand precision of the leaf GEMM of the measured build (default: "
                         "fp32, or fp16 for the 768-d workload)")
    ap.add_argument("--rescore-mult", type=int, default=0,
                    help="select rescore_mult*k by the GEMM distance, keep k by FP32 rescoring")
    ap.add_argument("--rescore-extra", type=int, default=0,
                    help="select k + rescore_extra by the GEMM distance, keep k by FP32 "
                         "rescoring (instead of --rescore-mult)")
    ap.add_argument("--variants", default="bf16:0,bf16:2,bf16:+4,fp8:2,fp32:0:2,fp32:0:1:a2a",
                    help="other forms (prec:rescore[:replicas[:a2a]], comma separated; rescore "
                         "is rescore_mult, or +e for rescore_extra e) built and timed after the "
                         "main one on the same workload (a2a: the All-to-All Prune leaf picker); "
                         "'' for none")
    ap.add_argument("--frontier", action="store_true",
                    help="also build (float32) with other fanouts, leaf k and l_max, and report "
                         "each one's build rate, the beam width reaching recall@10 >= 0.95 and "
                         "the search QPS there")
    ap.add_argument("--knn-graph", default="",
                    help="beam widths (comma separated): search every point of the main build's "
                         "graph for its 10 nearest other points (an approximate 10-NN graph), "
                         "timed, with recall@10 on a sample of 10,000 points")
    ap.add_argument("--no-precision", action="store_true",
                    help="skip the precision workload (1M x 96 vMF: FP32 vs bf16 and fp8 with "
                         "rescoring, error against FP64)")
    ap.add_argument("--precision-steps", type=int, default=3)
    ap.add_argument("--precision-queries", type=int, default=10000)
    ap.add_argument("--precision-leaves", type=int, default=40,
                    help="leaves of the precision workload whose picks are checked against FP64")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="after the timed steps, copy this many MiB once (a plain copy of known "
                         "size, used to scale hardware byte counters)")
    return ap.parse_args()


def ground_truth(torch, Xd, Qd, metric=0, k=10):
    """Exact k-th neighbour distance per query (squared L2, or negated inner
    product), FP64 on the GPU (evaluation only: the build never uses it)."""
    X64 = Xd.double()
    xn = (X64 * X64).sum(1)
    kth = torch.empty(Qd.shape[0], dtype=torch.float64, device="cuda")
    for q0 in range(0, Qd.shape[0], 512):
        q = Qd[q0:q0 + 512].double()
        if metric == 1:
            D = -(q @ X64.T)
            vals, ids = torch.topk(D, k, dim=1, largest=False)
            kth[q0:q0 + 512] = vals.max(1).values
        else:
            D = (q * q).sum(1, keepdim=True) + xn[None, :] - 2.0 * (q @ X64.T)
            vals, ids = torch.topk(D, k, dim=1, largest=False)
            # exact recomputation of the k winners by direct difference
            diff = X64[ids] - q[:, None, :]
            dd = (diff * diff).sum(-1)
            kth[q0:q0 + 512] = dd.max(1).values
        del D
    return kth


# Settings of the frontier: the paper's knobs around the workload's own
# (fanout {2,1,1,1}, leaf k 16, l_max 64, m 12 hash bits): the leaf k, the
# reservoir bound, single- or multi-level fanout, and the number of
# hyperplanes m of HashPrune's hash (the workload's hyperplanes are drawn for
# 16 and the first m are used).
FRONTIER = [
    {"fanout": (2, 1, 1, 1), "k": 16, "l_max": 64},
    {"fanout": (2, 1, 1, 1), "k": 8, "l_max": 64},
    {"fanout": (2, 1, 1, 1), "k": 12, "l_max": 64},
    {"fanout": (2, 1, 1, 1), "k": 24, "l_max": 64},
    {"fanout": (2, 1, 1, 1), "k": 16, "l_max": 32},
    {"fanout": (2, 1, 1, 1), "k": 16, "l_max": 48},
    {"fanout": (3, 1, 1, 1), "k": 16, "l_max": 64},
    {"fanout": (2, 2, 1, 1), "k": 16, "l_max": 64},
    {"fanout": (3, 2, 1, 1), "k": 12, "l_max": 64},
    {"fanout": (2, 1, 1, 1), "k": 16, "l_max": 64, "m": 8},
    {"fanout": (2, 1, 1, 1), "k": 16, "l_max": 64, "m": 10},
    {"fanout": (2, 1, 1, 1), "k": 16, "l_max": 64, "m": 14},
    {"fanout": (2, 1, 1, 1), "k": 16, "l_max": 64, "m": 16},
]


def knn_graph_stage(torch, np, idx, g, Xd, w, Ls, sample=10000):
    """Approximate 10-NN graph of the points (pipnn_knn_graph: every point
    searched on the built graph, its own id dropped), timed; recall@10 on a
    sample against exact ground truth (the 11th nearest including itself is
    the 10th nearest other point)."""
    n = Xd.shape[0]
    start = idx.start_node()
    rng = np.random.default_rng(2602)
    samp = np.sort(rng.choice(n, size=min(sample, n), replace=False)).astype(np.int64)
    sd = torch.from_numpy(samp).cuda()
    kth = ground_truth(torch, Xd, Xd[sd], w.metric, k=11)
    out = []
    for L in Ls:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ids, dist = idx.knn_graph(g, 10, max(11, L), start)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        hits = (dist[sd].double() <= kth[:, None]).sum().item()
        r = hits / (10.0 * len(samp))
        log(f"[bench] knn graph: L={L} {t:.2f} s ({n / t:.0f} points/s), recall@10 {r:.4f}")
        out.append({"L": L, "seconds": t, "points_per_s": n / t, "recall_at_10_sampled": r,
                    "sample": len(samp)})
    return out


# the sources of the float32 leaf kernel (four-lane layout) the committed
# counter runs were taken on
LEAF_KERNEL_SOURCES = ("knn_kernel.hpp", "knn_quad.hpp", "knn_fp32q.hip", "knn.hip")


def traffic_from_profiles(workload):
    """HBM bytes per leaf-kernel launch from committed counter runs, if they
    were taken on the current kernel source and on this workload."""
    path = os.path.join(ROOT, "profiles", "leaf_knn_hbm_traffic.json")
    csrc = os.path.join(ROOT, "paper_2602_21247_amd", "csrc")
    try:
        rec = json.load(open(path))
        h = hashlib.sha256(b"".join(open(os.path.join(csrc, f), "rb").read()
                                    for f in LEAF_KERNEL_SOURCES)).hexdigest()
        if rec.get("knn_hip_sha256") != h or workload not in rec.get("kernel", ""):
            return None
        return rec.get("bytes_per_launch")
    except Exception:
        return None


def cpu_model() -> str:
    """The host CPU's model name (lscpu, else /proc/cpuinfo)."""
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.lower().startswith("model name"):
                return line.split(":", 1)[1].strip()
    except Exception:
        pass
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except Exception:
        pass
    return "unknown"


def oracle_full_build(np, pi, cfg, threads_list):
    """The whole oracle pipeline (Alg. 4: partition, leaf pick, HashPrune,
    RobustPrune, with the sketches) on workload `cfg` at its full size, once
    per thread count; per-phase wall times from the oracle's own steady clock,
    and recall@10 of its graph at a few beam widths."""
    import oracle
    w = pi.WORKLOADS[cfg]
    X = pi.workload_points(cfg)
    H = pi.workload_hyperplanes(cfg)
    op = oracle.make_params(metric=w.metric, c_max=w.c_max, c_min=w.c_min,
                            leader_div=w.leader_div, leader_cap=w.leader_cap,
                            fanout=tuple(w.fanout), k=w.k, hash_bits=w.hash_bits, l_max=w.l_max,
                            R=w.R, alpha=w.alpha, seed=pi.workload_seed(cfg))
    runs = {}
    ref = None
    for th in threads_list:
        oracle.set_threads(th)
        oracle.phase_seconds(reset=True)
        ref = oracle.build_index(X, H, op)
        ph = oracle.phase_seconds(reset=True)
        wall = sum(ph[k] for k in ("sketches", "partition", "leaf_pick", "hashprune",
                                   "robustprune"))
        runs[str(oracle.get_threads())] = {"build_s": wall, "points_per_s": X.shape[0] / wall,
                                           "phase_s": {k: v for k, v in ph.items() if v > 0}}
    Q = pi.workload_queries(cfg)
    start, _ = oracle.start_node(X)
    _, gd = oracle.bruteforce_knn(X, Q, 10, metric=w.metric)
    curve = {}
    for L in (16, 32, 64, 128):
        ids, _, _ = oracle.beam_search(X, ref["graph"], Q, 10, L, start, metric=w.metric)
        curve[L] = round(oracle.recall_at_k(ids, X, Q, gd, metric=w.metric), 5)
    return {"workload": w.name, "n": int(X.shape[0]), "runs_by_threads": runs,
            "recall_at_10_by_L": curve}


def cpu_baseline(X, H, off, mem, res_np, stats, w, budget):
    """The FP64 oracle on a bounded sample of this build, phase by phase
    (each phase's wall time read from the oracle's own steady clock, scaled
    by the GPU build's unit counts), plus the whole oracle pipeline of the
    10,000-point correctness workload on one thread and on all threads."""
    import numpy as np

    import oracle
    import pipnn_inputs as pi
    oracle.lib()
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or (os.cpu_count() or 1)
    oracle.set_threads(threads)
    threads = oracle.get_threads()
    n, d = X.shape
    rng = np.random.default_rng(12345)
    notes = []
    total = 0.0

    def timed(phase, fn, *a, **kw):
        oracle.phase_seconds(reset=True)
        out = fn(*a, **kw)
        return out, oracle.phase_seconds(reset=True)[phase]

    # partition: point-to-leader distances with top-f selection (none when
    # the leaves are given)
    t_part = 0.0
    if stats["leader_dists"] > 0:
        ell = min(w.leader_cap, max(2, -(-n // w.leader_div)), n)
        leaders = X[rng.choice(n, ell, replace=False)]
        m = 2000
        _, dt = timed("bruteforce_knn", oracle.bruteforce_knn, leaders,
                      X[rng.choice(n, m, replace=False)], 2, metric=w.metric)
        m2 = int(min(n, max(m, m * budget / max(dt, 1e-3))))
        _, dt = timed("bruteforce_knn", oracle.bruteforce_knn, leaders,
                      X[rng.choice(n, m2, replace=False)], 2, metric=w.metric)
        t_part = dt * stats["leader_dists"] / float(m2 * ell)
        total += t_part
        notes.append(f"partition: {m2} points x {ell} leaders "
                     f"(x{stats['leader_dists'] / (m2 * ell):.0f})")

    # leaf pick: a random sample of the GPU build's leaves, grown after a
    # first timing so that it takes about `budget` seconds
    nl = len(off) - 1
    order = rng.permutation(nl)
    sizes = np.diff(off)
    pairs_tot = float((sizes.astype(np.float64) ** 2).sum())

    def leaf_sample(frac):
        pick, acc = [], 0.0
        for i in order:
            if acc >= pairs_tot * frac and len(pick) >= 4:
                break
            pick.append(i)
            acc += float(sizes[i]) ** 2
        s_off = np.concatenate([[0], np.cumsum(sizes[pick])]).astype(np.int64)
        s_mem = np.concatenate([mem[off[i]:off[i + 1]] for i in pick]).astype(np.uint32)
        return pick, acc, s_off, s_mem

    pick, acc, s_off, s_mem = leaf_sample(0.001)
    (cand, dist), dt = timed("leaf_pick", oracle.leaf_knn, X, s_off, s_mem, w.k, metric=w.metric)
    if dt < budget / 2 and acc < pairs_tot:
        pick, acc, s_off, s_mem = leaf_sample(min(1.0, acc / pairs_tot * budget / max(dt, 1e-3)))
        (cand, dist), dt = timed("leaf_pick", oracle.leaf_knn, X, s_off, s_mem, w.k,
                                 metric=w.metric)
    t_leaf = dt * pairs_tot / acc
    total += t_leaf
    notes.append(f"leaf pick: {len(pick)} leaves, {acc / pairs_tot * 100:.2f}% of pairs")

    # sketches of every point
    ns_sk = min(n, 100000)
    _, dt = timed("sketches", oracle.sketches, X[:ns_sk], H)
    t_sk = dt * n / ns_sk
    total += t_sk
    notes.append(f"sketches: {ns_sk} points")

    # HashPrune: the sampled leaves' records, ids renumbered densely
    dst, cnd, dv = oracle.bidirected_records(s_mem, cand, dist)
    uniq, inv = np.unique(np.concatenate([dst, cnd]), return_inverse=True)
    dst_c = inv[:len(dst)].astype(np.uint32)
    cnd_c = inv[len(dst):].astype(np.uint32)
    S = oracle.sketches(X[uniq], H)
    _, dt = timed("hashprune", oracle.hashprune, oracle.reservoir_init(len(uniq), w.l_max), S,
                  dst_c, cnd_c, dv)
    t_hp = dt * stats["records"] / max(1, len(dst))
    total += t_hp
    notes.append(f"HashPrune: {len(dst)} records ({len(dst) / max(1, stats['records']) * 100:.2f}%)")

    # RobustPrune: the reservoirs of the first points (grown like the leaf sample)
    ns = min(n, 20000)
    _, dt = timed("robustprune", oracle.robustprune, X, res_np[:ns], w.alpha, w.R,
                  metric=w.metric)
    if dt < budget / 2 and ns < n:
        ns = int(min(n, ns * budget / max(dt, 1e-3)))
        _, dt = timed("robustprune", oracle.robustprune, X, res_np[:ns], w.alpha, w.R,
                      metric=w.metric)
    t_rp = dt * n / ns
    total += t_rp
    notes.append(f"RobustPrune: {ns} points")
    full = oracle_full_build(np, pi, 1, [1, threads])
    oracle.set_threads(threads)
    return {
        "value": n / total, "unit": "points/s", "cores": threads, "kind": "oracle",
        "sample": "; ".join(notes) + "; each phase scaled by the GPU build's unit counts",
        "cpu_model": cpu_model(),
        "phase_s": {"sketches": t_sk, "partition": t_part, "leaf_pick": t_leaf,
                    "hashprune": t_hp, "robustprune": t_rp},
        "full_pipeline_small_workload": full,
    }


def rescore_kw(spec):
    """A form's rescoring from its spec: '0' none, 'r' rescore_mult r, '+e'
    rescore_extra e."""
    t = str(spec)
    if t.startswith("+"):
        return {"rescore_mult": 0, "rescore_extra": int(t[1:])}
    return {"rescore_mult": int(t), "rescore_extra": 0}


def rescore_label(spec):
    kw = rescore_kw(spec)
    return f"+{kw['rescore_extra']}" if kw["rescore_extra"] else f"x{kw['rescore_mult']}"


def precision_stage(args, torch, np, pp, pi):
    """The precision workload (1,000,000 unit vectors of 96 dimensions from a
    vMF mixture, L2): the float32 leaf GEMM, bf16 and OCP e4m3 with FP32
    rescoring of the top 2k, each built and timed the same way on the same
    points (the partition is float32 for all three: the 16-bit copies do not
    hold this data exactly), searched at the same beam widths, and the
    error of each form's leaf picks against the FP64 oracle's on a random
    sample of the leaves: the share of FP64 picks found, and the largest
    error of an emitted distance (against the FP64 distance of the same
    pair)."""
    import oracle
    cfg = 3
    w = pi.WORKLOADS[cfg]
    log(f"[bench] precision workload {w.name}: generating")
    X = pi.workload_points(cfg)
    H = pi.workload_hyperplanes(cfg)
    n = X.shape[0]
    Xd, Hd = torch.from_numpy(X).cuda(), torch.from_numpy(H).cuda()
    Qd = torch.from_numpy(pi.workload_queries(cfg, args.precision_queries)).cuda()
    kth = ground_truth(torch, Xd, Qd, w.metric)
    nq = Qd.shape[0]
    forms = []
    sample = None
    for prec, mult in (("fp32", 0), ("bf16", 2), ("bf16", "+4"), ("fp8", 2)):
        p = pp.default_params(metric=w.metric, c_max=w.c_max, c_min=w.c_min, k=w.k,
                              l_max=w.l_max, R=w.R, alpha=w.alpha, hash_bits=w.hash_bits,
                              leader_div=w.leader_div, leader_cap=w.leader_cap, fanout=w.fanout,
                              seed=pi.workload_seed(cfg), gemm_prec=PREC_CODES[prec],
                              **rescore_kw(mult))
        idx = pp.Index(Xd, Hd, p)
        res = torch.empty((n, w.l_max), dtype=torch.int64, device="cuda")

        def step():
            idx.prepare()
            pp.reservoir_init(n, w.l_max, out=res)
            off, mem = idx.partition()
            idx.build_leaves(off, mem, res)
            g, deg = idx.robustprune(res)
            return off, mem, g

        step()
        torch.cuda.synchronize()
        idx.set_profiling(True)
        t0 = time.perf_counter()
        for _ in range(args.precision_steps):
            off, mem, g = step()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1000.0 / args.precision_steps
        st = idx.stats()
        idx.set_profiling(False)
        start = idx.start_node()
        curve = {}
        for L in (64, 128, 256, 512):
            ids, dist, _ = idx.search(g, Qd, 10, L, start, want_cmps=False)
            curve[L] = round((dist.double() <= kth[:, None]).sum().item() / (nq * 10.0), 5)
        # picks of every leaf row, compared on a sample of leaves with FP64
        cand, dd = idx.leaf_pick(off, mem)
        torch.cuda.synchronize()
        off_h, mem_h = off.cpu().numpy(), mem.cpu().numpy().view(np.uint32)
        if sample is None:
            rng = np.random.default_rng(303)
            nl = len(off_h) - 1
            sample = np.sort(rng.choice(nl, min(nl, args.precision_leaves), replace=False))
        s_sizes = np.diff(off_h)[sample]
        s_off = np.concatenate([[0], np.cumsum(s_sizes)]).astype(np.int64)
        s_mem = np.concatenate([mem_h[off_h[i]:off_h[i + 1]] for i in sample])
        rows = np.concatenate([np.arange(off_h[i], off_h[i + 1]) for i in sample])
        ocand, odist = oracle.leaf_knn(X, s_off, s_mem, w.k, metric=w.metric)
        gc = cand.cpu().numpy().view(np.uint32)[rows]
        gd = dd.cpu().numpy()[rows].astype(np.float64)
        agree = float(np.mean([len(set(a[a != 0xFFFFFFFF]) & set(b[b != 0xFFFFFFFF]))
                               / max(1, (b != 0xFFFFFFFF).sum()) for a, b in zip(gc, ocand)]))
        # FP64 distance of each emitted pair, from the emitting row's point
        valid = gc != 0xFFFFFFFF
        Xs = X.astype(np.float64)
        src = np.repeat(s_mem.astype(np.int64), w.k).reshape(gc.shape)[valid]
        dst = gc[valid].astype(np.int64)
        d64 = ((Xs[src] - Xs[dst]) ** 2).sum(1)
        err = np.abs(gd[valid] - d64)
        rel = err / np.maximum(np.abs(d64), 1e-30)
        within = float(np.mean(err <= np.maximum(1e-5 * np.abs(d64), 1e-6)))
        f = {"prec": prec, **rescore_kw(mult), "ms_per_step": ms, "points_per_s": n / (ms / 1e3),
             "recall_at_10_by_L": curve,
             "leaf_gemm_tflops": 2.0 * st["leaf_pairs"] * w.d * args.precision_steps
             / max(1, st["leaf_knn_launches"]) / (st["ms_leaf_knn"] / max(1, st["leaf_knn_launches"])
                                                  / 1e3) / 1e12,
             "phase_ms": {k: st[k] / args.precision_steps for k in
                          ("ms_prepare", "ms_partition", "ms_leaf_knn", "ms_bin", "ms_merge",
                           "ms_robustprune")},
             "vs_fp64": {"leaves": int(len(sample)), "rows": int(len(rows)),
                         "pick_agreement": agree, "max_abs_dist_err": float(err.max()),
                         "max_rel_dist_err": float(rel.max()),
                         "share_within_1e-5_rel": within}}
        log(f"[bench] precision {prec} {rescore_label(mult)}: {ms:.2f} ms/build, recall {curve}, "
            f"picks vs FP64 {agree:.5f}, max rel err {rel.max():.2e}")
        forms.append(f)
        idx.close()
        del res
    return {"workload": w.name, "n": n, "d": w.d, "queries": nq, "forms": forms}


def kernel_rooflines(st, w, n, steps, res_valid, rp_elem, prec):
    """Achieved rate of each main kernel of one build against the roofline
    that bounds it, from the HIP-event phase times (ms per build) and the
    algorithmic work of the build:
      leaf pick: 2 d sum(s^2) flops (every pair of every leaf; MFMA peak of
        the operand's precision);
      partition: 2 d flops per point-to-leader distance (float32 MFMA);
      binning: 12 B per record (4 B of the pick and distance that yield it,
        8 B of slot written) + m 4 B of sketch per leaf member (HBM);
      merge: 8 B per binned record read + 2 l_max 8 B per point (reservoir
        read and written; HBM);
      RobustPrune: the candidates' rows (valid reservoir slots x d x the
        element size of the rows it reads: 1 B int8, 2 B of a 16-bit copy
        or 4 B float32) + l_max 8 B of reservoir and R 4 B of graph per point
        (HBM)."""
    d = w.d
    per = lambda k: st[k] / steps    # phase times are summed over the timed builds
    rec = st["records"]              # counts are those of the last build
    pairs = st["leaf_pairs"]
    hbm = 8000.0
    out = {}

    def put(name, ms, amount, unit, peak, bound):
        if ms <= 0:
            return
        a = amount / (ms / 1e3) / (1e12 if unit == "TFLOP/s" else 1e9)
        out[name] = {"bound": bound, "ms": ms, "achieved": a, "peak": peak, "unit": unit,
                     "frac": a / peak, "work": amount}

    put("leaf_knn", per("ms_leaf_knn"), 2.0 * d * pairs, "TFLOP/s", PEAK_MFMA_TFLOPS[prec], "mfma")
    if "leaf_knn" in out:
        out["leaf_knn"]["precision"] = prec
    # the partition multiplies the exact 16-bit copy where there is one
    part_prec = "fp32" if not st["operand_exact"] or d > 256 else (
        prec if prec in ("bf16", "fp16") else "fp16")
    put("partition", per("ms_partition"), 2.0 * d * st["leader_dists"], "TFLOP/s",
        PEAK_MFMA_TFLOPS[part_prec], "mfma")
    if "partition" in out:
        out["partition"]["precision"] = part_prec
    put("bin", per("ms_bin"), 12.0 * rec + st["n_members"] * w.hash_bits * 4.0, "GB/s", hbm, "hbm")
    put("merge", per("ms_merge"), 8.0 * rec + 16.0 * w.l_max * n, "GB/s", hbm, "hbm")
    put("robustprune", per("ms_robustprune"),
        res_valid * d * rp_elem + n * (8.0 * w.l_max + 4.0 * w.R), "GB/s", hbm, "hbm")
    return out


def serving_stage(args, torch, np, pp, pi, w, cfg, X, H, p_kw, L_serve):
    """Insert/query serving on the workload's index: the seeded request
    stream (80% k=10 query batches of floor(exp(U(0, ln 4097))) queries, 20%
    insertion batches of floor(exp(U(0, ln 50001))) fresh points of the same
    mixture) first arrives all at once (closed loop: the capacity in
    requests/s), then as a Poisson process at each of --serve-rates times
    that capacity, each on a fresh copy of the index that starts with room
    for one largest insertion and grows its capacity as insertions need it
    (admitted by free HBM). Per rate: p50/p99 latency per request class,
    inserts/s, QPS, capacity growths, and recall@10 of sampled queries
    against exact ground truth over the points committed at their epoch."""
    from paper_2602_21247_amd import serving
    rng = np.random.default_rng(5)
    n = X.shape[0]
    nreq = args.serve_requests
    kinds = rng.random(nreq) < 0.8
    sizes_q = np.floor(np.exp(rng.uniform(0, np.log(4097), nreq))).astype(int)
    sizes_i = np.floor(np.exp(rng.uniform(0, np.log(50001), nreq))).astype(int)
    n_ins = int(sizes_i[~kinds].sum())
    newpts = pi.integer_mixture(n_ins, w.d, 1000, pi.INT_MIXTURE_SIGMA, seed=5005,
                                center_seed=2) if cfg == 2 else pi.workload_points(cfg, n + n_ins)[n:]
    nq = int(sizes_q[kinds].sum())
    Qall = pi.workload_queries(cfg, nq)
    reqs_proto = []
    qo = io = 0
    for rid in range(nreq):
        if kinds[rid]:
            m = int(sizes_q[rid])
            reqs_proto.append(("query", Qall[qo:qo + m]))
            qo += m
        else:
            m = int(sizes_i[rid])
            reqs_proto.append(("insert", newpts[io:io + m]))
            io += m
    cap0 = n + 50_000   # room for one largest insertion; the server grows the rest

    def fresh():
        Xc = torch.empty((cap0, w.d), dtype=torch.float32, device="cuda")
        Xc[:n].copy_(torch.from_numpy(X))
        params = pp.default_params(**p_kw)
        idx = pp.Index(Xc[:n], torch.from_numpy(H).cuda(), params)
        off, mem = idx.partition()
        res = torch.empty((cap0, w.l_max), dtype=torch.int64, device="cuda")
        pp.reservoir_init(n, w.l_max, out=res[:n])
        idx.build_leaves(off, mem, res[:n])
        g = torch.full((cap0, w.R), -1, dtype=torch.int32, device="cuda")
        deg = torch.zeros(cap0, dtype=torch.int32, device="cuda")
        idx.robustprune(res[:n], g[:n], deg[:n])
        idx.reserve(cap0)
        start = idx.start_node()
        torch.cuda.synchronize()
        return idx, Xc, res, g, deg, start

    def run(arrivals):
        idx, Xc, res, g, deg, start = fresh()
        reqs = [serving.Request(i, kd, float(arrivals[i]), data)
                for i, (kd, data) in enumerate(reqs_proto)]
        srv = serving.Server(idx, Xc, res, g, deg, start, serving.ServerConfig(L=L_serve))
        t0 = time.perf_counter()
        out = srv.run(reqs)
        wall = time.perf_counter() - t0
        return out, wall, idx, srv

    def recall_by_epoch(out, srv, budget):
        """recall@10 of up to `budget` queries spread over the run's epochs,
        each against the points committed when it ran; overall and the
        lowest of the run's epoch quartiles."""
        commit_n = {0: n}
        for r in sorted((r for r in out.values() if r.kind == "insert" and r.status == "ok"),
                        key=lambda r: r.first_id):
            commit_n[r.batch + 1] = r.first_id + len(reqs_proto[r.rid][1])
        qreqs = sorted((r for r in out.values() if r.kind == "query"), key=lambda r: r.epoch)
        if not qreqs:
            return None, None, 0
        step = max(1, len(qreqs) * 40 // max(1, budget))
        picked = qreqs[::step]
        hits = tot = 0
        per_q = []
        for r in picked:
            if tot >= budget * 10:
                break
            ne = max(v for b, v in commit_n.items() if b <= r.epoch)
            Q = reqs_proto[r.rid][1][:64]
            kth = ground_truth(torch, srv.X[:ne], torch.from_numpy(Q).cuda(), w.metric)
            hq = int((torch.from_numpy(r.dist[:64]).cuda().double() <= kth[:, None]).sum().item())
            hits += hq
            tot += Q.shape[0] * 10
            per_q.append((r.epoch, hq / (Q.shape[0] * 10.0)))
        quart = np.array_split(np.array([v for _, v in per_q]), 4)
        low = min(float(np.mean(qv)) for qv in quart if len(qv))
        return hits / max(1, tot), low, tot // 10

    out, wall, idx, srv = run(np.zeros(nreq))
    capacity = nreq / wall
    idx.close()
    del srv
    log(f"[bench] serving: closed loop {nreq} requests in {wall:.2f} s "
        f"({capacity:.1f} requests/s)")
    ins_pts = sum(len(d) for kd, d in reqs_proto if kd == "insert")
    qs = sum(len(d) for kd, d in reqs_proto if kd == "query")
    rates = []
    for frac in [float(v) for v in args.serve_rates.split(",") if v.strip()]:
        rate = frac * capacity
        arr = np.cumsum(np.random.default_rng(55).exponential(1.0 / rate, nreq))
        out, wall, idx, srv = run(arr)
        summ = serving.summarize(out, wall)
        recall, low, sampled = recall_by_epoch(out, srv, args.serve_recall_queries)
        ent = {"load": frac, "offered_requests_per_s": rate, "wall_s": wall,
               "inserts_per_s": ins_pts / wall, "qps": qs / wall,
               "capacity_growths": len(srv.growths),
               "growth_ms": [round(t * 1e3, 1) for _, t in srv.growths],
               "final_capacity": srv.cap, "rejected": srv.rejected,
               "recall_at_10_sampled": recall, "recall_lowest_epoch_quartile": low,
               "recall_sample_queries": sampled}
        ent.update(summ)
        log(f"[bench] serving at {frac:.2f} x capacity ({rate:.1f} requests/s): {summ}; "
            f"recall@10 {recall:.4f}, growths {len(srv.growths)}")
        idx.close()
        del srv
        rates.append(ent)
    return {"requests_per_rate": nreq, "closed_loop_requests_per_s": capacity, "L": L_serve,
            "inserted_points": ins_pts, "queries": qs, "initial_capacity": cap0,
            "rates": rates}


def insert_p99(serve):
    """Insertion p99 of the serving stage at half its capacity (the load the
    headline latency is quoted at), else at the lowest load measured."""
    if not serve or not serve.get("rates"):
        return None
    rates = [r for r in serve["rates"] if "insert" in r]
    if not rates:
        return None
    half = [r for r in rates if abs(r["load"] - 0.5) < 1e-9]
    return (half or sorted(rates, key=lambda r: r["load"]))[0]["insert"]["p99_ms"]


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(sharding across GPUs is not built)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2602_21247_amd as pp
    import pipnn_inputs as pi

    if not torch.cuda.is_available():
        print("bench.py needs a ROCm GPU", file=sys.stderr)
        sys.exit(2)
    if not os.path.exists(pp.LIB_PATH):
        from paper_2602_21247_amd import hipbuild
        hipbuild.build()
    cfg = args.workload
    w = pi.WORKLOADS[cfg]
    if args.prec is None:
        args.prec = "fp16" if w.d > 256 else "fp32"
    n = args.n or w.n
    log(f"[bench] generating workload {cfg} ({w.name}) n={n}")
    X = pi.workload_points(cfg, n)
    H = pi.workload_hyperplanes(cfg)
    Xd = torch.from_numpy(X).cuda()
    Hd = torch.from_numpy(H).cuda()
    # hyperplanes for other hash widths m (frontier): the first m rows of a
    # 16-row draw with the workload's generator
    Hm = {}
    if args.frontier:
        H16 = pi.workload_hyperplanes(cfg, m=16)
        for o in FRONTIER:
            if "m" in o:
                Hm[o["m"]] = torch.from_numpy(np.ascontiguousarray(H16[:o["m"]])).cuda()
    Qd = kth = None
    if not args.no_recall:
        nq = args.queries or w.n_queries
        Qd = torch.from_numpy(pi.workload_queries(cfg, nq)).cuda()
        kth = ground_truth(torch, Xd, Qd, w.metric)

    leaves = None
    if cfg == 4:
        lo, lm = pi.workload_leaves(cfg, n, X=X)
        leaves = (torch.from_numpy(lo).cuda(), torch.from_numpy(lm.view(np.int32)).cuda())
        log(f"[bench] explicit leaves: {len(lo) - 1}, sizes {np.diff(lo).min()}..{np.diff(lo).max()}")

    def run_form(prec, mult, steps, warmup, keep=False, replicas=1, over=None, picker=0):
        """Build the whole index `warmup + steps` times with one leaf-GEMM
        form (and `replicas` independent partitions feeding the reservoirs);
        time the last `steps`; search the last graph for recall@10.
        With given leaves, the leaf kernel is autotuned on them, one eager
        build is profiled for the phase times, and the timed builds are
        replays of one captured HIP graph of the whole step. `over` replaces
        the workload's fanout, k or l_max."""
        over = over or {}
        fk, fl, ff = over.get("k", w.k), over.get("l_max", w.l_max), over.get("fanout", w.fanout)
        fm = over.get("m", w.hash_bits)
        p = pp.default_params(metric=w.metric, c_max=w.c_max, c_min=w.c_min, k=fk,
                              l_max=fl, R=w.R, alpha=w.alpha, hash_bits=fm,
                              leader_div=w.leader_div, leader_cap=w.leader_cap, fanout=ff,
                              seed=pi.workload_seed(cfg), gemm_prec=PREC_CODES[prec],
                              leaf_picker=picker, **rescore_kw(mult))
        idx = pp.Index(Xd, Hm.get(fm, Hd), p)
        res = torch.empty((n, fl), dtype=torch.int64, device="cuda")
        tune = None

        if leaves is None:
            def step():
                idx.prepare()
                pp.reservoir_init(n, fl, out=res)
                for r in range(replicas):
                    off, mem = idx.partition(r)
                    idx.build_leaves(off, mem, res)
                g, deg = idx.robustprune(res)
                return off, mem, g, deg

            for i in range(warmup):
                step()
                torch.cuda.synchronize()
                log(f"[bench] {prec} {rescore_label(mult)} r{replicas}: warmup {i + 1}/{warmup} done")
            torch.cuda.synchronize()
            idx.set_profiling(True)
            t0 = time.perf_counter()
            for i in range(steps):
                out = step()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            st = idx.stats()
            idx.set_profiling(False)
            off, mem, g, deg = out
        else:
            off, mem = leaves
            tune = idx.autotune(off, mem)
            log(f"[bench] {prec} {rescore_label(mult)} r{replicas}: autotune {tune}")
            g = torch.empty((n, w.R), dtype=torch.int32, device="cuda")
            deg = torch.empty(n, dtype=torch.int32, device="cuda")

            def step():
                idx.prepare()
                pp.reservoir_init(n, fl, out=res)
                idx.build_leaves(off, mem, res)
                idx.robustprune(res, g, deg)

            step()  # eager warm-up
            torch.cuda.synchronize()
            idx.set_profiling(True)
            step()  # eager, profiled: phase times and the leaf-kernel launch time
            torch.cuda.synchronize()
            st = idx.stats()
            st = {k: (v * steps if k.startswith("ms_") or k == "leaf_knn_launches" else v)
                  for k, v in st.items()}
            idx.set_profiling(False)
            idx.plan_leaves(off, mem)
            graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(graph):
                step()
            for i in range(warmup):
                graph.replay()
                torch.cuda.synchronize()
                log(f"[bench] {prec} {rescore_label(mult)} r{replicas}: warmup replay {i + 1}/{warmup} done")
            t0 = time.perf_counter()
            for i in range(steps):
                graph.replay()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
        ms = (t1 - t0) * 1000.0 / steps
        log(f"[bench] {prec} {rescore_label(mult)} r{replicas}{' a2a' if picker else ''}: {steps} steps, {ms:.2f} ms/step")
        # leaf kernel roofline: dense flops 2 s^2 d per leaf, per launch
        launches = max(1, st["leaf_knn_launches"])
        # leaf_pairs counts the last build_leaves call: one replica's leaves
        flops_per_launch = 2.0 * st["leaf_pairs"] * replicas * w.d * steps / launches
        avg_launch_s = st["ms_leaf_knn"] / launches / 1000.0
        achieved = flops_per_launch / avg_launch_s / 1e12
        phases = {k: st[k] / steps for k in ("ms_prepare", "ms_partition", "ms_leaf_knn",
                                              "ms_bin", "ms_merge", "ms_robustprune")}
        recall, l_at, curve, qps = None, None, {}, None
        if Qd is not None:
            start = idx.start_node()
            nq = Qd.shape[0]
            for L in RECALL_LS:
                ids, dist, cmps = idx.search(g, Qd, 10, L, start)
                hits = (dist.double() <= kth[:, None]).sum().item()
                r = hits / (nq * 10.0)
                curve[L] = {"recall": round(r, 5), "cmps": round(cmps.double().mean().item(), 1)}
                log(f"[bench] {prec} {rescore_label(mult)} r{replicas}: L={L} recall@10={r:.4f} cmps={curve[L]['cmps']}")
                if r >= 0.95:
                    l_at, recall = L, r
                    break
            if recall is None:
                recall = max(v["recall"] for v in curve.values())
            # search throughput at that beam width: the same batch once more, timed
            torch.cuda.synchronize()
            tq = time.perf_counter()
            idx.search(g, Qd, 10, l_at or RECALL_LS[-1], start, want_cmps=False)
            torch.cuda.synchronize()
            qps = nq / (time.perf_counter() - tq)
        form = {"prec": prec, **rescore_kw(mult), "replicas": replicas,
                "leaf_picker": "all-to-all-prune" if picker else "bi-directed-knn",
                "ms_per_step": ms,
                "value": n / (ms / 1000.0),
                "leaf_gemm_tflops": achieved, "peak": PEAK_MFMA_TFLOPS[prec],
                "frac": achieved / PEAK_MFMA_TFLOPS[prec], "recall_at_10": recall,
                "L_at_recall_0.95": l_at, "search_qps_at_L": qps, "recall_curve": curve,
                "phase_ms": phases, "stats": st, "autotune": tune}
        if over:
            form["params"] = {"fanout": list(ff), "k": fk, "l_max": fl, "m": fm}
        if keep:
            form["_out"] = (idx, res, off, mem, g, deg)
        else:
            idx.close()
        return form

    main_resc = f"+{args.rescore_extra}" if args.rescore_extra else str(args.rescore_mult)
    main_form = run_form(args.prec, main_resc, args.steps, args.warmup, keep=True)
    idx, res, off, mem, g, deg = main_form.pop("_out")
    st = main_form.pop("stats")
    ms = main_form["ms_per_step"]
    achieved = main_form["leaf_gemm_tflops"]
    if args.calibrate_copy_mib > 0:
        # a fill (writes N MiB) and a sum (reads N MiB) of known size
        src = torch.ones(args.calibrate_copy_mib * 262144, dtype=torch.float32, device="cuda")
        total = src.sum()
        torch.cuda.synchronize()
        log(f"[bench] calibration: {args.calibrate_copy_mib} MiB filled and summed ({total.item():.0f})")
        del src

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] timing the FP64 oracle on a sample")
        cpu = cpu_baseline(X, H, off.cpu().numpy(), mem.cpu().numpy().view(np.uint32),
                           res.cpu().numpy().view(np.uint64), st, w, args.cpu_budget)

    variants = []
    for spec in [v for v in args.variants.split(",") if v.strip()]:
        parts = spec.split(":")
        vp, vm = parts[0], parts[1]
        vr = int(parts[2]) if len(parts) > 2 else 1
        va = 1 if len(parts) > 3 and parts[3] == "a2a" else 0
        if (vp, rescore_kw(vm), vr, va) == (args.prec, rescore_kw(main_resc), 1, 0):
            continue
        if leaves is not None and (vr > 1 or va):
            continue  # explicit leaves: no partition to replicate; leaves above 2,048
        f = run_form(vp, vm, min(args.steps, 5) if va else args.steps, 1, replicas=vr,
                     picker=va)
        f.pop("stats")
        variants.append(f)

    frontier = None
    if args.frontier and leaves is None:
        frontier = []
        for o in FRONTIER:
            f = run_form("fp32", 0, 2, 1, over=o)
            f.pop("stats")
            f.pop("recall_curve")
            frontier.append(f)

    knn_graph = None
    if args.knn_graph:
        knn_graph = knn_graph_stage(torch, np, idx, g, Xd, w,
                                    [int(v) for v in args.knn_graph.split(",") if v.strip()])

    serve = None
    if not args.no_serving and cfg in (2, 3):
        p_kw = dict(metric=w.metric, c_max=w.c_max, c_min=w.c_min, k=w.k, l_max=w.l_max, R=w.R,
                    alpha=w.alpha, hash_bits=w.hash_bits, leader_div=w.leader_div,
                    leader_cap=w.leader_cap, fanout=w.fanout, seed=pi.workload_seed(cfg),
                    gemm_prec=PREC_CODES[args.prec], **rescore_kw(main_resc))
        L_serve = main_form["L_at_recall_0.95"] or 128
        serve = serving_stage(args, torch, np, pp, pi, w, cfg, X, H, p_kw, L_serve)

    precision = None
    if cfg == 2 and not args.no_precision:
        precision = precision_stage(args, torch, np, pp, pi)

    traffic = traffic_from_profiles(w.name) if args.prec == "fp32" else None
    peak = PEAK_MFMA_TFLOPS[args.prec]
    res_valid = int(((res & 0xFFFFFFFF) != 0xFFFFFFFF).sum().item())
    rp_elem = st["rp_row_bits"] / 8.0   # the rows RobustPrune reads: int8, 16-bit or float32
    roofs = kernel_rooflines(st, w, n, args.steps, res_valid, rp_elem, args.prec)
    dominant = max(roofs, key=lambda k: roofs[k]["ms"])
    main_roof = dict(roofs[dominant])
    main_roof["kernel"] = dominant
    main_roof["traffic"] = traffic if dominant == "leaf_knn" else None
    gemm = f"{args.prec}-mfma" + (f", fp32 rescore of top-{args.rescore_mult}k"
                                  if args.rescore_mult else
                                  f", fp32 rescore of top-(k+{args.rescore_extra})"
                                  if args.rescore_extra else "")
    line = {
        "metric": "build points/sec at recall@10>=0.95",
        "value": n / (ms / 1000.0),
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32"}.get(args.prec, args.prec),
        "data": "synthetic",
        "config": {"workload": w.name, "n": n, "d": w.d,
                   "metric": "L2" if w.metric == 0 else "IP", "c_max": w.c_max,
                   "leaves_per_point": 2, "k": w.k, "l_max": w.l_max, "R": w.R,
                   "alpha": w.alpha, "hash_bits": w.hash_bits, "gemm": gemm},
        "recall_at_10": main_form["recall_at_10"],
        "L_at_recall_0.95": main_form["L_at_recall_0.95"],
        "search_qps_at_L": main_form["search_qps_at_L"],
        "recall_curve": main_form["recall_curve"],
        "leaf_gemm_tflops": achieved,
        "insert_p99_ms": insert_p99(serve),
        "serving": serve,
        "phase_ms": main_form["phase_ms"],
        "build_stats": {k: st[k] for k in ("n_leaves", "n_members", "leader_dists", "levels",
                                           "leaf_pairs", "records")},
        "roofline": {k: main_roof[k] for k in ("bound", "achieved", "peak", "unit", "frac",
                                               "traffic", "kernel", "ms")},
        "rooflines": roofs,
        "cpu_baseline": cpu,
        "variants": variants,
    }
    if precision is not None:
        line["precision"] = precision
    if frontier is not None:
        line["frontier"] = frontier
    if knn_graph is not None:
        line["knn_graph"] = knn_graph
    print(json.dumps(line), flush=True)
    idx.close()


if __name__ == "__main__":
    main()
