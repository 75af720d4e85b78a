"""FP64 reference oracle for the PiPNN leaf hot path.

TEST INFRASTRUCTURE ONLY: only the tests, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package. The GPU
library never calls it, and it shares no code with the GPU library.

The arithmetic lives in ``pipnn_oracle.c`` (plain C, FP64, OpenMP over
independent points, leaves and queries); this module only marshals numpy
arrays through ctypes and chains the steps of the method (Alg. 4):
partition -> leaf pick -> HashPrune -> final RobustPrune.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pipnn_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
EMPTY_ID = 0xFFFFFFFF


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no FMA contraction, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
               "-shared", "-fPIC", "-Wall", "-Wno-unused-function", _SRC, "-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


class Params(C.Structure):
    _fields_ = [("metric", C.c_int32), ("c_max", C.c_int32), ("c_min", C.c_int32),
                ("leader_div", C.c_int32), ("leader_cap", C.c_int32),
                ("fanout", C.c_int32 * 4), ("k", C.c_int32), ("hash_bits", C.c_int32),
                ("l_max", C.c_int32), ("R", C.c_int32), ("alpha", C.c_float),
                ("pad_", C.c_int32), ("seed", C.c_uint64)]


def make_params(metric=0, c_max=1024, c_min=64, leader_div=200, leader_cap=1000,
                fanout=(2, 1, 1, 1), k=16, hash_bits=12, l_max=64, R=32, alpha=1.2,
                seed=0) -> Params:
    p = Params()
    p.metric, p.c_max, p.c_min = metric, c_max, c_min
    p.leader_div, p.leader_cap = leader_div, leader_cap
    fo = list(fanout) + [fanout[-1]] * (4 - len(fanout))
    for i in range(4):
        p.fanout[i] = int(fo[i])
    p.k, p.hash_bits, p.l_max, p.R = k, hash_bits, l_max, R
    p.alpha = alpha
    p.seed = seed
    return p


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        P = C.c_void_p
        i64, i32 = C.c_int64, C.c_int32
        L.orc_dist.restype = C.c_double
        L.orc_dist.argtypes = [P, P, i32, i32]
        L.orc_sketches.argtypes = [P, i64, i32, P, i32, P]
        L.orc_hash.restype = C.c_uint16
        L.orc_hash.argtypes = [P, P, i32]
        L.orc_hashes.argtypes = [P, i32, P, P, i64, P]
        L.orc_bf16.restype = C.c_uint16
        L.orc_bf16.argtypes = [C.c_double]
        L.orc_splitmix64.argtypes = [C.c_uint64, i64, P]
        L.orc_empty_slot.restype = C.c_uint64
        L.orc_reservoir_init.argtypes = [P, i64, i32]
        L.orc_reservoir_canonical.argtypes = [P, P, i64, i32]
        L.orc_hashprune_stream.restype = i32
        L.orc_hashprune_stream.argtypes = [P, i64, i32, P, i32, P, P, P, i64]
        L.orc_hashprune_closed.restype = i32
        L.orc_hashprune_closed.argtypes = [P, i64, i32, P, i32, P, P, P, i64]
        L.orc_partition.restype = i32
        L.orc_partition.argtypes = [P, i64, i32, C.POINTER(Params), P, i64, P, i64, P, P, P]
        L.orc_leaf_knn.argtypes = [P, i32, i32, P, P, i64, i32, P, P]
        L.orc_topk_rows.argtypes = [P, i64, i64, i32, P, P, P]
        L.orc_robustprune.argtypes = [P, i32, i32, P, i64, i32, C.c_float, i32, i32, P, P]
        L.orc_beam_search.argtypes = [P, i64, i32, i32, P, i32, P, i64, i32, i32, C.c_uint32,
                                      P, P, P]
        L.orc_bruteforce_knn.argtypes = [P, i64, i32, i32, P, i64, i32, P, P]
        L.orc_start_node.restype = C.c_uint32
        L.orc_start_node.argtypes = [P, i64, i32, P]
        L.orc_set_threads.argtypes = [i32]
        L.orc_bf16_rne.restype = C.c_uint16
        L.orc_bf16_rne.argtypes = [C.c_float]
        L.orc_fp16_rne.restype = C.c_uint16
        L.orc_fp16_rne.argtypes = [C.c_float]
        L.orc_e4m3_rne_sat.restype = C.c_uint8
        L.orc_e4m3_rne_sat.argtypes = [C.c_float]
        L.orc_bf16_value.restype = C.c_double
        L.orc_bf16_value.argtypes = [C.c_uint16]
        L.orc_fp16_value.restype = C.c_double
        L.orc_fp16_value.argtypes = [C.c_uint16]
        L.orc_e4m3_value.restype = C.c_double
        L.orc_e4m3_value.argtypes = [C.c_uint8]
        L.orc_quantize.argtypes = [P, i64, i32, i32, P, P, P]
        L.orc_leaf_knn_lowp.argtypes = [P, P, i32, i32, P, P, i64, i32, i32, i32, P, P]
        L.orc_leaf_reps.argtypes = [P, i32, P, P, i64, P]
        L.orc_robustprune_points.argtypes = [P, i32, i32, P, P, i64, i32, C.c_float, i32, P, P]
        L.orc_get_threads.restype = i32
        L.orc_leaf_all_to_all.argtypes = [P, i32, i32, P, P, i64, i32, C.c_float, P, P]
        L.orc_phase_seconds.restype = i32
        L.orc_phase_seconds.argtypes = [P, i32]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _f32(X):
    return np.ascontiguousarray(X, dtype=np.float32)


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


def get_threads() -> int:
    return int(lib().orc_get_threads())


PHASES = ("sketches", "partition", "leaf_pick", "hashprune", "robustprune", "beam_search",
          "bruteforce_knn")


def phase_seconds(reset: bool = True) -> dict:
    """Wall seconds spent in each phase function of the C oracle since the
    last reset (a steady clock read inside the C code)."""
    out = np.zeros(len(PHASES), dtype=np.float64)
    cnt = lib().orc_phase_seconds(_p(out), 1 if reset else 0)
    assert cnt == len(PHASES)
    return {k: float(v) for k, v in zip(PHASES, out)}


def dist(a, b, metric=0) -> float:
    a, b = _f32(a), _f32(b)
    return float(lib().orc_dist(_p(a), _p(b), a.shape[-1], metric))


def splitmix64(seed: int, count: int) -> np.ndarray:
    out = np.zeros(count, dtype=np.uint64)
    lib().orc_splitmix64(C.c_uint64(seed), count, _p(out))
    return out


def bf16(x: float) -> int:
    return int(lib().orc_bf16(float(x)))


def empty_slot() -> int:
    return int(lib().orc_empty_slot())


def sketches(X, H) -> np.ndarray:
    X, H = _f32(X), _f32(H)
    n, d = X.shape
    m = H.shape[0]
    S = np.zeros((n, m), dtype=np.float64)
    lib().orc_sketches(_p(X), n, d, _p(H), m, _p(S))
    return S


def hashes(S, dst, cand) -> np.ndarray:
    S = np.ascontiguousarray(S, dtype=np.float64)
    dst = np.ascontiguousarray(dst, dtype=np.uint32)
    cand = np.ascontiguousarray(cand, dtype=np.uint32)
    out = np.zeros(len(dst), dtype=np.uint16)
    lib().orc_hashes(_p(S), S.shape[1], _p(dst), _p(cand), len(dst), _p(out))
    return out


def reservoir_init(n: int, l_max: int) -> np.ndarray:
    r = np.zeros((n, l_max), dtype=np.uint64)
    lib().orc_reservoir_init(_p(r), n, l_max)
    return r


def reservoir_canonical(res) -> np.ndarray:
    res = np.ascontiguousarray(res, dtype=np.uint64)
    out = np.empty_like(res)
    lib().orc_reservoir_canonical(_p(res), _p(out), res.shape[0], res.shape[1])
    return out


def hashprune(res, S, dst, cand, dist_, closed: bool = False) -> np.ndarray:
    """Insert records into a copy of ``res`` (n x l_max uint64 slots)."""
    res = np.array(res, dtype=np.uint64, copy=True, order="C")
    S = np.ascontiguousarray(S, dtype=np.float64)
    dst = np.ascontiguousarray(dst, dtype=np.uint32)
    cand = np.ascontiguousarray(cand, dtype=np.uint32)
    dist_ = np.ascontiguousarray(dist_, dtype=np.float64)
    fn = lib().orc_hashprune_closed if closed else lib().orc_hashprune_stream
    rc = fn(_p(res), res.shape[0], res.shape[1], _p(S), S.shape[1], _p(dst), _p(cand),
            _p(dist_), len(dst))
    if rc != 0:
        raise ValueError("record id out of range")
    return res


def slot_fields(res):
    res = np.asarray(res, dtype=np.uint64)
    ids = (res & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    hsh = ((res >> np.uint64(32)) & np.uint64(0xFFFF)).astype(np.uint16)
    bfv = (res >> np.uint64(48)).astype(np.uint16)
    return ids, hsh, bfv


def replica_key(seed: int, r: int) -> int:
    """Root key of partition replica r (the paper's replication: an
    independent carving): the seed for r = 0, else the first splitmix64
    output from seed xor r * 0xD1B54A32D192ED03 (mod 2^64)."""
    if r == 0:
        return int(seed)
    return int(splitmix64((int(seed) ^ (r * 0xD1B54A32D192ED03)) & 0xFFFFFFFFFFFFFFFF, 1)[0])


def partition(X, params: Params, replica: int = 0):
    """Randomized Ball Carving (Alg. 5). Returns (offsets, members, leader_dists).
    Replica r > 0 is the same carving from root key replica_key(seed, r)."""
    if replica:
        q = Params.from_buffer_copy(params)
        q.seed = replica_key(params.seed, replica)
        params = q
    X = _f32(X)
    n, d = X.shape
    cap_l, cap_m = max(16, n // 8), 4 * n
    while True:
        off = np.zeros(cap_l + 1, dtype=np.int64)
        mem = np.zeros(cap_m, dtype=np.uint32)
        nl, nm, ld = C.c_int64(), C.c_int64(), C.c_int64()
        rc = lib().orc_partition(_p(X), n, d, C.byref(params), _p(off), cap_l, _p(mem), cap_m,
                                 C.byref(nl), C.byref(nm), C.byref(ld))
        if rc == 0:
            return off[:nl.value + 1].copy(), mem[:nm.value].copy(), int(ld.value)
        cap_l, cap_m = max(cap_l, nl.value), max(cap_m, nm.value)


def leaf_knn(X, offsets, members, k: int, metric: int = 0):
    """Bi-directed k-NN pick per leaf; returns (cand[total_members, k], dist)."""
    X = _f32(X)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    members = np.ascontiguousarray(members, dtype=np.uint32)
    tot = int(offsets[-1])
    cand = np.zeros((tot, k), dtype=np.uint32)
    dd = np.zeros((tot, k), dtype=np.float64)
    lib().orc_leaf_knn(_p(X), X.shape[1], metric, _p(offsets), _p(members), len(offsets) - 1,
                       k, _p(cand), _p(dd))
    return cand, dd


PREC_FP32, PREC_BF16, PREC_FP8, PREC_FP16 = 0, 1, 2, 3


def encode(x: float, prec: int) -> int:
    """One binary32 value encoded as a bf16 / fp16 / OCP e4m3 code (no scaling)."""
    f = {PREC_BF16: lib().orc_bf16_rne, PREC_FP16: lib().orc_fp16_rne,
         PREC_FP8: lib().orc_e4m3_rne_sat}[prec]
    return int(f(float(np.float32(x))))


def decode(code: int, prec: int) -> float:
    f = {PREC_BF16: lib().orc_bf16_value, PREC_FP16: lib().orc_fp16_value,
         PREC_FP8: lib().orc_e4m3_value}[prec]
    return float(f(int(code)))


def quantize(X, prec: int):
    """GEMM operand of the rows of X: (codes, inv_scale, xq) with codes
    uint16 (bf16/fp16), uint8 (fp8) or float32 (fp32), inv_scale float32 per
    row and xq the decoded operand in float64."""
    X = _f32(X)
    n, d = X.shape
    dt = {PREC_FP32: np.float32, PREC_BF16: np.uint16, PREC_FP16: np.uint16,
          PREC_FP8: np.uint8}[prec]
    codes = np.zeros((n, d), dtype=dt)
    inv = np.zeros(n, dtype=np.float32)
    xq = np.zeros((n, d), dtype=np.float64)
    lib().orc_quantize(_p(X), n, d, prec, _p(codes), _p(inv), _p(xq))
    return codes, inv, xq


def leaf_all_to_all(X, offsets, members, R_leaf: int, alpha: float, metric: int = 0):
    """All-to-All Prune leaf picker: per leaf member, lazy RobustPrune over
    the other members of its leaf (up to R_leaf admitted, in admission
    order); returns (cand, dist), (total members) x R_leaf like leaf_knn."""
    X = _f32(X)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    members = np.ascontiguousarray(members, dtype=np.uint32)
    tot = int(offsets[-1])
    cand = np.zeros((tot, R_leaf), dtype=np.uint32)
    dd = np.zeros((tot, R_leaf), dtype=np.float64)
    lib().orc_leaf_all_to_all(_p(X), X.shape[1], metric, _p(offsets), _p(members),
                              len(offsets) - 1, R_leaf, alpha, _p(cand), _p(dd))
    return cand, dd


def leaf_knn_lowp(X, xq, offsets, members, k: int, mult: int, metric: int = 0, extra: int = 0):
    """Leaf pick on the decoded operand xq with FP64 rescoring of the mult*k
    nearest, or with mult 0 of the k + extra nearest (both 0: no re-ranking);
    returns (cand, dist) like leaf_knn."""
    X = _f32(X)
    xq = np.ascontiguousarray(xq, dtype=np.float64)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    members = np.ascontiguousarray(members, dtype=np.uint32)
    tot = int(offsets[-1])
    cand = np.zeros((tot, k), dtype=np.uint32)
    dd = np.zeros((tot, k), dtype=np.float64)
    lib().orc_leaf_knn_lowp(_p(X), _p(xq), X.shape[1], metric, _p(offsets), _p(members),
                            len(offsets) - 1, k, mult, extra, _p(cand), _p(dd))
    return cand, dd


def bidirected_records(members, cand, dist_):
    """Expand per-row picks into the two records of each edge."""
    k = cand.shape[1]
    src = np.repeat(np.asarray(members, dtype=np.uint32), k)
    c = cand.reshape(-1)
    dv = dist_.reshape(-1)
    ok = c != EMPTY_ID
    src, c, dv = src[ok], c[ok], dv[ok]
    return (np.concatenate([src, c]), np.concatenate([c, src]), np.concatenate([dv, dv]))


def topk_rows(D, k: int, self_col=None):
    D = np.ascontiguousarray(D, dtype=np.float32)
    rows, cols = D.shape
    out = np.zeros((rows, k), dtype=np.uint32)
    val = np.zeros((rows, k), dtype=np.float32)
    sc = None if self_col is None else np.ascontiguousarray(self_col, dtype=np.int64)
    lib().orc_topk_rows(_p(D), rows, cols, k, None if sc is None else _p(sc), _p(out), _p(val))
    return out, val


def robustprune(X, res, alpha: float, R: int, metric: int = 0, lazy: bool = True):
    X = _f32(X)
    res = np.ascontiguousarray(res, dtype=np.uint64)
    n, l_max = res.shape
    g = np.zeros((n, R), dtype=np.uint32)
    deg = np.zeros(n, dtype=np.uint32)
    lib().orc_robustprune(_p(X), X.shape[1], metric, _p(res), n, l_max, alpha, R,
                          1 if lazy else 0, _p(g), _p(deg))
    return g, deg


def robustprune_points(X, res_rows, xs, alpha: float, R: int, metric: int = 0):
    """Lazy RobustPrune of points xs from their reservoir rows res_rows."""
    X = _f32(X)
    res_rows = np.ascontiguousarray(res_rows, dtype=np.uint64)
    xs = np.ascontiguousarray(xs, dtype=np.uint32)
    nx, l_max = res_rows.shape
    g = np.zeros((nx, R), dtype=np.uint32)
    deg = np.zeros(nx, dtype=np.uint32)
    lib().orc_robustprune_points(_p(X), X.shape[1], metric, _p(res_rows), _p(xs), nx, l_max,
                                 alpha, R, _p(g), _p(deg))
    return g, deg


def beam_search(X, graph, Q, k: int, L: int, start: int, metric: int = 0):
    X, Q = _f32(X), _f32(Q)
    graph = np.ascontiguousarray(graph, dtype=np.uint32)
    nq = Q.shape[0]
    ids = np.zeros((nq, k), dtype=np.uint32)
    dd = np.zeros((nq, k), dtype=np.float64)
    cm = np.zeros(nq, dtype=np.uint32)
    lib().orc_beam_search(_p(X), X.shape[0], X.shape[1], metric, _p(graph), graph.shape[1],
                          _p(Q), nq, k, L, start, _p(ids), _p(dd), _p(cm))
    return ids, dd, cm


def bruteforce_knn(X, Q, k: int, metric: int = 0):
    X, Q = _f32(X), _f32(Q)
    nq = Q.shape[0]
    ids = np.zeros((nq, k), dtype=np.uint32)
    dd = np.zeros((nq, k), dtype=np.float64)
    lib().orc_bruteforce_knn(_p(X), X.shape[0], X.shape[1], metric, _p(Q), nq, k, _p(ids),
                             _p(dd))
    return ids, dd


def start_node(X):
    X = _f32(X)
    dd = np.zeros(X.shape[0], dtype=np.float64)
    s = lib().orc_start_node(_p(X), X.shape[0], X.shape[1], _p(dd))
    return int(s), dd


def recall_at_k(found_ids, X, Q, gt_dist, metric: int = 0) -> float:
    """k@k recall (Preliminaries, Definition of k@k' recall). A returned id
    counts as a hit when its distance to the query is at most the k-th true
    distance, so exact ties with the k-th neighbour are not penalised."""
    X, Q = _f32(X), _f32(Q)
    nq, k = found_ids.shape
    hits = 0
    for qi in range(nq):
        kth = gt_dist[qi, k - 1]
        seen = set()
        for j in found_ids[qi]:
            j = int(j)
            if j == EMPTY_ID or j in seen:
                continue
            seen.add(j)
            if dist(Q[qi], X[j], metric) <= kth:
                hits += 1
    return hits / float(nq * k)


def build_index(X, H, params: Params, lazy: bool = True, replicas: int = 1):
    """Alg. 4 end to end: partition, pick, HashPrune, final RobustPrune.
    With replicas > 1, the records of that many independent partitions go
    into the same reservoirs. Returns a dict of every intermediate (the
    leaves, picks and records of the last replica)."""
    X = _f32(X)
    n = X.shape[0]
    S = sketches(X, H)
    res = reservoir_init(n, params.l_max)
    for r in range(replicas):
        off, mem, ld = partition(X, params, replica=r)
        cand, dd = leaf_knn(X, off, mem, params.k, params.metric)
        dst, cnd, dv = bidirected_records(mem, cand, dd)
        res = hashprune(res, S, dst, cnd, dv)
    g, deg = robustprune(X, res, params.alpha, params.R, params.metric, lazy=lazy)
    return dict(offsets=off, members=mem, leader_dists=ld, cand=cand, dist=dd, S=S,
                reservoirs=res, graph=g, degree=deg, records=(dst, cnd, dv))


def leaf_reps(X, offsets, members) -> np.ndarray:
    """Representative of each leaf (see orc_leaf_reps)."""
    X = _f32(X)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    members = np.ascontiguousarray(members, dtype=np.uint32)
    out = np.zeros(len(offsets) - 1, dtype=np.uint32)
    lib().orc_leaf_reps(_p(X), X.shape[1], _p(offsets), _p(members), len(offsets) - 1, _p(out))
    return out


def insert(X_all, n0: int, groups, offsets, members, res, H, k: int, alpha: float, R: int,
           fanout0: int = 2, metric: int = 0):
    """Insertion of points n0.. of X_all into an index built on the leaves
    (offsets, members) with reservoirs res (n0 x l_max), as this library
    defines it (the paper has none):
      1. every new point is routed to its min(fanout0, #leaves) nearest leaf
         representatives (exact distances, ties by leaf index);
      2. per (leaf, group), each new point of the group routed to the leaf
         picks its k nearest (distance, id) among the leaf's members and the
         group's new points routed there, itself excluded;
      3. both directed records of every pick go through HashPrune (starting
         from the old reservoirs; new points start empty);
      4. RobustPrune of every point that received a record.
    Returns (reservoirs n1 x l_max, touched ids, graph rows of the touched
    ids)."""
    X_all = _f32(X_all)
    n1 = X_all.shape[0]
    new = np.arange(n0, n1, dtype=np.int64)
    groups = np.zeros(len(new), dtype=np.int32) if groups is None else np.asarray(groups)
    reps = leaf_reps(X_all[:n0], offsets, members)
    nl = len(reps)
    f = min(fanout0, nl)
    rid, _ = bruteforce_knn(X_all[reps], X_all[new], f, metric)
    by = {}
    for i, p in enumerate(new):
        for L in rid[i]:
            by.setdefault((int(L), int(groups[i])), []).append(int(p))
    src, dst, dv = [], [], []
    for (L, g), pts in sorted(by.items()):
        cols = np.concatenate([np.asarray(members[offsets[L]:offsets[L + 1]], dtype=np.int64),
                               np.asarray(pts, dtype=np.int64)])
        kk = min(k + 1, len(cols))
        nb, nd = bruteforce_knn(X_all[cols], X_all[np.asarray(pts)], kk, metric)
        for r, p in enumerate(pts):
            got = [(cols[c], dd) for c, dd in zip(nb[r], nd[r]) if c != EMPTY_ID and cols[c] != p]
            for c, dd in got[:k]:
                src.append(p)
                dst.append(c)
                dv.append(dd)
    src, dst, dv = (np.asarray(src, dtype=np.uint32), np.asarray(dst, dtype=np.uint32),
                    np.asarray(dv, dtype=np.float64))
    l_max = res.shape[1]
    res1 = np.concatenate([np.asarray(res, dtype=np.uint64),
                           reservoir_init(n1 - n0, l_max)]) if n1 > n0 else res.copy()
    S = sketches(X_all, H)
    res1 = hashprune(res1, S, np.concatenate([src, dst]), np.concatenate([dst, src]),
                     np.concatenate([dv, dv]))
    touched = np.unique(np.concatenate([src.astype(np.int64), dst.astype(np.int64)]))
    g, _ = robustprune(X_all, res1, alpha, R, metric=metric)
    return res1, touched, g[touched]
