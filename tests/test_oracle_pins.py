"""Pins of the FP64 oracle to facts the paper and the mathematics fix.

Every check here compares the oracle with something other than itself:
golden values worked by hand from the paper's definitions, closed forms,
invariants, special cases that reduce to a textbook computation, and exact
brute force (int64 arithmetic) on tiny inputs.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import pipnn_inputs as pi

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.lib()
    oracle.set_threads(min(8, os.cpu_count() or 1))


def _int_points(n, d, seed, hi=16):
    rng = np.random.default_rng(seed)
    return rng.integers(0, hi, size=(n, d)).astype(np.float32)


def _exact_sqdist(A, B):
    """Exact squared L2 between integer-valued rows, in int64."""
    A = A.astype(np.int64)
    B = B.astype(np.int64)
    return ((A[:, None, :] - B[None, :, :]) ** 2).sum(-1)


def _knn_bruteforce(D, k, exclude_diag=False):
    """Row-wise k smallest by (value, column) via a lexicographic sort."""
    rows, cols = D.shape
    out = np.empty((rows, k), dtype=np.int64)
    colidx = np.arange(cols)
    for r in range(rows):
        order = np.lexsort((colidx, D[r]))
        if exclude_diag:
            order = order[order != r]
        out[r] = order[:k]
    return out


# --------------------------------------------------------------------------
# random stream and rounding

def test_splitmix64_reference_outputs():
    g = _gold("splitmix64_seed1234567.json")
    got = oracle.splitmix64(g["seed"], len(g["outputs"]))
    assert [int(v) for v in got] == [int(v) for v in g["outputs"]]


def test_bf16_hand_values():
    g = _gold("bf16_rne.json")
    for v, e in zip(g["values"], g["expected"]):
        v = float("inf") if v == "inf" else float(v)
        assert oracle.bf16(v) == e, (v, hex(oracle.bf16(v)), hex(e))


def test_bf16_matches_library_rne():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(5)
    vals = np.concatenate([rng.standard_normal(3000) * 10.0 ** rng.integers(-6, 7, 3000),
                           rng.uniform(0, 1e7, 1000)]).astype(np.float32)
    ref = torch.from_numpy(vals).to(torch.bfloat16).view(torch.int16).numpy().astype(np.uint16)
    got = np.array([oracle.bf16(float(v)) for v in vals], dtype=np.uint16)
    assert np.array_equal(got, ref)


# --------------------------------------------------------------------------
# dissimilarity

def test_dist_closed_forms():
    assert oracle.dist([0, 0], [3, 4]) == 25.0
    assert oracle.dist([1, 2, 3], [4, 5, 6], metric=1) == -32.0
    x = np.random.default_rng(0).standard_normal(50).astype(np.float32)
    assert oracle.dist(x, x) == 0.0
    y = np.random.default_rng(1).standard_normal(50).astype(np.float32)
    assert oracle.dist(x, y) == oracle.dist(y, x)


# --------------------------------------------------------------------------
# residualized hashing (Sec. 3)

def test_sketch_hash_equals_residual_hash_exactly():
    """With integer points and hyperplanes everything is exact, so the
    sketch form must give the residual form H_b . (c - p) >= 0 bit for bit."""
    rng = np.random.default_rng(3)
    X = rng.integers(0, 256, size=(60, 32)).astype(np.float32)
    H = np.rint(16 * rng.standard_normal((12, 32))).astype(np.float32)
    S = oracle.sketches(X, H)
    dst = np.repeat(np.arange(60), 60).astype(np.uint32)
    cand = np.tile(np.arange(60), 60).astype(np.uint32)
    got = oracle.hashes(S, dst, cand)
    resid = (X[cand].astype(np.int64) - X[dst].astype(np.int64)) @ H.astype(np.int64).T
    bits = (resid >= 0).astype(np.int64)
    want = (bits << np.arange(12)).sum(1)
    assert np.array_equal(got.astype(np.int64), want)


def test_reverse_hash_identity():
    """h_c(p) = not h_p(c) | [Sketch equal], bit by bit."""
    rng = np.random.default_rng(4)
    X = rng.integers(0, 4, size=(40, 8)).astype(np.float32)   # many equal sketch entries
    H = np.rint(2 * rng.standard_normal((10, 8))).astype(np.float32)
    S = oracle.sketches(X, H)
    a = np.repeat(np.arange(40), 40).astype(np.uint32)
    b = np.tile(np.arange(40), 40).astype(np.uint32)
    hab = oracle.hashes(S, a, b).astype(np.int64)
    hba = oracle.hashes(S, b, a).astype(np.int64)
    eq = ((S[a] == S[b]).astype(np.int64) << np.arange(10)).sum(1)
    assert np.array_equal(hba, (~hab & 0x3FF) | eq)


@pytest.mark.parametrize("theta,m", [(0.3, 12), (1.0, 6), (2.0, 4)])
def test_lsh_collision_law(theta, m):
    """P[h_p(c) = h_p(c')] = (1 - theta/pi)^m for Gaussian hyperplanes
    (Sec. 3, Why HashPrune works), checked within a 4.5-sigma binomial
    interval over many independent hyperplane draws."""
    rng = np.random.default_rng(11)
    d, trials = 16, 4000
    p = rng.standard_normal(d)
    u = rng.standard_normal(d); u /= np.linalg.norm(u)
    v = rng.standard_normal(d); v -= (v @ u) * u; v /= np.linalg.norm(v)
    c = p + 2.0 * u
    c2 = p + 3.0 * (math.cos(theta) * u + math.sin(theta) * v)
    X = np.stack([p, c, c2]).astype(np.float32)
    hits = 0
    for _ in range(trials):
        H = rng.standard_normal((m, d)).astype(np.float32)
        S = oracle.sketches(X, H)
        h = oracle.hashes(S, np.array([0, 0], np.uint32), np.array([1, 2], np.uint32))
        hits += int(h[0] == h[1])
    # the float32 rounding of the constructed points moves theta negligibly
    P = (1.0 - theta / math.pi) ** m
    sd = math.sqrt(P * (1 - P) / trials)
    assert abs(hits / trials - P) <= 4.5 * sd + 1e-3, (hits / trials, P)


# --------------------------------------------------------------------------
# HashPrune (Alg. 3 and the history-independence lemma)

def test_hashprune_hand_example():
    g = _gold("hashprune_quadrants.json")
    X = np.array(g["points"], dtype=np.float32)
    H = np.array(g["H"], dtype=np.float32)
    S = oracle.sketches(X, H)
    p = g["p"]
    cands = np.array(g["candidates"], dtype=np.uint32)
    dist = np.array([oracle.dist(X[p], X[c]) for c in cands])
    for closed in (False, True):
        res = oracle.hashprune(oracle.reservoir_init(len(X), g["l_max"]), S,
                               np.full(len(cands), p, np.uint32), cands, dist, closed=closed)
        ids, hs, bfv = oracle.slot_fields(res[p])
        assert list(ids) == g["expected_ids"]
        assert list(hs) == g["expected_hashes"]
        assert [oracle.bf16(v) for v in g["expected_dists"]] == list(bfv)


def _random_records(n, cnt, seed, dmax=1000):
    rng = np.random.default_rng(seed)
    dst = rng.integers(0, n, cnt).astype(np.uint32)
    cand = rng.integers(0, n, cnt).astype(np.uint32)
    # a distance per unordered pair, so repeated candidates agree
    a, b = np.minimum(dst, cand).astype(np.int64), np.maximum(dst, cand).astype(np.int64)
    dist = ((a * 7919 + b * 104729) % dmax).astype(np.float64) / 7.0
    return dst, cand, dist


def test_hashprune_history_independence_and_closed_form():
    n, l_max, m = 50, 8, 5
    rng = np.random.default_rng(21)
    X = rng.standard_normal((n, 6)).astype(np.float32)
    H = rng.standard_normal((m, 6)).astype(np.float32)
    S = oracle.sketches(X, H)
    dst, cand, dist = _random_records(n, 3000, 22)
    base = oracle.reservoir_init(n, l_max)
    closed = oracle.hashprune(base, S, dst, cand, dist, closed=True)
    for t in range(50):
        perm = np.random.default_rng(100 + t).permutation(len(dst))
        cuts = np.sort(np.random.default_rng(200 + t).integers(0, len(dst), 3))
        res = base
        for part in np.split(perm, cuts):
            res = oracle.hashprune(res, S, dst[part], cand[part], dist[part])
        assert np.array_equal(res, closed)
    # re-insertion of everything is a no-op
    again = oracle.hashprune(closed, S, dst, cand, dist)
    assert np.array_equal(again, closed)


def test_hashprune_invariants():
    n, l_max, m = 40, 6, 4
    rng = np.random.default_rng(31)
    X = rng.standard_normal((n, 5)).astype(np.float32)
    H = rng.standard_normal((m, 5)).astype(np.float32)
    S = oracle.sketches(X, H)
    dst, cand, dist = _random_records(n, 2500, 32, dmax=50)   # many equal distances
    res = oracle.hashprune(oracle.reservoir_init(n, l_max), S, dst, cand, dist)
    ids, hs, bfv = oracle.slot_fields(res)
    key = lambda b, i: ((int(b) ^ 0x8000) if not (b & 0x8000) else (~int(b) & 0xFFFF), int(i))
    for p in range(n):
        sel = (dst == p) & (cand != p)
        allh = oracle.hashes(S, dst[sel], cand[sel])
        bucket_min = {}
        for c, h, dv in zip(cand[sel], allh, dist[sel]):
            kk = key(oracle.bf16(dv), c)
            if h not in bucket_min or kk < bucket_min[h][0]:
                bucket_min[h] = (kk, int(c))
        valid = ids[p] != oracle.EMPTY_ID
        kept = list(zip(ids[p][valid], hs[p][valid], bfv[p][valid]))
        assert len(kept) == min(len(bucket_min), l_max)          # corrected output size
        assert len({h for _, h, _ in kept}) == len(kept)          # one slot per bucket
        for i, h, b in kept:                                      # kept = its bucket's min
            assert bucket_min[h] == (key(b, i), int(i))
        if len(kept) == l_max:                                    # full: unkept buckets lose
            worst = max(key(b, i) for i, _, b in kept)
            for h, (kk, _) in bucket_min.items():
                if h not in {hh for _, hh, _ in kept}:
                    assert kk > worst
        keys = [key(b, i) for i, _, b in kept]                   # canonical order
        assert keys == sorted(keys)
        assert np.all(ids[p][~valid] == oracle.EMPTY_ID)


def test_hashprune_special_cases():
    n, l_max = 30, 5
    rng = np.random.default_rng(41)
    X = rng.standard_normal((n, 4)).astype(np.float32)
    dst, cand, dist = _random_records(n, 800, 42)
    # m = 0: a single bucket, so the reservoir is {nearest}
    S0 = np.zeros((n, 0))
    r0 = oracle.hashprune(oracle.reservoir_init(n, l_max), S0, dst, cand, dist)
    ids0, _, _ = oracle.slot_fields(r0)
    for p in range(n):
        sel = (dst == p) & (cand != p)
        if not sel.any():
            assert np.all(ids0[p] == oracle.EMPTY_ID)
            continue
        c, dv = cand[sel], dist[sel]
        bf = np.array([oracle.bf16(v) for v in dv])
        best = min(zip(bf, c))[1]
        assert ids0[p][0] == best and np.all(ids0[p][1:] == oracle.EMPTY_ID)
    # every candidate in its own bucket (sketch = one-hot id code): plain top-l_max
    m = 16
    S = np.array([[(i >> b) & 1 for b in range(m)] for i in range(n)], dtype=np.float64) * 2 - 1
    S[:, 5:] = 0
    S[:, :5] = np.array([[(i >> b) & 1 for b in range(5)] for i in range(n)]) * 2 - 1.0
    rr = oracle.hashprune(oracle.reservoir_init(n, l_max), S, dst, cand, dist)
    idsr, _, _ = oracle.slot_fields(rr)
    for p in range(n):
        sel = (dst == p) & (cand != p)
        hs = oracle.hashes(S, dst[sel], cand[sel])
        if len(set(hs.tolist())) != len(set(cand[sel].tolist())):
            continue   # two candidates shared a hash: not this special case
        uniq = sorted({(oracle.bf16(v), int(c)) for c, v in zip(cand[sel], dist[sel])},
                      key=lambda t: (t[0], t[1]))
        seen, top = set(), []
        for b, c in uniq:
            if c not in seen:
                seen.add(c); top.append(c)
        assert list(idsr[p][:min(l_max, len(top))]) == top[:l_max]
    # l_max >= number of buckets: all bucket minima are kept
    big = oracle.hashprune(oracle.reservoir_init(n, 64), S, dst, cand, dist)
    idsb, _, _ = oracle.slot_fields(big)
    for p in range(n):
        sel = (dst == p) & (cand != p)
        hs = oracle.hashes(S, dst[sel], cand[sel])
        assert (idsb[p] != oracle.EMPTY_ID).sum() == len(set(hs.tolist()))


def test_hashprune_rejects_bad_ids():
    S = np.zeros((4, 2))
    with pytest.raises(ValueError):
        oracle.hashprune(oracle.reservoir_init(4, 2), S, np.array([5], np.uint32),
                         np.array([1], np.uint32), np.array([1.0]))


# --------------------------------------------------------------------------
# RobustPrune (Alg. 2) and the lazy form

def _res_from_ids(n, l_max, lists):
    res = oracle.reservoir_init(n, l_max)
    for p, ids in lists.items():
        for i, c in enumerate(ids):
            res[p, i] = np.uint64(c) | (np.uint64(0x7F80) << np.uint64(48))
    return res


def test_robustprune_hand_examples():
    g = _gold("robustprune_line.json")
    for case in g["cases"]:
        X = np.array(case["points"], dtype=np.float32)[:, None]
        res = _res_from_ids(len(X), 8, {case["x"]: case["candidates"]})
        for lazy in (False, True):
            gph, deg = oracle.robustprune(X, res, case["alpha"], case["R"], lazy=lazy)
            assert list(gph[case["x"], :deg[case["x"]]]) == case["expected"]


def test_robustprune_lazy_equals_standard():
    rng = np.random.default_rng(51)
    n, l_max = 300, 24
    X = rng.standard_normal((n, 8)).astype(np.float32)
    lists = {p: rng.choice(np.delete(np.arange(n), p), l_max, replace=False) for p in range(n)}
    res = _res_from_ids(n, l_max, lists)
    for alpha, R in [(1.2, 8), (1.0, 24), (2.0, 5)]:
        a, da = oracle.robustprune(X, res, alpha, R, lazy=False)
        b, db = oracle.robustprune(X, res, alpha, R, lazy=True)
        assert np.array_equal(a, b) and np.array_equal(da, db)


def test_robustprune_limits():
    """alpha -> infinity never prunes: the R nearest by (distance, id);
    alpha = 0 prunes every candidate farther than the first: {nearest}."""
    rng = np.random.default_rng(61)
    n, l_max, R = 120, 16, 6
    X = rng.integers(0, 30, size=(n, 5)).astype(np.float32)
    lists = {p: rng.choice(np.delete(np.arange(n), p), l_max, replace=False) for p in range(n)}
    res = _res_from_ids(n, l_max, lists)
    g_inf, _ = oracle.robustprune(X, res, 1e30, R)
    g_0, d0 = oracle.robustprune(X, res, 0.0, R)
    for p in range(n):
        c = np.array(lists[p])
        dv = _exact_sqdist(X[p:p + 1], X[c])[0]
        order = c[np.lexsort((c, dv))]
        assert list(g_inf[p]) == list(order[:R])
        nz = dv[np.lexsort((c, dv))]
        # with alpha = 0, any candidate at distance > 0 is pruned by the first
        keep = [order[0]] + [cc for cc, dd in zip(order[1:], nz[1:]) if dd == 0][:R - 1]
        assert list(g_0[p, :d0[p]]) == keep


# --------------------------------------------------------------------------
# leaf pick and brute force (Sec. 4.2; Definition of k-NN search)

def test_single_leaf_is_exact_knn():
    """With C_max >= n the whole set is one leaf, so the leaf pick is the
    exact k-NN of every point (computed here in int64)."""
    X = _int_points(200, 12, 71)
    prm = oracle.make_params(c_max=4096, k=7, seed=5)
    off, mem, ld = oracle.partition(X, prm)
    assert list(off) == [0, 200] and np.array_equal(mem, np.arange(200)) and ld == 0
    cand, dist = oracle.leaf_knn(X, off, mem, 7)
    D = _exact_sqdist(X, X)
    want = _knn_bruteforce(D, 7, exclude_diag=True)
    assert np.array_equal(cand.astype(np.int64), want)
    assert np.array_equal(dist, np.take_along_axis(D, want, 1).astype(np.float64))


def test_small_leaf_pads():
    X = _int_points(3, 4, 72)
    cand, dist = oracle.leaf_knn(X, np.array([0, 3]), np.arange(3, dtype=np.uint32), 5)
    assert np.all(cand[:, 2:] == oracle.EMPTY_ID) and np.all(cand[:, :2] != oracle.EMPTY_ID)


def test_bruteforce_and_topk_rows():
    X = _int_points(150, 6, 73)
    Q = _int_points(20, 6, 74)
    ids, dist = oracle.bruteforce_knn(X, Q, 10)
    D = _exact_sqdist(Q, X)
    assert np.array_equal(ids.astype(np.int64), _knn_bruteforce(D, 10))
    got, _ = oracle.topk_rows(D.astype(np.float32), 10)
    assert np.array_equal(got.astype(np.int64), _knn_bruteforce(D, 10))
    sc = np.arange(20)
    got2, _ = oracle.topk_rows(D[:, :20].astype(np.float32), 5, self_col=sc)
    assert np.array_equal(got2.astype(np.int64), _knn_bruteforce(D[:, :20], 5, exclude_diag=True))


# --------------------------------------------------------------------------
# Randomized Ball Carving (Alg. 5)

def test_partition_invariants_and_determinism():
    X = pi.workload_points(1, 6000)
    prm = oracle.make_params(c_max=512, c_min=32, seed=9)
    off, mem, _ = oracle.partition(X, prm)
    sizes = np.diff(off)
    assert sizes.max() <= 512 and sizes.min() >= 1
    counts = np.bincount(mem, minlength=6000)
    assert counts.min() >= 1 and counts.max() <= 2          # 1..prod(fanout) leaves per point
    for i in range(len(sizes)):
        seg = mem[off[i]:off[i + 1]]
        assert np.all(np.diff(seg.astype(np.int64)) > 0)    # ascending, no duplicates
    off2, mem2, _ = oracle.partition(X, prm)
    assert np.array_equal(off, off2) and np.array_equal(mem, mem2)
    prm3 = oracle.make_params(c_max=512, c_min=32, seed=10)
    off3, mem3, _ = oracle.partition(X, prm3)
    assert not (len(off3) == len(off) and np.array_equal(mem3, mem))


def test_partition_one_level_bruteforce():
    """One level of ball carving worked out independently: leaders from the
    pinned splitmix64 stream and a partial Fisher-Yates shuffle, exact int64
    distances, top-2 by (distance, leader index), buckets as leaves."""
    n, cmax = 900, 600
    X = _int_points(n, 5, 81, hi=50)
    prm = oracle.make_params(c_max=cmax, c_min=1, leader_div=100, seed=77)
    off, mem, ld = oracle.partition(X, prm)
    ell = -(-n // 100)
    r = oracle.splitmix64(77, ell)
    perm = list(range(n))
    for t in range(ell):
        j = t + ((int(r[t]) * (n - t)) >> 64)
        perm[t], perm[j] = perm[j], perm[t]
    leaders = perm[:ell]
    D = _exact_sqdist(X, X[leaders])
    top2 = _knn_bruteforce(D, 2)
    buckets = [sorted(np.nonzero((top2 == t).any(1))[0].tolist()) for t in range(ell)]
    if max(len(b) for b in buckets) > cmax:
        pytest.skip("draw recursed; the one-level case needs every bucket <= C_max")
    want = sorted(tuple(b) for b in buckets if b)
    got = sorted(tuple(mem[off[i]:off[i + 1]].tolist()) for i in range(len(off) - 1))
    assert got == want
    assert ld == n * ell                                   # |P| * l leader distances


def test_partition_merge_and_recursion_rules():
    X = pi.workload_points(1, 5000)
    prm = oracle.make_params(c_max=300, c_min=120, seed=3)
    off, mem, ld = oracle.partition(X, prm)
    sizes = np.diff(off)
    assert sizes.max() <= 300
    assert ld > 5000 * 25                                  # recursion happened below the root
    assert np.bincount(mem, minlength=5000).min() >= 1


def test_partition_merge_and_recursion_golden():
    """Hand-worked carving of 17 points on a line (tests/golden/
    partition_merge_recursion.json; Alg. 5 and Sec. 4.1): a merged group
    that holds one id twice, a group boundary set by the sum of bucket sizes
    (the union would still fit), a bucket of exactly C_min kept, a bucket of
    exactly C_max kept, a recursion whose leaders come from the derived child
    key (with a Fisher-Yates swap that lands on an already swapped position)
    and a no-progress bucket cut into runs of 4 and 3."""
    g = _gold("partition_merge_recursion.json")
    gamma, mask = 0x9E3779B97F4A7C15, (1 << 64) - 1
    x = g["points_1d"]
    for sp in g["subproblems"]:
        key = int(sp["key"])
        if "parent_key" in sp:      # child key from the pinned generator
            st = int(sp["parent_key"]) ^ (((sp["parent_t"] + 1) * gamma) & mask)
            assert int(oracle.splitmix64(st, 1)[0]) == key
        ids, ell = sp["ids"], sp["ell"]
        assert [int(v) for v in oracle.splitmix64(key, ell)] == [int(r) for r in sp["draws"]]
        perm = list(range(len(ids)))
        for t, r in enumerate(sp["draws"]):
            j = t + ((int(r) * (len(ids) - t)) >> 64)
            assert j == sp["j"][t]
            perm[t], perm[j] = perm[j], perm[t]
        assert [ids[perm[t]] for t in range(ell)] == sp["leaders"]
        # the worked buckets follow from the nearest leaders by (distance, t)
        buckets = [[] for _ in range(ell)]
        for p in ids:
            near = sorted(((x[p] - x[lid]) ** 2, t) for t, lid in enumerate(sp["leaders"]))
            for _, t in near[:sp["fanout"]]:
                buckets[t].append(p)
        assert buckets == sp["buckets"]
    X = np.array(x, dtype=np.float32)[:, None]
    P = g["params"]
    prm = oracle.make_params(c_max=P["c_max"], c_min=P["c_min"], leader_div=P["leader_div"],
                             leader_cap=P["leader_cap"], fanout=P["fanout"], seed=P["seed"])
    off, mem, ld = oracle.partition(X, prm)
    got = sorted(tuple(mem[off[i]:off[i + 1]].tolist()) for i in range(len(off) - 1))
    assert got == sorted(tuple(v) for v in g["expected_leaves"])
    assert ld == g["expected_leader_dists"]


def test_partition_no_progress_chunks():
    """All points identical: every point picks leaders 0 and 1, both buckets
    equal the parent, and each is cut into near-equal runs of ascending ids."""
    X = np.zeros((1000, 4), dtype=np.float32)
    prm = oracle.make_params(c_max=300, c_min=1, seed=1)
    off, mem, _ = oracle.partition(X, prm)
    sizes = np.diff(off)
    assert sorted(sizes.tolist()) == [250] * 8
    assert np.array_equal(np.sort(mem), np.repeat(np.arange(1000), 2))


# --------------------------------------------------------------------------
# BeamSearch (Alg. 1) and recall

def test_beam_search_wide_beam_is_exact():
    """On a connected graph with L >= n the search visits every point, so it
    returns the exact k nearest neighbours."""
    n = 120
    X = _int_points(n, 6, 91)
    Q = _int_points(15, 6, 92)
    R = 4
    rng = np.random.default_rng(93)
    g = np.full((n, R), oracle.EMPTY_ID, dtype=np.uint32)
    for p in range(n):
        g[p, 0] = (p + 1) % n                      # a ring keeps it connected
        g[p, 1] = (p - 1) % n
        g[p, 2:] = rng.choice(n, R - 2, replace=False)
    ids, dist, cmps = oracle.beam_search(X, g, Q, 10, n, 0)
    D = _exact_sqdist(Q, X)
    assert np.array_equal(ids.astype(np.int64), _knn_bruteforce(D, 10))
    assert np.all(cmps == n)


def test_beam_search_hand_trace():
    """Points on a line 0..5 joined as a path; query at 4.2 from source 0
    with L=2: the search walks the path and returns [4, 5]."""
    X = np.arange(6, dtype=np.float32)[:, None]
    g = np.full((6, 2), oracle.EMPTY_ID, dtype=np.uint32)
    for p in range(6):
        if p > 0:
            g[p, 0] = p - 1
        if p < 5:
            g[p, 1] = p + 1
    ids, dist, cmps = oracle.beam_search(X, g, np.array([[4.2]], np.float32), 2, 2, 0)
    assert list(ids[0]) == [4, 5]
    assert cmps[0] == 6


def test_start_node_symmetric():
    X = np.array([[-2, 0], [2, 0], [0, 0], [0, 3], [0, -3]], dtype=np.float32)
    s, d = oracle.start_node(X)
    assert s == 2 and d[2] == 0.0


def test_recall_definition():
    X = np.arange(20, dtype=np.float32)[:, None]
    Q = np.array([[0.0]], np.float32)
    gi, gd = oracle.bruteforce_knn(X, Q, 10)
    assert oracle.recall_at_k(gi, X, Q, gd) == 1.0
    half = gi.copy(); half[0, 5:] = np.arange(15, 20)
    assert oracle.recall_at_k(half, X, Q, gd) == 0.5


def test_partition_replicas():
    """Replication (an independent second carving): replica 0 is the plain
    partition, replica 1 another valid partition from the derived root key;
    the replicated build's reservoirs do not depend on the replicas' order
    (HashPrune is order-free), and a point's reservoir never holds fewer
    entries than with one replica (its records, so its buckets, only grow)."""
    X = pi.gaussian_mixture(1500, 16, 10, 0.3, seed=61, center_seed=61)
    H = pi.hyperplanes(12, 16, seed=62)
    p = oracle.make_params(c_max=200, c_min=16, k=8, l_max=24, R=12, seed=63)
    assert oracle.replica_key(63, 0) == 63
    assert oracle.replica_key(63, 1) == int(oracle.splitmix64(63 ^ 0xD1B54A32D192ED03, 1)[0])
    o0, m0, _ = oracle.partition(X, p)
    a0, b0, _ = oracle.partition(X, p, replica=0)
    o1, m1, _ = oracle.partition(X, p, replica=1)
    assert np.array_equal(o0, a0) and np.array_equal(m0, b0)
    s0 = sorted(tuple(m0[o0[i]:o0[i + 1]]) for i in range(len(o0) - 1))
    s1 = sorted(tuple(m1[o1[i]:o1[i + 1]]) for i in range(len(o1) - 1))
    assert s0 != s1
    assert np.diff(o1).max() <= 200 and set(np.unique(m1)) == set(range(1500))
    ref = oracle.build_index(X, H, p, replicas=2)
    S = oracle.sketches(X, H)
    res = oracle.reservoir_init(len(X), p.l_max)
    for r in (1, 0):
        o, m, _ = oracle.partition(X, p, replica=r)
        cand, dd = oracle.leaf_knn(X, o, m, p.k)
        res = oracle.hashprune(res, S, *oracle.bidirected_records(m, cand, dd))
    assert np.array_equal(res, ref["reservoirs"])
    one = oracle.build_index(X, H, p)
    ids2, _, bf2 = oracle.slot_fields(ref["reservoirs"])
    ids1, _, bf1 = oracle.slot_fields(one["reservoirs"])
    # per point, the two-replica reservoir's k-th key is no larger
    for i in range(0, 1500, 50):
        k1 = sorted(int(b) for b, c in zip(bf1[i], ids1[i]) if c != oracle.EMPTY_ID)
        k2 = sorted(int(b) for b, c in zip(bf2[i], ids2[i]) if c != oracle.EMPTY_ID)
        assert len(k2) >= len(k1)
