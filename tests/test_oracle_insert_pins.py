"""Pins of the oracle's insertion step (an extension of this library: the
paper builds only) to brute force on tiny integer inputs."""
import numpy as np

import oracle


def test_leaf_reps_is_member_nearest_to_mean():
    rng = np.random.default_rng(3)
    X = rng.integers(0, 20, size=(300, 12)).astype(np.float32)
    sizes = [1, 7, 50, 2, 90, 150]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    mem = rng.permutation(300).astype(np.uint32)
    reps = oracle.leaf_reps(X, off, mem)
    Xi = X.astype(np.int64)
    for L in range(len(sizes)):
        m = mem[off[L]:off[L + 1]]
        s = len(m)
        S = Xi[m].sum(0)
        score = ((s * Xi[m] - S) ** 2).sum(1)  # s^2 |x - mean|^2, exact in int64
        best = min(zip(score.tolist(), m.tolist()))[1]
        assert reps[L] == best


def _exact_knn_excluding(Xi, q, pool, k):
    d = ((Xi[pool] - Xi[q]) ** 2).sum(1)
    order = sorted((dd, c) for dd, c in zip(d.tolist(), pool.tolist()) if c != q)
    return [c for _, c in order[:k]]


def test_insert_single_leaf_is_exact_knn_and_groups_separate():
    rng = np.random.default_rng(4)
    n0, m, d, k = 120, 30, 8, 5
    X = rng.integers(0, 30, size=(n0 + m, d)).astype(np.float32)
    H = rng.integers(-16, 17, size=(6, d)).astype(np.float32)
    off = np.array([0, n0], dtype=np.int64)
    mem = np.arange(n0, dtype=np.uint32)
    res0 = oracle.reservoir_init(n0, 16)
    groups = np.array([i % 2 for i in range(m)], dtype=np.int32)
    res, touched, rows = oracle.insert(X, n0, groups, off, mem, res0, H, k, 1.2, 8)
    Xi = X.astype(np.int64)
    # every new point's reservoir holds exactly the records of its picks and
    # of the picks that chose it; its picks are its exact k nearest among
    # the old points and its own group's new points
    for i in range(m):
        p = n0 + i
        pool = np.concatenate([np.arange(n0), n0 + np.flatnonzero(groups == groups[i])])
        want = set(_exact_knn_excluding(Xi, p, pool, k))
        slots = res[p]
        ids = {int(v) & 0xFFFFFFFF for v in slots if (int(v) & 0xFFFFFFFF) != oracle.EMPTY_ID}
        other = n0 + np.flatnonzero(groups != groups[i])
        assert not (ids & set(other.tolist())), "a new point linked to another group"
        # HashPrune keeps at most one per hash bucket: every kept id is a
        # pick or a reverse pick, and the nearest pick is always kept
        assert _exact_knn_excluding(Xi, p, pool, 1)[0] in ids
        rev = {n0 + j for j in range(m) if groups[j] == groups[i]
               and p in _exact_knn_excluding(Xi, n0 + j, np.concatenate(
                   [np.arange(n0), n0 + np.flatnonzero(groups == groups[j])]), k)}
        assert ids <= want | rev
    assert set(range(n0, n0 + m)) <= set(touched.tolist())


def test_robustprune_points_equals_full_rows():
    rng = np.random.default_rng(1)
    X = rng.integers(0, 16, (400, 16)).astype(np.float32)
    off = np.array([0, 400])
    mem = np.arange(400, dtype=np.uint32)
    c, dd = oracle.leaf_knn(X, off, mem, 16)
    S = oracle.sketches(X, rng.integers(-16, 17, (12, 16)).astype(np.float32))
    d_, c_, v_ = oracle.bidirected_records(mem, c, dd)
    res = oracle.hashprune(oracle.reservoir_init(400, 64), S, d_, c_, v_)
    g, deg = oracle.robustprune(X, res, 1.2, 32)
    xs = np.array([5, 17, 399, 0], dtype=np.uint32)
    g2, deg2 = oracle.robustprune_points(X, res[xs], xs, 1.2, 32)
    assert np.array_equal(g2, g[xs]) and np.array_equal(deg2, deg[xs])
