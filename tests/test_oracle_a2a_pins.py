"""Pins of the oracle's All-to-All Prune leaf picker (Supplement, Picking
within Leaves, All-to-All Prune: RobustPrune of every leaf member over the
other members, lazy form): a hand-worked line example, equality with the
oracle's RobustPrune (itself pinned) fed the leaf as the reservoir, and the
special cases alpha -> infinity (the exact k nearest) and alpha = 0 (the
nearest alone)."""
import json
import os

import numpy as np

import oracle
import pipnn_inputs as pi

HERE = os.path.dirname(os.path.abspath(__file__))


def _line():
    g = json.load(open(os.path.join(HERE, "golden", "a2a_line.json")))
    X = np.zeros((5, 4), dtype=np.float32)
    X[:, 0] = g["points_on_a_line"]
    return g, X


def _rows(cand):
    return [[int(v) for v in r if v != oracle.EMPTY_ID] for r in cand]


def test_hand_worked_line():
    g, X = _line()
    off = np.array([0, 5], dtype=np.int64)
    mem = np.arange(5, dtype=np.uint32)
    for R, key in ((4, "expected_R4"), (1, "expected_R1")):
        cand, dist = oracle.leaf_all_to_all(X, off, mem, R, g["alpha"])
        assert _rows(cand) == g[key]
        # emitted distances are d(x, c) of the admitted candidates
        for i, r in enumerate(_rows(cand)):
            for t, c in enumerate(r):
                assert dist[i, t] == (X[i, 0] - X[c, 0]) ** 2


def _leaves(n, sizes, seed):
    rng = np.random.default_rng(seed)
    ids = rng.permutation(n)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    mem = np.concatenate([np.sort(ids[off[i]:off[i + 1]]) for i in range(len(sizes))])
    return off, mem.astype(np.uint32)


def test_equals_robustprune_with_the_leaf_as_reservoir():
    """Each member's list is the lazy RobustPrune (Alg. 2) of that member
    over a reservoir holding the leaf's other members."""
    X = pi.integer_mixture(600, 24, 6, 30.0, seed=3)
    off, mem = _leaves(600, [40, 63, 17, 2, 64, 33], seed=4)
    R, alpha, l_max = 8, 1.2, 64
    cand, _ = oracle.leaf_all_to_all(X, off, mem, R, alpha)
    for li in range(len(off) - 1):
        m = mem[off[li]:off[li + 1]]
        res = np.full((len(m), l_max), oracle.empty_slot(), dtype=np.uint64)
        for i in range(len(m)):
            others = np.delete(m, i)
            res[i, :len(others)] = others.astype(np.uint64) | np.uint64(0x7F80 << 48)
        g, deg = oracle.robustprune_points(X, res, m, alpha, R)
        assert np.array_equal(g, cand[off[li]:off[li + 1]]), li


def test_large_alpha_is_exact_knn_and_zero_alpha_the_nearest():
    X = pi.gaussian_mixture(500, 16, 5, 0.4, seed=5)
    off, mem = _leaves(500, [120, 200, 80, 100], seed=6)
    R = 6
    cand, dist = oracle.leaf_all_to_all(X, off, mem, R, 1e30)
    knn, kd = oracle.leaf_knn(X, off, mem, R)
    assert np.array_equal(cand, knn)
    assert np.array_equal(dist, kd)
    near, _ = oracle.leaf_all_to_all(X, off, mem, R, 0.0)
    assert np.array_equal(near[:, 0], knn[:, 0])
    assert np.all(near[:, 1:] == oracle.EMPTY_ID)


def test_member_order_within_a_leaf_does_not_matter():
    """Candidates are taken in (distance, id) order, so listing a leaf's
    members in another order gives every point the same list."""
    X = pi.integer_mixture(300, 8, 4, 20.0, seed=7)
    off = np.array([0, 300], dtype=np.int64)
    mem = np.arange(300, dtype=np.uint32)
    a, _ = oracle.leaf_all_to_all(X, off, mem, 10, 1.2)
    perm = np.random.default_rng(8).permutation(300).astype(np.uint32)
    b, _ = oracle.leaf_all_to_all(X, off, perm, 10, 1.2)
    assert np.array_equal(a[perm], b)
