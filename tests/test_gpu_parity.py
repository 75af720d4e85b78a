"""Parity of the gfx950 path (through the C ABI) with the FP64 oracle.

Integer-valued data (with integer hyperplanes) makes every distance, norm,
dot product and sketch exact in float32, so on it the GPU and the oracle
take every decision on the same values and must agree bit for bit:
partition, picks, hashes, reservoirs, RobustPrune lists and search results.
On real-valued data the discrete steps are checked by replaying the GPU's
own float32 values through the oracle, float results are held to
|d_gpu - d_64| <= max(1e-5 |d_64|, 1e-6), and recall@10 of the end graph to
within 0.3 points of the oracle's graph.
"""
import numpy as np
import pytest

import oracle
import pipnn_inputs as pi

torch = pytest.importorskip("torch")
import paper_2602_21247_amd as pp  # noqa: E402

pytestmark = pytest.mark.gpu

REL, ABS = 1e-5, 1e-6


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    pp.lib()
    oracle.set_threads(16)


def u32(t):
    return t.detach().cpu().numpy().view(np.uint32)


def u64(t):
    return t.detach().cpu().numpy().view(np.uint64)


def dev(a):
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint32:
        a = a.view(np.int32)
    if a.dtype == np.uint64:
        a = a.view(np.int64)
    return torch.from_numpy(a).cuda()


def int_points(n, d, seed, centers=40, sigma=30.0):
    return pi.integer_mixture(n, d, centers, sigma, seed=seed)


def quantized_gauss(n, d, seed):
    """Gaussian-mixture points rounded to multiples of 1/8: every distance
    and dot product is then exact in float32."""
    X = pi.gaussian_mixture(n, d, 20, 0.5, seed=seed)
    return (np.rint(X * 8.0) / 8.0).astype(np.float32)


def exact_sqdist(A, B):
    A = np.rint(A * 8).astype(np.int64)
    B = np.rint(B * 8).astype(np.int64)
    G = A @ B.T
    na = (A * A).sum(1)
    nb = (B * B).sum(1)
    return (na[:, None] + nb[None, :] - 2 * G).astype(np.float64) / 64.0


def topk_lex(D, k, exclude_diag):
    rows, cols = D.shape
    out = np.full((rows, k), 0xFFFFFFFF, dtype=np.uint32)
    ci = np.arange(cols)
    for r in range(rows):
        order = np.lexsort((ci, D[r]))
        if exclude_diag:
            order = order[order != r]
        m = min(k, len(order))
        out[r, :m] = order[:m]
    return out


def gpu_params(**kw):
    return pp.default_params(**kw)


def oracle_params(p):
    return oracle.make_params(metric=p.metric, c_max=p.c_max, c_min=p.c_min,
                              leader_div=p.leader_div, leader_cap=p.leader_cap,
                              fanout=tuple(p.fanout), k=p.k, hash_bits=p.hash_bits,
                              l_max=p.l_max, R=p.R, alpha=p.alpha, seed=p.seed)


def leaf_sets(off, mem):
    off = np.asarray(off)
    mem = np.asarray(mem).view(np.uint32) if np.asarray(mem).dtype == np.int32 else np.asarray(mem)
    return sorted(tuple(mem[off[i]:off[i + 1]].tolist()) for i in range(len(off) - 1))


# ---------------------------------------------------------------------------
# fused distance + selection kernel

@pytest.mark.parametrize("d", [128, 96, 40])
@pytest.mark.parametrize("nr,nc,k,diag", [(300, 300, 16, True), (257, 1000, 4, False),
                                          (70, 70, 32, True), (5, 3, 16, True),
                                          (129, 700, 16, False), (300, 300, 20, True),
                                          (257, 1000, 24, False), (300, 300, 12, True),
                                          (257, 1000, 2, False), (129, 700, 18, False)])
def test_knn_block_exact(d, nr, nc, k, diag):
    if diag:
        nc = nr
    X = int_points(1200, d, seed=11 + d)
    H = pi.hyperplanes(12, d, seed=5, integer=True)
    idx = pp.Index(dev(X), dev(H), gpu_params(k=k))
    rng = np.random.default_rng(d + nr)
    cols = np.sort(rng.choice(1200, nc, replace=False)).astype(np.uint32)
    rows = cols if diag else np.sort(rng.choice(1200, nr, replace=False)).astype(np.uint32)
    oc, od, om = idx.knn_block(dev(rows), dev(cols), k, diag, want_matrix=True)
    torch.cuda.synchronize()
    D = ((X[rows].astype(np.int64)[:, None, :] - X[cols].astype(np.int64)[None]) ** 2).sum(-1)
    want = topk_lex(D, k, diag)
    assert np.array_equal(u32(oc), want)
    assert np.array_equal(om.cpu().numpy(), D.astype(np.float32))
    got_d = od.cpu().numpy()
    valid = want != 0xFFFFFFFF
    assert np.array_equal(got_d[valid], np.take_along_axis(D, np.where(valid, want, 0), 1)[valid])
    assert np.all(np.isinf(got_d[~valid]))
    idx.close()


def test_knn_block_float_replay():
    X = pi.workload_points(1, 3000)
    H = pi.workload_hyperplanes(1)
    idx = pp.Index(dev(X), dev(H), gpu_params(k=16))
    ids = np.sort(np.random.default_rng(3).choice(3000, 700, replace=False)).astype(np.uint32)
    oc, od, om = idx.knn_block(dev(ids), dev(ids), 16, True, want_matrix=True)
    torch.cuda.synchronize()
    M = om.cpu().numpy()
    # the GPU's float32 GEMM distances, replayed through the oracle's selection
    sel, _ = oracle.topk_rows(M, 16, self_col=np.arange(700))
    assert np.array_equal(u32(oc), sel)
    # the GEMM distances are the norm-expansion form: within the worst-case
    # float32 rounding bound of a d-term dot product, (d+3) 2^-23 (|x|^2+|y|^2)
    Xd = X[ids].astype(np.float64)
    D64 = ((Xd[:, None, :] - Xd[None]) ** 2).sum(-1)
    nrm = (Xd * Xd).sum(1)
    bound = (X.shape[1] + 3) * 2.0 ** -23 * (nrm[:, None] + nrm[None])
    assert np.all(np.abs(M - D64) <= bound)
    assert np.median(np.abs(M - D64) / bound) < 0.05
    # emitted distances are FP32 direct differences: within the stated bound
    got = od.cpu().numpy()
    ref = np.take_along_axis(D64, u32(oc).astype(np.int64), 1)
    assert np.all(np.abs(got - ref) <= np.maximum(REL * np.abs(ref), ABS))
    idx.close()


def test_sketches():
    X = int_points(3000, 128, seed=21)
    H = pi.hyperplanes(12, 128, seed=2002, integer=True)
    idx = pp.Index(dev(X), dev(H), gpu_params())
    S = idx.get_sketches().cpu().numpy().astype(np.float64)
    assert np.array_equal(S, oracle.sketches(X, H))
    idx.close()
    Xf = pi.workload_points(1, 3000)
    Hf = pi.workload_hyperplanes(1)
    idx = pp.Index(dev(Xf), dev(Hf), gpu_params())
    S = idx.get_sketches().cpu().numpy().astype(np.float64)
    S64 = oracle.sketches(Xf, Hf)
    scale = np.abs(Xf.astype(np.float64)) @ np.abs(Hf.astype(np.float64)).T
    assert np.all(np.abs(S - S64) <= 1e-6 * scale + 1e-6)
    idx.close()


# ---------------------------------------------------------------------------
# HashPrune

def _records(n, cnt, seed):
    rng = np.random.default_rng(seed)
    dst = rng.integers(0, n, cnt).astype(np.uint32)
    cand = rng.integers(0, n, cnt).astype(np.uint32)
    a = np.minimum(dst, cand).astype(np.int64)
    b = np.maximum(dst, cand).astype(np.int64)
    dist = (((a * 7919 + b * 104729) % 5000) / 3.0).astype(np.float32)  # many ties
    return dst, cand, dist


@pytest.mark.parametrize("l_max,m", [(64, 12), (8, 3), (200, 16), (5, 1)])
def test_hashprune_insert_replay(l_max, m):
    n = 1500
    X = pi.workload_points(1, n)
    H = pi.hyperplanes(m, 128, seed=77)
    idx = pp.Index(dev(X), dev(H), gpu_params(l_max=l_max, hash_bits=m))
    S = idx.get_sketches().cpu().numpy().astype(np.float64)
    dst, cand, dist = _records(n, 120_000, m)
    want = oracle.hashprune(oracle.reservoir_init(n, l_max), S, dst, cand, dist.astype(np.float64),
                            closed=True)
    res = pp.reservoir_init(n, l_max)
    for part in np.array_split(np.arange(len(dst)), 3):
        idx.hashprune_insert(dev(dst[part]), dev(cand[part]), dev(dist[part]), res)
    torch.cuda.synchronize()
    assert np.array_equal(u64(res), want)
    # reversed order in one call, then everything again: same bytes
    res2 = pp.reservoir_init(n, l_max)
    r = slice(None, None, -1)
    idx.hashprune_insert(dev(dst[r]), dev(cand[r]), dev(dist[r]), res2)
    idx.hashprune_insert(dev(dst), dev(cand), dev(dist), res2)
    torch.cuda.synchronize()
    assert np.array_equal(u64(res2), want)
    assert np.array_equal(u64(idx.reservoir_canonical(res2)), want)
    idx.close()


def test_hashprune_hub_point_many_records():
    """One destination receiving far more records than an LDS chunk holds."""
    n = 5000
    X = pi.workload_points(1, n)
    H = pi.workload_hyperplanes(1)
    idx = pp.Index(dev(X), dev(H), gpu_params(l_max=64))
    S = idx.get_sketches().cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(8)
    cand = rng.integers(0, n, 20_000).astype(np.uint32)
    dst = np.zeros_like(cand)
    dist = rng.uniform(0, 100, 20_000).astype(np.float32)
    want = oracle.hashprune(oracle.reservoir_init(n, 64), S, dst, cand, dist.astype(np.float64))
    res = pp.reservoir_init(n, 64)
    idx.hashprune_insert(dev(dst), dev(cand), dev(dist), res)
    torch.cuda.synchronize()
    assert np.array_equal(u64(res), want)
    idx.close()


def test_hashprune_rejects_bad_id():
    X = pi.workload_points(1, 100)
    idx = pp.Index(dev(X), dev(pi.workload_hyperplanes(1)), gpu_params())
    res = pp.reservoir_init(100, 64)
    with pytest.raises(pp.PipnnError):
        idx.hashprune_insert(dev(np.array([1], np.uint32)), dev(np.array([100], np.uint32)),
                             dev(np.array([1.0], np.float32)), res)
    idx.close()


def test_reservoir_canonical_of_shuffled_slots():
    n, l_max = 300, 16
    X = pi.workload_points(1, n)
    idx = pp.Index(dev(X), dev(pi.workload_hyperplanes(1)), gpu_params(l_max=l_max))
    S = idx.get_sketches().cpu().numpy().astype(np.float64)
    dst, cand, dist = _records(n, 20_000, 9)
    want = oracle.hashprune(oracle.reservoir_init(n, l_max), S, dst, cand, dist.astype(np.float64))
    rng = np.random.default_rng(1)
    shuffled = np.stack([row[rng.permutation(l_max)] for row in want])
    got = u64(idx.reservoir_canonical(dev(shuffled)))
    assert np.array_equal(got, want)
    assert np.array_equal(oracle.reservoir_canonical(shuffled), want)
    idx.close()


# ---------------------------------------------------------------------------
# partition, pick, full build on exact data

PARTITION_CASES = [
    # (points, params)
    ("int", dict(c_max=512, c_min=48, leader_div=300, seed=7)),
    ("int", dict(c_max=256, c_min=200, leader_div=1000, seed=8, fanout=(2, 2, 1, 1))),
    ("quant", dict(c_max=1024, c_min=64, seed=9)),
    ("quant", dict(c_max=300, c_min=16, leader_div=50, leader_cap=40, seed=10)),
]


@pytest.mark.parametrize("kind,kw", PARTITION_CASES)
def test_partition_bit_exact(kind, kw):
    X = int_points(24000, 64, seed=31) if kind == "int" else quantized_gauss(12000, 48, seed=32)
    p = gpu_params(**kw)
    idx = pp.Index(dev(X), dev(pi.hyperplanes(12, X.shape[1], 1, integer=True)), p)
    off, mem = idx.partition()
    torch.cuda.synchronize()
    got = leaf_sets(off.cpu().numpy(), mem.cpu().numpy())
    ooff, omem, _ = oracle.partition(X, oracle_params(p))
    want = leaf_sets(ooff, omem)
    assert got == want
    assert max(len(x) for x in got) <= p.c_max
    idx.close()


def test_partition_hand_worked_golden():
    """The hand-worked carving of tests/golden/partition_merge_recursion.json
    (Alg. 5, Sec. 4.1: merge by the sum of sizes, a duplicate in a merged
    group, kept buckets of exactly C_min and C_max, recursion with a derived
    child key, a no-progress chunk) on the GPU planner: the same leaves."""
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden",
                           "partition_merge_recursion.json")) as f:
        g = json.load(f)
    X = np.array(g["points_1d"], dtype=np.float32)[:, None]
    P = g["params"]
    p = gpu_params(c_max=P["c_max"], c_min=P["c_min"], leader_div=P["leader_div"],
                   leader_cap=P["leader_cap"], fanout=tuple(P["fanout"]), seed=P["seed"])
    idx = pp.Index(dev(X), dev(pi.hyperplanes(12, 1, 1, integer=True)), p)
    off, mem = idx.partition()
    torch.cuda.synchronize()
    got = leaf_sets(off.cpu().numpy(), mem.cpu().numpy())
    assert got == sorted(tuple(v) for v in g["expected_leaves"])
    assert idx.stats()["leader_dists"] == g["expected_leader_dists"]
    idx.close()


def test_partition_single_leaf_and_duplicates():
    X = int_points(500, 16, seed=33)
    idx = pp.Index(dev(X), dev(pi.hyperplanes(4, 16, 1, integer=True)), gpu_params(c_max=1024))
    off, mem = idx.partition()
    assert off.cpu().tolist() == [0, 500] and np.array_equal(u32(mem), np.arange(500))
    idx.close()
    Z = np.zeros((1000, 8), dtype=np.float32)
    p = gpu_params(c_max=300, c_min=1, seed=1)
    idx = pp.Index(dev(Z), dev(pi.hyperplanes(4, 8, 1, integer=True)), p)
    off, mem = idx.partition()
    ooff, omem, _ = oracle.partition(Z, oracle_params(p))
    assert leaf_sets(off.cpu().numpy(), mem.cpu().numpy()) == leaf_sets(ooff, omem)
    idx.close()


@pytest.fixture(scope="module")
def exact_build():
    """Integer data with integer hyperplanes: the oracle's full build."""
    X = int_points(20000, 128, seed=41, centers=60, sigma=40.0)
    H = pi.hyperplanes(12, 128, seed=42, integer=True)
    p = gpu_params(c_max=1024, c_min=64, k=16, l_max=64, R=32, seed=43)
    ref = oracle.build_index(X, H, oracle_params(p))
    return X, H, p, ref


def test_leaf_pick_exact(exact_build):
    X, H, p, ref = exact_build
    idx = pp.Index(dev(X), dev(H), p)
    oc, od = idx.leaf_pick(dev(ref["offsets"]), dev(ref["members"]))
    torch.cuda.synchronize()
    assert np.array_equal(u32(oc), ref["cand"])
    gd = od.cpu().numpy()
    valid = ref["cand"] != oracle.EMPTY_ID
    assert np.array_equal(gd[valid].astype(np.float64), ref["dist"][valid])
    idx.close()


def test_full_build_bit_exact(exact_build):
    X, H, p, ref = exact_build
    idx, off, mem, res, g, deg = pp.build(dev(X), dev(H), p)
    torch.cuda.synchronize()
    assert leaf_sets(off.cpu().numpy(), mem.cpu().numpy()) == leaf_sets(ref["offsets"],
                                                                         ref["members"])
    assert np.array_equal(u64(res), ref["reservoirs"])
    assert np.array_equal(u32(g), ref["graph"])
    assert np.array_equal(u32(deg), ref["degree"])
    # search: same start, exact distances -> same beams, same comparison counts
    Q = int_points(300, 128, seed=44, centers=60, sigma=40.0)
    start, _ = oracle.start_node(X)
    for L in (16, 64):
        ids, dist, cmps = idx.search(g, dev(Q), 10, L, start)
        torch.cuda.synchronize()
        oi, odd, oc = oracle.beam_search(X, ref["graph"], Q, 10, L, start)
        assert np.array_equal(u32(ids), oi)
        assert np.array_equal(dist.cpu().numpy().astype(np.float64), odd)
        assert np.array_equal(u32(cmps), oc)
    idx.close()


@pytest.mark.parametrize("d", [37, 128])
def test_search_any_width_bit_exact(d):
    """BeamSearch (Alg. 1) on a built graph equals the oracle's on the same
    graph bit for bit -- ids, distances and comparison counts -- with rows
    read as 16-byte vectors (d = 128) or one value at a time (d = 37), at
    beam widths whose LDS layouts differ."""
    X = int_points(3000, d, seed=d)
    H = pi.hyperplanes(12, d, seed=5, integer=True)
    idx, off, mem, res, g, deg = pp.build(dev(X), dev(H), gpu_params())
    Q = int_points(200, d, seed=d + 1)
    start, _ = oracle.start_node(X)
    G = u32(g)
    for L in (10, 33, 100, 257):
        ids, dist, cmps = idx.search(g, dev(Q), 10, L, start)
        torch.cuda.synchronize()
        oi, odd, oc = oracle.beam_search(X, G, Q, 10, L, start)
        assert np.array_equal(u32(ids), oi), L
        assert np.array_equal(u32(cmps), oc), L
        assert np.array_equal(dist.cpu().numpy().astype(np.float64), odd), L
    idx.close()


def _drop_own(ids, dist, k):
    """Rows of k + 1 results of point i searched as a query: i's own id
    dropped (its first occurrence), else the last entry."""
    out_i = np.zeros((ids.shape[0], k), dtype=np.uint32)
    out_d = np.zeros((ids.shape[0], k), dtype=np.float64)
    for i in range(ids.shape[0]):
        row = list(zip(ids[i].tolist(), dist[i].tolist()))
        j = next((t for t, (v, _) in enumerate(row) if v == i), None)
        keep = row[:j] + row[j + 1:] if j is not None else row[:k]
        out_i[i] = [v for v, _ in keep]
        out_d[i] = [dd for _, dd in keep]
    return out_i, out_d


def test_knn_graph_bit_exact(exact_build):
    """Approximate 10-NN graph (Sec. 5, k-NN graph construction: every point
    searched on the built graph): equal to the oracle's BeamSearch of every
    point with its own id dropped, ids and distances bit for bit, and its
    recall against the exact 10 nearest other points reported."""
    X, H, p, ref = exact_build
    idx = pp.Index(dev(X), dev(H), p)
    g = dev(ref["graph"])
    start, _ = oracle.start_node(X)
    k = 10
    for L in (16, 48):
        ids, dist = idx.knn_graph(g, k, L, start)
        torch.cuda.synchronize()
        oi, od, _ = oracle.beam_search(X, ref["graph"], X, k + 1, L, start)
        wi, wd = _drop_own(oi, od, k)
        assert np.array_equal(u32(ids), wi), L
        assert np.array_equal(dist.cpu().numpy().astype(np.float64), wd), L
        # recall on a sample: exact 11 nearest including the point itself
        samp = np.arange(0, X.shape[0], 97)
        _, gd = oracle.bruteforce_knn(X, X[samp], k + 1)
        hits = sum(int((wd[i] <= gd[t, k]).sum()) for t, i in enumerate(samp))
        print(f"k-NN graph L={L}: recall@10 {hits / (k * len(samp)):.4f}")
    with pytest.raises(pp.PipnnError):
        idx.knn_graph(g, 10, 10, start)  # needs L > k
    idx.close()


def test_build_order_independence(exact_build):
    X, H, p, ref = exact_build
    idx = pp.Index(dev(X), dev(H), p)
    off, mem = ref["offsets"], ref["members"]
    nl = len(off) - 1
    sizes = np.diff(off)
    perm = np.random.default_rng(5).permutation(nl)
    new_off = np.concatenate([[0], np.cumsum(sizes[perm])]).astype(np.int64)
    new_mem = np.concatenate([mem[off[i]:off[i + 1]] for i in perm]).astype(np.uint32)
    res = pp.reservoir_init(len(X), p.l_max)
    half = nl // 2
    # two calls over the shuffled leaves, then a repeat of the first half
    o1 = new_off[:half + 1]
    idx.build_leaves(dev(o1), dev(new_mem[:o1[-1]]), res)
    o2 = new_off[half:] - new_off[half]
    idx.build_leaves(dev(o2), dev(new_mem[new_off[half]:]), res)
    idx.build_leaves(dev(o1), dev(new_mem[:o1[-1]]), res)
    torch.cuda.synchronize()
    assert np.array_equal(u64(res), ref["reservoirs"])
    idx.close()


@pytest.mark.parametrize("prec", ["bf16", "fp16", "fp32"])
def test_exact_16bit_operand_build(exact_build, prec):
    """Integer features of at most 8 significant bits survive bf16 / fp16
    encoding, so the 16-bit copy holds X exactly: the partition reads the
    copy, the leaf GEMM multiplies it (a float32 index keeps its float32
    leaf GEMM and an fp16 copy for the partition and RobustPrune while X is
    integral), RobustPrune loads its rows from it, and the whole build is
    still the oracle's bit for bit. A copy that does not hold X (the same
    data plus 1/3) keeps the float32 paths."""
    X, H, p, ref = exact_build
    code = {"bf16": pp.PREC_BF16, "fp16": pp.PREC_FP16, "fp32": pp.PREC_FP32}[prec]
    kw = {f: getattr(p, f) for f in ("c_max", "c_min", "k", "l_max", "R", "seed")}
    p16 = gpu_params(gemm_prec=code, **kw)
    idx, off, mem, res, g, deg = pp.build(dev(X), dev(H), p16)
    torch.cuda.synchronize()
    assert idx.stats()["operand_exact"] == 1
    assert leaf_sets(off.cpu().numpy(), mem.cpu().numpy()) == leaf_sets(ref["offsets"],
                                                                         ref["members"])
    assert np.array_equal(u64(res), ref["reservoirs"])
    assert np.array_equal(u32(g), ref["graph"])
    assert np.array_equal(u32(deg), ref["degree"])
    # RobustPrune alone on the oracle's reservoirs
    g2, deg2 = idx.robustprune(dev(ref["reservoirs"]))
    torch.cuda.synchronize()
    assert np.array_equal(u32(g2), ref["graph"])
    idx.close()
    Xf = (X + np.float32(1.0 / 3.0)).astype(np.float32)
    idx = pp.Index(dev(Xf), dev(H), p16)
    assert idx.stats()["operand_exact"] == 0
    idx.close()


@pytest.mark.parametrize("lo,hi,d,want", [
    (0, 255, 128, 1),      # d * 255^2 <= 2^23: the 8-bit workloads
    (0, 256, 128, 1),      # d * A^2 == 2^23 exactly
    (0, 257, 128, 0),      # d * A^2 > 2^23
    (-128, 127, 128, 1),
    (-200, 200, 128, 0),   # A fits, the range does not: d * W^2 > 2^24
    (0, 1020, 128, 0),
    (0, 511, 32, 1),       # fewer dimensions, wider values
])
def test_integer_check(lo, hi, d, want):
    """The check behind skipping the winners' recompute (every distance form
    an exact integer in float32): integral coordinates, d*A^2 <= 2^23 and
    d*W^2 <= 2^24. Non-integral data never passes; prepare takes the check
    again after the caller changes X in place."""
    rng = np.random.default_rng(abs(lo) * 7 + hi + d)
    X = rng.integers(lo, hi + 1, size=(3001, d)).astype(np.float32)
    X[0, 0], X[1, 1] = lo, hi            # the extremes are present
    H = pi.hyperplanes(8, d, 1, integer=True)
    Xd = dev(X)
    idx = pp.Index(Xd, dev(H), gpu_params(k=4))
    assert idx.stats()["data_int_exact"] == want
    Xd[5, 0] += 0.5                      # one non-integral coordinate
    idx.prepare()
    assert idx.stats()["data_int_exact"] == 0
    Xd[5, 0] -= 0.5
    idx.prepare()
    assert idx.stats()["data_int_exact"] == want
    idx.close()


def test_leaf_pick_without_recompute_matches_recompute(exact_build):
    """On integer data within the bound the leaf pick emits the GEMM distance
    (no recompute); the same leaves with rescoring (which always recomputes,
    and on exact distances keeps the same winners) give the same picks and
    the same distances, and both equal the oracle's."""
    X, H, p, ref = exact_build
    idx = pp.Index(dev(X), dev(H), p)
    assert idx.stats()["data_int_exact"] == 1
    oc, od = idx.leaf_pick(dev(ref["offsets"]), dev(ref["members"]))
    kw = {f: getattr(p, f) for f in ("c_max", "c_min", "k", "l_max", "R", "seed")}
    idx2 = pp.Index(dev(X), dev(H), gpu_params(rescore_mult=2, **kw))
    oc2, od2 = idx2.leaf_pick(dev(ref["offsets"]), dev(ref["members"]))
    torch.cuda.synchronize()
    assert np.array_equal(u32(oc), u32(oc2))
    assert np.array_equal(od.cpu().numpy(), od2.cpu().numpy())
    valid = ref["cand"] != oracle.EMPTY_ID
    assert np.array_equal(od.cpu().numpy()[valid].astype(np.float64), ref["dist"][valid])
    idx.close()
    idx2.close()


def test_replicated_build_bit_exact(exact_build):
    """Two independent partitions (replication) into the same reservoirs:
    the second carving's leaves and the final reservoirs and graph equal the
    oracle's replicated build bit for bit."""
    X, H, p, _ = exact_build
    ref = oracle.build_index(X, H, oracle_params(p), replicas=2)
    idx, off, mem, res, g, deg = pp.build(dev(X), dev(H), p, replicas=2)
    torch.cuda.synchronize()
    assert leaf_sets(off.cpu().numpy(), mem.cpu().numpy()) == leaf_sets(ref["offsets"],
                                                                         ref["members"])
    assert np.array_equal(u64(res), ref["reservoirs"])
    assert np.array_equal(u32(g), ref["graph"])
    assert np.array_equal(u32(deg), ref["degree"])
    idx.close()


def test_robustprune_exact_on_oracle_reservoirs(exact_build):
    X, H, p, ref = exact_build
    idx = pp.Index(dev(X), dev(H), p)
    g, deg = idx.robustprune(dev(ref["reservoirs"]))
    torch.cuda.synchronize()
    assert np.array_equal(u32(g), ref["graph"])
    assert np.array_equal(u32(deg), ref["degree"])
    idx.close()


@pytest.mark.parametrize("shift,span,d,bits,alpha", [(0, 256, 128, 8, 1.2), (100, 256, 64, 8, 1.0),
                                                     (-128, 256, 96, 8, 3.75),
                                                     (0, 256, 128, 8, 1.3),
                                                     (0, 300, 32, 16, 1.2)])
def test_robustprune_row_forms(shift, span, d, bits, alpha):
    """RobustPrune reads int8 rows (the coordinates minus the smallest one
    minus 128; the prune test in integer arithmetic with alpha's exact
    binary value) for integral data spanning at most 256 values, the exact
    fp16 copy for a wider integral span; every distance is the same integer
    in each form, so on the build's own reservoirs each gives the oracle's
    graph (whose test alpha * d(y,z) < d(x,z) is exact in FP64)."""
    rng = np.random.default_rng(span + d + shift + 1000)
    X = (rng.integers(0, span, size=(2500, d)) + shift).astype(np.float32)
    H = pi.hyperplanes(12, d, seed=d, integer=True)
    p = gpu_params(c_max=512, c_min=48, k=16, l_max=64, R=32, seed=9, alpha=alpha)
    idx, off, mem, res, g, deg = pp.build(dev(X), dev(H), p)
    torch.cuda.synchronize()
    assert idx.stats()["rp_row_bits"] == bits
    og, odeg = oracle.robustprune(X, u64(res), p.alpha, p.R)
    assert np.array_equal(u32(g), og)
    assert np.array_equal(u32(deg), odeg)
    idx.close()


def test_small_leaves_pad():
    X = int_points(50, 32, seed=51)
    p = gpu_params(k=16)
    idx = pp.Index(dev(X), dev(pi.hyperplanes(12, 32, 1, integer=True)), p)
    off = np.array([0, 1, 3, 6, 50], dtype=np.int64)
    mem = np.arange(50, dtype=np.uint32)
    oc, od = idx.leaf_pick(dev(off), dev(mem))
    cand, dd = oracle.leaf_knn(X, off, mem, 16)
    assert np.array_equal(u32(oc), cand)
    ok = cand != oracle.EMPTY_ID
    assert np.array_equal(od.cpu().numpy()[ok].astype(np.float64), dd[ok])
    idx.close()


def test_start_node_is_nearest_to_mean():
    X = pi.workload_points(1, 10000)
    idx = pp.Index(dev(X), dev(pi.workload_hyperplanes(1)), gpu_params())
    s = idx.start_node()
    o, d64 = oracle.start_node(X)
    assert d64[s] <= d64[o] * (1 + 1e-9) + 1e-9
    idx.close()


# ---------------------------------------------------------------------------
# real-valued data: the end graph's recall

def test_recall_parity_gauss_mixture_10k():
    w = pi.WORKLOADS[1]
    X = pi.workload_points(1)
    Q = pi.workload_queries(1)
    H = pi.workload_hyperplanes(1)
    p = gpu_params(c_max=w.c_max, c_min=w.c_min, k=w.k, l_max=w.l_max, R=w.R, alpha=w.alpha,
                   seed=pi.workload_seed(1))
    ref = oracle.build_index(X, H, oracle_params(p))
    idx, off, mem, res, g, deg = pp.build(dev(X), dev(H), p)
    G = u32(g)
    start, _ = oracle.start_node(X)
    gi, gd = oracle.bruteforce_knn(X, Q, 10)
    for L in (64, 128, 256):
        a, _, _ = oracle.beam_search(X, G, Q, 10, L, start)
        b, _, _ = oracle.beam_search(X, ref["graph"], Q, 10, L, start)
        ra = oracle.recall_at_k(a, X, Q, gd)
        rb = oracle.recall_at_k(b, X, Q, gd)
        print(f"L={L} gpu-graph recall {ra:.4f} oracle-graph recall {rb:.4f}")
        assert abs(ra - rb) <= 0.003
    # the GPU's own search on its graph agrees with the oracle's search on it
    ids, _, _ = idx.search(g, dev(Q), 10, 128, start)
    a, _, _ = oracle.beam_search(X, G, Q, 10, 128, start)
    rg = oracle.recall_at_k(u32(ids), X, Q, gd)
    ra = oracle.recall_at_k(a, X, Q, gd)
    assert abs(rg - ra) <= 0.003
    idx.close()
