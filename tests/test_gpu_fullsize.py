"""Parity at the benchmark's full size and launch configuration: the
1,000,000 x 128 integer-valued workload (every decision exact in float32),
built on the GPU exactly as bench.py times it, checked against the oracle
on sampled outputs it can compute one by one: the whole partition, the
picks of sampled leaves, the reservoirs and RobustPrune lists of sampled
points, and BeamSearch at the benchmark's beam width."""
import numpy as np
import pytest

import oracle
import pipnn_inputs as pi

torch = pytest.importorskip("torch")
import paper_2602_21247_amd as pp  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def full():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    oracle.set_threads(16)
    w = pi.WORKLOADS[2]
    X = pi.workload_points(2)
    H = pi.workload_hyperplanes(2)
    p = pp.default_params(metric=w.metric, c_max=w.c_max, c_min=w.c_min, k=w.k, l_max=w.l_max,
                          R=w.R, alpha=w.alpha, hash_bits=w.hash_bits, leader_div=w.leader_div,
                          leader_cap=w.leader_cap, fanout=w.fanout, seed=pi.workload_seed(2))
    idx = pp.Index(torch.from_numpy(X).cuda(), torch.from_numpy(H).cuda(), p)
    idx.prepare()
    off, mem = idx.partition()
    res = torch.empty((X.shape[0], w.l_max), dtype=torch.int64, device="cuda")
    pp.reservoir_init(X.shape[0], w.l_max, out=res)
    idx.build_leaves(off, mem, res)
    g, deg = idx.robustprune(res)
    torch.cuda.synchronize()
    yield dict(X=X, H=H, p=p, w=w, idx=idx, off=off.cpu().numpy(),
               mem=mem.cpu().numpy().view(np.uint32), res=res, g=g, deg=deg)
    idx.close()


def oracle_params(p):
    return oracle.make_params(metric=p.metric, c_max=p.c_max, c_min=p.c_min,
                              leader_div=p.leader_div, leader_cap=p.leader_cap,
                              fanout=tuple(p.fanout), k=p.k, hash_bits=p.hash_bits,
                              l_max=p.l_max, R=p.R, alpha=p.alpha, seed=p.seed)


def leaf_sets(off, mem):
    return sorted(tuple(mem[off[i]:off[i + 1]].tolist()) for i in range(len(off) - 1))


def test_fullsize_partition_is_the_oracles(full):
    ooff, omem, _ = oracle.partition(full["X"], oracle_params(full["p"]))
    assert leaf_sets(full["off"], full["mem"]) == leaf_sets(ooff, omem)


def test_fullsize_sampled_leaves_points_and_queries(full):
    X, H, p, w = full["X"], full["H"], full["p"], full["w"]
    off, mem = full["off"], full["mem"]
    rng = np.random.default_rng(17)
    # points to check, and every leaf that holds one of them (their records
    # come from those leaves only)
    pts = rng.choice(X.shape[0], 40, replace=False).astype(np.uint32)
    leaf_of = np.repeat(np.arange(len(off) - 1), np.diff(off))
    sel = np.unique(leaf_of[np.isin(mem, pts)])
    s_off = np.concatenate([[0], np.cumsum(np.diff(off)[sel])]).astype(np.int64)
    s_mem = np.concatenate([mem[off[L]:off[L + 1]] for L in sel])
    cand, dd = oracle.leaf_knn(X, s_off, s_mem, p.k)
    # 1. picks of those leaves (GPU leaf kernel in the build's configuration)
    oc, od = full["idx"].leaf_pick(torch.from_numpy(s_off).cuda(),
                                   torch.from_numpy(s_mem.view(np.int32)).cuda())
    torch.cuda.synchronize()
    assert np.array_equal(oc.cpu().numpy().view(np.uint32), cand)
    valid = cand != oracle.EMPTY_ID
    assert np.array_equal(od.cpu().numpy().astype(np.float64)[valid], dd[valid])
    # 2. reservoirs of the points: the closed form over their records
    dst, cnd, dv = oracle.bidirected_records(s_mem, cand, dd)
    keep = np.isin(dst, pts)
    S = oracle.sketches(X, H)
    ores = oracle.hashprune(oracle.reservoir_init(X.shape[0], p.l_max), S, dst[keep], cnd[keep],
                            dv[keep], closed=True)
    gres = full["res"][torch.from_numpy(pts.astype(np.int64)).cuda()]
    idx = full["idx"]
    canon = oracle.reservoir_canonical(gres.cpu().numpy().view(np.uint64))
    assert np.array_equal(canon, oracle.reservoir_canonical(ores[pts]))
    # 3. RobustPrune of the points from the GPU's reservoirs
    og, odeg = oracle.robustprune_points(X, full["res"].cpu().numpy().view(np.uint64)[pts], pts,
                                         p.alpha, p.R)
    G = full["g"].cpu().numpy().view(np.uint32)
    assert np.array_equal(G[pts], og)
    assert np.array_equal(full["deg"].cpu().numpy().view(np.uint32)[pts], odeg)
    # 4. BeamSearch at the benchmark's beam width, on the GPU graph
    Q = pi.workload_queries(2, 100)
    start = idx.start_node()
    ostart, _ = oracle.start_node(X)
    assert start == ostart
    ids, dist, cmps = idx.search(full["g"], torch.from_numpy(Q).cuda(), 10, 384, start)
    torch.cuda.synchronize()
    oi, odist, ocmps = oracle.beam_search(X, G, Q, 10, 384, start)
    assert np.array_equal(ids.cpu().numpy().view(np.uint32), oi)
    assert np.array_equal(dist.cpu().numpy().astype(np.float64), odist)
    assert np.array_equal(cmps.cpu().numpy().view(np.uint32), ocmps)
