"""Uneven leaves in one launch: wide reduced-precision operands (768-d fp16,
inner product), the persistent schedule, the leaf-kernel configurations the
autotuner chooses from, and a build captured in a HIP graph and replayed.

Every configuration must give the same picks bit for bit (the selection is
exact on the kernel's own distances whatever the schedule); graph replays
must equal the eager build bit for bit; the wide path is held to the
oracle by replaying its own GEMM distances and by the FP32 direct-difference
tolerance of its emitted distances.
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


def wide_params(**kw):
    w = pi.WORKLOADS[4]
    base = dict(metric=w.metric, c_max=w.c_max, c_min=w.c_min, k=w.k, l_max=w.l_max, R=w.R,
                alpha=w.alpha, hash_bits=w.hash_bits, seed=pi.workload_seed(4),
                gemm_prec=pp.PREC_FP16)
    base.update(kw)
    return pp.default_params(**base)


@pytest.fixture(scope="module")
def wide():
    n = 8000
    X16 = pi.workload_points(4, n)
    off, mem = pi.workload_leaves(4, n, X=X16)
    H = pi.workload_hyperplanes(4)
    return X16, H, off, mem


def test_wide_ip_block_replay(wide):
    X16, H, off, mem = wide
    X = X16.astype(np.float32)
    idx = pp.Index(dev(X16), dev(H), wide_params())
    ids = mem[off[3]:off[4]] if off[4] - off[3] >= 600 else mem[:900]
    ids = np.sort(ids[:900]).astype(np.uint32)
    k = 32
    oc, od, om = idx.knn_block(dev(ids), dev(ids), k, True, want_matrix=True)
    torch.cuda.synchronize()
    M = om.cpu().numpy()
    # fp16 holds X exactly; the GEMM distance is -x.y with FP32 accumulation
    Xd = X[ids].astype(np.float64)
    G = -(Xd @ Xd.T)
    d = X.shape[1]
    bound = (d + 3) * 2.0 ** -23 * (np.abs(Xd) @ np.abs(Xd).T)
    assert np.all(np.abs(M - G) <= bound)
    sel, _ = oracle.topk_rows(M, k, self_col=np.arange(len(ids)))
    assert np.array_equal(u32(oc), sel)
    ref = np.take_along_axis(G, u32(oc).astype(np.int64), 1)
    assert np.all(np.abs(od.cpu().numpy() - ref) <= np.maximum(REL * np.abs(ref), ABS))
    idx.close()


def test_wide_leaf_pick_against_fp64(wide):
    X16, H, off, mem = wide
    X = X16.astype(np.float32)
    p = wide_params()
    idx = pp.Index(dev(X16), dev(H), p)
    oc, od = idx.leaf_pick(dev(off), dev(mem))
    torch.cuda.synchronize()
    exact, ed = oracle.leaf_knn(X, off, mem, p.k, metric=1)
    got = u32(oc)
    agree = np.mean([len(set(a) & set(b)) / len(b) for a, b in zip(got, exact)])
    print(f"768-d fp16 inner-product picks: agreement with FP64 {agree:.5f}")
    assert agree >= 0.999
    gd = od.cpu().numpy().astype(np.float64)
    Xd = X.astype(np.float64)
    rows = np.repeat(mem, p.k)
    c = got.reshape(-1)
    ok = c != oracle.EMPTY_ID
    ref = -(Xd[rows[ok]] * Xd[c[ok]]).sum(1)
    assert np.all(np.abs(gd.reshape(-1)[ok] - ref) <= np.maximum(REL * np.abs(ref), ABS))
    idx.close()


@pytest.mark.parametrize("case", ["int128-fp32", "vmf96-bf16", "vmf96-bf16-extra", "wide768-fp16"])
def test_leaf_configs_give_identical_picks(case, wide):
    """Work-item size and schedule never change a pick. The two register
    layouts sum the GEMM products in different orders: on integer data
    (exact arithmetic) they agree bit for bit too, elsewhere their FP32
    distances of a pair agree bit for bit and the picks almost everywhere."""
    if case == "int128-fp32":
        X = pi.integer_mixture(20000, 128, 60, 40.0, seed=41)
        H = pi.hyperplanes(12, 128, seed=42, integer=True)
        p = pp.default_params(c_max=1024, k=16, seed=43)
        ref_idx = pp.Index(dev(X), dev(H), p)
        off, mem = ref_idx.partition()
        ref_idx.close()
        off, mem = off.cpu().numpy(), u32(mem)
        Xs = X
    elif case.startswith("vmf96-bf16"):
        Xs = pi.workload_points(3, 12000)
        H = pi.workload_hyperplanes(3)
        # 32 selected for rescoring, or 20 (four lanes: a list of 20; two: 32)
        resc = dict(rescore_extra=4) if case.endswith("extra") else dict(rescore_mult=2)
        p = pp.default_params(c_max=1024, k=16, seed=7, gemm_prec=pp.PREC_BF16, **resc)
        o = oracle.partition(Xs, oracle.make_params(c_max=1024, k=16, seed=7))
        off, mem = o[0], o[1]
    else:
        Xs, H, off, mem = wide
        p = wide_params()
    idx = pp.Index(dev(Xs), dev(H), p)
    outs = {}
    for layout in (pp.LAYOUT_PAIR, pp.LAYOUT_QUAD):
        for rows in (128, 64):
            for pers in (False, True):
                try:
                    idx.set_leaf_config(rows, pers, layout)
                except pp.PipnnError:
                    # 64-row items: two-lane layout at 65..128 dimensions only;
                    # the 768-d operand exists in the four-lane layout only
                    assert rows == 64 or (case == "wide768-fp16" and layout == pp.LAYOUT_PAIR)
                    continue
                oc, od = idx.leaf_pick(dev(off), dev(mem))
                torch.cuda.synchronize()
                outs[(layout, rows, pers)] = (u32(oc).copy(), od.cpu().numpy().copy())
    assert len(outs) >= 2
    for layout in (pp.LAYOUT_PAIR, pp.LAYOUT_QUAD):
        same = [v for k, v in outs.items() if k[0] == layout]
        for c, d in same[1:]:
            assert np.array_equal(c, same[0][0]), layout
            assert np.array_equal(d, same[0][1]), layout
    keys = sorted(outs)
    if keys[0][0] != keys[-1][0]:
        (c0, d0), (c1, d1) = outs[keys[0]], outs[keys[-1]]
        if case == "int128-fp32":
            assert np.array_equal(c0, c1) and np.array_equal(d0, d1)
        else:
            same_pick = c0 == c1
            print(case, f"layouts: same picks {same_pick.mean():.5f}")
            assert same_pick.mean() >= 0.999
            # where both layouts pick the same pair, its recomputed distance is the same
            assert np.array_equal(d0[same_pick], d1[same_pick])
    res = idx.autotune(dev(off), dev(mem))
    print(case, "autotune:", res)
    assert len(res) == len(outs) and all(r[3] > 0 for r in res)
    oc, od = idx.leaf_pick(dev(off), dev(mem))
    torch.cuda.synchronize()
    best = min(res, key=lambda r: r[3])
    assert np.array_equal(u32(oc), outs[(best[2], best[0], best[1])][0])
    idx.close()


def test_graph_replay_equals_eager(wide):
    X16, H, off, mem = wide
    p = wide_params()
    idx = pp.Index(dev(X16), dev(H), p)
    doff, dmem = dev(off), dev(mem)
    n = X16.shape[0]
    # eager reference
    res_e = pp.reservoir_init(n, p.l_max)
    idx.build_leaves(doff, dmem, res_e)
    g_e, deg_e = idx.robustprune(res_e)
    torch.cuda.synchronize()
    ref_res, ref_g = u64(res_e).copy(), u32(g_e).copy()
    # planned eager run gives the same
    idx.plan_leaves(doff, dmem)
    res = torch.empty((n, p.l_max), dtype=torch.int64, device="cuda")
    g = torch.empty((n, p.R), dtype=torch.int32, device="cuda")
    deg = torch.empty(n, dtype=torch.int32, device="cuda")
    pp.reservoir_init(n, p.l_max, out=res)
    idx.build_leaves(doff, dmem, res)
    idx.robustprune(res, g, deg)
    torch.cuda.synchronize()
    assert np.array_equal(u64(res), ref_res)
    # capture: reservoir init + leaf build + final prune
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        pp.reservoir_init(n, p.l_max, out=res)
        idx.build_leaves(doff, dmem, res)
        idx.robustprune(res, g, deg)
    for rep in range(3):
        res.fill_(0)
        g.fill_(0)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert np.array_equal(u64(res), ref_res), f"replay {rep}: reservoirs differ"
        assert np.array_equal(u32(g), ref_g), f"replay {rep}: graph differs"
        # eager work between replays
        oc, od = idx.leaf_pick(doff, dmem)
        torch.cuda.synchronize()
    idx.close()


def test_capture_without_plan_is_refused(wide):
    X16, H, off, mem = wide
    p = wide_params()
    idx = pp.Index(dev(X16), dev(H), p)
    res = torch.empty((X16.shape[0], p.l_max), dtype=torch.int64, device="cuda")
    doff, dmem = dev(off), dev(mem)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    err = None
    with torch.cuda.graph(graph):
        try:
            idx.build_leaves(doff, dmem, res)
        except pp.PipnnError as e:
            err = str(e)
    assert err is not None and "plan" in err
    idx.close()


def test_wide_build_recall_against_oracle_graph(wide):
    X16, H, off, mem = wide
    X = X16.astype(np.float32)
    p = wide_params()
    Q = pi.workload_queries(4, 1000).astype(np.float32)
    idx = pp.Index(dev(X16), dev(H), p)
    res = pp.reservoir_init(X.shape[0], p.l_max)
    idx.build_leaves(dev(off), dev(mem), res)
    g, deg = idx.robustprune(res)
    torch.cuda.synchronize()
    # the oracle's build on the same leaves
    cand, dd = oracle.leaf_knn(X, off, mem, p.k, metric=1)
    dst, cnd, dv = oracle.bidirected_records(mem, cand, dd)
    S = oracle.sketches(X, H)
    ores = oracle.hashprune(oracle.reservoir_init(X.shape[0], p.l_max), S, dst, cnd, dv)
    og, _ = oracle.robustprune(X, ores, p.alpha, p.R, metric=1)
    start, _ = oracle.start_node(X)
    _, gd = oracle.bruteforce_knn(X, Q, 10, metric=1)
    G = u32(g)
    same = np.mean(np.all(G == og, axis=1))
    for L in (32, 64, 128):
        a, _, _ = oracle.beam_search(X, G, Q, 10, L, start, metric=1)
        b, _, _ = oracle.beam_search(X, og, Q, 10, L, start, metric=1)
        ra = oracle.recall_at_k(a, X, Q, gd, metric=1)
        rb = oracle.recall_at_k(b, X, Q, gd, metric=1)
        print(f"identical graph rows {same:.4f}; L={L} gpu-graph recall {ra:.4f} "
              f"oracle-graph recall {rb:.4f}")
        assert abs(ra - rb) <= 0.003
    idx.close()


def test_wide_partition_invariants():
    n = 6000
    X16 = pi.workload_points(4, n)
    H = pi.workload_hyperplanes(4)
    p = wide_params(c_max=512)
    idx = pp.Index(dev(X16), dev(H), p)
    off, mem = idx.partition()
    off, mem = off.cpu().numpy(), u32(mem)
    sizes = np.diff(off)
    assert sizes.max() <= 512 and sizes.min() >= 1
    cnt = np.bincount(mem, minlength=n)
    assert cnt.min() >= 1 and cnt.max() <= 2
    idx.close()


def test_wide_robustprune_against_oracle(wide):
    """RobustPrune on 768-d fp16 inner-product data (the Gram of the GEMM
    operand on MFMA) against the oracle's FP64 RobustPrune on the same
    reservoirs: fp16 holds the data exactly, so the two differ only where
    float32 rounding flips an alpha test; adjacency agreement is held to a
    floor and reported."""
    X16, H, off, mem = wide
    X = X16.astype(np.float32)
    p = wide_params()
    cand, dd = oracle.leaf_knn(X, off, mem, p.k, metric=1)
    dst, cnd, dv = oracle.bidirected_records(mem, cand, dd)
    S = oracle.sketches(X, H)
    ores = oracle.hashprune(oracle.reservoir_init(X.shape[0], p.l_max), S, dst, cnd, dv)
    og, odeg = oracle.robustprune(X, ores, p.alpha, p.R, metric=1)
    idx = pp.Index(dev(X16), dev(H), p)
    g, deg = idx.robustprune(dev(ores))
    torch.cuda.synchronize()
    G = u32(g)
    same_rows = np.mean([np.array_equal(G[i], og[i]) for i in range(len(og))])
    jac = np.mean([len(set(G[i][G[i] != oracle.EMPTY_ID]) & set(og[i][og[i] != oracle.EMPTY_ID])) /
                   max(1, len(set(G[i][G[i] != oracle.EMPTY_ID]) | set(og[i][og[i] != oracle.EMPTY_ID])))
                   for i in range(len(og))])
    print(f"wide RobustPrune: identical lists {same_rows:.4f}, mean Jaccard {jac:.4f}, "
          f"mean degree gpu {u32(deg).mean():.2f} oracle {odeg.mean():.2f}")
    assert same_rows >= 0.98 and jac >= 0.995
    idx.close()


def test_graph_replay_equals_eager_rescored():
    """A captured build whose leaf pick rescores the top k + 4 of a bf16 GEMM
    (the FP32 recompute in the graph): every replay equals the eager build."""
    X = pi.workload_points(3, 12000)
    H = pi.workload_hyperplanes(3)
    p = pp.default_params(c_max=1024, k=16, seed=7, gemm_prec=pp.PREC_BF16, rescore_extra=4)
    o = oracle.partition(X, oracle.make_params(c_max=1024, k=16, seed=7))
    off, mem = o[0], o[1]
    idx = pp.Index(dev(X), dev(H), p)
    doff, dmem = dev(off), dev(mem)
    n = X.shape[0]
    res_e = pp.reservoir_init(n, p.l_max)
    idx.build_leaves(doff, dmem, res_e)
    g_e, _ = idx.robustprune(res_e)
    torch.cuda.synchronize()
    ref_res, ref_g = u64(res_e).copy(), u32(g_e).copy()
    idx.plan_leaves(doff, dmem)
    res = torch.empty((n, p.l_max), dtype=torch.int64, device="cuda")
    g = torch.empty((n, p.R), dtype=torch.int32, device="cuda")
    deg = torch.empty(n, dtype=torch.int32, device="cuda")
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        pp.reservoir_init(n, p.l_max, out=res)
        idx.build_leaves(doff, dmem, res)
        idx.robustprune(res, g, deg)
    for rep in range(3):
        res.fill_(0)
        g.fill_(0)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert np.array_equal(u64(res), ref_res), f"replay {rep}: reservoirs differ"
        assert np.array_equal(u32(g), ref_g), f"replay {rep}: graph differs"
        oc, od = idx.leaf_pick(doff, dmem)
        torch.cuda.synchronize()
    idx.close()
