"""An index over a caller's workspace: pipnn_workspace_bytes is the layout
the index uses, and the index allocates no device memory.

The 1M x 128 integer-mixture build (its workload parameters) runs on a
workspace of exactly pipnn_workspace_bytes for the smallest record batch
(one leaf of 65535 rows, about 31 batches) and for a whole-build batch. Each
gives the same leaves, canonical reservoirs and graph, bit for bit, as the
self-allocating index: HashPrune does not depend on the order or grouping of
its records (Alg. 3 with its history-independence lemma), and RobustPrune
(Alg. 2) is a function of the reservoir. The device's free memory stays the
same across creation, partition, build, RobustPrune and search. One page
less than the smallest layout is refused with ENOMEM.

A smaller case runs the other entry points on a workspace against the
self-allocating index: leaf picks of both pickers, the planned and captured
build, HashPrune insertion in chunks, the k-NN graph in chunks, 16-bit
queries and a 16-bit X; and the fixed capacity with the insertion epoch.
"""
import ctypes as C

import numpy as np
import pytest

import pipnn_inputs as pi

torch = pytest.importorskip("torch")
import paper_2602_21247_amd as pp  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    pp.lib()


def dev(a):
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint32:
        a = a.view(np.int32)
    return torch.from_numpy(a).cuda()


def u32(t):
    return t.detach().cpu().numpy().view(np.uint32)


def u64(t):
    return t.detach().cpu().numpy().view(np.uint64)


def workload_params(cfg, **kw):
    w = pi.WORKLOADS[cfg]
    return pp.default_params(metric=w.metric, c_max=w.c_max, c_min=w.c_min, k=w.k,
                             l_max=w.l_max, R=w.R, alpha=w.alpha, hash_bits=w.hash_bits,
                             leader_div=w.leader_div, leader_cap=w.leader_cap, fanout=w.fanout,
                             seed=pi.workload_seed(cfg), **kw)


def _outputs(n, p):
    return (torch.empty(n + 1, dtype=torch.int64, device="cuda"),
            torch.empty(2 * n, dtype=torch.int32, device="cuda"),
            torch.empty((n, p.l_max), dtype=torch.int64, device="cuda"),
            torch.empty((n, p.R), dtype=torch.int32, device="cuda"),
            torch.empty(n, dtype=torch.int32, device="cuda"))


def _build(idx, n, p, bufs):
    """Partition, leaf build and RobustPrune through the C ABI into
    preallocated outputs (nothing here allocates device memory)."""
    L, s = pp.lib(), pp._stream()
    off, mem, res, g, deg = bufs
    nl, nm = C.c_int64(), C.c_int64()
    pp._check(L.pipnn_partition(idx._h, pp._ptr(off), off.numel() - 1, pp._ptr(mem), mem.numel(),
                                C.byref(nl), C.byref(nm), s))
    pp._check(L.pipnn_reservoir_init(pp._ptr(res), n, p.l_max, s))
    pp._check(L.pipnn_build_leaves(idx._h, pp._ptr(off), pp._ptr(mem), nl.value, pp._ptr(res), s))
    pp._check(L.pipnn_robustprune(idx._h, pp._ptr(res), pp._ptr(g), pp._ptr(deg), s))
    return nl.value, nm.value


def _search(idx, g, Q, start, ids, dist):
    pp._check(pp.lib().pipnn_search(idx._h, pp._ptr(g), pp._ptr(Q), Q.shape[0], pp._dtype_code(Q),
                                    ids.shape[1], 64, start, pp._ptr(ids), pp._ptr(dist), None,
                                    pp._stream()))


@pytest.fixture(scope="module")
def int1m():
    return dev(pi.workload_points(2)), dev(pi.workload_hyperplanes(2))


def test_workload_build_in_exactly_the_reported_bytes(int1m):
    Xd, Hd = int1m
    n, d = Xd.shape
    p = workload_params(2)
    bufs = _outputs(n, p)
    off, mem, res, g, deg = bufs
    nq = 5000  # three search batches at 1M points (2,147 queries each)
    Q = dev(pi.workload_queries(2, nq))
    Qh = Q.to(torch.bfloat16)
    Qhf = Qh.float()
    ids = torch.empty((nq, 10), dtype=torch.int32, device="cuda")
    dist = torch.empty((nq, 10), dtype=torch.float32, device="cuda")
    # the self-allocating index
    ref = pp.Index(Xd, Hd, p)
    nl, nm = _build(ref, n, p, bufs)
    start = ref.start_node()
    _search(ref, g, Q, start, ids, dist)
    torch.cuda.synchronize()
    want = dict(off=u64(off[:nl + 1]).copy(), mem=u32(mem[:nm]).copy(),
                res=u64(ref.reservoir_canonical(res)).copy(), g=u32(g).copy(),
                deg=u32(deg).copy(), ids=u32(ids).copy())
    _search(ref, g, Qhf, start, ids, dist)
    torch.cuda.synchronize()
    want_h = u32(ids).copy()
    ref.close()
    canon = torch.empty_like(res)
    for mbr, rows in ((1, 65535), (0, 2 * n)):
        need = pp.workspace_bytes(p, n, d, max_batch_records=mbr)
        ws = torch.empty(need, dtype=torch.uint8, device="cuda")
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        idx = pp.Index(Xd, Hd, p, workspace=ws)
        assert _build(idx, n, p, bufs) == (nl, nm)
        assert idx.start_node() == start
        _search(idx, g, Q, start, ids, dist)
        torch.cuda.synchronize()
        free1 = torch.cuda.mem_get_info()[0]
        st = idx.stats()
        print(f"max_batch_records {mbr}: workspace {need / 2**20:.1f} MiB, batch rows "
              f"{st['batch_rows']}, free HBM change {free0 - free1} B")
        assert st["workspace_bytes"] == need and st["batch_rows"] == rows
        assert free0 == free1
        assert np.array_equal(u64(off[:nl + 1]), want["off"])
        assert np.array_equal(u32(mem[:nm]), want["mem"])
        assert np.array_equal(u32(g), want["g"]) and np.array_equal(u32(deg), want["deg"])
        assert np.array_equal(u32(ids), want["ids"])
        pp._check(pp.lib().pipnn_reservoir_canonical(idx._h, pp._ptr(res), pp._ptr(canon),
                                                     pp._stream()))
        assert np.array_equal(u64(canon), want["res"])
        # 16-bit queries: the float32 search of their float32 values
        _search(idx, g, Qh, start, ids, dist)
        torch.cuda.synchronize()
        assert np.array_equal(u32(ids), want_h)
        idx.close()
        del ws
    # one page below the smallest layout
    need = pp.workspace_bytes(p, n, d, max_batch_records=1)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    h = C.c_void_p()
    st = pp.lib().pipnn_create(C.byref(p), pp._ptr(Xd), n, d, 0, pp._ptr(Hd), pp._ptr(ws),
                               need - 4096, pp._stream(), C.byref(h))
    assert st == pp.ENOMEM and not h.value


SMALL_N = 20000


@pytest.fixture(scope="module")
def small():
    X = pi.workload_points(1, SMALL_N)
    H = pi.workload_hyperplanes(1)
    return X, H


def _pair(X, H, p):
    """A self-allocating index and one on a workspace of the smallest layout."""
    n, d = X.shape
    ws = torch.empty(pp.workspace_bytes(p, n, d, max_batch_records=1,
                                        x_dtype=pp._dtype_code(X)),
                     dtype=torch.uint8, device="cuda")
    return pp.Index(X, H, p), pp.Index(X, H, p, workspace=ws)


@pytest.mark.parametrize("picker", [pp.PICKER_KNN, pp.PICKER_ALL_TO_ALL])
def test_leaf_picks_and_build_on_a_workspace(small, picker):
    X, H = small
    p = pp.default_params(leaf_picker=picker)
    ref, idx = _pair(dev(X), dev(H), p)
    off, mem = ref.partition()
    off2, mem2 = idx.partition()
    assert np.array_equal(u64(off), u64(off2)) and np.array_equal(u32(mem), u32(mem2))
    a = ref.leaf_pick(off, mem)
    b = idx.leaf_pick(off, mem)
    torch.cuda.synchronize()
    assert np.array_equal(u32(a[0]), u32(b[0]))
    assert np.array_equal(a[1].cpu().numpy().view(np.uint32), b[1].cpu().numpy().view(np.uint32))
    r1 = pp.reservoir_init(SMALL_N, p.l_max)
    r2 = pp.reservoir_init(SMALL_N, p.l_max)
    ref.build_leaves(off, mem, r1)
    idx.build_leaves(off, mem, r2)
    g1, d1 = ref.robustprune(r1)
    g2, d2 = idx.robustprune(r2)
    torch.cuda.synchronize()
    assert np.array_equal(u64(ref.reservoir_canonical(r1)), u64(idx.reservoir_canonical(r2)))
    assert np.array_equal(u32(g1), u32(g2)) and np.array_equal(u32(d1), u32(d2))
    ref.close()
    idx.close()


def test_planned_and_captured_build_on_a_workspace(small):
    X, H = small
    p = pp.default_params()
    ref, idx = _pair(dev(X), dev(H), p)
    off, mem = ref.partition()
    r_ref = pp.reservoir_init(SMALL_N, p.l_max)
    ref.build_leaves(off, mem, r_ref)
    g_ref, _ = ref.robustprune(r_ref)
    torch.cuda.synchronize()
    want_res, want_g = u64(r_ref).copy(), u32(g_ref).copy()
    idx.plan_leaves(off, mem)
    res = torch.empty((SMALL_N, p.l_max), dtype=torch.int64, device="cuda")
    g = torch.empty((SMALL_N, p.R), dtype=torch.int32, device="cuda")
    deg = torch.empty(SMALL_N, dtype=torch.int32, device="cuda")
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        pp.reservoir_init(SMALL_N, p.l_max, out=res)
        idx.build_leaves(off, mem, res)
        idx.robustprune(res, g, deg)
    for rep in range(3):
        res.fill_(0)
        g.fill_(0)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert np.array_equal(u64(res), want_res), f"replay {rep}"
        assert np.array_equal(u32(g), want_g), f"replay {rep}"
    del graph
    ref.close()
    idx.close()


def test_hashprune_insert_and_knn_graph_in_chunks(small):
    """2.5M records against a bin slice of 2 x 65535 x 16 records: two
    chunks; a k-NN graph with k = 100 against result slices of 65 per point:
    two chunks of points."""
    X, H = small
    p = pp.default_params()
    ref, idx = _pair(dev(X), dev(H), p)
    rng = np.random.default_rng(5)
    cnt = 2_500_000
    dst = dev(rng.integers(0, SMALL_N, cnt).astype(np.uint32))
    cand = dev(rng.integers(0, SMALL_N, cnt).astype(np.uint32))
    dist = dev(rng.random(cnt).astype(np.float32))
    r1 = pp.reservoir_init(SMALL_N, p.l_max)
    r2 = pp.reservoir_init(SMALL_N, p.l_max)
    ref.hashprune_insert(dst, cand, dist, r1)
    idx.hashprune_insert(dst, cand, dist, r2)
    torch.cuda.synchronize()
    assert np.array_equal(u64(ref.reservoir_canonical(r1)), u64(idx.reservoir_canonical(r2)))
    off, mem = ref.partition()
    ref.build_leaves(off, mem, r1)
    g, _ = ref.robustprune(r1)
    start = ref.start_node()
    a_ids, a_d = ref.knn_graph(g, 100, 128, start)
    b_ids, b_d = idx.knn_graph(g, 100, 128, start)
    torch.cuda.synchronize()
    assert np.array_equal(u32(a_ids), u32(b_ids))
    assert np.array_equal(a_d.cpu().numpy().view(np.uint32), b_d.cpu().numpy().view(np.uint32))
    ref.close()
    idx.close()


def test_bf16_points_on_a_workspace(small):
    X, H = small
    Xh = dev(X).to(torch.bfloat16)
    p = pp.default_params(gemm_prec=pp.PREC_BF16)
    ref, idx = _pair(Xh, dev(H), p)
    off, mem = ref.partition()
    r1 = pp.reservoir_init(SMALL_N, p.l_max)
    r2 = pp.reservoir_init(SMALL_N, p.l_max)
    ref.build_leaves(off, mem, r1)
    idx.build_leaves(off, mem, r2)
    g1, _ = ref.robustprune(r1)
    g2, _ = idx.robustprune(r2)
    torch.cuda.synchronize()
    assert np.array_equal(u32(g1), u32(g2))
    ref.close()
    idx.close()


def test_fixed_capacity_and_epochs(small):
    X, H = small
    p = pp.default_params()
    ref, idx = _pair(dev(X), dev(H), p)
    off, mem = idx.partition()
    res = pp.reservoir_init(SMALL_N, p.l_max)
    idx.build_leaves(off, mem, res)
    g, deg = idx.robustprune(res)
    with pytest.raises(pp.PipnnError) as e:
        idx.reserve(SMALL_N + 1)
    assert e.value.status == pp.ESTATE
    idx.reserve(SMALL_N)  # within the capacity: nothing to do
    with pytest.raises(pp.PipnnError) as e:
        idx.insert(10, res, g, deg, epoch=1)
    assert e.value.status == pp.EOVERFLOW
    assert idx.stats()["epoch"] == 0
    # epochs: an empty insertion publishes its label; labels must increase
    idx.insert(0, res, g, deg, epoch=5)
    assert idx.stats()["epoch"] == 5 and idx.stats()["n_points"] == SMALL_N
    with pytest.raises(pp.PipnnError) as e:
        idx.insert(0, res, g, deg, epoch=5)
    assert e.value.status == pp.EINVAL
    ref.close()
    idx.close()
