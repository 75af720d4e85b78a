"""Serving: insertion (pipnn_insert) bit-exact against the oracle's
insertion on integer data, insertion order independence, and the
continuous-batching server giving every request the same result alone and
in the mix."""
import numpy as np
import pytest

import oracle
import pipnn_inputs as pi

torch = pytest.importorskip("torch")
import paper_2602_21247_amd as pp  # noqa: E402
from paper_2602_21247_amd import serving  # noqa: E402

pytestmark = pytest.mark.gpu


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


def oracle_params(p):
    return oracle.make_params(metric=p.metric, c_max=p.c_max, c_min=p.c_min,
                              leader_div=p.leader_div, leader_cap=p.leader_cap,
                              fanout=tuple(p.fanout), k=p.k, hash_bits=p.hash_bits,
                              l_max=p.l_max, R=p.R, alpha=p.alpha, seed=p.seed)


N0, CAP, D = 10000, 13000, 128


@pytest.fixture(scope="module")
def base():
    X = pi.integer_mixture(CAP, D, 60, 40.0, seed=51)
    H = pi.hyperplanes(12, D, seed=52, integer=True)
    p = pp.default_params(c_max=1024, c_min=64, k=16, l_max=64, R=32, seed=53)
    return X, H, p


def built(X, H, p, cap=CAP):
    """A GPU build on the first N0 points with buffers of capacity cap."""
    Xc = torch.from_numpy(X[:cap]).cuda()
    Hd = torch.from_numpy(H).cuda()
    idx = pp.Index(Xc[:N0], Hd, p)
    off, mem = idx.partition()
    res = torch.empty((cap, p.l_max), dtype=torch.int64, device="cuda")
    pp.reservoir_init(N0, p.l_max, out=res[:N0])
    idx.build_leaves(off, mem, res[:N0])
    g = torch.full((cap, p.R), -1, dtype=torch.int32, device="cuda")
    deg = torch.zeros(cap, dtype=torch.int32, device="cuda")
    idx.robustprune(res[:N0], g[:N0], deg[:N0])
    idx.reserve(cap)
    torch.cuda.synchronize()
    return idx, Xc, off, mem, res, g, deg


def canon(idx, res, n):
    out = torch.empty_like(res[:n])
    pp._check(pp.lib().pipnn_reservoir_canonical(idx._h, pp._ptr(res[:n]), pp._ptr(out),
                                                 pp._stream()))
    torch.cuda.synchronize()
    return u64(out)


def test_insert_bit_exact_against_oracle(base):
    X, H, p = base
    idx, Xc, off, mem, res, g, deg = built(X, H, p)
    res0 = canon(idx, res, N0).copy()
    g0 = u32(g[:N0]).copy()
    m = 1500
    groups = np.repeat(np.arange(3, dtype=np.int32), m // 3)
    idx.insert(m, res, g, deg, torch.from_numpy(groups).cuda())
    torch.cuda.synchronize()
    got_res = canon(idx, res, N0 + m)
    ores, touched, orows = oracle.insert(X[:N0 + m], N0, groups, off.cpu().numpy(),
                                         u32(mem), res0, H, p.k, p.alpha, p.R,
                                         fanout0=p.fanout[0])
    assert np.array_equal(got_res, oracle.reservoir_canonical(ores))
    G = u32(g[:N0 + m])
    assert np.array_equal(G[touched], orows)
    untouched = np.setdiff1d(np.arange(N0), touched)
    assert np.array_equal(G[untouched], g0[untouched])
    idx.close()


def test_failed_insert_leaves_index_usable(base):
    """An insertion that fails after its rows were routed (a leaf would grow
    past 65,535 columns) leaves the point count as it was: the next
    insertion, of other points in the same rows, still equals the oracle's
    insertion bit for bit."""
    X, H, p = base
    m_bad = 65_000
    cap = N0 + m_bad
    Xc = torch.zeros((cap, D), dtype=torch.float32, device="cuda")
    Xc[:N0] = torch.from_numpy(X[:N0]).cuda()
    Hd = torch.from_numpy(H).cuda()
    idx = pp.Index(Xc[:N0], Hd, p)
    off, mem = idx.partition()
    res = torch.empty((cap, p.l_max), dtype=torch.int64, device="cuda")
    pp.reservoir_init(N0, p.l_max, out=res[:N0])
    idx.build_leaves(off, mem, res[:N0])
    g = torch.full((cap, p.R), -1, dtype=torch.int32, device="cuda")
    deg = torch.zeros(cap, dtype=torch.int32, device="cuda")
    idx.robustprune(res[:N0], g[:N0], deg[:N0])
    idx.reserve(cap)
    torch.cuda.synchronize()
    res0 = canon(idx, res, N0).copy()
    # 65,000 copies of one point in one request: its two leaves would grow
    # past 65,535 columns
    Xc[N0:] = Xc[0]
    with pytest.raises(pp.PipnnError, match="65535"):
        idx.insert(m_bad, res, g, deg)
    torch.cuda.synchronize()
    assert idx.n == N0
    assert np.array_equal(canon(idx, res, N0), res0)
    m = 1200
    Xc[N0:N0 + m] = torch.from_numpy(X[N0:N0 + m]).cuda()
    groups = np.repeat(np.arange(2, dtype=np.int32), m // 2)
    idx.insert(m, res, g, deg, torch.from_numpy(groups).cuda())
    torch.cuda.synchronize()
    ores, touched, orows = oracle.insert(X[:N0 + m], N0, groups, off.cpu().numpy(), u32(mem),
                                         res0, H, p.k, p.alpha, p.R, fanout0=p.fanout[0])
    assert np.array_equal(canon(idx, res, N0 + m), oracle.reservoir_canonical(ores))
    assert np.array_equal(u32(g[:N0 + m])[touched], orows)
    idx.close()


def test_inserts_after_reserve_take_no_memory(base):
    """After pipnn_reserve, insertions up to the capacity reallocate none of
    the library's point-indexed scratch: free HBM is the same after every
    insertion of a series (the first one sizes the per-call buffers)."""
    X, H, p = base
    idx, Xc, off, mem, res, g, deg = built(X, H, p)
    sizes = [400, 300, 200, 150, 100]
    frees = []
    for m in sizes:
        idx.insert(m, res, g, deg)
        torch.cuda.synchronize()
        frees.append(torch.cuda.mem_get_info()[0])
    print("free HBM after each insertion:", frees)
    assert len(set(frees[1:])) == 1
    idx.close()


def test_insert_alone_equals_together(base):
    X, H, p = base
    m = 900
    groups = np.repeat(np.arange(3, dtype=np.int32), m // 3)
    # together: one call, three groups
    idx, Xc, off, mem, res, g, deg = built(X, H, p)
    idx.insert(m, res, g, deg, torch.from_numpy(groups).cuda())
    torch.cuda.synchronize()
    res_t, g_t = canon(idx, res, N0 + m), u32(g[:N0 + m]).copy()
    idx.close()
    # alone: three calls in a row
    idx, Xc, off, mem, res, g, deg = built(X, H, p)
    for gi in range(3):
        idx.insert(m // 3, res, g, deg)
    torch.cuda.synchronize()
    assert np.array_equal(canon(idx, res, N0 + m), res_t)
    assert np.array_equal(u32(g[:N0 + m]), g_t)
    idx.close()


def _requests(X, seed, n_req=40):
    rng = np.random.default_rng(seed)
    reqs, nxt, t = [], N0, 0.0
    for rid in range(n_req):
        t += rng.exponential(0.003)
        if rng.random() < 0.3 and nxt < CAP - 300:
            m = int(np.exp(rng.uniform(0, np.log(300))))
            reqs.append(serving.Request(rid, "insert", t, X[nxt:nxt + m]))
            nxt += m
        else:
            q = int(np.exp(rng.uniform(0, np.log(200))))
            Q = pi.integer_mixture(q, D, 60, 40.0, seed=1000 + rid)
            reqs.append(serving.Request(rid, "query", t, Q, k=10))
    return reqs


@pytest.mark.parametrize("grow", [False, True])
def test_server_same_alone_and_in_mix(base, grow):
    """Every request's result is the same alone and in the continuous-batching
    mix; with grow, the server starts with room for 64 more points only and
    grows the capacity (new X, reservoirs and graphs, pipnn_reserve with the
    new X) several times mid-stream, admitted by free HBM."""
    X, H, p = base
    reqs = _requests(X, seed=7)
    # the mix: continuous batching on two streams
    idx, Xc, off, mem, res, g, deg = built(X, H, p, cap=N0 + 64 if grow else CAP)
    start = idx.start_node()
    srv = serving.Server(idx, Xc, res, g, deg, start,
                         serving.ServerConfig(L=48, grow_factor=1.0))
    out = srv.run(reqs)
    n_mix = srv.n
    res, g = srv.res, srv.g
    g_mix = u32(g[:n_mix]).copy()
    res_mix = canon(idx, res, n_mix)
    summ = serving.summarize(out, 1.0)
    print("mix:", summ, "insert batches", len({r.batch for r in out.values() if r.kind == "insert"}),
          "query batches", len({r.batch for r in out.values() if r.kind == "query"}),
          "growths", srv.growths)
    assert srv.rejected == 0
    if grow:
        assert len(srv.growths) >= 2 and srv.cap >= n_mix
    idx.close()
    # alone: every insertion by itself, in the mix's commit order; each query
    # alone against the graph that held the same insertions
    ins = sorted((r for r in reqs if r.kind == "insert"), key=lambda r: out[r.rid].first_id)
    batches = sorted({out[r.rid].batch for r in ins})
    idx, Xc, off, mem, res, g, deg = built(X, H, p)
    by_epoch = {}
    for r in reqs:
        if r.kind == "query":
            by_epoch.setdefault(out[r.rid].epoch, []).append(r)

    def run_queries(epoch):
        for r in by_epoch.get(epoch, []):
            Qd = torch.from_numpy(r.data).cuda()
            ids, dist, _ = idx.search(g[:idx.n], Qd, r.k, 48, start)
            torch.cuda.synchronize()
            assert np.array_equal(u32(ids), out[r.rid].ids), f"query {r.rid} at epoch {epoch}"

    run_queries(0)
    for e, b in enumerate(batches):
        for r in ins:
            if out[r.rid].batch == b:
                idx.insert(len(r.data), res, g, deg)
        torch.cuda.synchronize()
        run_queries(e + 1)
    assert idx.n == n_mix
    assert np.array_equal(canon(idx, res, n_mix), res_mix)
    assert np.array_equal(u32(g[:n_mix]), g_mix)
    idx.close()
