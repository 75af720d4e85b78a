"""The All-to-All Prune leaf picker (Supplement, Picking within Leaves:
RobustPrune of every leaf member over the rest of its leaf, lazy form)
through the C ABI, against the FP64 oracle.

On integer data every GEMM distance is the exact distance, so the admitted
candidates, their order and their distances must equal the oracle's bit for
bit, for leaves of every size class the kernel has (1 .. 2,048 members), and
so must the reservoirs and the graph of a whole build with this picker. On
real-valued data the GEMM distances round, so near-tied candidates can be
taken in another order: the share of the oracle's picks found is held to a
floor and every emitted distance to the FP32 tolerance."""
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


def explicit_leaves(n, sizes, seed):
    rng = np.random.default_rng(seed)
    out = [np.sort(rng.choice(n, s, replace=False)) for s in sizes]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    return off, np.concatenate(out).astype(np.uint32)


SIZES = [2048, 1500, 1024, 700, 300, 129, 128, 65, 64, 63, 33, 2, 1]


def test_picks_bit_exact_every_size_class():
    X = pi.integer_mixture(6000, 128, 40, 30.0, seed=61)
    H = pi.hyperplanes(12, 128, seed=62, integer=True)
    off, mem = explicit_leaves(6000, SIZES, seed=63)
    for R, alpha in ((16, 1.2), (5, 1.0), (32, 1.5)):
        p = pp.default_params(k=R, alpha=alpha, leaf_picker=pp.PICKER_ALL_TO_ALL)
        idx = pp.Index(dev(X), dev(H), p)
        oc, od = idx.leaf_pick(dev(off), dev(mem))
        torch.cuda.synchronize()
        wc, wd = oracle.leaf_all_to_all(X, off, mem, R, alpha)
        got = u32(oc)
        assert np.array_equal(got, wc), f"R={R} alpha={alpha}"
        valid = wc != oracle.EMPTY_ID
        assert np.array_equal(od.cpu().numpy()[valid].astype(np.float64), wd[valid])
        print(f"R={R} alpha={alpha}: mean admitted {valid.sum(1).mean():.2f}")
        idx.close()


def test_build_bit_exact():
    """Reservoirs and graph of a build whose leaves pick by All-to-All Prune
    (one record per admitted candidate) equal the oracle's."""
    X = pi.integer_mixture(12000, 128, 60, 40.0, seed=71)
    H = pi.hyperplanes(12, 128, seed=72, integer=True)
    p = pp.default_params(c_max=1024, c_min=64, k=16, l_max=64, R=32, seed=73,
                          leaf_picker=pp.PICKER_ALL_TO_ALL)
    op = oracle.make_params(c_max=1024, c_min=64, k=16, l_max=64, R=32, seed=73)
    off, mem, _ = oracle.partition(X, op)
    cand, dd = oracle.leaf_all_to_all(X, off, mem, p.k, p.alpha)
    src = np.repeat(mem, p.k)
    ok = cand.reshape(-1) != oracle.EMPTY_ID
    S = oracle.sketches(X, H)
    ores = oracle.hashprune(oracle.reservoir_init(len(X), p.l_max), S, src[ok],
                            cand.reshape(-1)[ok], dd.reshape(-1)[ok])
    og, odeg = oracle.robustprune(X, ores, p.alpha, p.R)
    idx = pp.Index(dev(X), dev(H), p)
    res = pp.reservoir_init(len(X), p.l_max)
    idx.build_leaves(dev(off), dev(mem), res)
    g, deg = idx.robustprune(res)
    torch.cuda.synchronize()
    assert np.array_equal(u64(res), ores)
    assert np.array_equal(u32(g), og)
    assert np.array_equal(u32(deg), odeg)
    print(f"records {int(ok.sum())}, mean reservoir fill "
          f"{(u64(res) & 0xFFFFFFFF != 0xFFFFFFFF).sum(1).mean():.2f}, mean degree {odeg.mean():.2f}")
    # no planned or captured build, no insertion with this picker
    with pytest.raises(pp.PipnnError):
        idx.plan_leaves(dev(off), dev(mem))
    idx.close()


def test_real_valued_picks_against_fp64():
    X = pi.gaussian_mixture(5000, 64, 30, 0.3, seed=81)
    H = pi.hyperplanes(12, 64, seed=82)
    off, mem = explicit_leaves(5000, [1200, 600, 300, 100, 40], seed=83)
    p = pp.default_params(k=16, alpha=1.2, leaf_picker=pp.PICKER_ALL_TO_ALL)
    idx = pp.Index(dev(X), dev(H), p)
    oc, od = idx.leaf_pick(dev(off), dev(mem))
    torch.cuda.synchronize()
    wc, _ = oracle.leaf_all_to_all(X, off, mem, p.k, p.alpha)
    got, gd = u32(oc), od.cpu().numpy().astype(np.float64)
    same_rows = np.mean(np.all(got == wc, axis=1))
    agree = np.mean([len(set(a[a != oracle.EMPTY_ID]) & set(b[b != oracle.EMPTY_ID]))
                     / max(1, (b != oracle.EMPTY_ID).sum()) for a, b in zip(got, wc)])
    print(f"real-valued: identical lists {same_rows:.4f}, pick agreement {agree:.5f}")
    assert agree >= 0.99
    src = np.repeat(mem, p.k).reshape(got.shape)
    valid = got != oracle.EMPTY_ID
    Xd = X.astype(np.float64)
    d64 = ((Xd[src[valid]] - Xd[got[valid]]) ** 2).sum(1)
    assert np.all(np.abs(gd[valid] - d64) <= np.maximum(REL * np.abs(d64), ABS))
    idx.close()


def test_leaf_too_large_is_refused():
    X = pi.integer_mixture(3000, 32, 10, 20.0, seed=91)
    H = pi.hyperplanes(12, 32, seed=92, integer=True)
    off = np.array([0, 2100], dtype=np.int64)
    mem = np.arange(2100, dtype=np.uint32)
    idx = pp.Index(dev(X), dev(H), pp.default_params(leaf_picker=pp.PICKER_ALL_TO_ALL))
    with pytest.raises(pp.PipnnError, match="2048"):
        idx.leaf_pick(dev(off), dev(mem))
    idx.close()
