"""pipnn_hashprune_insert_static (HashPrune insertion with the library's
fixed per-device scratch, no device allocation) against
pipnn_hashprune_insert, through the C ABI.

Two calls in a row on the shared scratch, the second with a smaller index
and fewer records, must each give the same reservoirs byte for byte as the
allocating entry point; the FP64 oracle's closed form (Alg. 3 through the
history-independence lemma) is the third witness. A call whose scratch would
exceed the fixed size is refused on the host.
"""
import numpy as np
import pytest

import oracle
import pipnn_inputs as pi

torch = pytest.importorskip("torch")
import paper_2602_21247_amd as pp  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    pp.lib()
    oracle.set_threads(16)


def dev(a):
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint32:
        a = a.view(np.int32)
    return torch.from_numpy(a).cuda()


def u64(t):
    return t.detach().cpu().numpy().view(np.uint64)


def _records(n, cnt, seed):
    rng = np.random.default_rng(seed)
    dst = rng.integers(0, n, cnt).astype(np.uint32)
    cand = rng.integers(0, n, cnt).astype(np.uint32)
    a = np.minimum(dst, cand).astype(np.int64)
    b = np.maximum(dst, cand).astype(np.int64)
    dist = (((a * 7919 + b * 104729) % 5000) / 3.0).astype(np.float32)  # many ties
    return dst, cand, dist


def _case(n, n_rec, l_max, seed):
    X = pi.workload_points(1, n)
    H = pi.workload_hyperplanes(1)
    idx = pp.Index(dev(X), dev(H), pp.default_params(l_max=l_max, seed=seed))
    dst, cand, dist = _records(n, n_rec, seed)
    S = idx.get_sketches().cpu().numpy().astype(np.float64)
    want = oracle.hashprune(oracle.reservoir_init(n, l_max), S, dst, cand,
                            dist.astype(np.float64), closed=True)
    return idx, (dev(dst), dev(cand), dev(dist)), want


def test_static_scratch_insert_equals_allocating_insert():
    cases = [(9000, 400_000, 64, 3), (2500, 60_000, 24, 4)]  # the second call is smaller
    for i, (n, n_rec, l_max, seed) in enumerate(cases):
        print(f"case {i}: n={n} records={n_rec} l_max={l_max}", flush=True)
        idx, rec, want = _case(n, n_rec, l_max, seed)
        ref = idx.hashprune_insert(*rec, pp.reservoir_init(n, l_max))
        res = pp.reservoir_init(n, l_max)
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0] if i else None
        idx.hashprune_insert_static(*rec, res)
        torch.cuda.synchronize()
        if i:
            # after the first call has looked the array up, a call takes no memory
            assert torch.cuda.mem_get_info()[0] == free0
        assert np.array_equal(u64(res), u64(ref)), f"case {i}: differs from hashprune_insert"
        assert np.array_equal(u64(res), want), f"case {i}: differs from the oracle"
        # inserting the same records again changes nothing (Alg. 3 keeps one slot per bucket)
        idx.hashprune_insert_static(*rec, res)
        torch.cuda.synchronize()
        assert np.array_equal(u64(res), want)
        idx.close()


def test_static_scratch_size_limit():
    n = 1_000_000
    X = np.zeros((n, 32), dtype=np.float32)
    X[:, 0] = np.arange(n, dtype=np.float32)
    H = pi.hyperplanes(12, 32, seed=1)
    idx = pp.Index(dev(X), dev(H), pp.default_params())
    n_rec = 7_000_000  # 12 MB of per-point arrays + 56 MB of records > 64 MiB
    z = torch.zeros(n_rec, dtype=torch.int32, device="cuda")
    d = torch.zeros(n_rec, dtype=torch.float32, device="cuda")
    res = pp.reservoir_init(16, 64)  # never touched: the call is refused on the host
    with pytest.raises(pp.PipnnError, match="static scratch"):
        idx.hashprune_insert_static(z, z, d, res)
    idx.close()
