"""Pins of the oracle's reduced-precision GEMM operands and of the rescored
leaf pick.

The encoders are checked against the published format definitions (golden
values of the OCP E4M3 table), against independent library conversions
(torch's bfloat16 and float8_e4m3fn casts, numpy's float16 cast), and by
format properties (round trip, monotonicity, ties to even at every
midpoint). The rescored pick is checked against brute force on tiny inputs
and against the plain pick in the cases where the two must coincide.
"""
import json
import os

import numpy as np
import pytest
import torch

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden")
FP8, BF16, FP16 = oracle.PREC_FP8, oracle.PREC_BF16, oracle.PREC_FP16


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.lib()


def test_e4m3_spec_values():
    g = json.load(open(os.path.join(GOLD, "e4m3_spec.json")))
    for code, val in g["codes"].items():
        c = int(code, 16)
        assert oracle.decode(c, FP8) == val
        if val != 0.0:
            assert oracle.encode(val, FP8) == c
    for code in g["nan_codes"]:
        assert np.isnan(oracle.decode(int(code, 16), FP8))


def test_e4m3_roundtrip_monotone_and_ties_to_even():
    pos = [c for c in range(0x7F)]
    vals = [oracle.decode(c, FP8) for c in pos]
    assert all(b > a for a, b in zip(vals, vals[1:]))
    for c in range(256):
        if c in (0x7F, 0xFF):
            continue
        assert oracle.encode(oracle.decode(c, FP8), FP8) == c
    for c in range(0x7E):
        lo, hi = vals[c], vals[c + 1]
        mid = (lo + hi) / 2.0  # exact in binary32: both are short binary fractions
        assert float(np.float32(mid)) == mid
        even = c if c % 2 == 0 else c + 1
        assert oracle.encode(mid, FP8) == even
        assert oracle.encode(-mid, FP8) == even | 0x80
        below = float(np.nextafter(np.float32(mid), np.float32(0)))
        above = float(np.nextafter(np.float32(mid), np.float32(np.inf)))
        assert oracle.encode(below, FP8) == c
        assert oracle.encode(above, FP8) == c + 1


def test_e4m3_matches_library_cast_and_saturates():
    rng = np.random.default_rng(7)
    x = np.concatenate([
        rng.uniform(-463.9, 463.9, 4000),
        np.exp2(rng.uniform(-14, 8.85, 4000)) * rng.choice([-1, 1], 4000),
    ]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    ours = np.array([oracle.encode(v, FP8) for v in x], dtype=np.uint8)
    np.testing.assert_array_equal(ours, ref)
    # the library cast turns out-of-range values into NaN; this encoder
    # saturates at the largest finite value instead
    for v in (464.0, 480.0, 1e6, 3.4e38):
        assert oracle.encode(v, FP8) == 0x7E
        assert oracle.encode(-v, FP8) == 0xFE


def test_bf16_and_fp16_match_library_casts():
    rng = np.random.default_rng(8)
    x = np.concatenate([
        rng.standard_normal(3000),
        np.exp2(rng.uniform(-30, 20, 3000)) * rng.choice([-1, 1], 3000),
        np.exp2(rng.uniform(-26, -13, 1000)),          # fp16 subnormals
        np.array([65504.0, 65519.0, 65520.0, 7e4, 0.0, -0.0]),
    ]).astype(np.float32)
    bf = np.array([oracle.encode(v, BF16) for v in x], dtype=np.uint16)
    ref_bf = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    np.testing.assert_array_equal(bf, ref_bf)
    h = np.array([oracle.encode(v, FP16) for v in x], dtype=np.uint16)
    with np.errstate(over="ignore"):
        ref_h = x.astype(np.float16).view(np.uint16)
    np.testing.assert_array_equal(h, ref_h)
    dec = np.array([oracle.decode(c, FP16) for c in h])
    np.testing.assert_array_equal(dec, h.view(np.float16).astype(np.float64))
    decb = np.array([oracle.decode(c, BF16) for c in bf])
    ref_decb = torch.from_numpy(ref_bf.view(np.int16)).view(torch.bfloat16).to(torch.float64)
    np.testing.assert_array_equal(decb, ref_decb.numpy())


def test_quantize_fp8_scale_and_error_bound():
    rng = np.random.default_rng(9)
    X = (rng.standard_normal((200, 96)) * np.exp2(rng.uniform(-20, 20, (200, 1)))).astype(
        np.float32)
    X[3] = 0.0
    codes, inv, xq = oracle.quantize(X, FP8)
    assert inv[3] == 1.0 and not codes[3].any() and not xq[3].any()
    mx = np.abs(X).max(axis=1)
    for p in range(200):
        if p == 3:
            continue
        # the largest element saturates to +-448 in code space
        i = int(np.argmax(np.abs(X[p])))
        assert codes[p, i] & 0x7F == 0x7E
        assert inv[p] == np.float32(mx[p] / np.float32(448.0))
    # E4M3 keeps 3 fraction bits: relative error <= 2^-4 for normals, and
    # an absolute error <= 2^-10 * inv (half the subnormal step) below 2^-6
    err = np.abs(xq - X.astype(np.float64))
    bound = np.maximum(np.abs(X) * 2.0 ** -4, 2.0 ** -10 * inv[:, None]) * (1 + 1e-6)
    assert np.all(err <= bound)


def _bf_knn(A, B, k, self_skip=True):
    """Brute force: per row the k smallest (d, id) by float64 squared L2."""
    D = ((A[:, None, :] - B[None, :, :]) ** 2).sum(-1)
    out = []
    for i in range(len(A)):
        order = sorted(((D[i, j], j) for j in range(len(B)) if not (self_skip and j == i)))
        out.append([j for _, j in order[:k]])
    return out


@pytest.mark.parametrize("mult,extra", [(2, 0), (0, 1), (0, 3)])
def test_leaf_knn_lowp_equals_bruteforce_rescore(mult, extra):
    rng = np.random.default_rng(10)
    s, d, k = 40, 24, 4
    X = rng.standard_normal((s, d)).astype(np.float32)
    offsets = np.array([0, s], dtype=np.int64)
    members = np.arange(s, dtype=np.uint32)
    k1 = mult * k if mult else k + extra
    for prec in (BF16, FP8, FP16):
        _, _, xq = oracle.quantize(X, prec)
        cand, dist = oracle.leaf_knn_lowp(X, xq, offsets, members, k, mult, extra=extra)
        first = _bf_knn(xq, xq, k1)
        X64 = X.astype(np.float64)
        for i in range(s):
            rescored = sorted((((X64[i] - X64[j]) ** 2).sum(), j) for j in first[i])[:k]
            assert [j for _, j in rescored] == cand[i].tolist()
            np.testing.assert_allclose(dist[i], [v for v, _ in rescored], rtol=1e-12)


def test_leaf_knn_lowp_special_cases():
    rng = np.random.default_rng(11)
    s, d, k = 30, 16, 5
    offsets = np.array([0, s], dtype=np.int64)
    members = np.arange(s, dtype=np.uint32)
    # every candidate rescored: the exact k-NN of the original vectors
    X = rng.standard_normal((s, d)).astype(np.float32)
    _, _, xq = oracle.quantize(X, FP8)
    cand, _ = oracle.leaf_knn_lowp(X, xq, offsets, members, k, mult=6)
    exact, _ = oracle.leaf_knn(X, offsets, members, k)
    np.testing.assert_array_equal(cand, exact)
    # integers 0..255 are exact in bf16: the bf16 operand is the data itself
    Xi = rng.integers(0, 256, size=(s, d)).astype(np.float32)
    codes, inv, xq = oracle.quantize(Xi, BF16)
    np.testing.assert_array_equal(xq, Xi.astype(np.float64))
    for mult in (0, 2):
        c2, d2 = oracle.leaf_knn_lowp(Xi, xq, offsets, members, k, mult)
        c1, d1 = oracle.leaf_knn(Xi, offsets, members, k)
        np.testing.assert_array_equal(c2, c1)
        np.testing.assert_array_equal(d2, d1)
