"""Seeded synthetic inputs shaped like the PiPNN evaluation workloads.

This module is shared by the FP64 oracle, the tests and the benchmark. It
holds input generation only: no distance, hashing, partitioning or pruning
arithmetic of the method lives here, so neither the oracle nor the GPU path
can borrow the other's computation through it.

Workload shapes follow the dataset table of the experimental section
(BigANN: 128-d uint8, L2; DEEP: 96-d float32, L2; Wikipedia-Cohere: 768-d,
MIPS). None of those datasets is used; each generator below is a seeded
stand-in with the same dimensionality, value type and metric.

Seeds (numpy PCG64): data 1..5, queries 1001..1005, hyperplanes 2001..2005,
partition 3001..3005 for workload i.
"""
from __future__ import annotations

import dataclasses
import numpy as np

METRIC_L2 = 0
METRIC_IP = 1


@dataclasses.dataclass(frozen=True)
class Workload:
    """Sizes and hyper-parameters of one synthetic workload."""
    name: str
    n: int
    d: int
    n_queries: int
    metric: int
    c_max: int
    c_min: int
    k: int
    l_max: int
    R: int
    alpha: float
    hash_bits: int
    fanout: tuple
    leader_div: int = 200
    leader_cap: int = 1000


# The five workloads. Hyper-parameters: C_max, C_min, P_samp (as 1/leader_div),
# the leader cap, fanout by depth, leaf k, hash bits m, reservoir l_max, R, alpha.
# The inner-product workload prunes with alpha = 1: its dissimilarity -x.y is
# negative for similar unit vectors, where alpha > 1 tightens the pruning
# test instead of relaxing it.
WORKLOADS = {
    1: Workload("gauss-mixture-10k-d128-f32", 10_000, 128, 1_000, METRIC_L2,
                1024, 64, 16, 64, 32, 1.2, 12, (2, 1, 1, 1)),
    2: Workload("int-mixture-1M-d128-f32", 1_000_000, 128, 10_000, METRIC_L2,
                2048, 64, 16, 64, 32, 1.2, 12, (2, 1, 1, 1)),
    3: Workload("vmf-mixture-1M-d96-unit", 1_000_000, 96, 10_000, METRIC_L2,
                2048, 64, 16, 64, 32, 1.2, 12, (2, 1, 1, 1)),
    4: Workload("aniso-mixture-2M-d768-f16-ip", 2_000_000, 768, 1_000, METRIC_IP,
                4096, 64, 32, 96, 64, 1.0, 12, (2, 1, 1, 1)),
}

# Spread of the integer mixture around its centres. The value is a choice
# of this project: the workload description fixes only "integer features
# 0..255 from a clipped, rounded Gaussian mixture of 1,000 clusters".
INT_MIXTURE_SIGMA = 40.0


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def gaussian_mixture(n: int, d: int, n_centers: int, sigma: float, seed: int,
                     center_seed: int | None = None) -> np.ndarray:
    """Isotropic Gaussian mixture: centres ~ N(0, I), X = c + sigma * N(0, I).

    ``center_seed`` fixes the centres independently of ``seed`` so that points
    and queries can be drawn from the same mixture.
    """
    crng = _rng(seed if center_seed is None else center_seed)
    centers = crng.standard_normal((n_centers, d))
    rng = _rng(seed + 7919)
    labels = rng.integers(0, n_centers, size=n)
    X = centers[labels] + sigma * rng.standard_normal((n, d))
    return np.ascontiguousarray(X.astype(np.float32))


def integer_mixture(n: int, d: int, n_centers: int, sigma: float, seed: int,
                    center_seed: int | None = None) -> np.ndarray:
    """Clipped, rounded Gaussian mixture with integer values 0..255 stored
    as float32 (a BigANN-like uint8 stand-in). Centres ~ U[0, 255)^d."""
    crng = _rng(seed if center_seed is None else center_seed)
    centers = crng.uniform(0.0, 255.0, size=(n_centers, d))
    rng = _rng(seed + 7919)
    labels = rng.integers(0, n_centers, size=n)
    X = np.rint(centers[labels] + sigma * rng.standard_normal((n, d)))
    X = np.clip(X, 0, 255)
    return np.ascontiguousarray(X.astype(np.float32))


def vmf_mixture(n: int, d: int, n_centers: int, kappa: float, seed: int,
                center_seed: int | None = None) -> np.ndarray:
    """Unit vectors from a von Mises-Fisher mixture (a DEEP-like stand-in).

    Directions mu = normalize(N(0, I)). Samples use Wood's (1994) rejection
    sampler for the cosine w along mu, then a uniform direction orthogonal
    to mu.
    """
    crng = _rng(seed if center_seed is None else center_seed)
    mu = crng.standard_normal((n_centers, d))
    mu /= np.linalg.norm(mu, axis=1, keepdims=True)
    rng = _rng(seed + 7919)
    labels = rng.integers(0, n_centers, size=n)
    # Wood (1994): b, x0, c constants, then accept/reject on w.
    dm1 = d - 1.0
    b = dm1 / (2.0 * kappa + np.sqrt(4.0 * kappa * kappa + dm1 * dm1))
    x0 = (1.0 - b) / (1.0 + b)
    c = kappa * x0 + dm1 * np.log(1.0 - x0 * x0)
    w = np.empty(n)
    todo = np.arange(n)
    while todo.size:
        z = rng.beta(dm1 / 2.0, dm1 / 2.0, size=todo.size)
        ww = (1.0 - (1.0 + b) * z) / (1.0 - (1.0 - b) * z)
        u = rng.uniform(size=todo.size)
        ok = kappa * ww + dm1 * np.log(1.0 - x0 * ww) - c >= np.log(u)
        w[todo[ok]] = ww[ok]
        todo = todo[~ok]
    v = rng.standard_normal((n, d))
    m = mu[labels]
    v -= np.sum(v * m, axis=1, keepdims=True) * m
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    X = w[:, None] * m + np.sqrt(np.maximum(0.0, 1.0 - w * w))[:, None] * v
    X /= np.linalg.norm(X, axis=1, keepdims=True)
    return np.ascontiguousarray(X.astype(np.float32))


def anisotropic_mixture(n: int, d: int, n_centers: int, seed: int,
                        center_seed: int | None = None,
                        dtype=np.float16) -> np.ndarray:
    """Normalised anisotropic Gaussian mixture (a Wikipedia-Cohere-like
    768-d MIPS stand-in). Centres ~ N(0, I)/sqrt(d); noise z * sigma_j with
    sigma_j[i] = 0.25 * (pi_j(i) + 1)^-1/2 for a random permutation pi_j per
    cluster; rows are normalised, then rounded to ``dtype``."""
    crng = _rng(seed if center_seed is None else center_seed)
    centers = crng.standard_normal((n_centers, d)) / np.sqrt(d)
    scales = np.empty((n_centers, d))
    for j in range(n_centers):
        perm = crng.permutation(d)
        scales[j] = 0.25 / np.sqrt(perm + 1.0)
    rng = _rng(seed + 7919)
    labels = rng.integers(0, n_centers, size=n)
    out = np.empty((n, d), dtype=dtype)
    step = 1 << 16
    for s in range(0, n, step):
        e = min(n, s + step)
        lab = labels[s:e]
        Xb = centers[lab] + rng.standard_normal((e - s, d)) * scales[lab]
        Xb /= np.linalg.norm(Xb, axis=1, keepdims=True)
        out[s:e] = Xb.astype(dtype)
    return out


def hyperplanes(m: int, d: int, seed: int, integer: bool = False) -> np.ndarray:
    """Random hyperplane normals H (m x d) through the origin.

    Entries are N(0, 1). With ``integer`` they are rint(16 * N(0, 1)), which
    keeps sketches of integer data exact in float32 (|sum| < 2^24)."""
    rng = _rng(seed)
    H = rng.standard_normal((m, d))
    if integer:
        H = np.rint(16.0 * H)
    return np.ascontiguousarray(H.astype(np.float32))


def zipf_leaf_sizes(total: int, lo: int, hi: int, s: float, seed: int) -> np.ndarray:
    """Leaf sizes ~ truncated Zipf P(size) ~ size^-s on {lo..hi}, drawn until
    they cover ``total`` points (the last size is cut to fit)."""
    rng = _rng(seed)
    support = np.arange(lo, hi + 1)
    p = support.astype(np.float64) ** (-s)
    p /= p.sum()
    sizes = []
    acc = 0
    while acc < total:
        batch = rng.choice(support, size=4096, p=p)
        for v in batch:
            v = int(min(v, total - acc))
            if v < 2:
                if sizes:
                    sizes[-1] += v
                    acc += v
                break
            sizes.append(v)
            acc += v
            if acc >= total:
                break
    return np.asarray(sizes, dtype=np.int64)


def zipf_leaves(n: int, labels_order_key: np.ndarray, lo: int, hi: int, s: float,
                seed: int) -> tuple[np.ndarray, np.ndarray]:
    """Explicit leaves for the uneven-leaf workload: members are consecutive
    chunks of ``labels_order_key`` (an ordering of 0..n-1); chunk sizes are
    truncated-Zipf. Members are sorted ascending within each leaf.
    Returns CSR (offsets int64[n_leaves+1], members uint32[])."""
    sizes = zipf_leaf_sizes(n, lo, hi, s, seed)
    offsets = np.zeros(len(sizes) + 1, dtype=np.int64)
    np.cumsum(sizes, out=offsets[1:])
    members = np.empty(n, dtype=np.uint32)
    for i in range(len(sizes)):
        seg = labels_order_key[offsets[i]:offsets[i + 1]]
        members[offsets[i]:offsets[i + 1]] = np.sort(seg)
    return offsets, members


def mixture_labels(cfg: int, n: int) -> np.ndarray:
    """Mixture component of each point of ``workload_points(cfg, n)`` (the
    first draw of the stream that generated them)."""
    if cfg != 4:
        raise ValueError("labels are exposed for workload 4 only")
    return _rng(4 + 7919).integers(0, 200, size=n)


def rp_tree_order(X: np.ndarray, seed: int, leaf: int = 32) -> np.ndarray:
    """An ordering of the rows of X in which nearby points sit close: a
    random-projection tree (one random direction per level, every segment
    longer than ``leaf`` split at its median projection), read in order."""
    rng = _rng(seed)
    n, d = X.shape
    idx = np.arange(n, dtype=np.int64)
    start = np.zeros(n, dtype=np.int64)     # first position of each position's segment
    length = np.full(n, n, dtype=np.int64)  # its length
    pos = np.arange(n, dtype=np.int64)
    X32 = X if X.dtype == np.float32 else X.astype(np.float32)
    while length.max() > leaf:
        u = rng.standard_normal(d).astype(np.float32)
        proj = X32 @ u
        # sort every segment by projection (segments stay in place)
        idx = idx[np.lexsort((proj[idx], start))]
        split = length > leaf
        half = length // 2
        upper = split & (pos - start >= half)
        new_start = np.where(upper, start + half, start)
        new_len = np.where(split, np.where(upper, length - half, half), length)
        start, length = new_start, new_len
    return idx


def workload_leaves(cfg: int, n: int | None = None,
                    X: np.ndarray | None = None) -> tuple[np.ndarray, np.ndarray]:
    """Explicit uneven leaves of workload 4 (every point in two leaves): two
    orderings of the points, each cut into consecutive chunks of
    truncated-Zipf(1.2) sizes on 64..4096; members ascending within a leaf.
    The first ordering keeps each mixture component together and orders it
    by a random-projection tree; the second is a random-projection tree over
    all points, so leaves also join nearby points of different components.
    Returns one CSR over both. ``X``: the workload's points if already made."""
    if cfg != 4:
        raise ValueError("explicit leaves are defined for workload 4 only")
    w = WORKLOADS[cfg]
    nn = w.n if n is None else n
    if X is None:
        X = workload_points(cfg, nn)
    labels = mixture_labels(cfg, nn)
    offs, mems = [], []
    base = 0
    for j in range(2):
        tree = rp_tree_order(X, 4100 + j)
        rank = np.empty(nn, dtype=np.int64)
        rank[tree] = np.arange(nn)
        order = (np.lexsort((rank, labels)) if j == 0 else tree).astype(np.uint32)
        o, m = zipf_leaves(nn, order, 64, 4096, 1.2, seed=4200 + j)
        offs.append(o[:-1] + base if j == 0 else o + base)
        mems.append(m)
        base += nn
    return np.concatenate(offs).astype(np.int64), np.concatenate(mems).astype(np.uint32)


def workload_points(cfg: int, n: int | None = None) -> np.ndarray:
    """Points of workload ``cfg`` (optionally only the first ``n`` rows'
    worth, generated with the same mixture)."""
    w = WORKLOADS[cfg]
    nn = w.n if n is None else n
    if cfg == 1:
        return gaussian_mixture(nn, w.d, 100, 0.3, seed=1, center_seed=1)
    if cfg == 2:
        return integer_mixture(nn, w.d, 1000, INT_MIXTURE_SIGMA, seed=2, center_seed=2)
    if cfg == 3:
        return vmf_mixture(nn, w.d, 1000, 50.0, seed=3, center_seed=3)
    if cfg == 4:
        return anisotropic_mixture(nn, w.d, 200, seed=4, center_seed=4)
    raise ValueError(cfg)


def workload_queries(cfg: int, nq: int | None = None) -> np.ndarray:
    """Queries drawn from the same mixture as ``workload_points(cfg)``."""
    w = WORKLOADS[cfg]
    q = w.n_queries if nq is None else nq
    if cfg == 1:
        return gaussian_mixture(q, w.d, 100, 0.3, seed=1001, center_seed=1)
    if cfg == 2:
        return integer_mixture(q, w.d, 1000, INT_MIXTURE_SIGMA, seed=1002, center_seed=2)
    if cfg == 3:
        return vmf_mixture(q, w.d, 1000, 50.0, seed=1003, center_seed=3)
    if cfg == 4:
        return anisotropic_mixture(q, w.d, 200, seed=1004, center_seed=4)
    raise ValueError(cfg)


def workload_hyperplanes(cfg: int, m: int | None = None) -> np.ndarray:
    """Hyperplanes of workload ``cfg`` (its hash_bits rows, or ``m``): rows
    are drawn in order from one seeded stream, so the first rows of a larger
    draw equal a smaller draw."""
    w = WORKLOADS[cfg]
    return hyperplanes(m or w.hash_bits, w.d, seed=2000 + cfg, integer=(cfg == 2))


def workload_seed(cfg: int) -> int:
    """Seed of the randomized ball carving for workload ``cfg``."""
    return 3000 + cfg
