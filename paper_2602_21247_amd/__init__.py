"""Python binding of libpipnn (the PiPNN leaf hot path for gfx950).

Argument marshalling only: every step runs in the HIP kernels of
``libpipnn.so``; torch provides device memory and the stream. There is no
CPU fallback: importing works without a GPU (so the C ABI can be inspected),
but every call that touches the device needs the built library and a GPU.

The names mirror the C ABI in ``include/pipnn.h``.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpipnn.so")

METRIC_L2, METRIC_IP = 0, 1
DTYPE_F32, DTYPE_F16, DTYPE_BF16 = 0, 1, 2
PREC_FP32, PREC_BF16, PREC_FP8, PREC_FP16 = 0, 1, 2, 3
OK, EINVAL, ENOMEM, EOVERFLOW, EDEVICE, ESTATE = 0, -1, -2, -3, -4, -5
PICKER_KNN, PICKER_ALL_TO_ALL = 0, 1
LAYOUT_PAIR, LAYOUT_QUAD = 0, 1
EMPTY_ID = 0xFFFFFFFF
EMPTY_SLOT = 0x7F80 << 48 | 0xFFFFFFFF

EXPORTS = [
    "pipnn_version", "pipnn_last_error", "pipnn_default_params", "pipnn_workspace_bytes",
    "pipnn_create", "pipnn_destroy", "pipnn_partition", "pipnn_partition_replica",
    "pipnn_build_leaves",
    "pipnn_hashprune_insert", "pipnn_reservoir_init", "pipnn_reservoir_canonical",
    "pipnn_robustprune", "pipnn_start_node", "pipnn_search", "pipnn_get_sketches",
    "pipnn_knn_block", "pipnn_leaf_pick", "pipnn_prepare", "pipnn_set_profiling",
    "pipnn_get_stats", "pipnn_get_operand", "pipnn_plan_leaves", "pipnn_set_leaf_config",
    "pipnn_autotune", "pipnn_reserve", "pipnn_insert", "pipnn_hashprune_insert_static",
    "pipnn_knn_graph",
]


class PipnnError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"pipnn status {status}: {msg}")
        self.status = status


class Params(C.Structure):
    _fields_ = [("metric", C.c_int32), ("c_max", C.c_int32), ("c_min", C.c_int32),
                ("leader_div", C.c_int32), ("leader_cap", C.c_int32),
                ("fanout", C.c_int32 * 4), ("k", C.c_int32), ("hash_bits", C.c_int32),
                ("l_max", C.c_int32), ("R", C.c_int32), ("alpha", C.c_float),
                ("gemm_prec", C.c_int32), ("rescore_mult", C.c_int32),
                ("leaf_picker", C.c_int32), ("rescore_extra", C.c_int32),
                ("seed", C.c_uint64)]


class Stats(C.Structure):
    _fields_ = [("n_leaves", C.c_int64), ("n_members", C.c_int64), ("leader_dists", C.c_int64),
                ("levels", C.c_int32), ("leaf_knn_launches", C.c_int32),
                ("leaf_pairs", C.c_int64), ("records", C.c_int64),
                ("operand_exact", C.c_int32), ("data_int_exact", C.c_int32),
                ("ms_prepare", C.c_double), ("ms_partition", C.c_double),
                ("ms_leaf_knn", C.c_double), ("ms_bin", C.c_double), ("ms_merge", C.c_double),
                ("ms_robustprune", C.c_double), ("epoch", C.c_uint64), ("n_points", C.c_int64),
                ("workspace_bytes", C.c_int64), ("batch_rows", C.c_int64),
                ("rp_row_bits", C.c_int32), ("reserved_", C.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None


def lib():
    """Load libpipnn.so (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "python -m paper_2602_21247_amd.hipbuild")
        L = C.CDLL(LIB_PATH)
        P, i64, i32, u32 = C.c_void_p, C.c_int64, C.c_int32, C.c_uint32
        L.pipnn_version.restype = C.c_char_p
        L.pipnn_last_error.restype = C.c_char_p
        L.pipnn_default_params.argtypes = [C.POINTER(Params)]
        L.pipnn_workspace_bytes.restype = C.c_size_t
        L.pipnn_workspace_bytes.argtypes = [C.POINTER(Params), i64, i32, i32, i64]
        L.pipnn_create.argtypes = [C.POINTER(Params), P, i64, i32, i32, P, P, C.c_size_t, P,
                                   C.POINTER(P)]
        L.pipnn_destroy.argtypes = [P]
        L.pipnn_destroy.restype = None
        L.pipnn_partition.argtypes = [P, P, i64, P, i64, C.POINTER(i64), C.POINTER(i64), P]
        L.pipnn_partition_replica.argtypes = [P, i32, P, i64, P, i64, C.POINTER(i64),
                                              C.POINTER(i64), P]
        L.pipnn_build_leaves.argtypes = [P, P, P, i64, P, P]
        L.pipnn_hashprune_insert.argtypes = [P, P, P, P, i64, P, P]
        L.pipnn_hashprune_insert_static.argtypes = [P, P, P, P, i64, P, P]
        L.pipnn_reservoir_init.argtypes = [P, i64, i32, P]
        L.pipnn_reservoir_canonical.argtypes = [P, P, P, P]
        L.pipnn_robustprune.argtypes = [P, P, P, P, P]
        L.pipnn_start_node.argtypes = [P, C.POINTER(u32), P]
        L.pipnn_search.argtypes = [P, P, P, i64, i32, i32, i32, u32, P, P, P, P]
        L.pipnn_get_sketches.argtypes = [P, P, P]
        L.pipnn_knn_graph.argtypes = [P, P, i32, i32, u32, P, P, P]
        L.pipnn_knn_block.argtypes = [P, P, i64, P, i64, i32, i32, P, P, P, P]
        L.pipnn_leaf_pick.argtypes = [P, P, P, i64, P, P, P]
        L.pipnn_prepare.argtypes = [P, P]
        L.pipnn_set_profiling.argtypes = [P, i32]
        L.pipnn_get_stats.argtypes = [P, C.POINTER(Stats)]
        L.pipnn_get_operand.argtypes = [P, P, P, P, P]
        L.pipnn_plan_leaves.argtypes = [P, P, P, i64, P]
        L.pipnn_set_leaf_config.argtypes = [P, i32, i32, i32]
        L.pipnn_reserve.argtypes = [P, i64, P, P]
        L.pipnn_insert.argtypes = [P, i64, P, P, P, P, C.c_uint64, P]
        L.pipnn_autotune.argtypes = [P, P, P, i64, C.POINTER(TuneResult), i32, C.POINTER(i32), P]
        for name in EXPORTS:
            if name not in ("pipnn_version", "pipnn_last_error", "pipnn_default_params",
                            "pipnn_workspace_bytes", "pipnn_destroy"):
                getattr(L, name).restype = C.c_int32
        _lib = L
    return _lib


def _check(st: int):
    if st != 0:
        raise PipnnError(st, lib().pipnn_last_error().decode())


def version() -> str:
    return lib().pipnn_version().decode()


def default_params(**kw) -> Params:
    p = Params()
    lib().pipnn_default_params(C.byref(p))
    for key, v in kw.items():
        if key == "fanout":
            fo = list(v) + [1] * (4 - len(v))
            for i in range(4):
                p.fanout[i] = int(fo[i])
        else:
            setattr(p, key, v)
    return p


def workspace_bytes(params: Params, n: int, d: int, max_batch_records: int = 0,
                    x_dtype: int = 0) -> int:
    """pipnn_workspace_bytes: the workspace an index over n x d points (X of
    x_dtype) needs with build batches of max_batch_records records (0: a
    whole build in one batch)."""
    return int(lib().pipnn_workspace_bytes(C.byref(params), n, d, x_dtype, max_batch_records))


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("pipnn needs a ROCm GPU (torch.cuda is not available)")
    return torch


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


def _stream():
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dtype_code(t):
    torch = _torch()
    return {torch.float32: DTYPE_F32, torch.float16: DTYPE_F16, torch.bfloat16: DTYPE_BF16}[t.dtype]


def reservoir_init(n: int, l_max: int, out=None):
    torch = _torch()
    res = out if out is not None else torch.empty((n, l_max), dtype=torch.int64, device="cuda")
    _check(lib().pipnn_reservoir_init(_ptr(res), n, l_max, _stream()))
    return res


class TuneResult(C.Structure):
    _fields_ = [("rows_per_item", C.c_int32), ("persistent", C.c_int32), ("layout", C.c_int32),
                ("ms", C.c_float)]


class Index:
    """An index over device-resident points X (n x d) with hyperplanes H."""

    def __init__(self, X, H, params: Params, workspace=None):
        """workspace: a device tensor (contiguous, 256-byte aligned) whose
        bytes hold every device buffer of the index (see workspace_bytes);
        None: the index allocates its own."""
        torch = _torch()
        assert X.is_cuda and X.is_contiguous() and X.dim() == 2
        self.X = X
        self.H = H.to(device=X.device, dtype=torch.float32).contiguous()
        self.params = params
        self.n, self.d = X.shape
        self.epoch = 0
        self.workspace = workspace
        ws_bytes = 0
        if workspace is not None:
            assert workspace.is_cuda and workspace.is_contiguous()
            ws_bytes = workspace.numel() * workspace.element_size()
        h = C.c_void_p()
        _check(lib().pipnn_create(C.byref(params), _ptr(X), self.n, self.d, _dtype_code(X),
                                  _ptr(self.H), _ptr(workspace), ws_bytes, _stream(),
                                  C.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().pipnn_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- the hot path
    def prepare(self):
        _check(lib().pipnn_prepare(self._h, _stream()))

    def set_profiling(self, on: bool):
        _check(lib().pipnn_set_profiling(self._h, 1 if on else 0))

    def stats(self) -> dict:
        st = Stats()
        _check(lib().pipnn_get_stats(self._h, C.byref(st)))
        return st.as_dict()

    def plan_leaves(self, offsets, members):
        """Plan these leaves so that build_leaves on them can be captured."""
        _check(lib().pipnn_plan_leaves(self._h, _ptr(offsets), _ptr(members),
                                       offsets.numel() - 1, _stream()))

    def set_leaf_config(self, rows_per_item: int = 128, persistent: bool = False,
                        layout: int = LAYOUT_PAIR):
        _check(lib().pipnn_set_leaf_config(self._h, rows_per_item, 1 if persistent else 0,
                                           layout))

    def autotune(self, offsets, members):
        """Time every leaf-kernel configuration on these leaves and keep the
        fastest; returns [(rows_per_item, persistent, layout, ms), ...]."""
        out = (TuneResult * 16)()
        cnt = C.c_int32()
        _check(lib().pipnn_autotune(self._h, _ptr(offsets), _ptr(members), offsets.numel() - 1,
                                    out, 16, C.byref(cnt), _stream()))
        return [(out[i].rows_per_item, bool(out[i].persistent), out[i].layout, out[i].ms)
                for i in range(cnt.value)]

    def workspace_bytes(self, n: int, max_batch_records: int = 0) -> int:
        """pipnn_workspace_bytes for this index's parameters and X dtype at
        n points."""
        return workspace_bytes(self.params, n, self.d, max_batch_records, _dtype_code(self.X))

    def reserve(self, n_cap: int, X=None):
        """Room for n_cap points (the bound X must have n_cap rows). X: a new
        device tensor (same dtype and width, the current points in its first
        n rows) to bind instead of the current one."""
        if X is not None:
            assert X.is_cuda and X.is_contiguous() and X.dim() == 2 and X.shape[1] == self.d
            assert X.dtype == self.X.dtype and X.shape[0] >= n_cap
        _check(lib().pipnn_reserve(self._h, n_cap, None if X is None else _ptr(X), _stream()))
        if X is not None:
            self.X = X

    def insert(self, n_new: int, reservoirs, graph, degree, groups=None, epoch=None):
        """Insert rows [n, n + n_new) of X (already written by the caller)
        as snapshot `epoch` (default: the last one + 1)."""
        ep = self.epoch + 1 if epoch is None else int(epoch)
        _check(lib().pipnn_insert(self._h, n_new, None if groups is None else _ptr(groups),
                                  _ptr(reservoirs), _ptr(graph), _ptr(degree), ep, _stream()))
        self.n += n_new
        self.epoch = ep

    def partition(self, replica: int = 0):
        """Ball carving (Alg. 5); replica r > 0 is an independent carving
        with another root key."""
        torch = _torch()
        nl, nm = C.c_int64(), C.c_int64()
        cap_l, cap_m = max(16, self.n // 64), 2 * self.n
        for _ in range(2):
            off = torch.empty(cap_l + 1, dtype=torch.int64, device="cuda")
            mem = torch.empty(max(cap_m, 1), dtype=torch.int32, device="cuda")
            st = lib().pipnn_partition_replica(self._h, replica, _ptr(off), cap_l, _ptr(mem),
                                               cap_m, C.byref(nl), C.byref(nm), _stream())
            if st == 0:
                return off[: nl.value + 1], mem[: nm.value]
            if st != EOVERFLOW:
                _check(st)
            cap_l, cap_m = nl.value, nm.value
        _check(st)

    def build_leaves(self, offsets, members, reservoirs):
        _check(lib().pipnn_build_leaves(self._h, _ptr(offsets), _ptr(members),
                                        offsets.numel() - 1, _ptr(reservoirs), _stream()))
        return reservoirs

    def hashprune_insert(self, dst, cand, dist, reservoirs):
        _check(lib().pipnn_hashprune_insert(self._h, _ptr(dst), _ptr(cand), _ptr(dist),
                                            dst.numel(), _ptr(reservoirs), _stream()))
        return reservoirs

    def hashprune_insert_static(self, dst, cand, dist, reservoirs):
        """hashprune_insert with the library's fixed per-device scratch
        (no device allocation; see pipnn_hashprune_insert_static)."""
        _check(lib().pipnn_hashprune_insert_static(self._h, _ptr(dst), _ptr(cand), _ptr(dist),
                                                   dst.numel(), _ptr(reservoirs), _stream()))
        return reservoirs

    def reservoir_canonical(self, res):
        torch = _torch()
        out = torch.empty_like(res)
        _check(lib().pipnn_reservoir_canonical(self._h, _ptr(res), _ptr(out), _stream()))
        return out

    def robustprune(self, reservoirs, graph=None, degree=None):
        torch = _torch()
        g = graph if graph is not None else torch.empty((self.n, self.params.R),
                                                        dtype=torch.int32, device="cuda")
        deg = degree if degree is not None else torch.empty(self.n, dtype=torch.int32,
                                                            device="cuda")
        _check(lib().pipnn_robustprune(self._h, _ptr(reservoirs), _ptr(g), _ptr(deg), _stream()))
        return g, deg

    def start_node(self) -> int:
        out = C.c_uint32()
        _check(lib().pipnn_start_node(self._h, C.byref(out), _stream()))
        return int(out.value)

    def search(self, graph, Q, k: int, L: int, start: int, want_dist=True, want_cmps=True):
        torch = _torch()
        nq = Q.shape[0]
        ids = torch.empty((nq, k), dtype=torch.int32, device="cuda")
        dist = torch.empty((nq, k), dtype=torch.float32, device="cuda") if want_dist else None
        cmps = torch.empty(nq, dtype=torch.int32, device="cuda") if want_cmps else None
        _check(lib().pipnn_search(self._h, _ptr(graph), _ptr(Q), nq, _dtype_code(Q), k, L, start,
                                  _ptr(ids), _ptr(dist), _ptr(cmps), _stream()))
        return ids, dist, cmps

    def knn_graph(self, graph, k: int, L: int, start: int, want_dist=True):
        """k nearest other points of every indexed point, by searching each
        one on the graph (see pipnn_knn_graph): ids (n x k), dist (n x k)."""
        torch = _torch()
        ids = torch.empty((self.n, k), dtype=torch.int32, device="cuda")
        dist = torch.empty((self.n, k), dtype=torch.float32, device="cuda") if want_dist else None
        _check(lib().pipnn_knn_graph(self._h, _ptr(graph), k, L, start, _ptr(ids), _ptr(dist),
                                     _stream()))
        return ids, dist

    # ---- inspection
    def get_sketches(self):
        torch = _torch()
        out = torch.empty((self.n, self.params.hash_bits), dtype=torch.float32, device="cuda")
        _check(lib().pipnn_get_sketches(self._h, _ptr(out), _stream()))
        return out

    def get_operand(self):
        """The reduced-precision GEMM operand: (codes n x d as uint16 / uint8,
        per-point decode scale, squared norms of the decoded vectors)."""
        torch = _torch()
        prec = self.params.gemm_prec
        dt = torch.uint8 if prec == PREC_FP8 else torch.int16
        codes = torch.empty((self.n, self.d), dtype=dt, device="cuda")
        scale = torch.empty(self.n, dtype=torch.float32, device="cuda")
        norms = torch.empty(self.n, dtype=torch.float32, device="cuda")
        _check(lib().pipnn_get_operand(self._h, _ptr(codes), _ptr(scale), _ptr(norms),
                                       _stream()))
        return codes, scale, norms

    def knn_block(self, row_ids, col_ids, k: int, exclude_diag: bool, want_matrix=False):
        torch = _torch()
        nr, nc = row_ids.numel(), col_ids.numel()
        oc = torch.empty((nr, k), dtype=torch.int32, device="cuda")
        od = torch.empty((nr, k), dtype=torch.float32, device="cuda")
        om = torch.empty((nr, nc), dtype=torch.float32, device="cuda") if want_matrix else None
        _check(lib().pipnn_knn_block(self._h, _ptr(row_ids), nr, _ptr(col_ids), nc, k,
                                     1 if exclude_diag else 0, _ptr(oc), _ptr(od), _ptr(om),
                                     _stream()))
        return oc, od, om

    def leaf_pick(self, offsets, members):
        torch = _torch()
        tot = members.numel()
        k = self.params.k
        oc = torch.empty((tot, k), dtype=torch.int32, device="cuda")
        od = torch.empty((tot, k), dtype=torch.float32, device="cuda")
        _check(lib().pipnn_leaf_pick(self._h, _ptr(offsets), _ptr(members), offsets.numel() - 1,
                                     _ptr(oc), _ptr(od), _stream()))
        return oc, od


def build(X, H, params: Params, replicas: int = 1):
    """Alg. 4 on the GPU: partition, leaf pick + HashPrune, final RobustPrune.
    With replicas > 1, that many independent partitions feed the same
    reservoirs. Returns (index, offsets, members, reservoirs, graph, degree)
    with the last replica's leaves."""
    idx = Index(X, H, params)
    res = reservoir_init(idx.n, params.l_max)
    for r in range(replicas):
        off, mem = idx.partition(r)
        idx.build_leaves(off, mem, res)
    g, deg = idx.robustprune(res)
    return idx, off, mem, res, g, deg
