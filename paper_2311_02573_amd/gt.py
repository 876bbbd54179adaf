"""Python binding of the C interface in include/gt.h (argument marshalling only).

Every computation runs in the HIP kernels of libgt.so; PyTorch only provides
device memory and the current stream.  There is no CPU fallback: importing
this module raises if the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgt.so")

GT_OK, GT_ERR_INVALID_ARG, GT_ERR_INVALID_INPUT, GT_ERR_OUT_OF_MEMORY = 0, 1, 2, 3
GT_ERR_CAPACITY, GT_ERR_RESULT_OVERFLOW, GT_ERR_DEVICE = 4, 5, 6
STATUS_NAMES = {0: "GT_OK", 1: "GT_ERR_INVALID_ARG", 2: "GT_ERR_INVALID_INPUT",
                3: "GT_ERR_OUT_OF_MEMORY", 4: "GT_ERR_CAPACITY", 5: "GT_ERR_RESULT_OVERFLOW",
                6: "GT_ERR_DEVICE"}
GT_F32, GT_F16, GT_BF16 = 0, 1, 2
POOL_F32, POOL_BF16, POOL_FP8, POOL_MAX_F32, POOL_MAX_BF16 = 1, 2, 4, 8, 16
POOL_SIGNED = 32  # build-time flag: vectors of any sign, max/min pools
POOLS = {"f32": POOL_F32, "bf16": POOL_BF16, "fp8": POOL_FP8,
         "max_f32": POOL_MAX_F32, "max_bf16": POOL_MAX_BF16, "signed": POOL_SIGNED}
GT_MAX_LEVELS = 40

EXPORTS = ["gt_build_tree", "gt_insert", "gt_query_batch", "gt_query_batch_noalloc",
           "gt_exhaustive", "gt_call_bytes", "gt_batch_create_external",
           "gt_batch_submit_external", "gt_batch_info", "gt_batch_create",
           "gt_batch_submit", "gt_batch_poll", "gt_batch_finish", "gt_batch_destroy",
           "gt_get_stats", "gt_read_pools", "gt_set_option", "gt_destroy", "gt_last_error"]


class GTError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class GTStats(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64), ("capacity", ctypes.c_int64),
        ("d", ctypes.c_int32), ("d_pad", ctypes.c_int32),
        ("depth", ctypes.c_int32), ("head_level", ctypes.c_int32),
        ("pool_formats", ctypes.c_uint32),
        ("m_min", ctypes.c_double), ("epoch", ctypes.c_uint64),
        ("bytes_device", ctypes.c_int64),
        ("last_nq", ctypes.c_int32), ("last_tiles", ctypes.c_int32), ("last_format", ctypes.c_int32),
        ("entries", ctypes.c_int64 * GT_MAX_LEVELS), ("pairs", ctypes.c_int64 * GT_MAX_LEVELS),
        ("leaf_pairs", ctypes.c_int64), ("candidates", ctypes.c_int64),
        ("rechecked", ctypes.c_int64), ("results", ctypes.c_int64),
        ("ms_prep", ctypes.c_double), ("ms_frontier", ctypes.c_double),
        ("ms_leaf", ctypes.c_double), ("ms_recheck", ctypes.c_double),
        ("ms_compact", ctypes.c_double), ("ms_gemm", ctypes.c_double),
        ("ms_total", ctypes.c_double), ("frontier_launches", ctypes.c_int32),
        ("fp8_exp", ctypes.c_int32 * GT_MAX_LEVELS),
        ("unique_rows", ctypes.c_int64 * GT_MAX_LEVELS),
        ("dense_launches", ctypes.c_int32), ("ms_dense", ctypes.c_double),
        ("pool_width", ctypes.c_int32), ("shift_bound", ctypes.c_float),
    ]


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2311_02573_amd.build` "
                           "(there is no CPU fallback)")
    lib = ctypes.CDLL(path)
    vp, i64, i32, u32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32
    st = ctypes.c_int
    lib.gt_build_tree.restype = st
    lib.gt_build_tree.argtypes = [vp, i64, i32, ctypes.c_int, i64, u32, vp, ctypes.POINTER(vp)]
    lib.gt_insert.restype = st
    lib.gt_insert.argtypes = [vp, vp, i64, vp, ctypes.POINTER(i64)]
    lib.gt_query_batch.restype = st
    lib.gt_query_batch.argtypes = [vp, vp, i32, vp, ctypes.c_int, i64, vp, vp, vp,
                                   ctypes.POINTER(i64), vp]
    lib.gt_query_batch_noalloc.restype = st
    lib.gt_query_batch_noalloc.argtypes = [vp, vp, i32, vp, ctypes.c_int, i64, vp, vp, vp,
                                           ctypes.POINTER(i64), vp]
    lib.gt_exhaustive.restype = st
    lib.gt_exhaustive.argtypes = [vp, vp, i32, vp, i64, vp, vp, vp, ctypes.POINTER(i64), vp]
    lib.gt_call_bytes.restype = st
    lib.gt_call_bytes.argtypes = [vp, i32, ctypes.c_int, i64, i64, ctypes.POINTER(i64),
                                  ctypes.POINTER(i64)]
    lib.gt_batch_create_external.restype = st
    lib.gt_batch_create_external.argtypes = [vp, i32, ctypes.POINTER(vp)]
    lib.gt_batch_submit_external.restype = st
    lib.gt_batch_submit_external.argtypes = [vp, vp, i32, vp, ctypes.c_int, vp, i64, i64, vp]
    lib.gt_batch_info.restype = st
    lib.gt_batch_info.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64),
                                  ctypes.POINTER(i32)]
    lib.gt_batch_create.restype = st
    lib.gt_batch_create.argtypes = [vp, i32, ctypes.POINTER(vp)]
    lib.gt_batch_submit.restype = st
    lib.gt_batch_submit.argtypes = [vp, vp, i32, vp, ctypes.c_int, vp]
    lib.gt_batch_poll.restype = st
    lib.gt_batch_poll.argtypes = [vp, ctypes.POINTER(i32)]
    lib.gt_batch_finish.restype = st
    lib.gt_batch_finish.argtypes = [vp, i64, vp, vp, vp, ctypes.POINTER(i64)]
    lib.gt_batch_destroy.restype = None
    lib.gt_batch_destroy.argtypes = [vp]
    lib.gt_get_stats.restype = st
    lib.gt_get_stats.argtypes = [vp, ctypes.POINTER(GTStats)]
    lib.gt_read_pools.restype = st
    lib.gt_read_pools.argtypes = [vp, i32, i64, i64, ctypes.c_int, vp]
    lib.gt_set_option.restype = st
    lib.gt_set_option.argtypes = [vp, ctypes.c_char_p, i64]
    lib.gt_destroy.restype = None
    lib.gt_destroy.argtypes = [vp]
    lib.gt_last_error.restype = ctypes.c_char_p
    lib.gt_last_error.argtypes = []
    return lib


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        _lib = load_library()
    return _lib


def _check(status: int):
    if status != GT_OK:
        raise GTError(status, lib().gt_last_error().decode())


def _stream_ptr(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


_DTYPES = {torch.float32: GT_F32, torch.float16: GT_F16, torch.bfloat16: GT_BF16}


class Results:
    """CSR results on the device: query b has ids[offsets[b]:offsets[b+1]]."""

    def __init__(self, offsets, ids, sims, total):
        self.offsets, self.ids, self.sims, self.total = offsets, ids, sims, total

    def to_lists(self):
        off = self.offsets.cpu().numpy()
        ids = self.ids[: self.total].cpu().numpy()
        sims = self.sims[: self.total].cpu().numpy()
        return [(ids[off[b]:off[b + 1]], sims[off[b]:off[b + 1]]) for b in range(len(off) - 1)]


class GTIndex:
    """Owns one gt_index.  `feats` is a [n, d] CUDA tensor (float32/16, bfloat16)."""

    def __init__(self, feats: torch.Tensor, capacity: int = 0, pools=("f32", "bf16", "fp8"),
                 stream=None):
        if not feats.is_cuda:
            raise ValueError("features must be a device tensor")
        if feats.dtype not in _DTYPES:
            raise ValueError(f"unsupported dtype {feats.dtype}")
        feats = feats.contiguous()
        self.dtype = feats.dtype
        self.d = feats.shape[1]
        mask = 0
        for p in pools:
            mask |= POOLS[p]
        h = ctypes.c_void_p()
        _check(lib().gt_build_tree(ctypes.c_void_p(feats.data_ptr()), feats.shape[0], self.d,
                                   _DTYPES[feats.dtype], capacity, mask, _stream_ptr(stream),
                                   ctypes.byref(h)))
        self._h = h
        self._max_results = 1 << 16
        self.n = feats.shape[0]

    def close(self):
        if getattr(self, "_h", None):
            lib().gt_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def insert(self, feats: torch.Tensor, stream=None) -> int:
        if feats.dtype != self.dtype or feats.shape[1] != self.d:
            raise ValueError("inserted rows must match the index dtype and dimension")
        feats = feats.contiguous()
        first = ctypes.c_int64(-1)
        _check(lib().gt_insert(self._h, ctypes.c_void_p(feats.data_ptr()), feats.shape[0],
                               _stream_ptr(stream), ctypes.byref(first)))
        self.n = first.value + feats.shape[0]
        return first.value

    def _run(self, fn, q, rho, max_results, stream, *extra):
        q = q.contiguous()
        if q.dtype != torch.float32 or not q.is_cuda:
            raise ValueError("queries must be a float32 device tensor")
        nq = q.shape[0]
        rho_np = np.ascontiguousarray(np.broadcast_to(np.asarray(rho, dtype=np.float64), (nq,)))
        rho_arr = ctypes.c_void_p(rho_np.ctypes.data)
        dev = q.device
        offsets = torch.empty(nq + 1, dtype=torch.int64, device=dev)
        cap = max_results if max_results is not None else self._max_results
        total = ctypes.c_int64(0)
        while True:
            ids = torch.empty(max(cap, 1), dtype=torch.int64, device=dev)
            sims = torch.empty(max(cap, 1), dtype=torch.float32, device=dev)
            st = fn(self._h, ctypes.c_void_p(q.data_ptr()), nq, rho_arr, *extra, cap,
                    ctypes.c_void_p(offsets.data_ptr()), ctypes.c_void_p(ids.data_ptr()),
                    ctypes.c_void_p(sims.data_ptr()), ctypes.byref(total), _stream_ptr(stream))
            if st == GT_ERR_RESULT_OVERFLOW and max_results is None:
                cap = total.value
                self._max_results = max(self._max_results, cap)
                continue
            _check(st)
            return Results(offsets, ids, sims, total.value)

    def query(self, q: torch.Tensor, rho, pool: str = "bf16", max_results=None, stream=None):
        """Level-wise group-testing walk.  rho: float or per-query sequence."""
        return self._run(lambda h, qp, nq, r, fmt, *rest: lib().gt_query_batch(h, qp, nq, r, fmt, *rest),
                         q, rho, max_results, stream, POOLS[pool])

    def query_noalloc(self, q: torch.Tensor, rho, pool: str = "bf16", max_results=None,
                      stream=None):
        """The walk run in the library's fixed device scratch (no allocation by
        the library; the output tensors are allocated here, by the caller)."""
        return self._run(lambda h, qp, nq, r, fmt, *rest:
                         lib().gt_query_batch_noalloc(h, qp, nq, r, fmt, *rest),
                         q, rho, max_results, stream, POOLS[pool])

    def exhaustive(self, q: torch.Tensor, rho, max_results=None, stream=None):
        return self._run(lambda h, qp, nq, r, *rest: lib().gt_exhaustive(h, qp, nq, r, *rest),
                         q, rho, max_results, stream)

    def stats(self) -> dict:
        s = GTStats()
        _check(lib().gt_get_stats(self._h, ctypes.byref(s)))
        out = {}
        for name, _ in GTStats._fields_:
            v = getattr(s, name)
            out[name] = list(v) if name in ("entries", "pairs", "fp8_exp", "unique_rows") else v
        return out

    def read_pools(self, level: int, first: int = 0, count: int | None = None, pool: str = "f32"):
        """Stored pool rows of one level as a numpy array [count, width]: d_pad
        values, or pool_width for max pools above the leaves."""
        st = self.stats()
        if count is None:
            count = (1 << level) - first
        dt = {"f32": np.float32, "bf16": np.uint16, "fp8": np.uint8,
              "max_f32": np.float32, "max_bf16": np.uint16}[pool]
        w = st["pool_width"] if pool.startswith("max") and level < st["depth"] else st["d_pad"]
        out = np.empty((count, w), dtype=dt)
        _check(lib().gt_read_pools(self._h, level, first, count, POOLS[pool],
                                   ctypes.c_void_p(out.ctypes.data)))
        return out

    def set_option(self, key: str, value: int):
        _check(lib().gt_set_option(self._h, key.encode(), int(value)))


class Workspace:
    """A gt_batch: one asynchronous query call in flight at a time, on its own
    stream.  submit() returns at once; poll() says whether the result count is
    ready; finish() waits and returns Results."""

    def __init__(self, index: "GTIndex", max_queries: int, stream=None):
        self.index = index
        self.max_queries = max_queries
        self.stream = stream if stream is not None else torch.cuda.Stream()
        h = ctypes.c_void_p()
        _check(lib().gt_batch_create(index.handle, max_queries, ctypes.byref(h)))
        self._h = h
        self._q = None
        self._rho = None
        self._max_results = 1 << 16

    def close(self):
        if getattr(self, "_h", None):
            lib().gt_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, q: torch.Tensor, rho, pool: str = "bf16"):
        q = q.contiguous()
        if q.dtype != torch.float32 or not q.is_cuda:
            raise ValueError("queries must be a float32 device tensor")
        nq = q.shape[0]
        self._rho = np.ascontiguousarray(np.broadcast_to(np.asarray(rho, dtype=np.float64), (nq,)))
        self._q = q  # kept alive until finish
        self._pool = pool
        # the workspace's stream must see the queries written on the caller's stream
        self.stream.wait_stream(torch.cuda.current_stream())
        _check(lib().gt_batch_submit(self._h, ctypes.c_void_p(q.data_ptr()), nq,
                                     ctypes.c_void_p(self._rho.ctypes.data), POOLS[pool],
                                     ctypes.c_void_p(self.stream.cuda_stream)))
        self._nq = nq

    def poll(self) -> bool:
        done = ctypes.c_int32(0)
        _check(lib().gt_batch_poll(self._h, ctypes.byref(done)))
        return bool(done.value)

    def finish(self, max_results=None) -> Results:
        dev = self._q.device
        with torch.cuda.stream(self.stream):
            offsets = torch.empty(self._nq + 1, dtype=torch.int64, device=dev)
            cap = max_results if max_results is not None else self._max_results
            total = ctypes.c_int64(0)
            ids = torch.empty(max(cap, 1), dtype=torch.int64, device=dev)
            sims = torch.empty(max(cap, 1), dtype=torch.float32, device=dev)
            st = lib().gt_batch_finish(self._h, cap, ctypes.c_void_p(offsets.data_ptr()),
                                       ctypes.c_void_p(ids.data_ptr()), ctypes.c_void_p(sims.data_ptr()),
                                       ctypes.byref(total))
            if st == GT_ERR_RESULT_OVERFLOW and max_results is None:
                # the results are kept on the device: finish again with room for all
                need = total.value
                self._max_results = max(self._max_results, need + need // 4)
                ids = torch.empty(max(need, 1), dtype=torch.int64, device=dev)
                sims = torch.empty(max(need, 1), dtype=torch.float32, device=dev)
                st = lib().gt_batch_finish(self._h, need, ctypes.c_void_p(offsets.data_ptr()),
                                           ctypes.c_void_p(ids.data_ptr()),
                                           ctypes.c_void_p(sims.data_ptr()), ctypes.byref(total))
            _check(st)
        torch.cuda.current_stream().wait_stream(self.stream)
        res = Results(offsets, ids, sims, total.value)
        self._q = None
        return res


def call_bytes(index: "GTIndex", nq: int, pool: str = "bf16", frontier_entries: int = 0,
               pairs: int = 0):
    """(bytes, least bytes) of device memory for a call of nq queries given to
    ExternalWorkspace.submit with room for frontier_entries entries per level
    and `pairs` candidates (gt_call_bytes)."""
    b, m = ctypes.c_int64(0), ctypes.c_int64(0)
    _check(lib().gt_call_bytes(index.handle, nq, POOLS[pool], int(frontier_entries), int(pairs),
                               ctypes.byref(b), ctypes.byref(m)))
    return b.value, m.value


class ExternalWorkspace(Workspace):
    """A workspace whose device memory each call brings (gt_batch_create_external):
    submit(q, rho, pool, mem_ptr, mem_bytes, pairs) carves the call's buffers
    out of [mem_ptr, mem_ptr + mem_bytes), which the caller keeps reserved
    until finish() returns."""

    def __init__(self, index: "GTIndex", max_queries: int, stream=None):
        self.index = index
        self.max_queries = max_queries
        self.stream = stream if stream is not None else torch.cuda.Stream()
        h = ctypes.c_void_p()
        _check(lib().gt_batch_create_external(index.handle, max_queries, ctypes.byref(h)))
        self._h = h
        self._q = None
        self._rho = None
        self._max_results = 1 << 16

    def submit(self, q: torch.Tensor, rho, pool: str = "bf16", mem_ptr: int = 0, mem_bytes: int = 0,
               pairs: int = 0):
        q = q.contiguous()
        if q.dtype != torch.float32 or not q.is_cuda:
            raise ValueError("queries must be a float32 device tensor")
        nq = q.shape[0]
        self._rho = np.ascontiguousarray(np.broadcast_to(np.asarray(rho, dtype=np.float64), (nq,)))
        self._q = q  # read again by a continuation: kept until finish
        self._pool = pool
        self.stream.wait_stream(torch.cuda.current_stream())
        _check(lib().gt_batch_submit_external(self._h, ctypes.c_void_p(q.data_ptr()), nq,
                                              ctypes.c_void_p(self._rho.ctypes.data), POOLS[pool],
                                              ctypes.c_void_p(mem_ptr), int(mem_bytes), int(pairs),
                                              ctypes.c_void_p(self.stream.cuda_stream)))
        self._nq = nq

    def info(self) -> dict:
        """Of the last finished call: largest frontier level, results, tiles
        that ran one by one."""
        e, r, c = ctypes.c_int64(0), ctypes.c_int64(0), ctypes.c_int32(0)
        _check(lib().gt_batch_info(self._h, ctypes.byref(e), ctypes.byref(r), ctypes.byref(c)))
        return {"max_level_entries": e.value, "results": r.value, "continued_tiles": c.value}
