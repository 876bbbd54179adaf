"""Canonical float64 brute-force range scan (C, via ctypes) -- test infrastructure only.

Definition (problem statement, Sec. 1; similarity = cosine of non-negative
vectors, Sec. 2): for each query q and threshold rho, every row i with
cos(q, f_i) >= rho, where cos is computed in float64 with sequential sums over
the dimension (see range_oracle.c for the exact operation order).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "range_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_libs = {}

DTYPE_CODES = {"f32": 0, "f16": 1, "bf16": 2}


def build(force: bool = True) -> str:
    """Compile range_oracle.c with gcc (no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-shared",
                               "-fPIC", "-pthread", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load(path: str | None = None):
    """Load the oracle library (or a differently built copy of it at `path`)."""
    path = path or _LIB
    if path not in _libs:
        if path == _LIB and not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(path)
        vp, i64, i32, dp = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p
        lib.oracle_range_search.restype = vp
        lib.oracle_range_search.argtypes = [vp, ctypes.c_int, i64, i32, vp, i32, dp, ctypes.c_int]
        lib.oracle_result_count.restype = i64
        lib.oracle_result_count.argtypes = [vp, i32]
        lib.oracle_result_copy.argtypes = [vp, i32, vp, vp]
        lib.oracle_result_free.argtypes = [vp]
        lib.oracle_pair_cos.argtypes = [vp, ctypes.c_int, i32, vp, vp, vp, i64, vp]
        _libs[path] = lib
    return _libs[path]


def _feats_view(feats):
    """(pointer-holding contiguous array, dtype code).  16-bit torch tensors are
    passed as raw uint16 bits."""
    if isinstance(feats, np.ndarray):
        a = np.ascontiguousarray(feats, dtype=np.float32)
        return a, 0
    import torch

    t = feats.contiguous().cpu()
    if t.dtype == torch.float32:
        return t.numpy(), 0
    code = 1 if t.dtype == torch.float16 else 2
    return t.view(torch.int16).numpy().view(np.uint16), code


def default_threads() -> int:
    return max(1, len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count() or 1)


def range_search(feats, queries, rho, nthreads: int | None = None, lib_path: str | None = None):
    """Returns a list (one per query) of (ids int64 ascending, cos float64)."""
    lib = _load(lib_path)
    f, code = _feats_view(feats)
    n, d = f.shape
    q = np.ascontiguousarray(queries, dtype=np.float32).reshape(-1, d)
    nq = q.shape[0]
    r = np.ascontiguousarray(np.broadcast_to(np.asarray(rho, dtype=np.float64), (nq,)))
    h = lib.oracle_range_search(f.ctypes.data, code, n, d, q.ctypes.data, nq, r.ctypes.data,
                                nthreads or default_threads())
    out = []
    try:
        for j in range(nq):
            c = lib.oracle_result_count(h, j)
            ids = np.empty(c, np.int64)
            sims = np.empty(c, np.float64)
            if c:
                lib.oracle_result_copy(h, j, ids.ctypes.data, sims.ctypes.data)
            out.append((ids, sims))
    finally:
        lib.oracle_result_free(h)
    return out


def pair_cos(feats, queries, qidx, rows, lib_path: str | None = None):
    """Canonical float64 cosine for individual (query index, row) pairs."""
    lib = _load(lib_path)
    f, code = _feats_view(feats)
    d = f.shape[1]
    q = np.ascontiguousarray(queries, dtype=np.float32).reshape(-1, d)
    qi = np.ascontiguousarray(qidx, dtype=np.int64)
    ri = np.ascontiguousarray(rows, dtype=np.int64)
    out = np.empty(len(qi), np.float64)
    lib.oracle_pair_cos(f.ctypes.data, code, d, q.ctypes.data, qi.ctypes.data, ri.ctypes.data,
                        len(qi), out.ctypes.data)
    return out

