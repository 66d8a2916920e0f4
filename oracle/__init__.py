"""CPU oracle for TRS partitioning -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import this
package.  The GPU library never loads it and shares no code with it.

``build()`` compiles ``trs_oracle.c`` (plain C, gcc -O2) into ``_oracle.so`` next to it.
The Python wrappers below only marshal arguments; all arithmetic is in the C file (and,
for tiny cases, in the independent pure-Python brute force ``oracle.brute``).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "trs_oracle.c")
_LIB = os.path.join(_HERE, "_oracle.so")
_lib = None

MAXN = 64
MAXB = 65


class OrcParams(ctypes.Structure):
    _fields_ = [("n_threads", ctypes.c_int32), ("max_tile_cols", ctypes.c_int32),
                ("max_tile_rows", ctypes.c_int32), ("max_rs_per_tile", ctypes.c_int32),
                ("area_k", ctypes.c_int32), ("lambda_num", ctypes.c_int32),
                ("lambda_den", ctypes.c_int32), ("dtile", ctypes.c_int32),
                ("drs", ctypes.c_int32), ("prune", ctypes.c_int32), ("min_rs", ctypes.c_int32),
                ("span_tiles", ctypes.c_int32), ("space_budget", ctypes.c_int64)]


class OrcResult(ctypes.Structure):
    _fields_ = [("rank", ctypes.c_int64), ("t_min", ctypes.c_int64), ("t_sel", ctypes.c_int64),
                ("q_sel", ctypes.c_int64), ("n_enumerated", ctypes.c_int64),
                ("n_feasible", ctypes.c_int64), ("uniform_rank", ctypes.c_int64),
                ("t_unif", ctypes.c_int64), ("q_unif", ctypes.c_int64),
                ("status", ctypes.c_int32), ("tile_cols", ctypes.c_int32),
                ("tile_rows", ctypes.c_int32), ("n_rs", ctypes.c_int32),
                ("dtile_used", ctypes.c_int32), ("drs_used", ctypes.c_int32),
                ("col_bd", ctypes.c_int32 * MAXB), ("row_bd", ctypes.c_int32 * MAXB),
                ("rs", (ctypes.c_int32 * 4) * MAXN), ("rs_time", ctypes.c_int64 * MAXN)]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc.  Always recompiles unless force=False and it exists."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-Wall", "-shared", "-fPIC",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        L.orc_features.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, P, ctypes.c_int64,
                                   P, P, P, P, P, P]
        L.orc_cost_map.argtypes = [ctypes.c_int, P, P, ctypes.c_uint32, ctypes.c_uint32,
                                   ctypes.c_uint32, P]
        L.orc_space_size.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(OrcParams),
                                     ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32),
                                     ctypes.POINTER(ctypes.c_int32)]
        L.orc_search.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(OrcParams),
                                 P, P, P, ctypes.POINTER(OrcResult)]
        L.orc_literal_search.argtypes = L.orc_search.argtypes
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def ctu_dims(w: int, h: int, cs: int = 128) -> tuple[int, int]:
    return (w + cs - 1) // cs, (h + cs - 1) // cs


def features(luma: np.ndarray, cs: int = 128) -> dict:
    """Per-CTU s1, s2, grad, tex, mean, var (raster order) from a uint16 [h][w] plane."""
    luma = np.ascontiguousarray(luma, dtype=np.uint16)
    h, w = luma.shape
    W, H = ctu_dims(w, h, cs)
    out = {k: np.zeros(W * H, dtype=np.uint32) for k in ("s1", "grad", "tex", "mean", "var")}
    out["s2"] = np.zeros(W * H, dtype=np.uint64)
    rc = lib().orc_features(w, h, cs, _ptr(luma), w, _ptr(out["s1"]), _ptr(out["s2"]),
                            _ptr(out["grad"]), _ptr(out["tex"]), _ptr(out["mean"]), _ptr(out["var"]))
    if rc != 0:
        raise ValueError(f"orc_features failed: {rc}")
    return out


def cost_map(tex: np.ndarray, prev: np.ndarray | None, a: int = 200, b: int = 3,
             w_prev: int = 256) -> tuple[np.ndarray, int]:
    tex = np.ascontiguousarray(tex, dtype=np.uint32)
    cost = np.zeros_like(tex)
    pv = None if prev is None else np.ascontiguousarray(prev, dtype=np.uint32)
    rc = lib().orc_cost_map(tex.size, _ptr(tex), None if pv is None else _ptr(pv), a, b, w_prev,
                            _ptr(cost))
    return cost, rc


def make_params(n_threads, max_tile_cols, max_tile_rows, max_rs_per_tile, area_k=3,
                lam=(0, 1), dtile=-2, drs=-2, space_budget=1 << 24, prune=0,
                min_rs=0, span_tiles=0) -> OrcParams:
    num, den = lam
    return OrcParams(n_threads, max_tile_cols, max_tile_rows, max_rs_per_tile, area_k,
                     num, den, dtile, drs, prune, min_rs, span_tiles, space_budget)


def space_size(W: int, H: int, params: OrcParams) -> tuple[int, int, int]:
    n = ctypes.c_int64()
    dt = ctypes.c_int32()
    dr = ctypes.c_int32()
    rc = lib().orc_space_size(W, H, ctypes.byref(params), ctypes.byref(n), ctypes.byref(dt),
                              ctypes.byref(dr))
    if rc != 0:
        raise ValueError(f"orc_space_size failed: {rc}")
    return n.value, dt.value, dr.value


def search(w: int, h: int, params: OrcParams, cost: np.ndarray, s1: np.ndarray,
           s2: np.ndarray, cs: int = 128) -> dict:
    cost = np.ascontiguousarray(cost, dtype=np.uint32)
    s1 = np.ascontiguousarray(s1, dtype=np.uint32)
    s2 = np.ascontiguousarray(s2, dtype=np.uint64)
    res = OrcResult()
    rc = lib().orc_search(w, h, cs, ctypes.byref(params), _ptr(cost), _ptr(s1), _ptr(s2),
                          ctypes.byref(res))
    if rc < 0:
        raise ValueError(f"orc_search failed: {rc}")
    return result_dict(res)


def literal_search(w: int, h: int, params: OrcParams, cost: np.ndarray, s1: np.ndarray,
                   s2: np.ndarray, cs: int = 128) -> dict:
    """Exact two-step search over the literal space (every CTU boundary allowed) by the
    window / tile / strip / column decomposition; rank and n_feasible are -1."""
    cost = np.ascontiguousarray(cost, dtype=np.uint32)
    s1 = np.ascontiguousarray(s1, dtype=np.uint32)
    s2 = np.ascontiguousarray(s2, dtype=np.uint64)
    res = OrcResult()
    rc = lib().orc_literal_search(w, h, cs, ctypes.byref(params), _ptr(cost), _ptr(s1), _ptr(s2),
                                  ctypes.byref(res))
    if rc < 0:
        raise ValueError(f"orc_literal_search failed: {rc}")
    return result_dict(res)


def result_dict(res: OrcResult) -> dict:
    n = res.n_rs
    return dict(
        status=res.status, rank=res.rank, t_min=res.t_min, t_sel=res.t_sel, q_sel=res.q_sel,
        n_enumerated=res.n_enumerated, n_feasible=res.n_feasible,
        uniform_rank=res.uniform_rank, t_unif=res.t_unif, q_unif=res.q_unif,
        tile_cols=res.tile_cols, tile_rows=res.tile_rows, n_rs=n,
        dtile_used=res.dtile_used, drs_used=res.drs_used,
        col_bd=[res.col_bd[i] for i in range(res.tile_cols + 1)] if res.tile_cols else [],
        row_bd=[res.row_bd[j] for j in range(res.tile_rows + 1)] if res.tile_rows else [],
        rs=[tuple(res.rs[q][e] for e in range(4)) for q in range(n)],
        rs_time=[res.rs_time[q] for q in range(n)],
    )


def partition(luma: np.ndarray, prev: np.ndarray | None, params: OrcParams, cs: int = 128,
              a: int = 200, b: int = 3, w_prev: int = 256) -> dict:
    """Whole path for one frame: features -> cost map -> two-step search."""
    h, w = luma.shape
    f = features(luma, cs)
    cost, _ = cost_map(f["tex"], prev, a, b, w_prev)
    return search(w, h, params, cost, f["s1"], f["s2"], cs)
