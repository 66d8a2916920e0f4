"""ctypes binding of libtrs.so.

Argument marshalling only: every step of the partitioning path runs in the library's HIP
kernels.  PyTorch supplies device memory and the current HIP stream.  The module raises
at import of the library if libtrs.so is missing (build it with
``python -m paper_2012_14792_amd.build``); there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
import warnings

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtrs.so")

TRS_OK, TRS_ENOFEASIBLE = 0, 1
TRS_EINVAL, TRS_ERANGE, TRS_ENOSPACE, TRS_EWORKSPACE, TRS_EDEVICE, TRS_ENOTIMPL = -1, -2, -3, -4, -5, -6
MAX_RS = 64


class Frame(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("ctu_size", ctypes.c_int32), ("bit_depth", ctypes.c_int32)]


class Feat(ctypes.Structure):
    _fields_ = [("s1", ctypes.c_void_p), ("grad", ctypes.c_void_p), ("tex", ctypes.c_void_p),
                ("mean", ctypes.c_void_p), ("var", ctypes.c_void_p), ("s2", ctypes.c_void_p)]


class Blend(ctypes.Structure):
    _fields_ = [("a", ctypes.c_uint32), ("b", ctypes.c_uint32), ("w_prev", ctypes.c_uint32)]


class SearchParams(ctypes.Structure):
    _fields_ = [("n_threads", ctypes.c_int32), ("max_tile_cols", ctypes.c_int32),
                ("max_tile_rows", ctypes.c_int32), ("max_rs_per_tile", ctypes.c_int32),
                ("area_k", ctypes.c_int32), ("lambda_num", ctypes.c_int32),
                ("lambda_den", ctypes.c_int32), ("dtile", ctypes.c_int32), ("drs", ctypes.c_int32),
                ("sched_block", ctypes.c_int32), ("sched_item", ctypes.c_int32),
                ("prune", ctypes.c_int32), ("min_rs", ctypes.c_int32),
                ("span_tiles", ctypes.c_int32), ("space_budget", ctypes.c_int64)]


class PlanStats(ctypes.Structure):
    _fields_ = [("candidates", ctypes.c_int64), ("feasible", ctypes.c_int64),
                ("tile_lookups", ctypes.c_int64), ("items", ctypes.c_int64),
                ("records", ctypes.c_int64), ("record_slices", ctypes.c_int64),
                ("table_bytes", ctypes.c_int64), ("dtile", ctypes.c_int32), ("drs", ctypes.c_int32),
                ("records_max", ctypes.c_int32), ("entries_max", ctypes.c_int32)]


class Result(ctypes.Structure):
    _fields_ = [("rank", ctypes.c_int64), ("t_min", ctypes.c_int64), ("t_sel", ctypes.c_int64),
                ("q_sel", ctypes.c_int64), ("n_enumerated", ctypes.c_int64),
                ("n_feasible", ctypes.c_int64), ("n_step2", ctypes.c_int64),
                ("uniform_rank", ctypes.c_int64),
                ("t_unif", ctypes.c_int64), ("q_unif", ctypes.c_int64),
                ("status", ctypes.c_int32), ("tile_cols", ctypes.c_int32),
                ("tile_rows", ctypes.c_int32), ("n_rs", ctypes.c_int32),
                ("dtile_used", ctypes.c_int32), ("drs_used", ctypes.c_int32),
                ("col_bd", ctypes.c_int32 * (MAX_RS + 1)), ("row_bd", ctypes.c_int32 * (MAX_RS + 1)),
                ("rs", (ctypes.c_int32 * 4) * MAX_RS), ("rs_time", ctypes.c_int64 * MAX_RS)]


class BatchFrame(ctypes.Structure):
    _fields_ = [("frame", Frame), ("params", SearchParams), ("luma", ctypes.c_void_p),
                ("stride_elems", ctypes.c_int64), ("prev", ctypes.c_void_p), ("blend", Blend)]


class MLP(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in ("w1", "b1", "w2", "b2", "w3", "b3")]


class MLPGrads(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in ("w1", "b1", "w2", "b2", "w3", "b3")]


class MLPNorm(ctypes.Structure):
    _fields_ = [("mean", ctypes.c_float * 10), ("inv_std", ctypes.c_float * 10),
                ("lo", ctypes.c_float * 10), ("hi", ctypes.c_float * 10)]


RESULT_BYTES = ctypes.sizeof(Result)
_lib = None


class TrsError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {strerror(status)} ({status})")


def lib():
    """Load libtrs.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2012_14792_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P, S = ctypes.c_void_p, ctypes.c_int
        L.trs_features.argtypes = [ctypes.POINTER(Frame), P, ctypes.c_int64, Feat, P]
        L.trs_features.restype = S
        L.trs_cost_map.argtypes = [ctypes.POINTER(Frame), P, P, Blend, P, P, P]
        L.trs_cost_map.restype = S
        L.trs_search_workspace.argtypes = [ctypes.POINTER(Frame), ctypes.POINTER(SearchParams),
                                           ctypes.POINTER(ctypes.c_size_t)]
        L.trs_search_workspace.restype = S
        L.trs_search.argtypes = [ctypes.POINTER(Frame), ctypes.POINTER(SearchParams), P, P, P, P,
                                 ctypes.c_size_t, P, P]
        L.trs_search.restype = S
        L.trs_literal_workspace.argtypes = L.trs_search_workspace.argtypes
        L.trs_literal_workspace.restype = S
        L.trs_literal_search.argtypes = L.trs_search.argtypes
        L.trs_literal_search.restype = S
        L.trs_profile_read_literal.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64),
                                               ctypes.POINTER(ctypes.c_int64)]
        L.trs_profile_read_literal.restype = S
        L.trs_partition.argtypes = [ctypes.POINTER(Frame), ctypes.POINTER(SearchParams), P,
                                    ctypes.c_int64, P, Blend, Feat, P, P, P, ctypes.c_size_t, P, P]
        L.trs_partition.restype = S
        L.trs_space_size.argtypes = [ctypes.POINTER(Frame), ctypes.POINTER(SearchParams),
                                     ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32),
                                     ctypes.POINTER(ctypes.c_int32)]
        L.trs_space_size.restype = S
        L.trs_search_stats.argtypes = [ctypes.POINTER(Frame), ctypes.POINTER(SearchParams),
                                       ctypes.POINTER(PlanStats)]
        L.trs_search_stats.restype = S
        L.trs_decode.argtypes = [ctypes.POINTER(Frame), ctypes.POINTER(SearchParams),
                                 ctypes.c_int64, ctypes.POINTER(Result)]
        L.trs_decode.restype = S
        L.trs_release_plans.argtypes = []
        L.trs_release_plans.restype = None
        L.trs_profile_enable.argtypes = [S]
        L.trs_profile_enable.restype = None
        L.trs_profile_read.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_int64)]
        L.trs_profile_read.restype = S
        L.trs_lambda_policy.argtypes = [ctypes.POINTER(Frame), ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                        ctypes.POINTER(ctypes.c_int32)]
        L.trs_lambda_policy.restype = S
        i32p = ctypes.POINTER(ctypes.c_int32)
        L.trs_ra_schedule.argtypes = [ctypes.c_int32, ctypes.c_int32, i32p, i32p, i32p, i32p]
        L.trs_ra_schedule.restype = S
        L.trs_profile_read_batch.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
        L.trs_profile_read_batch.restype = S
        L.trs_batch_create.argtypes = [ctypes.POINTER(BatchFrame), ctypes.c_int32, ctypes.c_int32,
                                       ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p)]
        L.trs_batch_create.restype = S
        L.trs_batch_workspace.argtypes = [P, ctypes.POINTER(ctypes.c_size_t)]
        L.trs_batch_workspace.restype = S
        L.trs_batch_run.argtypes = [P, P, ctypes.c_size_t, P, P]
        L.trs_batch_run.restype = S
        L.trs_batch_features.argtypes = [P, P, ctypes.c_size_t, P]
        L.trs_batch_features.restype = S
        L.trs_batch_search.argtypes = [P, P, ctypes.c_size_t, P, P]
        L.trs_batch_search.restype = S
        L.trs_batch_frame_arrays.argtypes = [P, P, ctypes.c_int32, ctypes.POINTER(Feat),
                                             ctypes.POINTER(ctypes.c_void_p)]
        L.trs_batch_frame_arrays.restype = S
        L.trs_batch_destroy.argtypes = [P]
        L.trs_batch_destroy.restype = None
        L.trs_mlp_inputs.argtypes = [ctypes.POINTER(Frame), P, P, P, P, P, P]
        L.trs_mlp_inputs.restype = S
        L.trs_mlp_forward.argtypes = [ctypes.POINTER(MLP), ctypes.POINTER(MLPNorm), P, ctypes.c_int64,
                                      P, P, P, P]
        L.trs_mlp_forward.restype = S
        L.trs_mlp_backward_workspace.argtypes = [ctypes.c_int64, ctypes.POINTER(ctypes.c_size_t)]
        L.trs_mlp_backward_workspace.restype = S
        L.trs_mlp_backward.argtypes = [ctypes.POINTER(MLP), ctypes.POINTER(MLPNorm), P, P, P, P,
                                       ctypes.c_int64, MLPGrads, P, ctypes.c_size_t, P]
        L.trs_mlp_backward.restype = S
        L.trs_mlp_cost.argtypes = [ctypes.POINTER(Frame), P, P, ctypes.POINTER(MLPNorm), P, P, Blend,
                                   P, P, P]
        L.trs_mlp_cost.restype = S
        L.trs_strerror.argtypes = [S]
        L.trs_strerror.restype = ctypes.c_char_p
        _lib = L
    return _lib


def strerror(status: int) -> str:
    return lib().trs_strerror(int(status)).decode()


def check(status: int, where: str) -> int:
    if status < 0:
        raise TrsError(status, where)
    if status > 0:
        warnings.warn(f"{where}: {strerror(status)}", RuntimeWarning, stacklevel=3)
    return status


def make_frame(width: int, height: int, ctu_size: int = 128, bit_depth: int = 10) -> Frame:
    return Frame(width, height, ctu_size, bit_depth)


def make_params(n_threads: int, max_tile_cols: int, max_tile_rows: int, max_rs_per_tile: int,
                area_k: int = 3, lam=(0, 1), dtile: int = -2, drs: int = -2,
                sched_block: int = 0, sched_item: int = 0, space_budget: int = 1 << 24,
                prune: int = 0, min_rs: int = 0, span_tiles: int = 0) -> SearchParams:
    num, den = lam
    return SearchParams(n_threads, max_tile_cols, max_tile_rows, max_rs_per_tile, area_k,
                        num, den, dtile, drs, sched_block, sched_item, prune, min_rs,
                        span_tiles, space_budget)


# ---- host-only calls ---------------------------------------------------------------------

def trs_space_size(frame: Frame, params: SearchParams) -> tuple[int, int, int]:
    n, dt, dr = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32()
    check(lib().trs_space_size(ctypes.byref(frame), ctypes.byref(params), ctypes.byref(n),
                               ctypes.byref(dt), ctypes.byref(dr)), "trs_space_size")
    return n.value, dt.value, dr.value


def trs_search_workspace(frame: Frame, params: SearchParams) -> int:
    b = ctypes.c_size_t()
    check(lib().trs_search_workspace(ctypes.byref(frame), ctypes.byref(params), ctypes.byref(b)),
          "trs_search_workspace")
    return b.value


def trs_search_stats(frame: Frame, params: SearchParams) -> dict:
    st = PlanStats()
    check(lib().trs_search_stats(ctypes.byref(frame), ctypes.byref(params), ctypes.byref(st)),
          "trs_search_stats")
    return {k: getattr(st, k) for k, _ in PlanStats._fields_}


def trs_decode(frame: Frame, params: SearchParams, rank: int) -> dict:
    r = Result()
    check(lib().trs_decode(ctypes.byref(frame), ctypes.byref(params), int(rank), ctypes.byref(r)),
          "trs_decode")
    return result_dict(r)


def trs_profile_enable(on: bool) -> None:
    lib().trs_profile_enable(1 if on else 0)


def trs_profile_read() -> tuple[float, float, int]:
    a, b, n = ctypes.c_double(), ctypes.c_double(), ctypes.c_int64()
    check(lib().trs_profile_read(ctypes.byref(a), ctypes.byref(b), ctypes.byref(n)), "trs_profile_read")
    return a.value, b.value, n.value


BATCH_STAGES = ("features", "cost_sat", "step1", "tmin", "step2", "final")


def trs_profile_read_batch() -> tuple[dict, int]:
    """Summed milliseconds per batch launch stage since the last read, and the run count."""
    ms = (ctypes.c_double * 6)()
    n = ctypes.c_int64()
    check(lib().trs_profile_read_batch(ms, ctypes.byref(n)), "trs_profile_read_batch")
    return dict(zip(BATCH_STAGES, list(ms))), n.value


def trs_lambda_policy(frame: Frame, n_threads: int) -> tuple[int, int]:
    """(num, den) of the lambda Table 1 pairs with the frame's resolution and thread count."""
    num, den = ctypes.c_int32(), ctypes.c_int32()
    check(lib().trs_lambda_policy(ctypes.byref(frame), n_threads, ctypes.byref(num), ctypes.byref(den)),
          "trs_lambda_policy")
    return num.value, den.value


def trs_ra_schedule(gop_size: int, n_frames: int) -> dict:
    """Random-access GOP bookkeeping: coding order, temporal layer per frame, and per frame
    the co-TL reference (previously coded frame of the same layer) and the closest coded
    frame in display order (-1 where none exists)."""
    import numpy as np
    out = {k: np.zeros(max(n_frames, 1), np.int32)
           for k in ("coding_order", "layer", "cotl_ref", "closest_ref")}
    ptr = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    check(lib().trs_ra_schedule(gop_size, n_frames, ptr(out["coding_order"]), ptr(out["layer"]),
                                ptr(out["cotl_ref"]), ptr(out["closest_ref"])), "trs_ra_schedule")
    return out


def trs_release_plans() -> None:
    lib().trs_release_plans()


def result_dict(r: Result) -> dict:
    n = r.n_rs
    return dict(
        status=r.status, rank=r.rank, t_min=r.t_min, t_sel=r.t_sel, q_sel=r.q_sel,
        n_enumerated=r.n_enumerated, n_feasible=r.n_feasible, n_step2=r.n_step2,
        uniform_rank=r.uniform_rank,
        t_unif=r.t_unif, q_unif=r.q_unif, tile_cols=r.tile_cols, tile_rows=r.tile_rows,
        n_rs=n, dtile_used=r.dtile_used, drs_used=r.drs_used,
        col_bd=[r.col_bd[i] for i in range(r.tile_cols + 1)] if r.tile_cols else [],
        row_bd=[r.row_bd[j] for j in range(r.tile_rows + 1)] if r.tile_rows else [],
        rs=[tuple(r.rs[q][e] for e in range(4)) for q in range(n)],
        rs_time=[r.rs_time[q] for q in range(n)],
    )


# ---- device calls on torch tensors ---------------------------------------------------------

def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


def ctu_dims(frame: Frame) -> tuple[int, int]:
    cs = frame.ctu_size
    return (frame.width + cs - 1) // cs, (frame.height + cs - 1) // cs


def alloc_features(frame: Frame, device="cuda"):
    import torch
    W, H = ctu_dims(frame)
    n = W * H
    return {k: torch.empty(n, dtype=torch.int32, device=device) for k in ("s1", "grad", "tex", "mean", "var")} | \
        {"s2": torch.empty(n, dtype=torch.int64, device=device)}


def trs_features(frame: Frame, luma, feats: dict, stream=None) -> dict:
    """luma: 2-D uint16 (or int16) CUDA tensor [height, >= width], row stride a multiple of 8."""
    if luma.dim() != 2 or luma.element_size() != 2 or not luma.is_cuda:
        raise TrsError(TRS_EINVAL, "trs_features")
    if luma.stride(1) != 1:
        raise TrsError(TRS_EINVAL, "trs_features")
    f = Feat(feats["s1"].data_ptr(), feats["grad"].data_ptr(), feats["tex"].data_ptr(),
             feats["mean"].data_ptr(), feats["var"].data_ptr(), feats["s2"].data_ptr())
    check(lib().trs_features(ctypes.byref(frame), _ptr(luma), luma.stride(0), f, _stream(stream)),
          "trs_features")
    return feats


def trs_cost_map(frame: Frame, tex, prev, blend: Blend, cost, flags=None, stream=None):
    check(lib().trs_cost_map(ctypes.byref(frame), _ptr(tex), None if prev is None else _ptr(prev),
                             blend, _ptr(cost), None if flags is None else _ptr(flags),
                             _stream(stream)), "trs_cost_map")
    return cost


def trs_search(frame: Frame, params: SearchParams, cost, s1, s2, workspace, out, stream=None):
    """Enqueue the search; `out` is a CUDA uint8 tensor of RESULT_BYTES bytes."""
    check(lib().trs_search(ctypes.byref(frame), ctypes.byref(params), _ptr(cost), _ptr(s1), _ptr(s2),
                           _ptr(workspace), workspace.numel() * workspace.element_size(),
                           _ptr(out), _stream(stream)), "trs_search")
    return out


def trs_literal_workspace(frame: Frame, params: SearchParams) -> int:
    n = ctypes.c_size_t()
    check(lib().trs_literal_workspace(ctypes.byref(frame), ctypes.byref(params), ctypes.byref(n)),
          "trs_literal_workspace")
    return n.value


def trs_literal_search(frame: Frame, params: SearchParams, cost, s1, s2, workspace, out, stream=None):
    """Enqueue the exact search over the literal space (params.dtile = params.drs = -1)."""
    check(lib().trs_literal_search(ctypes.byref(frame), ctypes.byref(params), _ptr(cost), _ptr(s1),
                                   _ptr(s2), _ptr(workspace), workspace.numel() * workspace.element_size(),
                                   _ptr(out), _stream(stream)), "trs_literal_search")
    return out


LITERAL_STAGES = ("prefix_rects", "tiles1", "units1", "tiles2", "units2", "pick", "final")


def trs_profile_read_literal() -> tuple[dict, int, tuple[int, int]]:
    """Summed per-stage ms of the literal searches made while profiling was on, their count, and
    the DP relaxations of the units that step 1 and step 2 ran (summed over the searches)."""
    ms = (ctypes.c_double * len(LITERAL_STAGES))()
    n = ctypes.c_int64()
    relax = (ctypes.c_int64 * 2)()
    check(lib().trs_profile_read_literal(ms, ctypes.byref(n), relax), "trs_profile_read_literal")
    return dict(zip(LITERAL_STAGES, list(ms))), n.value, (relax[0], relax[1])


def _feat(feats: dict) -> Feat:
    return Feat(feats["s1"].data_ptr(), feats["grad"].data_ptr(), feats["tex"].data_ptr(),
                feats["mean"].data_ptr(), feats["var"].data_ptr(), feats["s2"].data_ptr())


def trs_partition(frame: Frame, params: SearchParams, luma, prev, blend: Blend, feats: dict, cost,
                  workspace, out, flags=None, stream=None):
    """Enqueue the whole per-frame path (features -> cost map -> search) in one call."""
    if luma.dim() != 2 or luma.element_size() != 2 or not luma.is_cuda or luma.stride(1) != 1:
        raise TrsError(TRS_EINVAL, "trs_partition")
    check(lib().trs_partition(ctypes.byref(frame), ctypes.byref(params), _ptr(luma), luma.stride(0),
                              None if prev is None else _ptr(prev), blend, _feat(feats), _ptr(cost),
                              None if flags is None else _ptr(flags), _ptr(workspace),
                              workspace.numel() * workspace.element_size(), _ptr(out),
                              _stream(stream)), "trs_partition")
    return out


def read_result(out) -> dict:
    """Copy a device trs_result to the host (synchronises on it) and decode it."""
    raw = bytes(out.cpu().numpy().tobytes())
    r = Result.from_buffer_copy(raw)
    d = result_dict(r)
    if d["status"] == TRS_ENOFEASIBLE:
        warnings.warn("trs_search: no area-feasible partition; uniform partition returned",
                      RuntimeWarning, stacklevel=2)
    return d


class Partitioner:
    """Whole per-frame path on one device: features -> cost map -> two-step search.

    Holds device buffers for one frame geometry and parameter set.
    """

    def __init__(self, width, height, params: SearchParams, ctu_size=128, bit_depth=10,
                 blend=(200, 3, 256), device="cuda"):
        import torch
        self.frame = make_frame(width, height, ctu_size, bit_depth)
        self.params = params
        self.blend = Blend(*blend)
        self.W, self.H = ctu_dims(self.frame)
        self.feats = alloc_features(self.frame, device)
        self.cost = torch.empty(self.W * self.H, dtype=torch.int32, device=device)
        self.flags = torch.zeros(1, dtype=torch.int32, device=device)
        ws = trs_search_workspace(self.frame, params)
        self.ws = torch.empty(ws, dtype=torch.uint8, device=device)
        self.out = torch.empty(RESULT_BYTES, dtype=torch.uint8, device=device)

    def enqueue(self, luma, prev, out=None, stream=None):
        """Enqueue one frame (one trs_partition call); returns the device result buffer."""
        dst = self.out if out is None else out
        trs_partition(self.frame, self.params, luma, prev, self.blend, self.feats, self.cost,
                      self.ws, dst, self.flags, stream)
        return dst

    def enqueue_separate(self, luma, prev, out=None, stream=None):
        """The same path through the three separate calls."""
        dst = self.out if out is None else out
        trs_features(self.frame, luma, self.feats, stream)
        trs_cost_map(self.frame, self.feats["tex"], prev, self.blend, self.cost, self.flags, stream)
        trs_search(self.frame, self.params, self.cost, self.feats["s1"], self.feats["s2"], self.ws,
                   dst, stream)
        return dst

    def __call__(self, luma, prev, stream=None) -> dict:
        self.enqueue(luma, prev, stream=stream)
        return read_result(self.out)


class Batch:
    """The batched form: every frame of a list through the whole path in six launches.

    frames: list of dicts with keys width, height, params (SearchParams), luma (2-D CUDA
    uint16/int16 tensor), prev (CUDA int32 tensor or None) and optional blend (a, b, w_prev),
    ctu_size.  The tensors must stay alive and in place while the batch is used.
    """

    def __init__(self, frames, block: int = 0, wgs_per_cu: int = 0, device="cuda"):
        import torch
        self._keep = []
        arr = (BatchFrame * len(frames))()
        for i, fr in enumerate(frames):
            luma = fr["luma"]
            if luma.dim() != 2 or luma.element_size() != 2 or not luma.is_cuda or luma.stride(1) != 1:
                raise TrsError(TRS_EINVAL, "Batch")
            prev = fr.get("prev")
            arr[i].frame = make_frame(fr["width"], fr["height"], fr.get("ctu_size", 128), 10)
            arr[i].params = fr["params"]
            arr[i].luma = luma.data_ptr()
            arr[i].stride_elems = luma.stride(0)
            arr[i].prev = None if prev is None else prev.data_ptr()
            arr[i].blend = Blend(*fr.get("blend", (200, 3, 256)))
            self._keep += [luma, prev]
        h = ctypes.c_void_p()
        check(lib().trs_batch_create(arr, len(frames), block, wgs_per_cu, ctypes.byref(h)), "trs_batch_create")
        self._h = h
        self.n = len(frames)
        nb = ctypes.c_size_t()
        check(lib().trs_batch_workspace(h, ctypes.byref(nb)), "trs_batch_workspace")
        self.ws = torch.empty(nb.value, dtype=torch.uint8, device=device)
        self.out = torch.empty((self.n, RESULT_BYTES), dtype=torch.uint8, device=device)

    def enqueue(self, stream=None):
        check(lib().trs_batch_run(self._h, _ptr(self.ws), self.ws.numel(), _ptr(self.out), _stream(stream)),
              "trs_batch_run")
        return self.out

    def enqueue_features(self, stream=None):
        """The feature launch of every frame (first part of enqueue)."""
        check(lib().trs_batch_features(self._h, _ptr(self.ws), self.ws.numel(), _stream(stream)),
              "trs_batch_features")

    def enqueue_search(self, stream=None):
        """The five launches after the features (second part of enqueue)."""
        check(lib().trs_batch_search(self._h, _ptr(self.ws), self.ws.numel(), _ptr(self.out), _stream(stream)),
              "trs_batch_search")
        return self.out

    def results(self) -> list:
        raw = self.out.cpu().numpy()
        return [result_dict(Result.from_buffer_copy(bytes(raw[i].tobytes()))) for i in range(self.n)]

    def frame_arrays(self, i: int) -> tuple[Feat, int]:
        feat, cost = Feat(), ctypes.c_void_p()
        check(lib().trs_batch_frame_arrays(self._h, _ptr(self.ws), i, ctypes.byref(feat), ctypes.byref(cost)),
              "trs_batch_frame_arrays")
        return feat, cost.value

    def capture(self):
        """A CUDA/HIP graph whose replay runs the whole batch."""
        import torch
        self.enqueue()
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            with torch.cuda.graph(g, stream=s):
                self.enqueue()
        torch.cuda.current_stream().wait_stream(s)
        return g

    def close(self):
        if getattr(self, "_h", None):
            lib().trs_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- learned CTU time predictor ------------------------------------------------------------

def _mlp(ws) -> MLP:
    return MLP(*(w.data_ptr() for w in ws))


def trs_mlp_inputs(frame: Frame, feats: dict, prev, x, stream=None):
    check(lib().trs_mlp_inputs(ctypes.byref(frame), _ptr(feats["tex"]), _ptr(feats["var"]),
                               _ptr(feats["mean"]), _ptr(prev), _ptr(x), _stream(stream)), "trs_mlp_inputs")
    return x


def trs_mlp_forward(weights, norm: MLPNorm, x, y, z1=None, z2=None, stream=None):
    check(lib().trs_mlp_forward(ctypes.byref(_mlp(weights)), ctypes.byref(norm), _ptr(x), x.shape[0], _ptr(y),
                                None if z1 is None else _ptr(z1), None if z2 is None else _ptr(z2),
                                _stream(stream)), "trs_mlp_forward")
    return y


def trs_mlp_backward(weights, norm: MLPNorm, x, z1, z2, dy, grads, workspace=None, stream=None):
    import torch
    n = x.shape[0]
    if workspace is None:
        nb = ctypes.c_size_t()
        check(lib().trs_mlp_backward_workspace(n, ctypes.byref(nb)), "trs_mlp_backward_workspace")
        workspace = torch.empty(nb.value, dtype=torch.uint8, device=x.device)
    g = MLPGrads(*(t.data_ptr() for t in grads))
    check(lib().trs_mlp_backward(ctypes.byref(_mlp(weights)), ctypes.byref(norm), _ptr(x), _ptr(z1), _ptr(z2),
                                 _ptr(dy), n, g, _ptr(workspace), workspace.numel(), _stream(stream)),
          "trs_mlp_backward")
    return grads


def trs_mlp_cost(frame: Frame, y, x, norm: MLPNorm, tex, prev, blend: Blend, cost, n_fallback=None, stream=None):
    check(lib().trs_mlp_cost(ctypes.byref(frame), _ptr(y), _ptr(x), ctypes.byref(norm), _ptr(tex),
                             None if prev is None else _ptr(prev), blend, _ptr(cost),
                             None if n_fallback is None else _ptr(n_fallback), _stream(stream)), "trs_mlp_cost")
    return cost
