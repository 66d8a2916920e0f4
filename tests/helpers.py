"""Shared test helpers: seeded inputs, GPU calls through the C ABI, result comparison."""
from __future__ import annotations

import numpy as np

from paper_2012_14792_amd import binding as B
from paper_2012_14792_amd import synth

RESULT_KEYS = ["status", "rank", "t_min", "t_sel", "q_sel", "n_enumerated", "n_feasible",
               "uniform_rank", "t_unif", "q_unif", "tile_cols", "tile_rows", "n_rs",
               "dtile_used", "drs_used", "col_bd", "row_bd", "rs", "rs_time"]


def to_device(luma: np.ndarray):
    """uint16 [h, w] -> CUDA int16 view with a row stride rounded up to 8 samples."""
    import torch
    h, w = luma.shape
    ws = (w + 7) // 8 * 8
    buf = torch.zeros((h, ws), dtype=torch.int16)
    buf[:, :w] = torch.from_numpy(luma.view(np.int16))
    return buf.cuda()[:, :w]


def u32(t) -> np.ndarray:
    return t.cpu().numpy().view(np.uint32)


def u64(t) -> np.ndarray:
    return t.cpu().numpy().view(np.uint64)


def gpu_features(frame, luma_dev) -> dict:
    feats = B.alloc_features(frame)
    B.trs_features(frame, luma_dev, feats)
    out = {k: u32(v) for k, v in feats.items() if k != "s2"}
    out["s2"] = u64(feats["s2"])
    return out


def gpu_cost(frame, tex: np.ndarray, prev: np.ndarray | None, blend=(200, 3, 256)):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(tex, np.uint32).view(np.int32)).cuda()
    p = None if prev is None else torch.from_numpy(np.ascontiguousarray(prev, np.uint32).view(np.int32)).cuda()
    cost = torch.empty_like(t)
    flags = torch.zeros(1, dtype=torch.int32, device="cuda")
    B.trs_cost_map(frame, t, p, B.Blend(*blend), cost, flags)
    return u32(cost), int(flags.item())


def gpu_search(frame, params, cost: np.ndarray, s1: np.ndarray, s2: np.ndarray) -> dict:
    import torch
    dev = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a).view(dt)).cuda()
    c = dev(np.asarray(cost, np.uint32), np.int32)
    a = dev(np.asarray(s1, np.uint32), np.int32)
    b = dev(np.asarray(s2, np.uint64), np.int64)
    ws = torch.empty(B.trs_search_workspace(frame, params), dtype=torch.uint8, device="cuda")
    out = torch.empty(B.RESULT_BYTES, dtype=torch.uint8, device="cuda")
    B.trs_search(frame, params, c, a, b, ws, out)
    return B.read_result(out)


def gpu_literal(frame, params, cost: np.ndarray, s1: np.ndarray, s2: np.ndarray) -> dict:
    """The exact literal-space search on the GPU for one frame (host arrays in, result out)."""
    import torch
    dev = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a).view(dt)).cuda()
    c = dev(np.asarray(cost, np.uint32), np.int32)
    a = dev(np.asarray(s1, np.uint32), np.int32)
    b = dev(np.asarray(s2, np.uint64), np.int64)
    ws = torch.empty(B.trs_literal_workspace(frame, params), dtype=torch.uint8, device="cuda")
    out = torch.empty(B.RESULT_BYTES, dtype=torch.uint8, device="cuda")
    B.trs_literal_search(frame, params, c, a, b, ws, out)
    return B.read_result(out)


def oracle_params(orc, p: "B.SearchParams"):
    return orc.make_params(p.n_threads, p.max_tile_cols, p.max_tile_rows, p.max_rs_per_tile,
                           p.area_k, (p.lambda_num, p.lambda_den), p.dtile, p.drs, p.space_budget, p.prune,
                           p.min_rs, p.span_tiles)


def assert_same_result(gpu: dict, ref: dict, ctx: str = ""):
    for k in RESULT_KEYS:
        g, r = gpu[k], ref[k]
        if isinstance(r, list):
            r = [tuple(x) if isinstance(x, (list, tuple)) else x for x in r]
            g = [tuple(x) if isinstance(x, (list, tuple)) else x for x in g]
        assert g == r, f"{ctx}: field {k}: gpu {g} != oracle {r}"


def sequence_inputs(orc, cfg: dict, frames, eps_seed_offset: int = 1000):
    """(f, luma, prev) for the requested frames of a config's sequence.

    prev for frame f is the synthetic measured time map of frame f - 1 (frame 0 uses its
    own), computed from the oracle's texture of that frame.
    """
    w, h = cfg["width"], cfg["height"]
    gen = synth.SequenceGenerator(w, h, cfg["seed"], cfg["drift"])
    W, H = (w + 127) // 128, (h + 127) // 128
    nf = max(frames) + 1
    eps = synth.ar1_eps(W * H, max(nf, 1), cfg["seed"] + eps_seed_offset)
    for f in frames:
        luma = gen.frame(f)
        src = max(f - 1, 0)
        tex = orc.features(gen.frame(src) if src != f else luma)["tex"]
        prev = synth.ctu_times(tex, eps[src])
        yield f, luma, prev
