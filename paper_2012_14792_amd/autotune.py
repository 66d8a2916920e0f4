"""Schedule autotuner for the search kernels.

A schedule is (work-group size, target candidates per work item) for per-frame searches,
and (work-group size, resident work-groups per CU) for the batched form.  Schedules change
speed only: every candidate schedule's results must equal the reference schedule's in every
field, or tuning stops with an error.  The one exception is n_step2, the number of
candidates step 2 scored, which depends on how the space is cut into work items.

Results are cached as JSON keyed by GPU architecture, frame geometry and search parameters:

    python -m paper_2012_14792_amd.autotune --workload uhd_seq
    python -m paper_2012_14792_amd.autotune --workload uhd_batch
    python -m paper_2012_14792_amd.autotune --workload batch512

`load(key)` returns a cached schedule (or None); `tuned_params(...)` fills one in.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_CACHE = os.path.join(HERE, "tuned.json")

PER_FRAME_CANDIDATES = [(256, 512), (256, 256), (256, 1024), (128, 256), (128, 512),
                        (512, 1024), (64, 128), (64, 256)]
BATCH_CANDIDATES = [(256, 0), (128, 0), (64, 0), (256, 4), (128, 8), (64, 16), (64, 24), (512, 0)]


def cache_path() -> str:
    return os.environ.get("TRS_TUNE_CACHE", DEFAULT_CACHE)


def arch() -> str:
    import torch
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def frame_key(width, height, params) -> str:
    p = params
    return (f"{arch()}|{width}x{height}|N{p.n_threads}|C{p.max_tile_cols}R{p.max_tile_rows}"
            f"K{p.max_rs_per_tile}|k{p.area_k}|w{p.dtile},{p.drs}" + (f"|p{p.prune}" if p.prune else "")
            + (f"|n{p.min_rs}" if p.min_rs else ""))


def load_all() -> dict:
    try:
        with open(cache_path()) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def load(key: str):
    return load_all().get(key)


def store(key: str, value: dict) -> None:
    data = load_all()
    data[key] = value
    tmp = cache_path() + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(tmp, cache_path())


def tuned_params(width, height, params):
    """`params` with the cached per-frame schedule filled in (unchanged if none)."""
    from . import binding as B
    hit = load(frame_key(width, height, params))
    if not hit:
        return params
    p = B.SearchParams.from_buffer_copy(params)
    p.sched_block, p.sched_item = hit["sched_block"], hit["sched_item"]
    return p


def _decisions(outs) -> list:
    from . import binding as B
    raw = outs.cpu().numpy()
    res = []
    for i in range(raw.shape[0]):
        d = B.result_dict(B.Result.from_buffer_copy(bytes(raw[i].tobytes())))
        d.pop("n_step2")
        res.append(d)
    return res


def _time_graph(g, reps):
    import torch
    g.replay()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        g.replay()
    torch.cuda.synchronize()
    return (time.perf_counter() - t) / reps


def tune_per_frame(width, height, params, lumas, prevs, streams=8, reps=20,
                   candidates=PER_FRAME_CANDIDATES, log=print) -> dict:
    """Time every candidate schedule on the given frames (graph of per-frame launches
    over `streams` streams); returns the fastest and the table."""
    import torch

    from . import binding as B
    F = len(lumas)
    outs_ref = None
    table = []
    for blk, item in candidates:
        p = B.SearchParams.from_buffer_copy(params)
        p.sched_block, p.sched_item = blk, item
        parts = [B.Partitioner(width, height, p) for _ in range(streams)]
        sts = [torch.cuda.Stream() for _ in range(streams)]
        outs = torch.empty((F, B.RESULT_BYTES), dtype=torch.uint8, device="cuda")

        def step():
            base = torch.cuda.current_stream()
            for st in sts:
                st.wait_stream(base)
            for f in range(F):
                with torch.cuda.stream(sts[f % streams]):
                    parts[f % streams].enqueue(lumas[f], prevs[f], out=outs[f])
            for st in sts:
                base.wait_stream(st)

        step()
        torch.cuda.synchronize()
        if outs_ref is None:
            outs_ref = _decisions(outs)
        elif _decisions(outs) != outs_ref:
            raise RuntimeError(f"schedule {blk}/{item} changed a result")
        g = torch.cuda.CUDAGraph()
        cap = torch.cuda.Stream()
        cap.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(cap):
            with torch.cuda.graph(g, stream=cap):
                step()
        torch.cuda.current_stream().wait_stream(cap)
        dt = _time_graph(g, reps)
        table.append({"sched_block": blk, "sched_item": item, "frames_per_s": F / dt})
        log(f"  block {blk:4d} item {item:5d}: {F / dt:10.1f} frames/s")
    best = max(table, key=lambda r: r["frames_per_s"])
    return {"best": best, "table": table}


def tune_batch(items, reps=50, candidates=BATCH_CANDIDATES, log=print) -> dict:
    """Time the batched form under each (block, wgs_per_cu); results must not change."""
    import torch

    from . import binding as B
    ref = None
    table = []
    for blk, wgs in candidates:
        b = B.Batch(items, block=blk, wgs_per_cu=wgs)
        b.enqueue()
        torch.cuda.synchronize()
        if ref is None:
            ref = b.out.clone()
        elif not torch.equal(b.out, ref):
            raise RuntimeError(f"batch schedule {blk}/{wgs} changed a result")
        g = b.capture()
        dt = _time_graph(g, reps)
        table.append({"block": blk, "wgs_per_cu": wgs, "frames_per_s": len(items) / dt})
        log(f"  block {blk:4d} wgs/CU {wgs:3d}: {len(items) / dt:10.1f} frames/s")
        b.close()
    best = max(table, key=lambda r: r["frames_per_s"])
    return {"best": best, "table": table}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", choices=["uhd_seq", "uhd_batch", "batch512", "all"], default="all")
    ap.add_argument("--frames", type=int, default=32)
    args = ap.parse_args(argv)
    sys.path.insert(0, os.path.dirname(HERE))
    import numpy as np
    import torch

    from . import binding as B
    from . import synth

    torch.cuda.set_device(0)
    log = lambda m: print(m, file=sys.stderr, flush=True)   # noqa: E731
    report = {}
    if args.workload in ("uhd_seq", "all"):
        # per-frame schedules for every (size, N) of the workloads
        for name, (w, h) in synth.SIZES.items():
            gen = synth.SequenceGenerator(w, h, synth.batch_sequence_seed(name), 8.0)
            nfr = max(4, args.frames // (4 if name == "8k" else 1))
            lumas = [torch.from_numpy(gen.frame(f).view(np.int16)).cuda() for f in range(nfr)]
            W, H = synth.ctu_grid(w, h)
            rng = np.random.default_rng(0)
            prevs = [torch.from_numpy(rng.integers(200, 3000, W * H).astype(np.int32)).cuda()
                     for _ in range(nfr)]
            for N in (4, 8, 16):
                C, R, K = synth.BOUNDS[N]
                p = B.make_params(N, C, R, K, lam=synth.LAMBDA[(name, N)])
                log(f"{name} N={N}:")
                res = tune_per_frame(w, h, p, lumas, prevs, log=log)
                store(frame_key(w, h, p), {"sched_block": res["best"]["sched_block"],
                                           "sched_item": res["best"]["sched_item"]})
                report[f"{name}_N{N}"] = res
    if args.workload in ("uhd_batch", "all"):
        # the batched form over the 64-frame 4K sequence
        cfg = synth.CONFIGS["uhd_n8"]
        w, h = cfg["width"], cfg["height"]
        gen = synth.SequenceGenerator(w, h, cfg["seed"], cfg["drift"])
        W, H = synth.ctu_grid(w, h)
        rng = np.random.default_rng(0)
        p = tuned_params(w, h, B.make_params(cfg["n_threads"], cfg["max_tile_cols"], cfg["max_tile_rows"],
                                             cfg["max_rs_per_tile"], lam=cfg["lam"]))
        items = [dict(width=w, height=h, params=p, luma=torch.from_numpy(gen.frame(f).view(np.int16)).cuda(),
                      prev=torch.from_numpy(rng.integers(200, 3000, W * H).astype(np.int32)).cuda())
                 for f in range(64)]
        log("uhd_seq64 batched:")
        res = tune_batch(items, log=log)
        store(f"{arch()}|uhd_seq64", {"block": res["best"]["block"], "wgs_per_cu": res["best"]["wgs_per_cu"]})
        report["uhd_seq64"] = res
    if args.workload in ("batch512", "all"):
        spec = synth.batch_workload(512)
        gens = {n: synth.SequenceGenerator(*synth.SIZES[n], synth.batch_sequence_seed(n), 8.0)
                for n in ("fhd", "uhd", "8k")}
        items = []
        rng = np.random.default_rng(1)
        for n, k, N in spec:
            w, h = synth.SIZES[n]
            W, H = synth.ctu_grid(w, h)
            C, R, K = synth.BOUNDS[N]
            p = tuned_params(w, h, B.make_params(N, C, R, K, lam=synth.LAMBDA[(n, N)]))
            items.append(dict(width=w, height=h, params=p,
                              luma=torch.from_numpy(gens[n].frame(k).view(np.int16)).cuda(),
                              prev=torch.from_numpy(rng.integers(200, 3000, W * H).astype(np.int32)).cuda()))
        log("batch512:")
        res = tune_batch(items, log=log)
        store(f"{arch()}|batch512", {"block": res["best"]["block"], "wgs_per_cu": res["best"]["wgs_per_cu"]})
        report["batch512"] = res
    print(json.dumps({k: v["best"] for k, v in report.items()}))


if __name__ == "__main__":
    main()
