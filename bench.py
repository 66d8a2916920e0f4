#!/usr/bin/env python3
"""Throughput of the TRS partitioning path on one MI355X.

Workload: the 4K sequence -- 64 frames of 3840x2160 10-bit luma (30 x 17 CTUs of 128),
N = 8 slices/threads, tile grids up to 6 x 4, up to 4 slices per tile, lambda = 1/10, the
ladder rule's (3, 1) window: 5,914,718 candidates per frame.  One step = every frame of
the sequence through features -> predicted time map -> two-step exhaustive search, inputs
(luma and previous-frame CTU times) resident in HBM.  The step runs in one of two forms,
both timed, both checked against each other:

  batched  one trs_batch_run over all frames (six launches, persistent search kernels)
  streams  one trs_partition launch sequence per frame, frames spread over 8 streams

Prints one JSON line: frames/s (4K frames partitioned per second) of the chosen form
(default batched) with candidates scored per second, the dominant kernel's roofline
fraction (HIP events around it, on its stream), and the CPU oracle timed on a bounded
sample of the same workload on the host's cores.

Other workloads: --workload batch512 (512 mixed 1080p/4K/8K frames with mixed N) and
--workload mlp (training steps of the learned CTU-time predictor).
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_ALU_TOPS = round(256 * 64 * 2.4e9 / 1e12, 2)   # 32-bit VALU lane-ops: CUs x lanes/clk x clock
PEAK_HBM_GBS = 8000.0
# HBM bytes per launch from rocprofv3 FETCH_SIZE (x 2.00) + WRITE_SIZE (x 1.00) on this workload,
# the factors read from a 1 GiB device copy in the same runs; a kernel changed since the
# counters were taken has no entry.
TRAFFIC = {
    "k_features_batch<128>": 1223334195,     # 64 frames: 596,811.9 KiB fetched, 1,038.5 KiB written
    "k_features<128>": 16889037,             # 1 frame: 8,239.5 KiB fetched, 14.2 KiB written
}
METRIC = "4K frames partitioned/s + TRS candidates scored/s (1 GPU, bit-exact vs oracle)"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--frames", type=int, default=64)
    ap.add_argument("--cpu-frames", type=int, default=0, help="oracle sample size (0: 4 x cores)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-threads", type=int, default=16, help="oracle worker threads (cap)")
    ap.add_argument("--sched-block", type=int, default=0)
    ap.add_argument("--sched-item", type=int, default=0)
    ap.add_argument("--streams", type=int, default=8, help="frames in flight (one stream each)")
    ap.add_argument("--workload", default="uhd_seq", choices=["uhd_seq", "batch512", "mlp", "literal"],
                    help="uhd_seq: the 64-frame 4K sequence; batch512: 512 mixed frames in one batch; "
                         "mlp: training steps of the learned CTU-time predictor; literal: exact search "
                         "of 4K frames over the literal space (every CTU boundary allowed)")
    ap.add_argument("--mlp-batch", type=int, default=65536)
    ap.add_argument("--span-tiles", type=int, default=0,
                    help="literal workload: RS may also be blocks of tiles stacked in one tile column")
    ap.add_argument("--prune", type=int, default=0,
                    help="optional pruning rules (bit 0: slice heights, bit 1: mean areas); 0 = the paper's method")
    ap.add_argument("--pipeline", type=int, default=0,
                    help="batched form: sub-batches pipelined over streams (0: tuned, else 1)")
    ap.add_argument("--form", default="batched", choices=["batched", "streams"],
                    help="4K sequence: one batched launch sequence per step, or per-frame launches "
                         "over --streams streams")
    ap.add_argument("--batch-frames", type=int, default=512)
    ap.add_argument("--wgs-per-cu", type=int, default=0)
    ap.add_argument("--copy-probe", action="store_true",
                    help="copy 1 GiB once before timing (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.workload == "batch512":
        return run_batch(args)
    if args.workload == "mlp":
        return run_mlp(args)
    if args.workload == "literal":
        return run_literal(args)
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build partitions frames on a single MI355X "
              "and has no multi-GPU path (frames would shard across GPUs with no communication).",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2012_14792_amd import autotune
    from paper_2012_14792_amd import binding as B
    from paper_2012_14792_amd import synth

    cfg = synth.CONFIGS["uhd_n8"]
    w, h, F = cfg["width"], cfg["height"], args.frames
    torch.cuda.set_device(0)
    params = B.make_params(cfg["n_threads"], cfg["max_tile_cols"], cfg["max_tile_rows"],
                           cfg["max_rs_per_tile"], lam=cfg["lam"], sched_block=args.sched_block,
                           sched_item=args.sched_item, prune=args.prune)
    if not (args.sched_block or args.sched_item):
        params = autotune.tuned_params(w, h, params)       # cached schedule, if any
    frame = B.make_frame(w, h)
    stats = B.trs_search_stats(frame, params)
    W, H = B.ctu_dims(frame)

    # ---- inputs: seeded synthetic sequence, rendered on the host, resident in HBM ----------
    t0 = time.perf_counter()
    gen = synth.SequenceGenerator(w, h, cfg["seed"], cfg["drift"])
    with cf.ThreadPoolExecutor(8) as ex:
        frames = list(ex.map(gen.frame, range(F)))
    luma = torch.empty((F, h, w), dtype=torch.int16, device="cuda")
    for f in range(F):
        luma[f].copy_(torch.from_numpy(frames[f].view(np.int16)))
    # measured CTU times: the synthetic time model on each frame's texture (GPU features)
    texs = []
    for f in range(F):
        feats = B.alloc_features(frame)
        B.trs_features(frame, luma[f], feats)
        texs.append(feats["tex"].cpu().numpy().view(np.uint32))
    eps = synth.ar1_eps(W * H, F, cfg["seed"] + 1000)
    truth = [synth.ctu_times(texs[f], eps[f]) for f in range(F)]
    prev_np = [truth[max(f - 1, 0)] for f in range(F)]
    prev = torch.stack([torch.from_numpy(p.view(np.int32)) for p in prev_np]).cuda()
    torch.cuda.synchronize()
    log(f"inputs ready: {F} frames {w}x{h} in {time.perf_counter() - t0:.1f} s; "
        f"{stats['candidates']} candidates/frame, {stats['items']} work items")

    if args.copy_probe:
        src = torch.ones(1 << 30, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("copy probe: 1 GiB device-to-device copy done")

    # ---- form 1: per-frame launch sequences over S streams (default priority) --------------
    # frames are independent: each stream runs whole frames with its own buffers, so the
    # kernels of up to S frames overlap
    S = max(1, args.streams)
    parts = [B.Partitioner(w, h, params) for _ in range(S)]
    part = parts[0]
    outs = torch.empty((F, B.RESULT_BYTES), dtype=torch.uint8, device="cuda")
    streams = [torch.cuda.Stream() for _ in range(S)]

    def step_streams():
        base = torch.cuda.current_stream()
        for st in streams:
            st.wait_stream(base)
        for f in range(F):
            k = f % S
            with torch.cuda.stream(streams[k]):
                parts[k].enqueue(luma[f], prev[f], out=outs[f])
        for st in streams:
            base.wait_stream(st)

    for _ in range(max(args.warmup, 1)):
        step_streams()
    torch.cuda.synchronize()
    g_streams = capture(step_streams)

    # ---- form 2: the batched form, every frame in one six-launch sequence --------------------
    tuned = (autotune.load(f"{autotune.arch()}|uhd_seq{F}") or {}) if not args.sched_block else {}
    block = args.sched_block or tuned.get("block", 0)
    wgs = args.wgs_per_cu or tuned.get("wgs_per_cu", 0)
    # K sub-batches of consecutive frames, one stream each.  Their feature launches run one
    # after another (each waits for the previous one's), and each sub-batch's search follows
    # its own features, so one sub-batch's search can overlap the next one's features.
    K = max(1, min(F, args.pipeline or tuned.get("pipeline", 1)))
    cuts = [F * k // K for k in range(K + 1)]
    batches = [B.Batch([dict(width=w, height=h, params=params, luma=luma[f], prev=prev[f])
                        for f in range(cuts[k], cuts[k + 1])], block=block, wgs_per_cu=wgs) for k in range(K)]
    bstreams = [torch.cuda.Stream() for _ in range(K)] if K > 1 else None

    def step_batch():
        if K == 1:
            batches[0].enqueue()
            return
        base = torch.cuda.current_stream()
        for st in bstreams:
            st.wait_stream(base)
        done_features = None
        for bt, st in zip(batches, bstreams):
            if done_features is not None:
                st.wait_event(done_features)
            bt.enqueue_features(stream=st)
            done_features = torch.cuda.Event()
            done_features.record(st)
            bt.enqueue_search(stream=st)
        for st in bstreams:
            base.wait_stream(st)

    def batch_out():
        return torch.cat([bt.out for bt in batches])

    for _ in range(max(args.warmup, 1)):
        step_batch()
    torch.cuda.synchronize()
    g_batch = capture(step_batch)

    # single-frame latency: one trs_partition launch sequence on one stream (the paper's use,
    # a frame partitioned just before it is encoded), graph-replayed back to back
    one = B.Partitioner(w, h, params)
    one_out = torch.empty(B.RESULT_BYTES, dtype=torch.uint8, device="cuda")
    one.enqueue(luma[1], prev[1], out=one_out)
    torch.cuda.synchronize()
    g_one = capture(lambda: one.enqueue(luma[1], prev[1], out=one_out))
    reps_one = max(200, 20 * args.steps)
    _, el_one = time_graph(g_one, args.warmup, reps_one, 1)
    latency_us = el_one / reps_one * 1e6
    fps_streams, el_streams = time_graph(g_streams, args.warmup, args.steps, F)
    outs_streams = outs.clone()
    fps_batch, el_batch = time_graph(g_batch, args.warmup, args.steps, F)
    outs_batch = batch_out()
    log(f"per-frame launches over {S} streams: {fps_streams:.1f} frames/s; batched: {fps_batch:.1f} frames/s")
    batched = args.form == "batched"
    fps, elapsed = (fps_batch, el_batch) if batched else (fps_streams, el_streams)
    graph_outs = outs_batch if batched else outs_streams
    forms_equal = bool(torch.equal(outs_batch, outs_streams))

    # ---- eager runs of the reported form with HIP events around its kernels ----------------
    # (events on the stream the kernels are launched on: torch's current stream)
    B.trs_profile_enable(True)
    t0 = time.perf_counter()
    if batched:
        for _ in range(args.steps):
            step_batch()
        torch.cuda.synchronize()
        eager_elapsed = time.perf_counter() - t0
        B.trs_profile_enable(False)
        stage_ms, runs = B.trs_profile_read_batch()
        kms = {k: v / max(runs, 1) for k, v in stage_ms.items()}
        eager_out = batch_out()
        launch_frames = F / K
    else:
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(F)]
        feat_ms = 0.0
        for _ in range(args.steps):
            for f in range(F):
                ev[f][0].record()
                B.trs_features(frame, luma[f], part.feats)
                ev[f][1].record()
                B.trs_cost_map(frame, part.feats["tex"], prev[f], part.blend, part.cost, part.flags)
                B.trs_search(frame, params, part.cost, part.feats["s1"], part.feats["s2"], part.ws, outs[f])
            torch.cuda.synchronize()
            feat_ms += sum(a.elapsed_time(b) for a, b in ev)
        eager_elapsed = time.perf_counter() - t0
        B.trs_profile_enable(False)
        ms1, ms2, n_search = B.trs_profile_read()
        n = F * args.steps
        kms = {"features": feat_ms / n, "step1": ms1 / max(n_search, 1), "step2": ms2 / max(n_search, 1)}
        eager_out = outs
        launch_frames = 1
    eager_equals_graph = bool(torch.equal(eager_out, graph_outs))
    res_all = [B.result_dict(B.Result.from_buffer_copy(bytes(graph_outs[f].cpu().numpy().tobytes())))
               for f in range(F)]
    step2_frac = sum(r["n_step2"] for r in res_all) / max(1, sum(r["n_feasible"] for r in res_all))
    log(f"eager {args.form}: {F * args.steps / eager_elapsed:.1f} frames/s; kernel ms "
        + " ".join(f"{k} {v:.4f}" for k, v in kms.items()))

    # ---- roofline of each measured kernel; the longest one is reported as dominant ---------
    # features: HBM bytes per frame = every luma sample once + the per-CTU outputs
    feat_bytes = 2 * w * h + W * H * (5 * 4 + 8)
    # step 1: per feasible candidate one 64-bit max per tile (3 lane-ops) and a 64-bit
    # minimum (3); per record slice one rectangle sum and max (10)
    ops1 = 3 * stats["tile_lookups"] + 3 * stats["feasible"] + 10 * stats["record_slices"]
    # step 2 (work items not skipped by the Eq. 4 bound): per candidate and tile a 64-bit
    # max and add (5); per candidate the bound test and key compare (6); per record slice
    # three rectangle sums, the exact floor(S1^2 / n) and the sums (40)
    ops2 = step2_frac * (5 * stats["tile_lookups"] + 6 * stats["feasible"] + 40 * stats["record_slices"])
    kblock = (block or 256) if batched else (params.sched_block or 256)
    fk = "k_features_batch<128>" if batched else "k_features<128>"
    kernels = {
        fk: {"bound": "hbm", "avg_ms": kms["features"], "work": feat_bytes * launch_frames,
             "peak": PEAK_HBM_GBS, "unit": "GB/s", "scale": 1e9},
        (f"k_step1_units<{kblock}> (step 1)" if batched else f"k_search<{kblock}, false> (step 1)"): {
            "bound": "alu", "avg_ms": kms["step1"], "work": ops1 * launch_frames,
            "peak": PEAK_ALU_TOPS, "unit": "Tops/s", "scale": 1e12},
        (f"k_step2_live<{kblock}> (step 2)" if batched else f"k_search<{kblock}, true> (step 2)"): {
            "bound": "alu", "avg_ms": kms["step2"], "work": ops2 * launch_frames,
            "peak": PEAK_ALU_TOPS, "unit": "Tops/s", "scale": 1e12},
    }
    table = {}
    for name, k in kernels.items():
        ach = k["work"] / (k["avg_ms"] * 1e-3) / k["scale"] if k["avg_ms"] > 0 else 0.0
        table[name] = {"bound": k["bound"], "achieved": round(ach, 3), "peak": k["peak"], "unit": k["unit"],
                       "frac": round(ach / k["peak"], 4), "avg_ms": round(k["avg_ms"], 5),
                       "work_per_launch": int(k["work"])}
    dom = max(kernels, key=lambda n: kernels[n]["avg_ms"])
    roofline = dict(table[dom])
    roofline["kernel"] = dom
    roofline["traffic"] = TRAFFIC.get(dom)

    # ---- CPU oracle on a bounded sample, on the host's cores ------------------------------
    cpu = None
    parity = None
    if not args.no_cpu_baseline:
        import oracle
        cores = min(len(os.sched_getaffinity(0)), args.cpu_threads)
        n_cpu = min(F, args.cpu_frames or 4 * cores)
        oparams = oracle.make_params(cfg["n_threads"], cfg["max_tile_cols"], cfg["max_tile_rows"],
                                     cfg["max_rs_per_tile"], lam=cfg["lam"], prune=args.prune)
        otex = [oracle.features(frames[f])["tex"] for f in range(n_cpu)]
        oprev = [synth.ctu_times(otex[max(f - 1, 0)], eps[max(f - 1, 0)]) for f in range(n_cpu)]
        log(f"cpu baseline: oracle on {n_cpu} frames with {cores} threads")
        t0 = time.perf_counter()
        with cf.ThreadPoolExecutor(cores) as ex:
            refs = list(ex.map(lambda f: oracle.partition(frames[f], oprev[f], oparams), range(n_cpu)))
        wall = time.perf_counter() - t0
        cpu = {"value": round(n_cpu / wall, 4), "unit": "4K frames/s", "cores": cores, "kind": "oracle",
               "sample": f"frames 0..{n_cpu - 1} of the same 64-frame 4K sequence, whole path "
                         f"(features, time map, two-step search), one frame per thread, "
                         f"{wall:.1f} s wall ({wall * cores:.0f} thread-seconds)"}
        ok = 0
        for f in range(n_cpu):
            g = res_all[f]
            r = refs[f]
            same = all(g[k] == r[k] for k in ("rank", "t_min", "t_sel", "q_sel", "n_feasible", "rs_time")) \
                and [tuple(x) for x in g["rs"]] == [tuple(x) for x in r["rs"]]
            ok += same
        parity = (f"{ok}/{n_cpu} graph-replayed frames bit-exact vs oracle; eager == graph: {eager_equals_graph}; "
                  f"batched == per-frame on {F} frames: {forms_equal}")
        log(parity)

    res = {
        "metric": METRIC,
        "value": round(fps, 3),
        "unit": "4K frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": f"4K sequence: {F} frames 3840x2160 10-bit, CTU 128 (30x17), "
                               f"N=8 slices, tiles <= 6x4, <= 4 slices/tile, lambda=1/10, "
                               f"window ({stats['dtile']},{stats['drs']}), "
                               f"{stats['candidates']} candidates/frame ({stats['feasible']} area-feasible)",
                   "frames": F, "width": w, "height": h, "n_threads": 8,
                   "candidates_per_frame": stats["candidates"], "work_items": stats["items"],
                   "form": args.form, "sub_batches": K if batched else None, "prune": args.prune,
                   "wgs_per_cu": wgs if batched else None,
                   "timing": (f"HIP graph of one step ({K} batched runs over {F} frames, pipelined over "
                              f"{K} streams), replayed once per step"
                              if batched else
                              f"HIP graph of one step ({F} trs_partition calls over {S} streams), replayed K times")},
        "candidates_scored_per_s": round(fps * stats["candidates"], 1),
        "feasible_scored_per_s": round(fps * stats["feasible"], 1),
        "batched_value": round(fps_batch, 3),
        "per_frame_streams_value": round(fps_streams, 3),
        "single_frame_latency_us": round(latency_us, 2),
        "eager_value": round(F * args.steps / eager_elapsed, 3),
        "kernel_ms": {k: round(v, 5) for k, v in kms.items()},
        "step2_fraction": round(step2_frac, 4),
        "roofline": roofline,
        "roofline_kernels": table,
        "cpu_baseline": cpu,
        "parity": parity,
    }
    print(json.dumps(res), flush=True)


def capture(fn):
    """A HIP graph of one call of fn (captured on a side stream)."""
    import torch
    g = torch.cuda.CUDAGraph()
    cap = torch.cuda.Stream()
    cap.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(cap):
        with torch.cuda.graph(g, stream=cap):
            fn()
    torch.cuda.current_stream().wait_stream(cap)
    return g


def time_graph(g, warmup, steps, frames_per_step):
    """K replays bracketed by device synchronisation; returns (frames/s, seconds)."""
    import torch
    for _ in range(warmup):
        g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        g.replay()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    return frames_per_step * steps / el, el


def run_batch(args):
    """512 frames of 1080p / 4K / 8K (1:2:1), N drawn from {4, 8, 16}: one batched launch
    sequence (six launches, persistent search kernels) per step, graph-replayed, against
    the same frames as per-frame trs_partition launches over several streams."""
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2012_14792_amd import autotune
    from paper_2012_14792_amd import binding as B
    from paper_2012_14792_amd import synth

    torch.cuda.set_device(0)
    spec = synth.batch_workload(args.batch_frames)
    tuned = (autotune.load(f"{autotune.arch()}|batch512") or {}) if not args.sched_block else {}
    block = args.sched_block or tuned.get("block", 0)
    wgs = args.wgs_per_cu or tuned.get("wgs_per_cu", 0)
    t0 = time.perf_counter()
    gens = {n: synth.SequenceGenerator(*synth.SIZES[n], synth.batch_sequence_seed(n), 8.0)
            for n in ("fhd", "uhd", "8k")}
    with cf.ThreadPoolExecutor(16) as ex:
        frames_np = list(ex.map(lambda t: gens[t[0]].frame(t[1]), spec))
    lumas = [torch.from_numpy(fr.view(np.int16)).cuda() for fr in frames_np]
    prevs = [torch.zeros(synth.ctu_grid(*synth.SIZES[n])[0] * synth.ctu_grid(*synth.SIZES[n])[1],
                         dtype=torch.int32, device="cuda") for n, _, _ in spec]
    params = []
    for n, _, N in spec:
        C, R, K = synth.BOUNDS[N]
        p = B.make_params(N, C, R, K, lam=synth.LAMBDA[(n, N)], sched_block=args.sched_block,
                          sched_item=args.sched_item)
        if not (args.sched_block or args.sched_item):
            p = autotune.tuned_params(*synth.SIZES[n], p)
        params.append(p)
    items = [dict(width=synth.SIZES[n][0], height=synth.SIZES[n][1], params=params[i], luma=lumas[i],
                  prev=prevs[i]) for i, (n, _, _) in enumerate(spec)]
    batch = B.Batch(items, block=block, wgs_per_cu=wgs)
    # measured times of each frame from its texture (GPU features of the batch itself)
    batch.enqueue()
    torch.cuda.synchronize()
    base = batch.ws.data_ptr()
    tex = []
    for i, (n, _, _) in enumerate(spec):
        feat, _ = batch.frame_arrays(i)
        W, H = synth.ctu_grid(*synth.SIZES[n])
        off = feat.tex - base
        tex.append(batch.ws[off:off + 4 * W * H].cpu().numpy().view(np.uint32).copy())
    pos = {(n, k): i for i, (n, k, _) in enumerate(spec)}
    eps = {n: synth.ar1_eps(synth.ctu_grid(*synth.SIZES[n])[0] * synth.ctu_grid(*synth.SIZES[n])[1],
                            sum(1 for t in spec if t[0] == n), 4000 + j) for j, n in enumerate(("fhd", "uhd", "8k"))}
    prev_np = []
    for i, (n, k, _) in enumerate(spec):
        src = pos[(n, max(k - 1, 0))]
        pv = synth.ctu_times(tex[src], eps[n][max(k - 1, 0)])
        prev_np.append(pv)
        prevs[i].copy_(torch.from_numpy(pv.view(np.int32)))
    torch.cuda.synchronize()
    log(f"batch inputs ready: {len(spec)} frames in {time.perf_counter() - t0:.1f} s; "
        f"ws {batch.ws.numel() / 2**20:.1f} MiB")

    # batched: graph of one batch run
    g = batch.capture()
    for _ in range(args.warmup):
        g.replay()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        g.replay()
    torch.cuda.synchronize()
    el_b = time.perf_counter() - t1
    fps_b = len(spec) * args.steps / el_b
    batch_out = batch.out.clone()
    log(f"batched: {fps_b:.1f} frames/s")

    # per-frame launches of the same frames, over streams, graph-replayed
    S = max(1, args.streams)
    streams = [torch.cuda.Stream() for _ in range(S)]
    parts = {}
    outs = torch.empty_like(batch.out)

    def part_for(i, k):
        key = (spec[i][0], spec[i][2], k)
        if key not in parts:
            parts[key] = B.Partitioner(items[i]["width"], items[i]["height"], params[i])
        return parts[key]

    def step():
        b0 = torch.cuda.current_stream()
        for st in streams:
            st.wait_stream(b0)
        for i in range(len(spec)):
            k = i % S
            with torch.cuda.stream(streams[k]):
                part_for(i, k).enqueue(lumas[i], prevs[i], out=outs[i])
        for st in streams:
            b0.wait_stream(st)

    step()
    torch.cuda.synchronize()
    gp = torch.cuda.CUDAGraph()
    cap = torch.cuda.Stream()
    cap.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(cap):
        with torch.cuda.graph(gp, stream=cap):
            step()
    torch.cuda.current_stream().wait_stream(cap)
    for _ in range(args.warmup):
        gp.replay()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(args.steps):
        gp.replay()
    torch.cuda.synchronize()
    el_p = time.perf_counter() - t2
    fps_p = len(spec) * args.steps / el_p
    same = bool(torch.equal(batch_out, outs))
    log(f"per-frame launches: {fps_p:.1f} frames/s; batched == per-frame on all frames: {same}")

    cpu = None
    parity = None
    res = [B.result_dict(B.Result.from_buffer_copy(bytes(batch_out[i].cpu().numpy().tobytes())))
           for i in range(len(spec))]
    if not args.no_cpu_baseline:
        import oracle
        cores = min(len(os.sched_getaffinity(0)), args.cpu_threads)
        n_cpu = min(len(spec), args.cpu_frames or cores)
        oparams = [oracle.make_params(p.n_threads, p.max_tile_cols, p.max_tile_rows, p.max_rs_per_tile,
                                      lam=(p.lambda_num, p.lambda_den)) for p in params[:n_cpu]]
        oprev = []
        for i in range(n_cpu):
            n, k, _ = spec[i]
            src = frames_np[pos[(n, max(k - 1, 0))]]
            oprev.append(synth.ctu_times(oracle.features(src)["tex"], eps[n][max(k - 1, 0)]))
        log(f"cpu baseline: oracle on {n_cpu} batch frames with {cores} threads")
        t3 = time.perf_counter()
        with cf.ThreadPoolExecutor(cores) as ex:
            refs = list(ex.map(lambda i: oracle.partition(frames_np[i], oprev[i], oparams[i]), range(n_cpu)))
        wall = time.perf_counter() - t3
        cpu = {"value": round(n_cpu / wall, 4), "unit": "frames/s", "cores": cores, "kind": "oracle",
               "sample": f"the first {n_cpu} frames of the 512-frame batch (mixed sizes and N), whole "
                         f"path, one frame per thread, {wall:.1f} s wall"}
        ok = sum(all(res[i][k] == refs[i][k] for k in ("rank", "t_min", "t_sel", "q_sel", "n_feasible",
                                                        "rs_time"))
                 and [tuple(x) for x in res[i]["rs"]] == [tuple(x) for x in refs[i]["rs"]]
                 for i in range(n_cpu))
        parity = f"{ok}/{n_cpu} frames bit-exact vs oracle; batched == per-frame on {len(spec)} frames: {same}"
        log(parity)
    cands = sum(r["n_enumerated"] for r in res)
    feas = sum(r["n_feasible"] for r in res)
    out = {
        "metric": "mixed-batch frames partitioned/s (1 GPU, bit-exact vs oracle)",
        "value": round(fps_b, 3), "unit": "frames/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(el_b / args.steps * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": f"batch of {len(spec)} frames: 1080p/4K/8K 1:2:1, N from {{4,8,16}}, "
                               f"one batched launch sequence (persistent search) per step, graph-replayed",
                   "frames": len(spec), "candidates": cands, "feasible": feas,
                   "block": block or 256, "wgs_per_cu": wgs},
        "per_frame_value": round(fps_p, 3),
        "batched_over_per_frame": round(fps_b / fps_p, 3),
        "candidates_scored_per_s": round(cands * args.steps / el_b, 1),
        "cpu_baseline": cpu,
        "parity": parity,
    }
    print(json.dumps(out), flush=True)


# fp32 FMA-counted flops per sample of the perceptron's matrix products (10 -> 64 -> 64 -> 1)
MLP_FWD_FLOPS = 2 * (64 * 10 + 64 * 64 + 64)
# backward: dz1 = W2^T dz2, dW2, dW1, dW3 (the products; GELU derivatives not counted)
MLP_BWD_FLOPS = 2 * (64 * 64 + 64 * 64 + 64 * 10 + 64)
PEAK_FP32_TFLOPS = 157.3


def run_mlp(args):
    """Training steps of the learned per-CTU time predictor: forward kernel, backward
    kernels, torch's Adam, on batches of `--mlp-batch` samples drawn from a resident pool of
    inputs shaped like the training pairs.  Also times one 4K frame's inference (inputs,
    forward, time map)."""
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2012_14792_amd import binding as B
    from paper_2012_14792_amd.mlp import TimeMLP

    torch.cuda.set_device(0)
    nb = args.mlp_batch
    pool = 1 << 21
    g = torch.Generator(device="cuda").manual_seed(7)
    # inputs in the ranges of the training pairs: textures, variances, means, times (us)
    scale = torch.tensor([500, 4000, 1000, 500, 500, 500, 500, 3000, 3000, 1], device="cuda")
    X = torch.rand((pool, 10), generator=g, device="cuda") * scale
    T = torch.rand(pool, generator=g, device="cuda") * 3
    m = TimeMLP(seed=0)
    m.fit_norm(X)
    opt = torch.optim.Adam(m.parameters(), lr=1e-3, fused=True, capturable=True)
    idx = [torch.randint(0, pool, (nb,), generator=g, device="cuda") for _ in range(16)]
    xs = [X[i].contiguous() for i in idx]
    ts = [T[i].contiguous() for i in idx]

    def step(k):
        y = m(xs[k % 16])
        loss = torch.mean((y - ts[k % 16]) ** 2)
        opt.zero_grad(set_to_none=True)
        loss.backward()
        opt.step()

    # warm-up on a side stream (the optimiser state is created here), then eager timing
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        for k in range(max(args.warmup, 1)):
            step(k)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(k)
    torch.cuda.synchronize()
    el_eager = time.perf_counter() - t0
    sps_eager = nb * args.steps / el_eager
    # the same steps as one HIP graph of 16 steps (one per resident batch), replayed: the
    # host's launch overhead leaves the timed region
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        for k in range(16):
            step(k)
    graph.replay()
    torch.cuda.synchronize()
    reps = max(1, (args.steps + 15) // 16)
    t0 = time.perf_counter()
    for _ in range(reps):
        graph.replay()
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / (16 * reps) * args.steps
    sps = nb * args.steps / el
    log(f"mlp training: {sps / 1e6:.2f} M samples/s graph-replayed ({el / args.steps * 1e3:.3f} ms/step of {nb}); "
        f"eager {sps_eager / 1e6:.2f} M samples/s")

    # kernel durations with events on the launching stream, at the training batch size
    ws = [p.detach() for p in m.parameters()]
    y = torch.empty(nb, device="cuda")
    z1 = torch.empty((64, nb), device="cuda")
    z2 = torch.empty((64, nb), device="cuda")
    dy = torch.randn(nb, device="cuda")
    grads = [torch.empty_like(p) for p in ws]
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    reps = max(args.steps, 10)
    B.trs_mlp_forward(ws, m.norm, xs[0], y, z1, z2)
    B.trs_mlp_backward(ws, m.norm, xs[0], z1, z2, dy, grads)
    torch.cuda.synchronize()
    fwd_ms = bwd_ms = 0.0
    for _ in range(reps):
        e[0].record()
        B.trs_mlp_forward(ws, m.norm, xs[0], y, z1, z2)
        e[1].record()
        B.trs_mlp_backward(ws, m.norm, xs[0], z1, z2, dy, grads)
        e[2].record()
        torch.cuda.synchronize()
        fwd_ms += e[0].elapsed_time(e[1])
        bwd_ms += e[1].elapsed_time(e[2])
    fwd_ms /= reps
    bwd_ms /= reps
    fwd_tf = MLP_FWD_FLOPS * nb / (fwd_ms * 1e-3) / 1e12
    bwd_tf = MLP_BWD_FLOPS * nb / (bwd_ms * 1e-3) / 1e12

    # one 4K frame's inference: inputs -> forward -> time map (2040 CTUs)
    frame = B.make_frame(3840, 2160)
    W, H = B.ctu_dims(frame)
    feats = B.alloc_features(frame)
    lum = torch.randint(0, 1024, (2160, 3840), dtype=torch.int16, generator=g, device="cuda")
    B.trs_features(frame, lum, feats)
    prev = torch.randint(200, 3000, (W * H,), dtype=torch.int32, generator=g, device="cuda")
    x4 = torch.empty((W * H, 10), device="cuda")
    cost = torch.empty(W * H, dtype=torch.int32, device="cuda")

    def infer():
        B.trs_mlp_inputs(frame, feats, prev, x4)
        m.cost_map(frame, x4, feats["tex"], prev, cost=cost)

    infer()
    torch.cuda.synchronize()
    e[0].record()
    for _ in range(reps):
        infer()
    e[1].record()
    torch.cuda.synchronize()
    inf_us = e[0].elapsed_time(e[1]) / reps * 1e3

    cpu = None
    if not args.no_cpu_baseline:
        from oracle import mlp_ref
        n_cpu = 1 << 16
        p = {k: v.cpu().double().numpy() for k, v in zip(("w1", "b1", "w2", "b2", "w3", "b3"), ws)}
        xc = X[:n_cpu].cpu().double().numpy()
        mean = np.array(list(m.norm.mean))
        inv = np.array(list(m.norm.inv_std))
        dyc = dy[:n_cpu].cpu().double().numpy() if nb >= n_cpu else np.ones(n_cpu)
        t1 = time.perf_counter()
        reps_cpu = 0
        while True:
            _, cache = mlp_ref.forward(p, xc, mean, inv)
            mlp_ref.backward(p, cache, dyc)
            reps_cpu += 1
            if time.perf_counter() - t1 > 10.0:
                break
        wall = time.perf_counter() - t1
        cores = min(len(os.sched_getaffinity(0)), args.cpu_threads)
        cpu = {"value": round(n_cpu * reps_cpu / wall, 1), "unit": "samples/s (forward + backward)",
               "cores": cores, "kind": "oracle",
               "sample": f"FP64 reference forward + backward on {n_cpu} samples, {reps_cpu} passes, "
                         f"{wall:.1f} s wall (numpy matrix products may use up to {cores} threads)"}
        log(f"cpu baseline: {cpu['value']:.0f} samples/s")

    out = {
        "metric": "learned CTU-time predictor training samples/s (forward + backward + Adam, 1 GPU)",
        "value": round(sps, 1), "unit": "samples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(el / args.steps * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"10-64-64-1 GELU perceptron, batches of {nb} samples from a resident "
                               f"pool of {pool} synthetic inputs", "batch": nb},
        "eager_value": round(sps_eager, 1),
        "timing": f"{16 * reps} training steps as {reps} replays of a 16-step HIP graph",
        "kernel_ms": {"forward": round(fwd_ms, 5), "backward": round(bwd_ms, 5)},
        "roofline": {"bound": "alu", "kernel": "k_mlp_fwd", "achieved": round(fwd_tf, 3),
                     "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s", "frac": round(fwd_tf / PEAK_FP32_TFLOPS, 4),
                     "traffic": None},
        "roofline_kernels": {"backward (3 kernels)": {"bound": "alu", "achieved": round(bwd_tf, 3),
                                                      "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                                                      "frac": round(bwd_tf / PEAK_FP32_TFLOPS, 4)}},
        "inference_us_4k_frame": round(inf_us, 2),
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


# DP relaxations of the literal-space search and the lane-ops charged to each.  Tile tables: a
# step-1 relaxation is a 64-bit max and a 64-bit compare-select (6 lane-ops), a step-2 one adds
# a 64-bit sum and compares (Q, T~) lexicographically (10).  Units: step 1 with 32-bit times is
# a max and a min (2 lane-ops; 6 with 64-bit times), step 2 on packed (Q, T~) keys is two 64-bit
# masks, a 64-bit min of them, a 64-bit add and subtract and a 64-bit compare-select (14).
LIT_OPS = {"tiles1": 6, "tiles2": 10, "units1_u32": 2, "units1_u64": 6, "units2": 14}


def literal_relaxations(w, h, N, Cm, Rm, Km, area_k=3, cs=128):
    """(tile-table relaxations, unit relaxations) of one step of the literal search, counted
    from the loop bounds of the three DPs: split rows per (window, strip, row pair, k), and per
    (window, row boundaries) the strip DP over tiles and the column DP over (columns, RS)."""
    from math import comb
    W, H = (w + cs - 1) // cs, (h + cs - 1) // cs
    Cm, Rm, Km = min(Cm, W), min(Rm, H), min(Km, H)
    cw = [min(cs, w - x * cs) for x in range(W)]
    rh = [min(cs, h - y * cs) for y in range(H)]
    widths = {sum(cw[a:b]) for a in range(W) for b in range(a + 1, W + 1)}
    heights = {sum(rh[a:b]) for a in range(H) for b in range(a + 1, H + 1)}
    areas = {x * y for x in widths for y in heights}
    n_win = 1 if area_k == 0 else sum(1 for a in areas if N * a <= w * h < area_k * N * a)
    S = W * (W + 1) // 2
    per_strip = sum(max(0, (y - y0) - q + 1) if q > 1 else 1
                    for y0 in range(H) for y in range(y0 + 1, H + 1) for q in range(1, Km + 1))
    tiles = n_win * S * per_strip
    knap = sum(min(Km, K) for K in range(N + 1))
    colB = sum((x - i + 1) * n for x in range(1, W + 1) for i in range(1, min(x, Cm) + 1)
               for n in range(1, N + 1))
    units = 0
    for r in range(1, Rm + 1):
        nY = comb(H - 1, r - 1)
        colA = sum(x * r * knap for x in range(1, W + 1))
        units += n_win * nY * (colA + colB)
    return tiles, units


def run_literal(args):
    """4K frames searched exactly over the literal space (5.4e9 candidates per frame): per
    frame the feature kernel, the time map and trs_literal_search, frames one after another
    on one stream with one workspace."""
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2012_14792_amd import binding as B
    from paper_2012_14792_amd import synth

    torch.cuda.set_device(0)
    w, h, N, C, R, K, lam = 3840, 2160, 8, 6, 4, 4, (1, 10)
    F = 8 if args.frames == 64 else args.frames
    frame = B.make_frame(w, h)
    W, H = B.ctu_dims(frame)
    params = B.make_params(N, C, R, K, lam=lam, dtile=-1, drs=-1, span_tiles=args.span_tiles)
    gen = synth.SequenceGenerator(w, h, 2, 8.0)
    lum_np = [gen.frame(f) for f in range(F + 1)]
    luma = [torch.from_numpy(x.view(np.int16)).cuda() for x in lum_np]
    feats = [B.alloc_features(frame) for _ in range(F + 1)]
    for f in range(F + 1):
        B.trs_features(frame, luma[f], feats[f])
    eps = synth.ar1_eps(W * H, F + 1, 2000)
    truth = [synth.ctu_times(feats[f]["tex"].cpu().numpy().view(np.uint32), eps[f]) for f in range(F + 1)]
    prev = [torch.from_numpy(truth[f].view(np.int32)).cuda() for f in range(F + 1)]
    cost = [torch.empty(W * H, dtype=torch.int32, device="cuda") for _ in range(F + 1)]
    ws = torch.empty(B.trs_literal_workspace(frame, params), dtype=torch.uint8, device="cuda")
    out = torch.empty((F + 1, B.RESULT_BYTES), dtype=torch.uint8, device="cuda")
    blend = B.Blend(200, 3, 256)

    def step():
        for f in range(1, F + 1):
            B.trs_features(frame, luma[f], feats[f])
            B.trs_cost_map(frame, feats[f]["tex"], prev[f - 1], blend, cost[f])
            B.trs_literal_search(frame, params, cost[f], feats[f]["s1"], feats[f]["s2"], ws, out[f])

    for _ in range(max(args.warmup, 1)):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    fps = F * args.steps / el
    log(f"literal search: {fps:.1f} 4K frames/s ({el / args.steps / F * 1e3:.3f} ms per frame)")

    # stage durations with events on the launching stream, one eager pass
    B.trs_profile_enable(1)
    step()
    torch.cuda.synchronize()
    B.trs_profile_enable(0)
    st, runs, (run1, run2) = B.trs_profile_read_literal()
    st = {k: v / runs for k, v in st.items()}
    run1, run2 = run1 / runs, run2 / runs               # relaxations of the units run, per frame
    tiles, units = literal_relaxations(w, h, N, C, R, K)
    wide = any(int(c.cpu().numpy().view(np.uint32).astype(np.int64).sum()) >= 2**32 - 1 for c in cost[1:])
    ops = {"tiles1": tiles * LIT_OPS["tiles1"], "tiles2": tiles * LIT_OPS["tiles2"],
           "units1": run1 * LIT_OPS["units1_u64" if wide else "units1_u32"], "units2": run2 * LIT_OPS["units2"]}
    dom = max(ops, key=lambda k: st[k])
    ach = ops[dom] / (st[dom] * 1e-3) / 1e12
    res = [B.read_result(out[f]) for f in range(1, F + 1)]
    log("stages (ms per frame): " + ", ".join(f"{k} {v:.3f}" for k, v in st.items()))
    # the same frames over the ladder space (the default search) for comparison
    lad_p = B.make_params(N, C, R, K, lam=lam)
    lws = torch.empty(B.trs_search_workspace(frame, lad_p), dtype=torch.uint8, device="cuda")
    lout = torch.empty(B.RESULT_BYTES, dtype=torch.uint8, device="cuda")
    better_t = better_q = 0
    for f in range(1, F + 1):
        B.trs_search(frame, lad_p, cost[f], feats[f]["s1"], feats[f]["s2"], lws, lout)
        lr = B.read_result(lout)
        assert res[f - 1]["t_min"] <= lr["t_min"], "literal T~min above the ladder's"
        better_t += res[f - 1]["t_min"] < lr["t_min"]
        better_q += res[f - 1]["q_sel"] < lr["q_sel"]
    log(f"literal vs ladder: lower T~min on {better_t}/{F} frames, lower Q on {better_q}/{F}")

    cpu, parity = None, "not checked (--no-cpu-baseline)"
    if not args.no_cpu_baseline:
        import oracle as orc
        f = 1
        fo = orc.features(lum_np[f])
        c_np, _ = orc.cost_map(fo["tex"], truth[f - 1])
        t1 = time.perf_counter()
        ref = orc.literal_search(w, h, orc.make_params(N, C, R, K, lam=lam, dtile=-1, drs=-1,
                                                       span_tiles=args.span_tiles), c_np, fo["s1"], fo["s2"])
        wall = time.perf_counter() - t1
        keys = ("status", "t_min", "t_sel", "q_sel", "n_enumerated", "tile_cols", "tile_rows",
                "col_bd", "row_bd", "rs", "rs_time", "t_unif", "q_unif")
        same = all(res[f - 1][k] == ref[k] for k in keys)
        parity = f"frame {f} bit-exact vs oracle: {same}"
        cpu = {"value": round(1.0 / wall, 4), "unit": "4K frames/s", "cores": 1, "kind": "oracle",
               "sample": f"frame {f}: oracle literal-space search by the same decomposition in plain C, "
                         f"one thread, {wall:.1f} s"}
        log(f"cpu baseline: {wall:.1f} s per frame; {parity}")

    out_j = {
        "metric": "4K frames/s, exact search over the literal space (every CTU boundary allowed)",
        "value": round(fps, 2), "unit": "4K frames/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(el / args.steps * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": f"{F} frames of the 3840x2160 drifting sequence (seed 2), N=8, tiles <= 6x4, "
                               f"<= 4 RS per tile, lambda 1/10, literal space"
                               + (" with RS spanning tiles of one tile column" if args.span_tiles else "")
                               + f" ({res[0]['n_enumerated']} candidates/frame)",
                   "frames_per_step": F},
        "stage_ms_per_frame": {k: round(v, 4) for k, v in st.items()},
        "relaxations_per_frame": {"tiles (each step)": tiles, "units (each step, every unit)": units,
                                  "units run (step 1)": round(run1), "units run (step 2)": round(run2)},
        "roofline": {"bound": "alu", "kernel": {"units1": "k_lit_units<1>", "units2": "k_lit_units<2>",
                                                "tiles1": "k_lit_tiles<1>", "tiles2": "k_lit_tiles<2>"}[dom],
                     "achieved": round(ach, 3), "peak": PEAK_ALU_TOPS, "unit": "T lane-ops/s",
                     "frac": round(ach / PEAK_ALU_TOPS, 4), "traffic": None},
        "t_min_frames": [r["t_min"] for r in res],
        "literal_better_than_ladder": {"t_min": better_t, "q": better_q, "frames": F},
        "parity": parity,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out_j), flush=True)


if __name__ == "__main__":
    main()
