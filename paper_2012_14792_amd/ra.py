"""Random-access sequences: which earlier frame's CTU times predict the current frame's.

Section 2.1 of the paper takes the predicted time of a CTU from the co-located CTU of the
co-TL frame (the previously coded frame of the same temporal layer), since in random-access
coding the frames of one layer share their coding parameters; the related works it cites use
the closest frame in time.  `trs_ra_schedule` gives both references for a dyadic GOP.

Synthetic stand-in for an RA encoder's times: the seeded per-CTU model round((a + b tex) e^eps)
of the other workloads with (a, b) set per temporal layer: deeper layers are coded at higher QP,
take less time, and their time depends less on texture (`layer_model`).  A factor common to a
whole frame would not matter: scaling a time map leaves every decision unchanged (T~min, the
Eq. 4 bound and every T~(P) scale together, Q does not depend on times); what a reference frame
must predict is the spatial pattern.  The per-layer values are a modelling choice of this module,
not values from the paper.

    python -m paper_2012_14792_amd.ra          # co-TL vs closest-frame estimator, one GPU
"""
from __future__ import annotations

import numpy as np

from . import synth


def layer_model(layer: int) -> tuple[float, float]:
    """(a, b) of the time model a + b tex for temporal layer `layer` (synthetic): both shrink
    with depth, b faster than a."""
    return 200.0 * 0.85 ** layer, 3.0 * 0.6 ** layer


def layer_times(tex: np.ndarray, eps: np.ndarray, layer: int) -> np.ndarray:
    """Synthetic measured CTU times (us) of a frame in temporal layer `layer`, uint32."""
    a, b = layer_model(layer)
    t = np.rint((a + b * np.asarray(tex, np.float64)) * np.exp(eps))
    return np.clip(t, 1, 2**31 - 1).astype(np.uint32)


def sequence(size: str = "fhd", gop: int = 16, n_frames: int = 33, seed: int = 70, device="cuda"):
    """Frames of a seeded drifting sequence with their features and per-layer times.
    Returns (schedule, lumas, times) with times[p] the uint32 map of frame p (display order)."""
    from . import binding as B
    w, h = synth.SIZES[size]
    W, H = synth.ctu_grid(w, h)
    sched = B.trs_ra_schedule(gop, n_frames)
    gen = synth.TorchSequenceGenerator(w, h, seed, 8.0, device)
    eps = synth.ar1_eps(W * H, n_frames, seed + 1000)
    frame = B.make_frame(w, h)
    feats = B.alloc_features(frame, device)
    lumas, times = [], []
    for p in range(n_frames):
        luma = gen.frame(p)
        B.trs_features(frame, luma, feats)
        tex = feats["tex"].cpu().numpy().view(np.uint32)
        times.append(layer_times(tex, eps[p], int(sched["layer"][p])))
        lumas.append(luma)
    return sched, lumas, times


def report(size: str = "fhd", n_threads: int = 4, gop: int = 16, n_frames: int = 33, seed: int = 70,
           device="cuda", keep_decisions: bool = False) -> dict:
    """For every frame that has both references, partition it (batched GPU path, Table 1's
    lambda) with each reference's times as the prediction, and compare the estimators: mean
    relative per-CTU error of the prediction, and the speed-up sigma (sum of 1-thread times over
    sum of slowest-RS times, realized times) of the chosen partitions."""
    import torch

    from . import binding as B
    from .speedup import sequence_speedup
    w, h = synth.SIZES[size]
    W, H = synth.ctu_grid(w, h)
    sched, lumas, times = sequence(size, gop, n_frames, seed, device)
    C, R, K = synth.BOUNDS[n_threads]
    lam = B.trs_lambda_policy(B.make_frame(w, h), n_threads)
    params = B.make_params(n_threads, C, R, K, lam=lam)
    order = [int(p) for p in sched["coding_order"]]
    targets = [p for p in order if sched["cotl_ref"][p] >= 0 and sched["closest_ref"][p] >= 0]
    out = {"size": size, "n_threads": n_threads, "gop": gop, "frames": len(targets),
           "lambda": f"{lam[0]}/{lam[1]}"}
    truth = [times[p].reshape(H, W).astype(np.int64) for p in targets]
    for name in ("cotl", "closest"):
        refs = [int(sched[f"{name}_ref"][p]) for p in targets]
        items = [dict(width=w, height=h, params=params, luma=lumas[p],
                      prev=torch.from_numpy(times[q].view(np.int32)).to(device))
                 for p, q in zip(targets, refs)]
        batch = B.Batch(items)
        batch.enqueue()
        torch.cuda.synchronize()
        res = batch.results()
        batch.close()
        rel = [np.abs(times[q].astype(np.float64) - times[p]) / times[p] for p, q in zip(targets, refs)]
        # the same after dividing each map by its sum (the spatial pattern alone)
        shape = []
        for p, q in zip(targets, refs):
            tp, tq = times[p] / times[p].sum(dtype=np.float64), times[q] / times[q].sum(dtype=np.float64)
            shape.append(np.abs(tq - tp) / tp)
        out[name] = {"ctu_rel_err": float(np.mean(np.concatenate(rel))),
                     "pattern_rel_err": float(np.mean(np.concatenate(shape))),
                     "sigma": sequence_speedup([r["rs"] for r in res], truth),
                     "mean_display_distance": float(np.mean([abs(p - q) for p, q in zip(targets, refs)]))}
        if keep_decisions:
            out[name]["decisions"] = list(zip(targets, refs, res))
    out["inputs"] = (sched, lumas, times) if keep_decisions else None
    return out


def main():
    import argparse
    import json
    import sys
    ap = argparse.ArgumentParser()
    ap.add_argument("--frames", type=int, default=65)
    ap.add_argument("--gop", type=int, default=16)
    args = ap.parse_args()
    rows = []
    for size, n in (("fhd", 4), ("fhd", 8), ("uhd", 8), ("uhd", 16)):
        r = report(size, n, args.gop, args.frames)
        r.pop("inputs")
        rows.append(r)
        print(f"{size} N={n:2d} lambda {r['lambda']:>5s}: "
              + " | ".join(f"{e}: err {r[e]['ctu_rel_err']:.3f} pattern {r[e]['pattern_rel_err']:.3f} "
                           f"sigma {r[e]['sigma']:.3f}" for e in ("cotl", "closest")), file=sys.stderr)
    print(json.dumps(rows))


if __name__ == "__main__":
    main()
