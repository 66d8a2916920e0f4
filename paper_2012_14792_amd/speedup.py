"""Synthetic analog of the paper's speed-up measures (Section 3.2, Eq. 5 and Eq. 6).

The paper measures the speed-up sigma of an N-thread encoder as the ratio of the 1-thread to
the N-thread encoding time (Eq. 5, averaged over four QPs), and bounds it with Amdahl's law for
a sequential share s of the encoder (Eq. 6).  Without an encoder, the synthetic stand-in uses
the realized CTU times of the seeded time model: one thread takes the sum of a frame's CTU
times, N threads (one rectangular slice each) take the largest slice sum (Eq. 1 with the true
times), and a sequence's time is the sum over its frames.  The Amdahl-capped variant adds a
sequential share s of the 1-thread time to every frame.

    python -m paper_2012_14792_amd.speedup            # Table-1-shaped report on one GPU
"""
from __future__ import annotations

import numpy as np


def sigma_max(n: int, s: float) -> float:
    """Eq. 6: the Amdahl bound for n threads and a sequential share s (0 <= s <= 1)."""
    return 1.0 / (s + (1.0 - s) / n)


def region_times(rects, times_hw: np.ndarray) -> list[int]:
    """Sum of CTU times over each rectangle (x0, y0, x1, y1), half open, in CTUs."""
    return [int(times_hw[y0:y1, x0:x1].sum()) for (x0, y0, x1, y1) in rects]


def uniform_rects(W: int, H: int, n: int) -> list[tuple[int, int, int, int]]:
    """The uniform grid of n tiles, one slice each: c_u x r_u = n with r_u the largest
    divisor not above sqrt(n); boundaries floor(i W / c_u), floor(j H / r_u)."""
    ru = max(d for d in range(1, int(n ** 0.5) + 1) if n % d == 0)
    cu = n // ru
    return [(i * W // cu, j * H // ru, (i + 1) * W // cu, (j + 1) * H // ru)
            for j in range(ru) for i in range(cu)]


def sequence_speedup(frames_rects, frames_times, s: float = 0.0) -> float:
    """sigma over a sequence: sum of 1-thread times over sum of N-thread times, where a frame's
    N-thread time is its largest region sum and both carry the sequential share s of the
    1-thread time (s = 0: the partition's own balance; s > 0: the Amdahl-capped analog)."""
    t_one = t_par = 0.0
    for rects, t in zip(frames_rects, frames_times):
        total = float(t.sum())
        t_one += total
        t_par += s * total + (1.0 - s) * max(region_times(rects, t))
    return t_one / t_par


def report(n_frames: int = 16, s: float = 0.04, sizes=("fhd", "uhd", "8k"), threads=(4, 8, 16),
           device="cuda", keep_decisions: bool = False, prune: int = 0) -> dict:
    """For every (resolution, N) of the workloads: sigma of the uniform grid and of the chosen
    partitions, with and without the sequential share, and the Eq. 6 bound.  Partitions come
    from the batched GPU path on a seeded drifting sequence with the previous frame's realized
    times as the estimate; realized times follow the seeded AR(1) model."""
    import torch

    from . import binding as B
    from . import synth

    out = {}
    for name in sizes:
        w, h = synth.SIZES[name]
        W, H = synth.ctu_grid(w, h)
        gen = synth.TorchSequenceGenerator(w, h, synth.batch_sequence_seed(name) + 100, 8.0, device)
        eps = synth.ar1_eps(W * H, n_frames + 1, 9000 + len(out))
        frame = B.make_frame(w, h)
        feats = B.alloc_features(frame, device)
        lumas, truth = [], []
        for f in range(n_frames + 1):
            luma = gen.frame(f)
            B.trs_features(frame, luma, feats)
            truth.append(synth.ctu_times(feats["tex"].cpu().numpy().view(np.uint32), eps[f]))
            lumas.append(luma)
        for N in threads:
            C, R, K = synth.BOUNDS[N]
            params = B.make_params(N, C, R, K, lam=synth.LAMBDA[(name, N)], prune=prune)
            items = [dict(width=w, height=h, params=params, luma=lumas[f],
                          prev=torch.from_numpy(truth[f - 1].view(np.int32)).to(device))
                     for f in range(1, n_frames + 1)]
            batch = B.Batch(items)
            batch.enqueue()
            torch.cuda.synchronize()
            res = batch.results()
            batch.close()
            times = [truth[f].reshape(H, W).astype(np.int64) for f in range(1, n_frames + 1)]
            chosen = [r["rs"] for r in res]
            unif = [uniform_rects(W, H, N)] * n_frames
            out[f"{name}_N{N}"] = {
                "lambda": "/".join(map(str, synth.LAMBDA[(name, N)])),
                "sigma_uniform": sequence_speedup(unif, times),
                "sigma_proposed": sequence_speedup(chosen, times),
                "sigma_uniform_amdahl": sequence_speedup(unif, times, s),
                "sigma_proposed_amdahl": sequence_speedup(chosen, times, s),
                "sigma_max": sigma_max(N, s),
            }
            if keep_decisions:
                out[f"{name}_N{N}"]["decisions"] = res
                out[f"{name}_N{N}"]["inputs"] = (lumas, truth)
    return out


def main():
    import argparse
    import json
    import sys
    ap = argparse.ArgumentParser()
    ap.add_argument("--frames", type=int, default=16)
    ap.add_argument("--prune", type=int, default=0, help="pruning rules (bit 0 heights, bit 1 means)")
    args = ap.parse_args()
    res = report(n_frames=args.frames, prune=args.prune)
    print(f"{'workload':10s} {'lambda':>6s} {'uniform':>8s} {'proposed':>9s} {'unif(s)':>8s} "
          f"{'prop(s)':>8s} {'max(s)':>7s}", file=sys.stderr)
    for k, v in res.items():
        print(f"{k:10s} {v['lambda']:>6s} {v['sigma_uniform']:8.3f} {v['sigma_proposed']:9.3f} "
              f"{v['sigma_uniform_amdahl']:8.3f} {v['sigma_proposed_amdahl']:8.3f} {v['sigma_max']:7.3f}",
              file=sys.stderr)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
