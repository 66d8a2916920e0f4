"""Seeded synthetic inputs: 10-bit luma frames and per-CTU encoding-time maps.

The paper measures on JVET common-test-condition sequences (FHD and UHD, Section 3.1),
which are not available here.  These generators produce frames of the same resolutions,
bit depth and CTU grid, with spatially varying texture, and CTU times that are temporally
correlated (the property the co-located-CTU estimator of Section 2.1 relies on).

This module is the only code shared by the oracle-side tests and the GPU path.  It holds
none of the partitioning method's arithmetic: no features, no cost map, no search.  The
time model takes a per-CTU texture array as an *input*; callers supply it.

Frame recipe (fixed draw order from ``numpy.random.Generator(PCG64(seed))``):
  1. 8 sinusoids: period P ~ logU[4, 256] px, angle ~ U[0, pi), phase ~ U[0, 2 pi),
     amplitude ~ U[20, 80].  Drawn as four arrays of length 8 in that order.
  2. 20 blobs: centre x ~ U[0, w), centre y ~ U[0, h), sigma ~ U[8, 200],
     amplitude ~ U[50, 300], speed ~ U[0, drift_max], heading ~ U[0, 2 pi).
     Drawn as six arrays of length 20 in that order.
  3. For each blob in order: a noise patch u ~ U[-1, 1] of shape (2R+1, 2R+1), R = ceil(3 sigma).
  Luma = clip(rint(512 + sum of sinusoids + sum of blob patches), 0, 1023) as uint16.
  A blob contributes a * exp(-r^2 / (2 sigma^2)) * u inside its (2R+1)^2 window and nothing
  outside it; at frame f its window is centred at round(centre + f * velocity), so the noise
  moves with the blob.  Sinusoids do not move.

Time recipe: T_f(c) = round((200 + 3 tex_f(c)) * exp(eps_f(c))) microseconds, with
eps_0 ~ N(0, 0.3^2) and eps_f = rho eps_{f-1} + sqrt(1 - rho^2) N(0, 0.3^2).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "FrameSpec", "SequenceGenerator", "make_frame", "ar1_eps", "ctu_times",
    "CONFIGS", "ctu_grid",
]


@dataclasses.dataclass(frozen=True)
class FrameSpec:
    width: int
    height: int
    ctu: int = 128
    bit_depth: int = 10


def ctu_grid(width: int, height: int, ctu: int = 128) -> tuple[int, int]:
    """Number of CTU columns and rows covering the frame (partial CTUs count)."""
    return (width + ctu - 1) // ctu, (height + ctu - 1) // ctu


class SequenceGenerator:
    """A drifting-blob sequence; ``frame(f)`` renders frame f (f >= 0)."""

    def __init__(self, width: int, height: int, seed: int, drift_max: float = 0.0,
                 n_sin: int = 8, n_blobs: int = 20, base: float = 512.0):
        self.width, self.height = int(width), int(height)
        rng = np.random.Generator(np.random.PCG64(seed))
        period = np.exp(rng.uniform(math.log(4.0), math.log(256.0), n_sin))
        angle = rng.uniform(0.0, math.pi, n_sin)
        phase = rng.uniform(0.0, 2.0 * math.pi, n_sin)
        amp = rng.uniform(20.0, 80.0, n_sin)
        bx = rng.uniform(0.0, width, n_blobs)
        by = rng.uniform(0.0, height, n_blobs)
        bsig = rng.uniform(8.0, 200.0, n_blobs)
        bamp = rng.uniform(50.0, 300.0, n_blobs)
        bspeed = rng.uniform(0.0, drift_max, n_blobs) if drift_max > 0 else np.zeros(n_blobs)
        bhead = rng.uniform(0.0, 2.0 * math.pi, n_blobs)
        self.blobs = []
        for i in range(n_blobs):
            rad = int(math.ceil(3.0 * bsig[i]))
            noise = rng.uniform(-1.0, 1.0, (2 * rad + 1, 2 * rad + 1))
            yy, xx = np.mgrid[-rad:rad + 1, -rad:rad + 1]
            env = np.exp(-(xx * xx + yy * yy) / (2.0 * bsig[i] ** 2))
            patch = (bamp[i] * env * noise).astype(np.float32)
            vx = bspeed[i] * math.cos(bhead[i])
            vy = bspeed[i] * math.sin(bhead[i])
            self.blobs.append((bx[i], by[i], vx, vy, rad, patch))
        # Static sinusoid field, float32, computed once per sequence.
        ys = np.arange(height, dtype=np.float64)[:, None]
        xs = np.arange(width, dtype=np.float64)[None, :]
        fld = np.full((height, width), base, dtype=np.float64)
        for k in range(n_sin):
            arg = (xs * math.cos(angle[k]) + ys * math.sin(angle[k])) * (2.0 * math.pi / period[k])
            fld += amp[k] * np.sin(arg + phase[k])
        self.base = fld.astype(np.float32)

    def frame(self, f: int = 0) -> np.ndarray:
        h, w = self.height, self.width
        img = self.base.copy()
        for (bx, by, vx, vy, rad, patch) in self.blobs:
            cx = int(round(bx + f * vx))
            cy = int(round(by + f * vy))
            x0, y0 = cx - rad, cy - rad
            x1, y1 = cx + rad + 1, cy + rad + 1
            sx0, sy0 = max(x0, 0), max(y0, 0)
            sx1, sy1 = min(x1, w), min(y1, h)
            if sx0 >= sx1 or sy0 >= sy1:
                continue
            img[sy0:sy1, sx0:sx1] += patch[sy0 - y0:sy1 - y0, sx0 - x0:sx1 - x0]
        np.rint(img, out=img)
        np.clip(img, 0.0, 1023.0, out=img)
        return img.astype(np.uint16)


def make_frame(width: int, height: int, seed: int) -> np.ndarray:
    """A single still frame (frame 0 of a non-drifting sequence)."""
    return SequenceGenerator(width, height, seed).frame(0)


def ar1_eps(n_ctu: int, n_frames: int, seed: int, rho: float = 0.8,
            sigma: float = 0.3) -> np.ndarray:
    """AR(1) log-noise per CTU, shape (n_frames, n_ctu); marginal N(0, sigma^2)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    eps = np.empty((n_frames, n_ctu), dtype=np.float64)
    eps[0] = rng.normal(0.0, sigma, n_ctu)
    s = math.sqrt(1.0 - rho * rho)
    for f in range(1, n_frames):
        eps[f] = rho * eps[f - 1] + s * rng.normal(0.0, sigma, n_ctu)
    return eps


def ctu_times(tex: np.ndarray, eps: np.ndarray, a: float = 200.0, b: float = 3.0) -> np.ndarray:
    """Synthetic measured CTU times in microseconds: round((a + b tex) e^eps), uint32."""
    t = np.rint((a + b * np.asarray(tex, dtype=np.float64)) * np.exp(eps))
    return np.clip(t, 1, 2**31 - 1).astype(np.uint32)


# Workload configurations (sizes, thread budgets and search bounds).
CONFIGS = {
    "fhd_n4": dict(width=1920, height=1080, frames=1, n_threads=4, max_tile_cols=3,
                   max_tile_rows=3, max_rs_per_tile=2, lam=(0, 1), seed=1, drift=0.0),
    "uhd_n8": dict(width=3840, height=2160, frames=64, n_threads=8, max_tile_cols=6,
                   max_tile_rows=4, max_rs_per_tile=4, lam=(1, 10), seed=2, drift=8.0),
    "8k_n16": dict(width=7680, height=4320, frames=32, n_threads=16, max_tile_cols=8,
                   max_tile_rows=6, max_rs_per_tile=4, lam=(1, 10), seed=3, drift=8.0),
}


# Search bounds per thread budget (tile columns, tile rows, slices per tile) and the lambda
# chosen per (resolution, N): Table 1 picks lambda per resolution and thread count; 16
# threads take the 12-thread choice.
BOUNDS = {4: (3, 3, 2), 8: (6, 4, 4), 16: (8, 6, 4)}
LAMBDA = {("fhd", 4): (0, 1), ("fhd", 8): (3, 10), ("fhd", 16): (1, 10),
          ("uhd", 4): (0, 1), ("uhd", 8): (1, 10), ("uhd", 16): (1, 10),
          ("8k", 4): (0, 1), ("8k", 8): (1, 10), ("8k", 16): (1, 10)}
SIZES = {"fhd": (1920, 1080), "uhd": (3840, 2160), "8k": (7680, 4320)}


def batch_workload(n_frames: int = 512, seed: int = 4, mix=(1, 2, 1)):
    """The mixed batch: sizes in proportion fhd:uhd:8k = mix, in seeded order, and a thread
    budget drawn from {4, 8, 16} per frame.

    Returns a list of (size, index_within_size, N).  Frame i of a size is frame i of that
    size's drifting sequence (generator seed `seed` * 10 + size number, drift 8 px/frame).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    tot = sum(mix)
    counts = [n_frames * m // tot for m in mix]
    counts[1] += n_frames - sum(counts)
    names = ["fhd"] * counts[0] + ["uhd"] * counts[1] + ["8k"] * counts[2]
    order = rng.permutation(len(names))
    ns = rng.choice([4, 8, 16], size=n_frames)
    seen = {"fhd": 0, "uhd": 0, "8k": 0}
    out = []
    for i, k in enumerate(order):
        name = names[k]
        out.append((name, seen[name], int(ns[i])))
        seen[name] += 1
    return out


def batch_sequence_seed(name: str, seed: int = 4) -> int:
    return seed * 10 + ["fhd", "uhd", "8k"].index(name)


class TorchSequenceGenerator:
    """SequenceGenerator's sequence rendered on a torch device (for bulk training data).

    The random draws are those of SequenceGenerator (same generator, same order); the
    sinusoid field is evaluated on the device in float64, so frames agree with
    SequenceGenerator's up to the rounding of that field.
    """

    def __init__(self, width: int, height: int, seed: int, drift_max: float = 0.0,
                 device="cuda", n_sin: int = 8, n_blobs: int = 20, base: float = 512.0):
        import torch
        self.width, self.height, self.device = int(width), int(height), device
        rng = np.random.Generator(np.random.PCG64(seed))
        period = np.exp(rng.uniform(math.log(4.0), math.log(256.0), n_sin))
        angle = rng.uniform(0.0, math.pi, n_sin)
        phase = rng.uniform(0.0, 2.0 * math.pi, n_sin)
        amp = rng.uniform(20.0, 80.0, n_sin)
        bx = rng.uniform(0.0, width, n_blobs)
        by = rng.uniform(0.0, height, n_blobs)
        bsig = rng.uniform(8.0, 200.0, n_blobs)
        bamp = rng.uniform(50.0, 300.0, n_blobs)
        bspeed = rng.uniform(0.0, drift_max, n_blobs) if drift_max > 0 else np.zeros(n_blobs)
        bhead = rng.uniform(0.0, 2.0 * math.pi, n_blobs)
        self.blobs = []
        for i in range(n_blobs):
            rad = int(math.ceil(3.0 * bsig[i]))
            noise = torch.from_numpy(rng.uniform(-1.0, 1.0, (2 * rad + 1, 2 * rad + 1))).to(device)
            r = torch.arange(-rad, rad + 1, dtype=torch.float64, device=device)
            env = torch.exp(-(r[None, :] ** 2 + r[:, None] ** 2) / (2.0 * bsig[i] ** 2))
            patch = (bamp[i] * env * noise).to(torch.float32)
            self.blobs.append((bx[i], by[i], bspeed[i] * math.cos(bhead[i]),
                               bspeed[i] * math.sin(bhead[i]), rad, patch))
        ys = torch.arange(height, dtype=torch.float64, device=device)[:, None]
        xs = torch.arange(width, dtype=torch.float64, device=device)[None, :]
        fld = torch.full((height, width), base, dtype=torch.float64, device=device)
        for k in range(n_sin):
            arg = (xs * math.cos(angle[k]) + ys * math.sin(angle[k])) * (2.0 * math.pi / period[k])
            fld += amp[k] * torch.sin(arg + phase[k])
        self.base = fld.to(torch.float32)

    def frame(self, f: int = 0):
        """Frame f as an int16 tensor [height, width] holding 10-bit values."""
        import torch
        h, w = self.height, self.width
        img = self.base.clone()
        for (bx, by, vx, vy, rad, patch) in self.blobs:
            cx = int(round(bx + f * vx))
            cy = int(round(by + f * vy))
            x0, y0 = cx - rad, cy - rad
            x1, y1 = cx + rad + 1, cy + rad + 1
            sx0, sy0 = max(x0, 0), max(y0, 0)
            sx1, sy1 = min(x1, w), min(y1, h)
            if sx0 >= sx1 or sy0 >= sy1:
                continue
            img[sy0:sy1, sx0:sx1] += patch[sy0 - y0:sy1 - y0, sx0 - x0:sx1 - x0]
        return torch.clamp(torch.round(img), 0.0, 1023.0).to(torch.int16)
