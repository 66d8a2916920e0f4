"""Pins for the oracle's per-CTU features and cost map (CPU only).

Each check comes from something other than the oracle's own formula: closed forms on
constructed frames, the textbook definitions of mean and population variance evaluated
with exact rationals, and a pixel-by-pixel Python recount.
"""
from fractions import Fraction

import numpy as np
import pytest

from oracle import brute
from paper_2012_14792_amd import synth


def _blocks(luma, cs):
    h, w = luma.shape
    W, H = (w + cs - 1) // cs, (h + cs - 1) // cs
    for cy in range(H):
        for cx in range(W):
            yield cy * W + cx, luma[cy * cs:(cy + 1) * cs, cx * cs:(cx + 1) * cs]


@pytest.mark.parametrize("v", [0, 1, 511, 1023])
def test_constant_frame(orc, v):
    luma = np.full((300, 260), v, dtype=np.uint16)       # partial CTUs on both edges
    f = orc.features(luma)
    for c, blk in _blocks(luma, 128):
        n = blk.size
        assert f["s1"][c] == v * n
        assert f["s2"][c] == v * v * n
        assert f["grad"][c] == 0 and f["tex"][c] == 0 and f["var"][c] == 0
        assert f["mean"][c] == v


def test_horizontal_ramp_gradient(orc):
    # p(x, y) = x: every horizontal forward difference is 1, vertical ones are 0.
    w, h = 300, 200
    luma = np.tile(np.arange(w, dtype=np.uint16), (h, 1))
    f = orc.features(luma)
    W = 3
    for cy in range(2):
        for cx in range(3):
            cw = min(128, w - 128 * cx)
            ch = min(128, h - 128 * cy)
            # columns x with x + 1 < w contribute 1 each
            cols = cw if cx < W - 1 else cw - 1
            assert f["grad"][cy * W + cx] == cols * ch


def test_vertical_ramp_gradient(orc):
    w, h = 200, 300
    luma = np.tile(np.arange(h, dtype=np.uint16)[:, None], (1, w))
    f = orc.features(luma)
    W = 2
    for cy in range(3):
        for cx in range(2):
            cw = min(128, w - 128 * cx)
            ch = min(128, h - 128 * cy)
            rows = ch if cy < 2 else ch - 1
            assert f["grad"][cy * W + cx] == rows * cw


def test_checkerboard_gradient_is_maximal(orc):
    w, h = 256, 256
    yy, xx = np.mgrid[0:h, 0:w]
    luma = np.where((xx + yy) % 2 == 0, 0, 1023).astype(np.uint16)
    f = orc.features(luma)
    # every forward difference inside the frame has magnitude 1023
    # CTU (0,0): 128*128 horizontal terms, 128*128 vertical terms (neighbours exist)
    assert f["grad"][0] == 1023 * 2 * 128 * 128
    # CTU (1,1): last column/row have no right/bottom neighbour
    assert f["grad"][3] == 1023 * (127 * 128 + 128 * 127)


def test_gradient_uses_halo_across_ctu_boundary(orc):
    # A step edge exactly on the CTU boundary x = 128 is charged to the left CTU.
    luma = np.zeros((128, 256), dtype=np.uint16)
    luma[:, 128:] = 1000
    f = orc.features(luma)
    assert f["grad"][0] == 1000 * 128
    assert f["grad"][1] == 0


@pytest.mark.parametrize("seed,w,h,cs", [(0, 300, 260, 128), (1, 200, 136, 64), (2, 130, 70, 32)])
def test_mean_variance_texture_definitions(orc, seed, w, h, cs):
    luma = synth.make_frame(w, h, seed)
    f = orc.features(luma, cs)
    n_px, s1, s2, g = brute.ctu_stats_pixels(luma, cs)
    W = (w + cs - 1) // cs
    for c, blk in _blocks(luma, cs):
        vals = [int(v) for v in blk.ravel()]
        n = len(vals)
        mu = Fraction(sum(vals), n)
        pop_var = sum((Fraction(v) - mu) ** 2 for v in vals) / n   # textbook definition
        assert f["mean"][c] == int(mu)                               # floor (non-negative)
        assert f["var"][c] == int(pop_var)
        cy, cx = divmod(c, W)
        assert f["s1"][c] == s1[cy][cx] and f["s2"][c] == s2[cy][cx]
        assert f["grad"][c] == g[cy][cx]
        assert f["tex"][c] == g[cy][cx] // n_px[cy][cx]


def test_cost_map_identity_and_texture_model(orc):
    rng = np.random.default_rng(7)
    tex = rng.integers(0, 400, 135).astype(np.uint32)
    prev = rng.integers(1, 5000, 135).astype(np.uint32)
    c, rc = orc.cost_map(tex, prev, 200, 3, 256)      # the paper's co-located estimator
    assert rc == 0 and np.array_equal(c, prev)
    c, rc = orc.cost_map(tex, prev, 200, 3, 0)        # pure texture model
    assert rc == 0 and np.array_equal(c, 200 + 3 * tex)
    c, rc = orc.cost_map(tex, None, 17, 5, 128)       # no previous frame: model only
    assert rc == 0 and np.array_equal(c, 17 + 5 * tex)


def test_cost_map_blend_rounding(orc):
    # w = 64: (64 * 1000 + 192 * (200 + 3 * 10) + 128) / 256 = (64000 + 44160 + 128) / 256 = 423.0
    # w = 1 :  (1 * 7 + 255 * 200 + 128) / 256 = 51135 / 256 = 199.74 -> 199
    tex = np.array([10, 0], dtype=np.uint32)
    prev = np.array([1000, 7], dtype=np.uint32)
    c, _ = orc.cost_map(tex[:1], prev[:1], 200, 3, 64)
    assert c[0] == 423
    c, _ = orc.cost_map(tex[1:], prev[1:], 200, 3, 1)
    assert c[0] == 199


def test_cost_map_overflow_guard(orc):
    tex = np.array([2**31], dtype=np.uint32)
    c, rc = orc.cost_map(tex, None, 0, 1, 256)
    assert rc == -2 and c[0] == 2**31 - 1
    c, rc = orc.cost_map(np.array([1], np.uint32), None, 2**31 - 1, 0, 256)
    assert rc == 0 and c[0] == 2**31 - 1
