"""The synthetic speed-up analog (Section 3.2, Eq. 5 and Eq. 6) on the host: the Amdahl bound
against the values the paper prints, closed forms of the sequence speed-up, and the uniform
grid against the library's own decode of the uniform rank."""
import json
import os

import numpy as np
import pytest

from paper_2012_14792_amd import binding as B
from paper_2012_14792_amd import speedup as SP

HERE = os.path.dirname(os.path.abspath(__file__))


def test_sigma_max_matches_printed_bounds():
    g = json.load(open(os.path.join(HERE, "golden", "amdahl_eq6.json")))
    for n, ref in zip(g["n"], g["sigma_max"]):
        assert round(SP.sigma_max(n, g["s"]), g["printed_decimals"]) == ref
    assert SP.sigma_max(8, 0.0) == 8.0 and SP.sigma_max(8, 1.0) == 1.0


@pytest.mark.parametrize("n", [4, 8, 16])
def test_balanced_partition_reaches_the_bound(n):
    # n equal regions of equal CTU times: sigma = n, and with a sequential share s the
    # sequence speed-up equals Eq. 6 exactly
    t = np.full((4, 4 * n), 7, dtype=np.int64)
    rects = [(4 * i, 0, 4 * i + 4, 4) for i in range(n)]
    assert SP.sequence_speedup([rects] * 3, [t] * 3) == pytest.approx(n, rel=1e-12)
    assert SP.sequence_speedup([rects] * 3, [t] * 3, 0.04) == pytest.approx(SP.sigma_max(n, 0.04), rel=1e-12)


def test_unbalanced_sequence_by_hand():
    # frame 1: regions 6 and 2 (total 8, parallel 6); frame 2: regions 3 and 5 (total 8, parallel 5)
    t1 = np.array([[1, 2, 1], [1, 2, 1]], dtype=np.int64)
    t2 = np.array([[1, 1, 3], [1, 0, 2]], dtype=np.int64)
    r1 = [(0, 0, 2, 2), (2, 0, 3, 2)]
    r2 = [(0, 0, 2, 2), (2, 0, 3, 2)]
    assert SP.region_times(r1, t1) == [6, 2] and SP.region_times(r2, t2) == [3, 5]
    assert SP.sequence_speedup([r1, r2], [t1, t2]) == pytest.approx(16 / 11)
    assert SP.sequence_speedup([r1, r2], [t1, t2], 0.5) == pytest.approx(16 / (8 + 5.5))


@pytest.mark.parametrize("wh,n", [((1920, 1080), 4), ((3840, 2160), 8), ((7680, 4320), 16), ((1920, 1080), 6)])
def test_uniform_grid_matches_library_decode(wh, n):
    w, h = wh
    frame = B.make_frame(w, h)
    C, R, K = {4: (3, 3, 2), 6: (3, 3, 2), 8: (6, 4, 4), 16: (8, 6, 4)}[n]
    params = B.make_params(n, C, R, K)
    W, H = B.ctu_dims(frame)
    stats = B.trs_search_stats(frame, params)
    assert stats["candidates"] > 0
    ref = SP.uniform_rects(W, H, n)
    # the uniform grid's rank (from the oracle) decodes, in the library, to the same rectangles
    res = B.trs_decode(frame, params, _uniform_rank(frame, params))
    assert [tuple(r) for r in res["rs"]] == ref


def _uniform_rank(frame, params):
    import oracle
    W, H = B.ctu_dims(frame)
    op = oracle.make_params(params.n_threads, params.max_tile_cols, params.max_tile_rows,
                            params.max_rs_per_tile)
    flat = np.zeros(W * H, dtype=np.uint32)
    r = oracle.search(frame.width, frame.height, op, flat + 1, flat, flat.astype(np.uint64))
    return r["uniform_rank"]
