"""Pins for the exact search over the literal candidate space (every CTU boundary allowed),
which the oracle solves by decomposition (area windows, tiles, column strips, columns) instead
of listing the candidates (CPU only).

Pinned against the plain definition: the oracle's exhaustive two-step search run on the same
literal space (dtile = drs = -1), itself pinned to the pure-Python brute force, wherever that
finishes; and against properties that hold at any size (the chosen partition tiles the frame,
passes the area rule and the Eq. 4 bound, and scores what is reported; the literal optimum is
never worse than the optimum over the smaller ladder space)."""
import numpy as np
import pytest

from paper_2012_14792_amd import synth

LAMS = [(0, 1), (1, 10), (3, 10), (-1, 1)]


def _inputs(orc, w, h, seed):
    luma = synth.make_frame(w, h, seed)
    f = orc.features(luma)
    W, H = orc.ctu_dims(w, h)
    prev = synth.ctu_times(f["tex"], synth.ar1_eps(W * H, 1, seed + 1000)[0])
    cost, _ = orc.cost_map(f["tex"], prev)
    return luma, f, cost


def _check_partition(orc, w, h, f, cost, p, d):
    """The partition tiles the frame, passes the area rule, respects the Eq. 4 bound, and its
    RS times and Q recomputed from the per-CTU arrays equal the reported ones."""
    W, H = orc.ctu_dims(w, h)
    cover = np.zeros((H, W), np.int32)
    cw = [min(128, w - 128 * x) for x in range(W)]
    rh = [min(128, h - 128 * y) for y in range(H)]
    T = np.asarray(cost, np.int64).reshape(H, W)
    S1 = np.asarray(f["s1"], np.int64).reshape(H, W)
    S2 = np.asarray(f["s2"], np.uint64).astype(object).reshape(H, W)
    areas, q, times = [], 0, []
    for (x0, y0, x1, y1) in d["rs"]:
        cover[y0:y1, x0:x1] += 1
        a = sum(cw[x0:x1]) * sum(rh[y0:y1])
        s1 = int(S1[y0:y1, x0:x1].sum())
        s2 = sum(int(v) for v in S2[y0:y1, x0:x1].ravel())
        areas.append(a)
        q += s2 - (s1 * s1) // a
        times.append(int(T[y0:y1, x0:x1].sum()))
    assert (cover == 1).all()
    assert len(d["rs"]) == p.n_threads == d["n_rs"]
    assert d["tile_cols"] <= p.max_tile_cols and d["tile_rows"] <= p.max_tile_rows
    if p.area_k:
        assert p.area_k * min(areas) > max(areas)
    assert times == d["rs_time"] and max(times) == d["t_sel"] and q == d["q_sel"]
    if p.lambda_num >= 0:
        assert d["t_sel"] * p.lambda_den <= d["t_min"] * (p.lambda_den + p.lambda_num)


@pytest.mark.parametrize("w,h,N,C,R,K,seed", [(640, 512, 3, 3, 3, 2, 0), (768, 600, 4, 3, 3, 2, 1),
                                              (1024, 768, 5, 3, 3, 3, 3), (1920, 1080, 4, 3, 3, 2, 1),
                                              (896, 640, 6, 3, 3, 3, 4), (1280, 768, 8, 4, 3, 4, 5)])
@pytest.mark.parametrize("lam", LAMS)
@pytest.mark.parametrize("area_k", [3, 0, 2])
def test_matches_exhaustive_search_of_the_literal_space(orc, w, h, N, C, R, K, seed, lam, area_k):
    luma, f, cost = _inputs(orc, w, h, seed)
    p = orc.make_params(N, C, R, K, area_k=area_k, lam=lam, dtile=-1, drs=-1)
    e = orc.search(w, h, p, cost, f["s1"], f["s2"])
    d = orc.literal_search(w, h, p, cost, f["s1"], f["s2"])
    assert d["n_enumerated"] == e["n_enumerated"]
    assert (d["status"], d["t_min"], d["t_sel"], d["q_sel"]) == (e["status"], e["t_min"], e["t_sel"], e["q_sel"])
    assert (d["t_unif"], d["q_unif"]) == (e["t_unif"], e["q_unif"])
    # the optimum is a unique set of rectangles on these frames (equal rectangle sets may come
    # from different tile grids: one tile of k slices or k tiles of one slice)
    assert sorted(d["rs"]) == sorted(e["rs"])
    if d["status"] == 0:
        _check_partition(orc, w, h, f, cost, p, d)
    assert d["rank"] == -1 and d["n_feasible"] == -1


def test_matches_brute_force_directly(orc):
    from fractions import Fraction

    from oracle import brute
    w, h = 768, 600
    luma, f, cost = _inputs(orc, w, h, 2)
    p = orc.make_params(4, 3, 3, 2, lam=(1, 10), dtile=-1, drs=-1)
    d = orc.literal_search(w, h, p, cost, f["s1"], f["s2"])
    b = brute.brute_search(luma, cost, 128, 4, 3, 3, 2, lam=Fraction(1, 10))
    assert (d["t_min"], d["t_sel"], d["q_sel"]) == (b["t_min"], b["t_sel"], b["q_sel"])
    assert sorted(d["rs"]) == sorted(b["rs"])


@pytest.mark.parametrize("w,h,N,C,R,K,seed", [(1920, 1080, 8, 6, 4, 4, 1), (2560, 1440, 8, 6, 4, 4, 2)])
def test_literal_optimum_is_never_worse_than_the_ladder(orc, w, h, N, C, R, K, seed):
    """The ladder space is a subset of the literal space: T~min can only drop, and with
    lambda = inf the chosen Q can only drop."""
    luma, f, cost = _inputs(orc, w, h, seed)
    for lam in [(1, 10), (-1, 1)]:
        lit = orc.make_params(N, C, R, K, lam=lam, dtile=-1, drs=-1)
        d = orc.literal_search(w, h, lit, cost, f["s1"], f["s2"])
        e = orc.search(w, h, orc.make_params(N, C, R, K, lam=lam), cost, f["s1"], f["s2"])
        assert e["n_enumerated"] < d["n_enumerated"]
        assert d["t_min"] <= e["t_min"]
        if lam[0] < 0:
            assert d["q_sel"] <= e["q_sel"]
        _check_partition(orc, w, h, f, cost, lit, d)


def test_no_feasible_partition_returns_the_uniform_grid(orc):
    w, h = 896, 640
    luma, f, cost = _inputs(orc, w, h, 4)
    p = orc.make_params(6, 3, 3, 3, area_k=2, dtile=-1, drs=-1)
    d = orc.literal_search(w, h, p, cost, f["s1"], f["s2"])
    e = orc.search(w, h, p, cost, f["s1"], f["s2"])
    assert d["status"] == e["status"] == 1 and d["t_min"] == -1
    assert d["rs"] == e["rs"] and (d["t_sel"], d["q_sel"]) == (e["t_unif"], e["q_unif"])


def test_rejects_what_it_does_not_cover(orc):
    luma, f, cost = _inputs(orc, 640, 512, 0)
    for kw in (dict(prune=1), dict(min_rs=1)):
        p = orc.make_params(3, 3, 3, 2, dtile=-1, drs=-1, **kw)
        with pytest.raises(ValueError):
            orc.literal_search(640, 512, p, cost, f["s1"], f["s2"])


@pytest.mark.parametrize("w,h,N,C,R,K,seed", [(384, 512, 3, 2, 3, 2, 0), (512, 640, 4, 3, 3, 2, 1),
                                              (640, 512, 3, 3, 2, 2, 2), (384, 768, 4, 2, 4, 2, 3),
                                              (512, 512, 2, 2, 3, 2, 4)])
@pytest.mark.parametrize("lam", [(0, 1), (1, 10), (-1, 1)])
@pytest.mark.parametrize("area_k", [3, 0])
def test_spanning_blocks_match_brute_force(orc, w, h, N, C, R, K, seed, lam, area_k):
    """RS that may also be blocks of complete tiles stacked in one tile column: the oracle's DP
    (blocks as one more choice in the strip DP) against the brute force, which lists every
    covering of every tile column; the count of the space is checked against the list."""
    from fractions import Fraction

    from oracle import brute
    luma, f, cost = _inputs(orc, w, h, seed)
    p = orc.make_params(N, C, R, K, area_k=area_k, lam=lam, dtile=-1, drs=-1, span_tiles=1)
    d = orc.literal_search(w, h, p, cost, f["s1"], f["s2"])
    b = brute.brute_spanning(luma, cost, 128, N, C, R, K, lam=None if lam[0] < 0 else Fraction(*lam),
                             area_k=area_k)
    assert d["n_enumerated"] == b["n_enumerated"]
    if b["rank"] is None:
        assert d["status"] == 1
        return
    assert (d["t_min"], d["t_sel"], d["q_sel"]) == (b["t_min"], b["t_sel"], b["q_sel"])
    assert sorted(d["rs"]) == sorted(b["rs"])
    assert d["n_rs"] == N


def test_spanning_blocks_widen_the_space(orc):
    """Blocks only add candidates: T~min cannot rise; on this frame it falls (a tall tile column
    is one RS while its neighbour is cut at a row boundary the first one does not need)."""
    w, h = 384, 768
    luma, f, cost = _inputs(orc, w, h, 3)
    plain = orc.literal_search(w, h, orc.make_params(4, 2, 4, 2, dtile=-1, drs=-1), cost, f["s1"], f["s2"])
    span = orc.literal_search(w, h, orc.make_params(4, 2, 4, 2, dtile=-1, drs=-1, span_tiles=1), cost,
                              f["s1"], f["s2"])
    assert span["n_enumerated"] > plain["n_enumerated"]
    assert span["t_min"] < plain["t_min"]
    bd = span["row_bd"]
    assert any(any(r[1] < y < r[3] for y in bd) for r in span["rs"])    # an RS across a row boundary
