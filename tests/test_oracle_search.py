"""Pins for the oracle's two-step TRS search (CPU only).

What pins it, none of which re-types the oracle's own code:
  * an independent pure-Python brute force (itertools enumeration sorted by the canonical
    key, direct sums over CTUs and pixels) on tiny grids and on the 1080p / N = 4 workload;
  * textbook special cases: with a single tile column and row, no area rule and one RS per
    CTU-row band, step 1 is the linear-partition (painter's) problem and step 2 with
    lambda = inf is the optimal contiguous k-segmentation under SSE, both solved here by DP;
  * an independent generating-polynomial count of the candidate space;
  * invariants that hold for any frame (Eq. 1 sums, Eq. 4 bound, monotonicity in lambda).
"""
from fractions import Fraction
import functools

import numpy as np
import pytest

from oracle import brute
from paper_2012_14792_amd import synth

LAMS = [(0, 1), (1, 10), (3, 10), (-1, 1)]


def _inputs(orc, w, h, seed, cs=128, flat=None):
    luma = synth.make_frame(w, h, seed) if flat is None else np.full((h, w), flat, np.uint16)
    f = orc.features(luma, cs)
    W, H = orc.ctu_dims(w, h, cs)
    eps = synth.ar1_eps(W * H, 1, seed + 1000)[0]
    prev = synth.ctu_times(f["tex"], eps)
    cost, rc = orc.cost_map(f["tex"], prev)
    assert rc == 0
    return luma, f, cost


def _frac(lam):
    return None if lam[0] < 0 else Fraction(*lam)


@pytest.mark.parametrize("w,h,N,seed", [(640, 512, 3, 0), (640, 512, 3, 5), (768, 600, 4, 1),
                                        (768, 600, 4, 2), (512, 640, 4, 3), (896, 384, 5, 4)])
@pytest.mark.parametrize("lam", LAMS)
def test_matches_brute_force_tiny(orc, w, h, N, seed, lam):
    luma, f, cost = _inputs(orc, w, h, seed)
    p = orc.make_params(N, 3, 3, 2, lam=lam)
    o = orc.search(w, h, p, cost, f["s1"], f["s2"])
    b = brute.brute_search(luma, cost, 128, N, 3, 3, 2, lam=_frac(lam))
    assert o["n_enumerated"] == b["n_enumerated"]
    assert o["n_feasible"] == b["n_feasible"]
    if b["rank"] is None:
        assert o["status"] == 1
        return
    assert (o["rank"], o["t_min"], o["t_sel"], o["q_sel"]) == (b["rank"], b["t_min"], b["t_sel"], b["q_sel"])
    assert o["rs"] == b["rs"]


def test_matches_brute_force_windows(orc):
    # fixed windows instead of the literal space
    w, h = 1024, 768
    luma, f, cost = _inputs(orc, w, h, 11)
    for dt, dr in [(1, 0), (2, 1), (0, 0)]:
        p = orc.make_params(4, 3, 3, 2, lam=(1, 10), dtile=dt, drs=dr)
        o = orc.search(w, h, p, cost, f["s1"], f["s2"])
        b = brute.brute_search(luma, cost, 128, 4, 3, 3, 2, lam=Fraction(1, 10), dt=dt, dr=dr)
        assert o["n_enumerated"] == b["n_enumerated"] and o["n_feasible"] == b["n_feasible"]
        assert (o["rank"], o["t_min"], o["q_sel"], o["rs"]) == (b["rank"], b["t_min"], b["q_sel"], b["rs"])


def test_matches_brute_force_fhd_n4(orc):
    """The 1080p, 4-thread workload: 3,416 candidates, brute force end to end."""
    cfg = synth.CONFIGS["fhd_n4"]
    w, h = cfg["width"], cfg["height"]
    luma, f, cost = _inputs(orc, w, h, cfg["seed"])
    for lam in [(0, 1), (-1, 1)]:
        p = orc.make_params(4, 3, 3, 2, lam=lam)
        o = orc.search(w, h, p, cost, f["s1"], f["s2"])
        b = brute.brute_search(luma, cost, 128, 4, 3, 3, 2, lam=_frac(lam))
        assert o["n_enumerated"] == b["n_enumerated"] == 3416
        assert o["n_feasible"] == b["n_feasible"]
        assert (o["rank"], o["t_min"], o["t_sel"], o["q_sel"], o["rs"]) == \
            (b["rank"], b["t_min"], b["t_sel"], b["q_sel"], b["rs"])


# ---- textbook special cases -------------------------------------------------------------

def _painter_dp(rows, k):
    """min over contiguous k-segmentations of the max segment sum (linear partition)."""
    n = len(rows)
    pre = [0]
    for v in rows:
        pre.append(pre[-1] + v)

    @functools.lru_cache(None)
    def best(i, k):            # rows i..n-1 into k non-empty segments
        if k == 1:
            return pre[n] - pre[i]
        return min(max(pre[j] - pre[i], best(j, k - 1)) for j in range(i + 1, n - k + 2))
    return best(0, k)


def _sse_dp(n_rows, s1_rows, s2_rows, k):
    """min over contiguous k-segmentations of sum of ceil(SSE) (Fisher / Bellman)."""
    m = len(s1_rows)

    def seg(i, j):
        n = sum(n_rows[i:j])
        a = sum(s1_rows[i:j])
        return sum(s2_rows[i:j]) - (a * a) // n

    @functools.lru_cache(None)
    def best(i, k):
        if k == 1:
            return seg(i, m)
        return min(seg(i, j) + best(j, k - 1) for j in range(i + 1, m - k + 2))
    return best(0, k)


@pytest.mark.parametrize("seed,N", [(0, 2), (1, 3), (2, 5), (3, 8)])
def test_single_tile_reduces_to_linear_partition_and_segmentation(orc, seed, N):
    w, h = 1280, 1280          # 10 x 10 CTUs, one tile, N full-width bands
    luma, f, cost = _inputs(orc, w, h, seed)
    W = H = 10
    T = np.asarray(cost, dtype=np.int64).reshape(H, W)
    S1 = np.asarray(f["s1"], dtype=object).reshape(H, W)
    S2 = np.asarray(f["s2"], dtype=object).reshape(H, W)
    rows_t = [int(v) for v in T.sum(axis=1)]
    rows_1 = [int(sum(S1[y])) for y in range(H)]
    rows_2 = [int(sum(S2[y])) for y in range(H)]
    rows_n = [128 * w] * H
    p = orc.make_params(N, 1, 1, N, area_k=0, lam=(0, 1), dtile=-1, drs=-1)
    o = orc.search(w, h, p, cost, f["s1"], f["s2"])
    assert o["t_min"] == _painter_dp(rows_t, N)
    p = orc.make_params(N, 1, 1, N, area_k=0, lam=(-1, 1), dtile=-1, drs=-1)
    o = orc.search(w, h, p, cost, f["s1"], f["s2"])
    assert o["q_sel"] == _sse_dp(rows_n, rows_1, rows_2, N)
    import math
    assert o["n_enumerated"] == math.comb(H - 1, N - 1)


# ---- independent count of the candidate space --------------------------------------------

def _count_space(W, H, N, Cm, Rm, Km, dt, dr):
    """Generating-polynomial count; windows as in the space definition (None = unbounded)."""
    def nvec(L, m, d):
        return len(brute.boundary_vectors(L, m, d)) if m <= L else 0
    tot = 0
    for c in range(1, Cm + 1):
        for r in range(1, Rm + 1):
            if not (c * r <= N <= Km * c * r):
                continue
            nx = nvec(W, c, dt)
            sm = 0
            for Y in (brute.boundary_vectors(H, r, dt) if r <= H else []):
                yb = (0,) + Y + (H,)
                poly = {0: 1}
                for j in range(r):
                    hj = yb[j + 1] - yb[j]
                    P = {k: nvec(hj, k, dr) for k in range(1, min(Km, hj) + 1)}
                    for _ in range(c):
                        q = {}
                        for a, va in poly.items():
                            for k, vk in P.items():
                                if a + k <= N and vk:
                                    q[a + k] = q.get(a + k, 0) + va * vk
                        poly = q
                sm += poly.get(N, 0)
            tot += nx * sm
    return tot


@pytest.mark.parametrize("W,H,N,Cm,Rm,Km", [(15, 9, 4, 3, 3, 2), (30, 17, 8, 6, 4, 4),
                                            (15, 9, 8, 6, 4, 4), (30, 17, 4, 3, 3, 2),
                                            (60, 34, 8, 6, 4, 4)])
def test_space_size_and_ladder(orc, W, H, N, Cm, Rm, Km):
    p = orc.make_params(N, Cm, Rm, Km)
    n, dt, dr = orc.space_size(W, H, p)
    rungs = [(None, None), (3, 1), (2, 1), (1, 1), (1, 0), (0, 0)]
    sizes = []
    for a, b in rungs:
        if a is None and W * H > 300 and N > 4:
            sizes.append(float("inf"))      # literal space: far above the budget
            continue
        sizes.append(_count_space(W, H, N, Cm, Rm, Km, a, b))
    pick = next((i for i, s in enumerate(sizes) if s <= 1 << 24), 5)
    exp_dt, exp_dr = (-1 if rungs[pick][0] is None else rungs[pick][0],
                      -1 if rungs[pick][1] is None else rungs[pick][1])
    assert (dt, dr) == (exp_dt, exp_dr)
    assert n == sizes[pick]


# ---- invariants -------------------------------------------------------------------------

@pytest.mark.parametrize("seed", [0, 1, 2])
def test_invariants(orc, seed):
    w, h = 1920, 1080
    luma, f, cost = _inputs(orc, w, h, seed + 20)
    W, H = 15, 9
    total_t = int(np.asarray(cost, np.int64).sum())
    prev_q = None
    for lam in LAMS:
        p = orc.make_params(4, 3, 3, 2, lam=lam)
        o = orc.search(w, h, p, cost, f["s1"], f["s2"])
        assert o["status"] == 0
        # regions tile the CTU grid exactly once
        cover = np.zeros((H, W), np.int32)
        for (x0, y0, x1, y1) in o["rs"]:
            cover[y0:y1, x0:x1] += 1
        assert (cover == 1).all()
        assert len(o["rs"]) == 4
        assert sum(o["rs_time"]) == total_t          # Eq. 1: region times sum to the frame total
        assert max(o["rs_time"]) == o["t_sel"]
        assert o["t_min"] <= o["t_unif"]               # the uniform grid is a candidate
        if lam[0] == 0:
            assert o["t_sel"] == o["t_min"]
        if lam[0] >= 0:
            assert o["t_sel"] * lam[1] <= o["t_min"] * (lam[1] + lam[0])   # Eq. 4
        if prev_q is not None:
            assert o["q_sel"] <= prev_q                # more freedom never hurts Eq. 2
        prev_q = o["q_sel"]


def test_flat_frame_quality_term_vanishes(orc):
    w, h = 768, 600
    luma, f, cost = _inputs(orc, w, h, 3, flat=700)
    p = orc.make_params(4, 3, 3, 2, lam=(-1, 1))
    o = orc.search(w, h, p, cost, f["s1"], f["s2"])
    b = brute.brute_search(luma, cost, 128, 4, 3, 3, 2, lam=None)
    assert o["q_sel"] == 0
    # Q ties everywhere: the choice is the smallest T, then the smallest rank
    assert o["rank"] == b["rank"]
    assert o["t_sel"] == o["t_min"]


def test_no_feasible_candidate_returns_uniform(orc):
    w, h = 1920, 1080
    luma, f, cost = _inputs(orc, w, h, 4)
    p = orc.make_params(4, 3, 3, 2, area_k=1)   # 1 * A_min > A_max is impossible
    o = orc.search(w, h, p, cost, f["s1"], f["s2"])
    assert o["status"] == 1 and o["n_feasible"] == 0
    assert o["tile_cols"] == 2 and o["tile_rows"] == 2
    assert o["col_bd"] == [0, 7, 15] and o["row_bd"] == [0, 4, 9]
    assert o["rank"] == o["uniform_rank"] >= 0
    assert o["t_sel"] == o["t_unif"] == max(o["rs_time"])


@pytest.mark.parametrize("w,h,N,seed", [(768, 600, 4, 1), (896, 640, 4, 7), (1024, 768, 5, 8)])
@pytest.mark.parametrize("prune", [1, 2, 3])
def test_pruning_rules_match_brute_force(orc, w, h, N, seed, prune):
    """The optional pruning rules (the authors' commented notes): the oracle and the
    independent brute force agree on the feasible set and the decision; each rule only
    removes candidates and both together remove at least what each removes."""
    luma, f, cost = _inputs(orc, w, h, seed)
    counts = {}
    for pr in (0, prune):
        p = orc.make_params(N, 3, 3, 2, lam=(1, 10), prune=pr)
        o = orc.search(w, h, p, cost, f["s1"], f["s2"])
        b = brute.brute_search(luma, cost, 128, N, 3, 3, 2, lam=Fraction(1, 10), prune=pr)
        assert o["n_enumerated"] == b["n_enumerated"] and o["n_feasible"] == b["n_feasible"]
        counts[pr] = o["n_feasible"]
        if b["rank"] is None:
            assert o["status"] == 1
            continue
        assert (o["rank"], o["t_min"], o["t_sel"], o["q_sel"], o["rs"]) == \
            (b["rank"], b["t_min"], b["t_sel"], b["q_sel"], b["rs"])
    assert counts[prune] <= counts[0]
    if prune == 3:
        n1 = orc.search(w, h, orc.make_params(N, 3, 3, 2, prune=1), cost, f["s1"], f["s2"])["n_feasible"]
        n2 = orc.search(w, h, orc.make_params(N, 3, 3, 2, prune=2), cost, f["s1"], f["s2"])["n_feasible"]
        assert counts[3] <= min(n1, n2)


def test_pruning_heights_by_hand():
    """Bit 0 on a hand-checked geometry: 1 x 1 tile grid of a 128 x 640 frame (5 CTU rows),
    4 slices: splits (1, 2, 3) give heights 128, 128, 128, 256 (kept: 256 = 2 x 128), splits
    (1, 2, 4)... every candidate with a slice of 3 rows (384 > 2 x 128) next to a 1-row slice is
    dropped."""
    luma = np.full((640, 128), 100, np.uint16)
    cost = [100] * 5
    all4 = brute.enumerate_candidates(1, 5, 4, 1, 1, 4, None, None)
    kept = []
    for cand in all4:
        rs = brute.regions_of(1, 5, cand)
        if brute.coherent(cand, rs, lambda q: 128 * 128 * (q[3] - q[1]), [128] * 5, 1):
            kept.append(cand[4][0][1])
    # 4 slices in 5 rows: one slice has 2 rows, the others 1 row: 256 <= 2 x 128, all kept
    assert len(all4) == 4 and len(kept) == 4
    all2 = brute.enumerate_candidates(1, 5, 2, 1, 1, 2, None, None)
    kept2 = [c[4][0][1] for c in all2
             if brute.coherent(c, brute.regions_of(1, 5, c), lambda q: 0, [128] * 5, 1)]
    # 2 slices: splits at 1 (1 + 4 rows) and 4 (4 + 1) break the rule, 2 and 3 (2 + 3) keep it
    assert sorted(kept2) == [(2,), (3,)]
    b = brute.brute_search(luma, cost, 128, 2, 1, 1, 2, lam=None, area_k=0, prune=1)
    assert b["n_feasible"] == 2


@pytest.mark.parametrize("wh,N,C,R,K", [((1920, 1080), 4, 3, 3, 2), ((1920, 1080), 8, 6, 4, 4),
                                        ((3840, 2160), 8, 6, 4, 4)])
@pytest.mark.parametrize("prune", [1, 2, 3])
def test_plan_applies_pruning_like_the_oracle(orc, wh, N, C, R, K, prune):
    """The library's plan (host only) keeps exactly the candidates the oracle keeps."""
    from paper_2012_14792_amd import binding as B
    w, h = wh
    frame = B.make_frame(w, h)
    st = B.trs_search_stats(frame, B.make_params(N, C, R, K, prune=prune))
    W, H = orc.ctu_dims(w, h, 128)
    flat = np.zeros(W * H, np.uint32)
    o = orc.search(w, h, orc.make_params(N, C, R, K, prune=prune), flat + 1, flat, flat.astype(np.uint64))
    assert st["feasible"] == o["n_feasible"]
    assert st["candidates"] == o["n_enumerated"]


@pytest.mark.parametrize("w,h,N,lo,seed,prune", [(768, 600, 4, 1, 1, 0), (640, 512, 4, 2, 0, 0),
                                                 (896, 384, 5, 3, 4, 0), (768, 600, 4, 1, 2, 3),
                                                 (1024, 768, 5, 1, 8, 2)])
@pytest.mark.parametrize("lam", [(0, 1), (3, 10), (-1, 1)])
def test_idle_threads_match_brute_force(orc, w, h, N, lo, seed, prune, lam):
    """RS counts in [min_rs, N] (N - n threads idle): the oracle and the independent brute
    force (candidates filtered on their own RS count) agree on the space, the feasible set
    and the decision, with and without the pruning rules (bit 1 compares against the other
    tiles of the candidate's own RS count)."""
    luma, f, cost = _inputs(orc, w, h, seed)
    p = orc.make_params(N, 3, 3, 2, lam=lam, prune=prune, min_rs=lo)
    o = orc.search(w, h, p, cost, f["s1"], f["s2"])
    b = brute.brute_search(luma, cost, 128, N, 3, 3, 2, lam=_frac(lam), prune=prune, n_lo=lo)
    assert o["n_enumerated"] == b["n_enumerated"]
    assert o["n_feasible"] == b["n_feasible"]
    if b["rank"] is None:
        assert o["status"] == 1
        return
    assert (o["rank"], o["t_min"], o["t_sel"], o["q_sel"], o["rs"]) == \
        (b["rank"], b["t_min"], b["t_sel"], b["q_sel"], b["rs"])
    assert o["n_rs"] == len(o["rs"]) and lo <= o["n_rs"] <= N


@pytest.mark.parametrize("W,H,N,C,R,K,dt,dr", [(15, 9, 4, 3, 3, 2, -1, -1), (30, 17, 8, 6, 4, 4, 3, 1),
                                               (60, 34, 16, 8, 6, 4, 1, 0), (8, 8, 6, 3, 3, 3, -1, -1)])
def test_idle_thread_space_is_union_of_exact_spaces(orc, W, H, N, C, R, K, dt, dr):
    """At fixed windows, the space with RS counts in [lo, N] is the disjoint union of the
    exact-count spaces for n = lo .. N (a candidate with n RS has c r <= n <= Kmax c r), so
    the sizes add up; the exact-count sizes come from separate runs with N = n."""
    for lo in sorted({1, max(1, N // 2), N}):
        n_union = orc.space_size(W, H, orc.make_params(N, C, R, K, dtile=dt, drs=dr, min_rs=lo))[0]
        parts = sum(orc.space_size(W, H, orc.make_params(n, C, R, K, dtile=dt, drs=dr))[0]
                    for n in range(lo, N + 1))
        assert n_union == parts


def test_idle_threads_widen_step_one(orc):
    """More candidates can only lower the step-1 minimum: T~min over [lo, N] RS is the
    minimum of the exact-count minima, and the partition chosen with lambda = inf has the
    smallest Q over the union."""
    w, h, N = 1024, 768, 5
    luma, f, cost = _inputs(orc, w, h, 8)
    per_n = [orc.search(w, h, orc.make_params(n, 3, 3, 2, dtile=-1, drs=-1, lam=(-1, 1)),
                        cost, f["s1"], f["s2"]) for n in range(2, N + 1)]
    u = orc.search(w, h, orc.make_params(N, 3, 3, 2, dtile=-1, drs=-1, lam=(-1, 1), min_rs=2),
                   cost, f["s1"], f["s2"])
    feas = [r for r in per_n if r["status"] == 0]
    assert u["t_min"] == min(r["t_min"] for r in feas)
    assert u["q_sel"] == min(r["q_sel"] for r in feas)
    assert u["n_feasible"] == sum(r["n_feasible"] for r in per_n)


def test_idle_threads_on_a_frame_smaller_than_n(orc):
    """A 3 x 2 CTU frame cannot hold 8 RS: the exact space is empty, while with min_rs <= 6
    the space holds partitions into 1..6 RS, and the oracle equals the brute force."""
    w, h = 384, 256
    luma, f, cost = _inputs(orc, w, h, 3)
    assert orc.space_size(3, 2, orc.make_params(8, 3, 2, 2, dtile=-1, drs=-1))[0] == 0
    for lo, size in ((1, 22), (4, 12), (6, 2)):
        p = orc.make_params(8, 3, 2, 2, lam=(1, 10), dtile=-1, drs=-1, min_rs=lo)
        assert orc.space_size(3, 2, p)[0] == size
        o = orc.search(w, h, p, cost, f["s1"], f["s2"])
        b = brute.brute_search(luma, cost, 128, 8, 3, 2, 2, lam=Fraction(1, 10), n_lo=lo)
        assert o["n_enumerated"] == b["n_enumerated"] == size
        assert (o["rank"], o["t_min"], o["q_sel"], o["rs"]) == (b["rank"], b["t_min"], b["q_sel"], b["rs"])
        assert o["n_rs"] == 6


@pytest.mark.parametrize("lam", LAMS)
def test_decision_is_invariant_to_scaling_the_time_map(orc, lam):
    """Multiplying every predicted CTU time by the same integer scales T~min, the Eq. 4 bound
    and every T~(P) alike and leaves Q alone, so the chosen partition does not change."""
    w, h = 1920, 1080
    luma, f, cost = _inputs(orc, w, h, 13)
    p = orc.make_params(4, 3, 3, 2, lam=lam)
    a = orc.search(w, h, p, cost, f["s1"], f["s2"])
    b = orc.search(w, h, p, (np.asarray(cost, np.uint32) * 7).astype(np.uint32), f["s1"], f["s2"])
    assert (b["rank"], b["rs"], b["q_sel"]) == (a["rank"], a["rs"], a["q_sel"])
    assert (b["t_min"], b["t_sel"]) == (7 * a["t_min"], 7 * a["t_sel"])
