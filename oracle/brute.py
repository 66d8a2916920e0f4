"""Pure-Python brute force for tiny TRS problems -- TEST INFRASTRUCTURE ONLY.

Independent of the C oracle: it lists every candidate partition with itertools, orders
them by sorting on the canonical key (shape, X, Y, per-tile (k, Z) choices), and scores
each one with direct sums over pixels / CTUs (no prefix sums), in Python integers.

Definitions followed: Eq. 1 (region time = sum of CTU times, partition time = max over
regions), Eq. 3 (step 1 minimum), Eq. 4 (time bound with lambda), Eq. 2 (within-region luma
SSE, evaluated as sum over regions of S2 - floor(S1^2 / n)), and the area balance rule
k * A_min > A_max of Section 2.3.
"""
from __future__ import annotations

import itertools
from fractions import Fraction

import numpy as np


def ctu_stats_pixels(luma: np.ndarray, cs: int):
    """Per-CTU (n, S1, S2, G) by visiting every pixel, Python ints."""
    h, w = luma.shape
    W, H = (w + cs - 1) // cs, (h + cs - 1) // cs
    L = [[int(v) for v in row] for row in luma.tolist()]
    n = [[0] * W for _ in range(H)]
    s1 = [[0] * W for _ in range(H)]
    s2 = [[0] * W for _ in range(H)]
    g = [[0] * W for _ in range(H)]
    for y in range(h):
        row = L[y]
        nxt = L[y + 1] if y + 1 < h else None
        cy = y // cs
        for x in range(w):
            cx = x // cs
            p = row[x]
            n[cy][cx] += 1
            s1[cy][cx] += p
            s2[cy][cx] += p * p
            if x + 1 < w:
                g[cy][cx] += abs(row[x + 1] - p)
            if nxt is not None:
                g[cy][cx] += abs(nxt[x] - p)
    return n, s1, s2, g


def boundary_vectors(L: int, m: int, d: int | None):
    """All strictly increasing (b_1..b_{m-1}) in [1, L-1], each within d of floor(i L / m)."""
    out = []
    for combo in itertools.combinations(range(1, L), m - 1):
        if d is None or all(abs(b - (i * L) // m) <= d for i, b in enumerate(combo, start=1)):
            out.append(combo)
    return sorted(out)


def enumerate_candidates(W, H, N, Cmax, Rmax, Kmax, dt, dr, n_lo=None):
    """Every candidate as a canonical key, sorted (the sort defines the rank).  The RS count
    of a candidate runs over [n_lo, N] (default: exactly N; fewer RS leave threads idle)."""
    n_lo = N if n_lo is None else n_lo
    cands = []
    for c in range(1, Cmax + 1):
        for r in range(1, Rmax + 1):
            if not any(c * r <= n <= Kmax * c * r for n in range(n_lo, N + 1)):
                continue
            Xs = boundary_vectors(W, c, dt)
            Ys = boundary_vectors(H, r, dt)
            for X in Xs:
                for Y in Ys:
                    yb = (0,) + Y + (H,)
                    per_tile = []
                    for j in range(r):
                        hj = yb[j + 1] - yb[j]
                        opts = []
                        for k in range(1, min(Kmax, hj) + 1):
                            for Z in boundary_vectors(hj, k, dr):
                                opts.append((k, Z))
                        per_tile.extend([opts] * c)
                    for choice in itertools.product(*per_tile):
                        if n_lo <= sum(k for k, _ in choice) <= N:
                            cands.append((c, r, X, Y, choice))
    cands.sort(key=lambda t: (t[0], t[1], t[2], t[3], t[4]))
    return cands


def regions_of(W, H, cand):
    c, r, X, Y, choice = cand
    xb = (0,) + X + (W,)
    yb = (0,) + Y + (H,)
    rs = []
    for j in range(r):
        for i in range(c):
            k, Z = choice[j * c + i]
            zb = (0,) + Z + (yb[j + 1] - yb[j],)
            for q in range(k):
                rs.append((xb[i], yb[j] + zb[q], xb[i + 1], yb[j] + zb[q + 1]))
    return rs


def coherent(cand, rs, area, row_px, prune):
    """The authors' commented pruning notes as rules (pixel units): bit 0, the tallest slice of
    every tile is at most twice its shortest; bit 1, every tile's mean slice area is within
    [1/1.5, 1.5] times the mean slice area of the other tiles (when they hold any slice)."""
    if not prune:
        return True
    choice = cand[4]
    tiles, pos = [], 0
    for k, _ in choice:
        tiles.append(rs[pos:pos + k])
        pos += k
    heights = [[sum(row_px[y] for y in range(q[1], q[3])) for q in t] for t in tiles]
    if prune & 1 and any(max(hs) > 2 * min(hs) for hs in heights):
        return False
    if prune & 2:
        tile_area = [sum(area(q) for q in t) for t in tiles]
        total = sum(tile_area)
        for t, a in zip(tiles, tile_area):
            k, rest = len(t), len(rs) - len(t)
            if rest <= 0:
                continue
            mean_cur, mean_rem = Fraction(a, k), Fraction(total - a, rest)
            if mean_cur > Fraction(3, 2) * mean_rem or mean_cur < mean_rem / Fraction(3, 2):
                return False
    return True


def brute_search(luma, cost, cs, N, Cmax, Rmax, Kmax, lam=Fraction(0), area_k=3,
                 dt=None, dr=None, prune=0, n_lo=None):
    """Returns dict(rank, t_min, t_sel, q_sel, rs, n_enumerated, n_feasible).

    `cost` is the per-CTU time map (raster, length W*H); lam is a Fraction or None (= inf).
    """
    h, w = luma.shape
    W, H = (w + cs - 1) // cs, (h + cs - 1) // cs
    n, s1, s2, _ = ctu_stats_pixels(luma, cs)
    T = [[int(cost[y * W + x]) for x in range(W)] for y in range(H)]
    row_px = [min(cs, h - y * cs) for y in range(H)]
    cands = enumerate_candidates(W, H, N, Cmax, Rmax, Kmax, dt, dr, n_lo)

    def rsum(a, rect):
        x0, y0, x1, y1 = rect
        return sum(a[y][x] for y in range(y0, y1) for x in range(x0, x1))

    scored = []
    for rank, cand in enumerate(cands):
        rs = regions_of(W, H, cand)
        areas = [rsum(n, q) for q in rs]
        feasible = (area_k == 0 or area_k * min(areas) > max(areas)) and \
            coherent(cand, rs, lambda q: rsum(n, q), row_px, prune)
        t = max(rsum(T, q) for q in rs)
        qv = sum(rsum(s2, q) - (rsum(s1, q) ** 2) // rsum(n, q) for q in rs)
        scored.append((rank, feasible, t, qv, rs))
    feas = [s for s in scored if s[1]]
    out = dict(n_enumerated=len(cands), n_feasible=len(feas))
    if not feas:
        out.update(rank=None)
        return out
    tmin = min(s[2] for s in feas)
    if lam is None:
        pool = feas
    else:
        pool = [s for s in feas if s[2] <= tmin * (1 + lam)]
    best = min(pool, key=lambda s: (s[3], s[2], s[0]))
    out.update(rank=best[0], t_min=tmin, t_sel=best[2], q_sel=best[3], rs=best[4])
    return out


def enumerate_spanning(W, H, N, Cmax, Rmax, Kmax):
    """The literal space in which an RS may also be a block of two or more complete tiles stacked
    in one tile column: every (c, r, X, Y) and, per tile column, every way to cover its r tiles
    from top to bottom with single tiles cut into k slices (any split rows) or blocks of >= 2
    tiles; N RS in all.  Each candidate is (c, r, X, Y, columns), a column being a tuple of
    ('t', j, k, Z) and ('b', a, b) items."""
    def coverings(yb, j, r):
        if j == r:
            yield ()
            return
        hj = yb[j + 1] - yb[j]
        for k in range(1, min(Kmax, hj) + 1):
            for Z in boundary_vectors(hj, k, None):
                for rest in coverings(yb, j + 1, r):
                    yield (('t', j, k, Z),) + rest
        for b in range(j + 2, r + 1):
            for rest in coverings(yb, b, r):
                yield (('b', j, b),) + rest

    def count_rs(col):
        return sum(it[2] if it[0] == 't' else 1 for it in col)

    out = []
    for c in range(1, Cmax + 1):
        for r in range(1, Rmax + 1):
            for X in boundary_vectors(W, c, None):
                for Y in boundary_vectors(H, r, None):
                    yb = (0,) + Y + (H,)
                    cols = [(col, count_rs(col)) for col in coverings(yb, 0, r)]
                    for choice in itertools.product(cols, repeat=c):
                        if sum(n for _, n in choice) == N:
                            out.append((c, r, X, Y, tuple(col for col, _ in choice)))
    return out


def spanning_regions(W, H, cand):
    """RS rectangles of a spanning candidate, tiles in raster order: a block is listed at its top
    tile, a cut tile lists its slices top to bottom."""
    c, r, X, Y, cols = cand
    xb = (0,) + X + (W,)
    yb = (0,) + Y + (H,)
    at = {}
    for i, col in enumerate(cols):
        for it in col:
            at[(it[1], i)] = it
    rs = []
    for j in range(r):
        for i in range(c):
            it = at.get((j, i))
            if it is None:
                continue
            if it[0] == 'b':
                rs.append((xb[i], yb[it[1]], xb[i + 1], yb[it[2]]))
            else:
                _, _, k, Z = it
                zb = (0,) + Z + (yb[j + 1] - yb[j],)
                for q in range(k):
                    rs.append((xb[i], yb[j] + zb[q], xb[i + 1], yb[j] + zb[q + 1]))
    return rs


def brute_spanning(luma, cost, cs, N, Cmax, Rmax, Kmax, lam=Fraction(0), area_k=3):
    """Two-step search over enumerate_spanning's candidates with direct sums (as brute_search)."""
    h, w = luma.shape
    W, H = (w + cs - 1) // cs, (h + cs - 1) // cs
    n, s1, s2, _ = ctu_stats_pixels(luma, cs)
    T = [[int(cost[y * W + x]) for x in range(W)] for y in range(H)]
    cands = enumerate_spanning(W, H, N, Cmax, Rmax, Kmax)

    def rsum(a, rect):
        x0, y0, x1, y1 = rect
        return sum(a[y][x] for y in range(y0, y1) for x in range(x0, x1))

    scored = []
    for rank, cand in enumerate(cands):
        rs = spanning_regions(W, H, cand)
        areas = [rsum(n, q) for q in rs]
        feasible = area_k == 0 or area_k * min(areas) > max(areas)
        t = max(rsum(T, q) for q in rs)
        qv = sum(rsum(s2, q) - (rsum(s1, q) ** 2) // rsum(n, q) for q in rs)
        scored.append((rank, feasible, t, qv, rs))
    feas = [s for s in scored if s[1]]
    out = dict(n_enumerated=len(cands), n_feasible=len(feas))
    if not feas:
        out.update(rank=None)
        return out
    tmin = min(s[2] for s in feas)
    pool = feas if lam is None else [s for s in feas if s[2] <= tmin * (1 + lam)]
    best = min(pool, key=lambda s: (s[3], s[2], s[0]))
    out.update(rank=best[0], t_min=tmin, t_sel=best[2], q_sel=best[3], rs=best[4])
    return out
