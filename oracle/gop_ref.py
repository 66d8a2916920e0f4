"""Random-access GOP reference selection, written from the definitions -- TEST INFRASTRUCTURE ONLY.

Section 2.1 of the paper predicts a CTU's time from the co-located CTU of the co-TL frame: the
previously coded frame of the same temporal layer (the related works it cites use the closest
frame in time instead).  The hierarchy is the dyadic one of random-access coding with GOP size
G: a frame's temporal layer is the depth at which the recursive halving of its GOP reaches it
(the GOP's last frame at depth 0), and frames are coded GOP by GOP, key frame first, then each
halving point before the two halves it creates, left half first.
"""
from __future__ import annotations


def layers(G: int, n: int) -> list[int]:
    """Layer of every frame by recursive halving of each GOP interval (depth of the midpoint)."""
    lay = [0] * n

    def halve(lo, hi, depth):
        if hi - lo < 2:
            return
        mid = (lo + hi) // 2
        if mid < n:
            lay[mid] = depth
        halve(lo, mid, depth + 1)
        halve(mid, hi, depth + 1)

    for base in range(0, n, G):
        halve(base, base + G, 1)
    return lay


def coding_order(G: int, n: int) -> list[int]:
    order = [0]

    def halve(lo, hi):
        if hi - lo < 2:
            return []
        mid = (lo + hi) // 2
        return [mid] + halve(lo, mid) + halve(mid, hi)

    for base in range(0, n - 1, G):
        order += [p for p in [base + G] + halve(base, base + G) if p < n]
    return order


def references(G: int, n: int) -> tuple[list[int], list[int]]:
    """(co-TL reference, closest coded frame) per frame in display order, -1 where none."""
    lay, order = layers(G, n), coding_order(G, n)
    cotl, closest = [-1] * n, [-1] * n
    done = []
    for p in order:
        same = [q for q in done if lay[q] == lay[p]]
        cotl[p] = same[-1] if same else -1
        if done:
            closest[p] = min(done, key=lambda q: (abs(q - p), q))
        done.append(p)
    return cotl, closest
