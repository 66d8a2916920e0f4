"""Random-access GOP reference selection (Section 2.1, the co-TL estimator): the oracle is
pinned to closed forms and invariants of the dyadic hierarchy, then the library's host
routine trs_ra_schedule is compared with it (CPU only)."""
import numpy as np
import pytest

from oracle import gop_ref
from paper_2012_14792_amd import binding as B


@pytest.mark.parametrize("G", [1, 2, 4, 8, 16, 32, 64])
def test_layers_closed_form(G):
    """Layer = log2 G - (trailing zero bits of p) for frames off the GOP grid, 0 on it."""
    n = 3 * G + 5
    lg = G.bit_length() - 1
    expect = [0 if p % G == 0 else lg - ((p & -p).bit_length() - 1) for p in range(n)]
    assert gop_ref.layers(G, n) == expect


def test_gop16_coding_order():
    """The hierarchical-B order of a 16-frame GOP: key frame, then halving points depth first."""
    assert gop_ref.coding_order(16, 17) == [0, 16, 8, 4, 2, 1, 3, 6, 5, 7, 12, 10, 9, 11, 14, 13, 15]


@pytest.mark.parametrize("G,n", [(16, 65), (16, 50), (32, 97), (8, 3), (4, 1), (2, 9)])
def test_coding_order_invariants(G, n):
    """A permutation of the frames in which each frame comes after the two frames bounding its
    halving interval (the references a hierarchical-B frame needs), GOP by GOP."""
    order = gop_ref.coding_order(G, n)
    assert sorted(order) == list(range(n))
    pos = {p: i for i, p in enumerate(order)}
    for p in range(1, n):
        if p % G == 0:
            assert pos[p] > pos[p - G]
            continue
        step = p & -p
        lo, hi = p - step, p + step
        assert pos[lo] < pos[p]
        if hi < n:
            assert pos[hi] < pos[p]
        assert all(pos[q] < pos[p] for q in range(0, (p // G) * G + 1, G))


def test_low_delay_gop_of_one():
    """G = 1: display order is coding order, one layer, both references are the previous frame."""
    cotl, closest = gop_ref.references(1, 10)
    assert gop_ref.coding_order(1, 10) == list(range(10))
    assert cotl == closest == [-1] + list(range(9))


def test_gop16_references_by_hand():
    cotl, closest = gop_ref.references(16, 33)
    # layer 4 (odd frames) is coded 1, 3, 5, 7, 9, ...: frame 3's co-TL frame is 1
    assert cotl[1] == -1 and cotl[3] == 1 and cotl[5] == 3 and cotl[17] == 15
    # frame 24 (layer 1) follows frame 8; frame 32 (layer 0) follows 16; frame 16 follows 0
    assert cotl[24] == 8 and cotl[32] == 16 and cotl[16] == 0
    # closest coded frames: 16 -> 0, 8 -> 0 (tie 0 / 16 at distance 8: the earlier), 1 -> 0
    assert closest[16] == 0 and closest[8] == 0 and closest[1] == 0 and closest[3] == 2


@pytest.mark.parametrize("G,n", [(1, 7), (2, 2), (4, 21), (8, 64), (16, 65), (16, 50), (32, 129),
                                 (64, 200), (256, 300)])
def test_library_matches_oracle(G, n):
    got = B.trs_ra_schedule(G, n)
    cotl, closest = gop_ref.references(G, n)
    assert got["coding_order"].tolist() == gop_ref.coding_order(G, n)
    assert got["layer"].tolist() == gop_ref.layers(G, n)
    assert got["cotl_ref"].tolist() == cotl
    assert got["closest_ref"].tolist() == closest


@pytest.mark.parametrize("G,n", [(0, 8), (3, 8), (512, 8), (16, 0), (-4, 8)])
def test_library_rejects_bad_arguments(G, n):
    with pytest.raises(B.TrsError) as e:
        B.trs_ra_schedule(G, n)
    assert e.value.status == B.TRS_EINVAL
