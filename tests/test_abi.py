"""CPU tests of the C ABI: exports, host-only entry points and host-side error paths.

No kernel is launched here.  The host-only calls (space size, workspace query, rank
decode) are checked against the oracle and against the brute-force enumeration order.
"""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import brute
from paper_2012_14792_amd import binding as B
from paper_2012_14792_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(B.LIB_PATH):
        from paper_2012_14792_amd import build
        build.build()
    return B.lib()


def test_every_declared_entry_point_is_exported(lib):
    hdr = open(os.path.join(ROOT, "include", "trs.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    names = set(re.findall(r"\b(trs_[a-z_]+)\s*\(", hdr))
    assert {"trs_features", "trs_cost_map", "trs_search", "trs_search_workspace", "trs_space_size",
            "trs_decode", "trs_release_plans", "trs_strerror"} <= names
    raw = ctypes.CDLL(B.LIB_PATH)
    for n in sorted(names):
        assert hasattr(raw, n), n


def test_strerror(lib):
    for s in range(-6, 2):
        assert B.strerror(s) and B.strerror(s) != "unknown status"
    assert B.strerror(-99) == "unknown status"


@pytest.mark.parametrize("w,h,N,C,R,K", [(1920, 1080, 4, 3, 3, 2), (3840, 2160, 8, 6, 4, 4),
                                         (1920, 1080, 16, 8, 6, 4), (3840, 2160, 4, 3, 3, 2),
                                         (640, 512, 3, 3, 3, 2), (1000, 700, 5, 3, 3, 3)])
def test_space_size_matches_oracle(lib, orc, w, h, N, C, R, K):
    fr, pr = B.make_frame(w, h), B.make_params(N, C, R, K)
    W, H = B.ctu_dims(fr)
    assert B.trs_space_size(fr, pr) == orc.space_size(W, H, orc.make_params(N, C, R, K))


@pytest.mark.parametrize("w,h,N,C,R,K,lo", [(1920, 1080, 8, 6, 4, 4, 4), (3840, 2160, 8, 6, 4, 4, 6),
                                            (3840, 2160, 12, 6, 4, 4, 9), (7680, 4320, 16, 8, 6, 4, 1),
                                            (384, 256, 8, 3, 2, 2, 1)])
def test_space_size_with_idle_threads_matches_oracle(lib, orc, w, h, N, C, R, K, lo):
    fr, pr = B.make_frame(w, h), B.make_params(N, C, R, K, min_rs=lo)
    W, H = B.ctu_dims(fr)
    assert B.trs_space_size(fr, pr) == orc.space_size(W, H, orc.make_params(N, C, R, K, min_rs=lo))


@pytest.mark.parametrize("w,h,N,C,R,K,lo", [(768, 600, 4, 3, 3, 2, 1), (640, 512, 5, 3, 3, 2, 2),
                                            (384, 256, 8, 3, 2, 2, 1)])
def test_decode_with_idle_threads_follows_canonical_order(lib, w, h, N, C, R, K, lo):
    """With RS counts in [min_rs, N], every rank still decodes to the candidate the brute
    force puts at that position."""
    fr, pr = B.make_frame(w, h), B.make_params(N, C, R, K, dtile=-1, drs=-1, min_rs=lo)
    W, H = B.ctu_dims(fr)
    cands = brute.enumerate_candidates(W, H, N, C, R, K, None, None, lo)
    assert B.trs_space_size(fr, pr)[0] == len(cands)
    for rank, cand in enumerate(cands):
        d = B.trs_decode(fr, pr, rank)
        assert d["rs"] == brute.regions_of(W, H, cand), rank
        assert d["n_rs"] == len(d["rs"]) >= lo


@pytest.mark.parametrize("w,h,N,C,R,K,dt,dr", [(640, 512, 3, 3, 3, 2, -1, -1),
                                               (768, 600, 4, 3, 3, 2, -1, -1),
                                               (1024, 768, 4, 3, 3, 2, 1, 0),
                                               (1152, 896, 5, 3, 3, 3, 2, 1),
                                               (1920, 1080, 4, 3, 3, 2, -2, -2)])
def test_decode_follows_canonical_order(lib, w, h, N, C, R, K, dt, dr):
    """Every rank decodes to the candidate the brute force puts at that position."""
    fr, pr = B.make_frame(w, h), B.make_params(N, C, R, K, dtile=dt, drs=dr)
    W, H = B.ctu_dims(fr)
    n, dtu, dru = B.trs_space_size(fr, pr)
    cands = brute.enumerate_candidates(W, H, N, C, R, K, None if dtu < 0 else dtu,
                                       None if dru < 0 else dru)
    assert n == len(cands)
    for rank, cand in enumerate(cands):
        d = B.trs_decode(fr, pr, rank)
        assert d["rs"] == brute.regions_of(W, H, cand), rank
        assert d["tile_cols"] == cand[0] and d["tile_rows"] == cand[1]
        assert d["col_bd"] == [0, *cand[2], W] and d["row_bd"] == [0, *cand[3], H]


def test_decode_of_oracle_winner_uhd(lib, orc):
    """The oracle's chosen rank on a 4K frame decodes to the oracle's slices."""
    cfg = synth.CONFIGS["uhd_n8"]
    w, h = cfg["width"], cfg["height"]
    luma = synth.SequenceGenerator(w, h, cfg["seed"], cfg["drift"]).frame(3)
    f = orc.features(luma)
    W, H = orc.ctu_dims(w, h)
    prev = synth.ctu_times(f["tex"], synth.ar1_eps(W * H, 1, 77)[0])
    cost, _ = orc.cost_map(f["tex"], prev)
    op = orc.make_params(8, 6, 4, 4, lam=cfg["lam"])
    o = orc.search(w, h, op, cost, f["s1"], f["s2"])
    d = B.trs_decode(B.make_frame(w, h), B.make_params(8, 6, 4, 4, lam=cfg["lam"]), o["rank"])
    assert d["rs"] == o["rs"] and d["col_bd"] == o["col_bd"] and d["row_bd"] == o["row_bd"]
    assert d["n_enumerated"] == o["n_enumerated"]


def test_workspace_is_small_and_schedule_dependent(lib):
    fr = B.make_frame(3840, 2160)
    a = B.trs_search_workspace(fr, B.make_params(8, 6, 4, 4, sched_item=1024))
    b = B.trs_search_workspace(fr, B.make_params(8, 6, 4, 4, sched_item=65536))
    assert 0 < b < a < 64 << 20


# ---- host-side error paths (no kernel is launched) ------------------------------------------

@pytest.mark.parametrize("frame", [(0, 1080, 128, 10), (1920, 0, 128, 10), (1920, 1080, 96, 10),
                                   (1920, 1080, 128, 7), (1920, 1080, 128, 13), (9000, 1080, 128, 10)])
def test_invalid_frame(lib, frame):
    with pytest.raises(B.TrsError) as e:
        B.trs_space_size(B.Frame(*frame), B.make_params(4, 3, 3, 2))
    assert e.value.status == B.TRS_EINVAL


@pytest.mark.parametrize("kw", [dict(n_threads=0), dict(n_threads=65), dict(max_tile_cols=0),
                                dict(max_rs_per_tile=0), dict(area_k=-1), dict(lam=(1, 0)),
                                dict(lam=(70000, 1)), dict(dtile=-3, drs=0), dict(dtile=-2, drs=1),
                                dict(sched_block=96), dict(sched_item=-5), dict(min_rs=-1),
                                dict(min_rs=5), dict(prune=4)])
def test_invalid_params(lib, kw):
    base = dict(n_threads=4, max_tile_cols=3, max_tile_rows=3, max_rs_per_tile=2)
    base.update(kw)
    with pytest.raises(B.TrsError) as e:
        B.trs_search_workspace(B.make_frame(1920, 1080), B.make_params(**base))
    assert e.value.status == B.TRS_EINVAL


def test_empty_space(lib):
    # 8 slices cannot be cut from a 2 x 1 CTU frame with at most 2 slices per tile
    with pytest.raises(B.TrsError) as e:
        B.trs_search_workspace(B.make_frame(256, 128), B.make_params(8, 3, 3, 2))
    assert e.value.status == B.TRS_ENOSPACE


def test_decode_rank_out_of_range(lib):
    fr, pr = B.make_frame(1920, 1080), B.make_params(4, 3, 3, 2)
    for bad in (-1, 3416):
        with pytest.raises(B.TrsError) as e:
            B.trs_decode(fr, pr, bad)
        assert e.value.status == B.TRS_EINVAL


def test_search_rejects_missing_or_small_workspace(lib):
    L = B.lib()
    fr, pr = B.make_frame(1920, 1080), B.make_params(4, 3, 3, 2)
    fake = ctypes.c_void_p(0x1000)
    st = L.trs_search(ctypes.byref(fr), ctypes.byref(pr), fake, fake, fake, None, 0, fake, None)
    assert st == B.TRS_EWORKSPACE
    need = B.trs_search_workspace(fr, pr)
    st = L.trs_search(ctypes.byref(fr), ctypes.byref(pr), fake, fake, fake, ctypes.c_void_p(0x10000),
                      need - 1, fake, None)
    assert st == B.TRS_EWORKSPACE
    st = L.trs_search(ctypes.byref(fr), ctypes.byref(pr), fake, fake, fake, ctypes.c_void_p(0x10010),
                      need, fake, None)
    assert st == B.TRS_EWORKSPACE                                   # misaligned
    st = L.trs_search(ctypes.byref(fr), ctypes.byref(pr), None, fake, fake, ctypes.c_void_p(0x10000),
                      need, fake, None)
    assert st == B.TRS_EINVAL


def test_features_rejects_bad_layout(lib):
    L = B.lib()
    fr = B.make_frame(1920, 1080)
    feat = B.Feat(*(0x2000 for _ in range(6)))
    assert L.trs_features(ctypes.byref(fr), ctypes.c_void_p(0x1000), 1919, feat, None) == B.TRS_EINVAL
    assert L.trs_features(ctypes.byref(fr), ctypes.c_void_p(0x1000), 1924, feat, None) == B.TRS_EINVAL
    assert L.trs_features(ctypes.byref(fr), ctypes.c_void_p(0x1008), 1920, feat, None) == B.TRS_EINVAL
    bad = B.Feat(0x2000, 0x2000, 0, 0x2000, 0x2000, 0x2000)
    assert L.trs_features(ctypes.byref(fr), ctypes.c_void_p(0x1000), 1920, bad, None) == B.TRS_EINVAL
    assert L.trs_cost_map(ctypes.byref(fr), ctypes.c_void_p(0x1000), None, B.Blend(200, 3, 257),
                          ctypes.c_void_p(0x2000), None, None) == B.TRS_EINVAL


def test_lambda_policy_matches_table1():
    """trs_lambda_policy returns the lambda Table 1 prints for each resolution and n, and maps
    other thread counts and sizes to the nearest row and column."""
    import json
    from fractions import Fraction
    g = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "table1_lambda.json")))
    for col, (w, h) in (("fhd", (1920, 1080)), ("uhd", (3840, 2160))):
        for n, lam in g[col].items():
            num, den = B.trs_lambda_policy(B.make_frame(w, h), int(n))
            assert Fraction(num, den) == Fraction(*lam), (col, n)
    assert B.trs_lambda_policy(B.make_frame(7680, 4320), 16) == B.trs_lambda_policy(B.make_frame(3840, 2160), 12)
    assert B.trs_lambda_policy(B.make_frame(1280, 720), 6) == B.trs_lambda_policy(B.make_frame(1920, 1080), 8)
    assert B.trs_lambda_policy(B.make_frame(1920, 1080), 2) == (0, 10)
    with pytest.raises(B.TrsError):
        B.trs_lambda_policy(B.make_frame(1920, 1080), 0)


def test_workload_lambdas_follow_the_policy():
    from fractions import Fraction
    for (size, n), lam in synth.LAMBDA.items():
        w, h = synth.SIZES[size]
        assert Fraction(*B.trs_lambda_policy(B.make_frame(w, h), n)) == Fraction(*lam), (size, n)


def test_literal_search_rejects_what_it_does_not_cover(lib):
    fr = B.make_frame(1920, 1080)
    cases = [(dict(dtile=3, drs=1), B.TRS_EINVAL), (dict(dtile=-1, drs=-1, prune=1), B.TRS_ENOTIMPL),
             (dict(dtile=-1, drs=-1, min_rs=2), B.TRS_ENOTIMPL)]
    for kw, status in cases:
        with pytest.raises(B.TrsError) as e:
            B.trs_literal_workspace(fr, B.make_params(4, 3, 3, 2, **kw))
        assert e.value.status == status
    with pytest.raises(B.TrsError) as e:
        B.trs_literal_workspace(B.make_frame(7680, 4320), B.make_params(16, 8, 6, 4, dtile=-1, drs=-1))
    assert e.value.status == B.TRS_ENOTIMPL


def test_literal_profile_read_without_searches(lib):
    """With no literal search profiled the read returns zero stages, zero runs and zero
    relaxations; a missing output pointer is rejected."""
    st, runs, relax = B.trs_profile_read_literal()
    assert runs == 0 and relax == (0, 0) and all(v == 0 for v in st.values())
    ms = (ctypes.c_double * len(B.LITERAL_STAGES))()
    n = ctypes.c_int64()
    assert lib.trs_profile_read_literal(ms, ctypes.byref(n), None) == B.TRS_EINVAL
