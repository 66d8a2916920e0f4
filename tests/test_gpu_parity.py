"""GPU parity: the HIP path through the C ABI against the CPU oracle, bit-exact.

Features, costs and scores are integers, so every field of every result must match:
rank, T~min, T~(P), Q(P), counts, tile grid, slice rectangles and slice times.
"""
import numpy as np
import pytest

from helpers import (assert_same_result, gpu_cost, gpu_features, gpu_search, oracle_params,
                     sequence_inputs, to_device)
from paper_2012_14792_amd import binding as B
from paper_2012_14792_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    B.lib()
    yield
    torch.cuda.synchronize()


# ---- features ----------------------------------------------------------------------------

@pytest.mark.parametrize("w,h,cs,seed", [(1920, 1080, 128, 1), (3840, 2160, 128, 2),
                                         (7680, 4320, 128, 3), (1000, 700, 128, 4),
                                         (1001, 333, 128, 5), (640, 360, 64, 6), (333, 200, 32, 7),
                                         (8, 8, 128, 8), (130, 1, 128, 9), (1, 130, 32, 10)])
def test_features_bit_exact(orc, w, h, cs, seed):
    luma = synth.make_frame(w, h, seed)
    fr = B.make_frame(w, h, cs)
    g = gpu_features(fr, to_device(luma))
    o = orc.features(luma, cs)
    for k in ("s1", "s2", "grad", "tex", "mean", "var"):
        assert np.array_equal(g[k], o[k]), k


def test_features_extreme_values(orc):
    rng = np.random.default_rng(0)
    luma = np.where(rng.random((517, 389)) < 0.5, 0, 1023).astype(np.uint16)
    g = gpu_features(B.make_frame(389, 517), to_device(luma))
    o = orc.features(luma)
    for k in o:
        assert np.array_equal(g[k], o[k]), k
    luma12 = rng.integers(0, 4096, (300, 300)).astype(np.uint16)
    g = gpu_features(B.make_frame(300, 300, 128, 12), to_device(luma12))
    o = orc.features(luma12)
    for k in o:
        assert np.array_equal(g[k], o[k]), k


# ---- cost map ----------------------------------------------------------------------------

@pytest.mark.parametrize("blend", [(200, 3, 256), (200, 3, 0), (200, 3, 128), (17, 5, 1), (0, 1, 255)])
def test_cost_map_bit_exact(orc, blend):
    rng = np.random.default_rng(3)
    fr = B.make_frame(3840, 2160)
    n = 30 * 17
    tex = rng.integers(0, 2000, n).astype(np.uint32)
    prev = rng.integers(1, 100000, n).astype(np.uint32)
    for pv in (prev, None):
        g, flag = gpu_cost(fr, tex, pv, blend)
        o, rc = orc.cost_map(tex, pv, *blend)
        assert np.array_equal(g, o) and flag == 0 and rc == 0


def test_cost_map_overflow_flag(orc):
    fr = B.make_frame(256, 128)
    tex = np.array([2**31, 5], np.uint32)
    prev = np.array([2**32 - 1, 7], np.uint32)
    for pv, blend in [(None, (0, 1, 256)), (prev, (0, 1, 256)), (prev, (10, 2**20, 100))]:
        g, flag = gpu_cost(fr, tex, pv, blend)
        o, rc = orc.cost_map(tex, pv, *blend)
        assert np.array_equal(g, o) and flag == 1 and rc == -2


# ---- search ------------------------------------------------------------------------------

def _search_both(orc, w, h, params, luma, prev, cs=128):
    f = orc.features(luma, cs)
    cost, _ = orc.cost_map(f["tex"], prev)
    o = orc.search(w, h, oracle_params(orc, params), cost, f["s1"], f["s2"], cs)
    g = gpu_search(B.make_frame(w, h, cs), params, cost, f["s1"], f["s2"])
    return g, o


@pytest.mark.parametrize("w,h,N,seed", [(640, 512, 3, 0), (768, 600, 4, 1), (512, 640, 4, 3),
                                        (896, 384, 5, 4), (1280, 1280, 6, 5)])
@pytest.mark.parametrize("lam", [(0, 1), (1, 10), (3, 10), (-1, 1)])
def test_search_small_grids(orc, w, h, N, seed, lam):
    luma = synth.make_frame(w, h, seed)
    W, H = (w + 127) // 128, (h + 127) // 128
    prev = synth.ctu_times(orc.features(luma)["tex"], synth.ar1_eps(W * H, 1, seed)[0])
    p = B.make_params(N, 3, 3, min(N, 3), lam=lam)
    g, o = _search_both(orc, w, h, p, luma, prev)
    assert_same_result(g, o, f"{w}x{h} N={N} lam={lam}")


@pytest.mark.parametrize("lam", [(0, 1), (1, 10), (3, 10), (-1, 1)])
@pytest.mark.parametrize("N,C,R,K", [(4, 3, 3, 2), (8, 6, 4, 4), (16, 8, 6, 4), (12, 6, 4, 4)])
def test_search_fhd(orc, lam, N, C, R, K):
    cfg = synth.CONFIGS["fhd_n4"]
    w, h = cfg["width"], cfg["height"]
    luma = synth.make_frame(w, h, cfg["seed"])
    prev = synth.ctu_times(orc.features(luma)["tex"], synth.ar1_eps(135, 1, 1001)[0])
    g, o = _search_both(orc, w, h, B.make_params(N, C, R, K, lam=lam), luma, prev)
    assert_same_result(g, o, f"fhd N={N} lam={lam}")


@pytest.mark.parametrize("frames", [[0, 1], [31, 63]])
def test_search_uhd_sequence(orc, frames):
    cfg = synth.CONFIGS["uhd_n8"]
    w, h = cfg["width"], cfg["height"]
    p = B.make_params(8, 6, 4, 4, lam=cfg["lam"])
    for f, luma, prev in sequence_inputs(orc, cfg, frames):
        g, o = _search_both(orc, w, h, p, luma, prev)
        assert g["n_enumerated"] == 5914718
        assert_same_result(g, o, f"uhd frame {f}")


def test_search_8k_frame(orc):
    cfg = synth.CONFIGS["8k_n16"]
    w, h = cfg["width"], cfg["height"]
    p = B.make_params(16, 8, 6, 4, lam=cfg["lam"])
    for f, luma, prev in sequence_inputs(orc, cfg, [5]):
        g, o = _search_both(orc, w, h, p, luma, prev)
        assert g["n_enumerated"] == 16133022
        assert_same_result(g, o, f"8k frame {f}")


def test_full_path_matches_oracle_partition(orc):
    """luma + previous times -> features -> cost map -> search, all on the GPU."""
    import torch
    cfg = synth.CONFIGS["uhd_n8"]
    w, h = cfg["width"], cfg["height"]
    p = B.make_params(8, 6, 4, 4, lam=cfg["lam"])
    part = B.Partitioner(w, h, p)
    for f, luma, prev in sequence_inputs(orc, cfg, [7]):
        pv = torch.from_numpy(prev.view(np.int32)).cuda()
        g = part(to_device(luma), pv)
        o = orc.partition(luma, prev, oracle_params(orc, p))
        assert_same_result(g, o, f"full path frame {f}")


def test_special_cases(orc):
    w, h = 1920, 1080
    luma = synth.make_frame(w, h, 12)
    prev = synth.ctu_times(orc.features(luma)["tex"], synth.ar1_eps(135, 1, 12)[0])
    # no area rule
    g, o = _search_both(orc, w, h, B.make_params(8, 6, 4, 4, area_k=0, lam=(1, 10)), luma, prev)
    assert_same_result(g, o, "area_k=0")
    # nothing feasible: uniform partition with status 1
    with pytest.warns(RuntimeWarning):
        g, o = _search_both(orc, w, h, B.make_params(4, 3, 3, 2, area_k=1), luma, prev)
    assert g["status"] == 1 and o["status"] == 1
    assert_same_result(g, o, "no feasible")
    # flat frame: Q = 0 everywhere, choice by time then rank
    flat = np.full((h, w), 300, np.uint16)
    g, o = _search_both(orc, w, h, B.make_params(8, 6, 4, 4, lam=(-1, 1)), flat, prev)
    assert g["q_sel"] == 0
    assert_same_result(g, o, "flat")
    # fixed windows and textbook single-tile space
    g, o = _search_both(orc, w, h, B.make_params(8, 6, 4, 4, lam=(1, 10), dtile=2, drs=1), luma, prev)
    assert_same_result(g, o, "windows 2,1")
    g, o = _search_both(orc, w, h, B.make_params(5, 1, 1, 5, area_k=0, dtile=-1, drs=-1), luma, prev)
    assert_same_result(g, o, "single tile")
    # small CTUs
    g, o = _search_both(orc, 1000, 600, B.make_params(6, 4, 3, 3, lam=(1, 10)),
                        synth.make_frame(1000, 600, 13),
                        synth.ctu_times(orc.features(synth.make_frame(1000, 600, 13), 64)["tex"],
                                        synth.ar1_eps(16 * 10, 1, 13)[0]), cs=64)
    assert_same_result(g, o, "ctu 64")


def test_schedules_do_not_change_the_decision(orc):
    cfg = synth.CONFIGS["uhd_n8"]
    w, h = cfg["width"], cfg["height"]
    (f, luma, prev), = list(sequence_inputs(orc, cfg, [2]))
    fo = orc.features(luma)
    cost, _ = orc.cost_map(fo["tex"], prev)
    ref = None
    for blk in (64, 128, 256, 512):
        for item in (256, 4096, 65536):
            p = B.make_params(8, 6, 4, 4, lam=cfg["lam"], sched_block=blk, sched_item=item)
            g = gpu_search(B.make_frame(w, h), p, cost, fo["s1"], fo["s2"])
            if ref is None:
                ref = g
                o = orc.search(w, h, oracle_params(orc, p), cost, fo["s1"], fo["s2"])
                assert_same_result(g, o, "schedule reference")
            assert_same_result(g, ref, f"block {blk} item {item}")


def test_repeated_runs_are_bit_identical(orc):
    import torch
    w, h = 3840, 2160
    luma = synth.make_frame(w, h, 21)
    fo = orc.features(luma)
    prev = synth.ctu_times(fo["tex"], synth.ar1_eps(510, 1, 21)[0])
    p = B.make_params(8, 6, 4, 4, lam=(1, 10))
    part = B.Partitioner(w, h, p)
    pv = torch.from_numpy(prev.view(np.int32)).cuda()
    d = to_device(luma)
    outs = []
    for _ in range(3):
        out = torch.empty(B.RESULT_BYTES, dtype=torch.uint8, device="cuda")
        part.enqueue(d, pv, out=out)
        outs.append(out)
    torch.cuda.synchronize()
    assert all(torch.equal(outs[0], o) for o in outs[1:])


def test_separate_calls_match_fused_call(orc):
    import torch
    cfg = synth.CONFIGS["uhd_n8"]
    w, h = cfg["width"], cfg["height"]
    p = B.make_params(8, 6, 4, 4, lam=cfg["lam"])
    part = B.Partitioner(w, h, p)
    (f, luma, prev), = list(sequence_inputs(orc, cfg, [9]))
    d = to_device(luma)
    pv = torch.from_numpy(prev.view(np.int32)).cuda()
    a = torch.empty(B.RESULT_BYTES, dtype=torch.uint8, device="cuda")
    b = torch.empty(B.RESULT_BYTES, dtype=torch.uint8, device="cuda")
    part.enqueue(d, pv, out=a)
    part.enqueue_separate(d, pv, out=b)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    assert_same_result(B.read_result(a), orc.partition(luma, prev, oracle_params(orc, p)), "fused")


def test_graph_replay_matches_eager(orc):
    """Every replay of a captured multi-frame graph equals the eager results."""
    import torch
    cfg = synth.CONFIGS["uhd_n8"]
    w, h = cfg["width"], cfg["height"]
    p = B.make_params(8, 6, 4, 4, lam=cfg["lam"])
    part = B.Partitioner(w, h, p)
    frames = list(sequence_inputs(orc, cfg, [3, 4, 5, 6]))
    lumas = [to_device(l) for _, l, _ in frames]
    prevs = [torch.from_numpy(pv.view(np.int32)).cuda() for _, _, pv in frames]
    eager = torch.empty((len(frames), B.RESULT_BYTES), dtype=torch.uint8, device="cuda")
    for i in range(len(frames)):
        part.enqueue(lumas[i], prevs[i], out=eager[i])
    torch.cuda.synchronize()
    graphed = torch.zeros_like(eager)
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            for i in range(len(frames)):
                part.enqueue(lumas[i], prevs[i], out=graphed[i])
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    for rep in range(3):
        graphed.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(graphed, eager), f"replay {rep}"
        # eager work between replays reuses the same workspace
        part.enqueue(lumas[0], prevs[0], out=eager[0])
        torch.cuda.synchronize()
    for i, (f, luma, prev) in enumerate(frames):
        assert_same_result(B.read_result(graphed[i]), orc.partition(luma, prev, oracle_params(orc, p)),
                           f"graph frame {f}")


@pytest.mark.parametrize("name,N,C,R,K,lam", [("fhd", 8, 6, 4, 4, (3, 10)), ("uhd", 8, 6, 4, 4, (1, 10)),
                                               ("fhd", 4, 3, 3, 2, (0, 1))])
@pytest.mark.parametrize("prune", [1, 2, 3])
def test_search_with_pruning_rules_matches_oracle(orc, name, N, C, R, K, lam, prune):
    """The optional pruning rules change the feasible set at plan time; per-frame searches and
    a batch holding frames with different rule sets both give the oracle's results."""
    import torch
    w, h = synth.SIZES[name]
    frame = B.make_frame(w, h)
    gen = synth.SequenceGenerator(w, h, 40 + prune, 8.0)
    luma = gen.frame(1)
    f = orc.features(luma)
    W, H = B.ctu_dims(frame)
    prev = synth.ctu_times(orc.features(gen.frame(0))["tex"], synth.ar1_eps(W * H, 1, 5)[0])
    cost, _ = orc.cost_map(f["tex"], prev)
    params = B.make_params(N, C, R, K, lam=lam, prune=prune)
    ref = orc.search(w, h, oracle_params(orc, params), cost, f["s1"], f["s2"])
    gf = gpu_features(frame, to_device(luma))
    got = gpu_search(frame, params, cost, gf["s1"], gf["s2"])
    assert_same_result(got, ref, f"{name} prune {prune}")
    # the same frame in a batch next to an unpruned copy
    items = [dict(width=w, height=h, params=params, luma=to_device(luma),
                  prev=torch.from_numpy(prev.view(np.int32)).cuda()),
             dict(width=w, height=h, params=B.make_params(N, C, R, K, lam=lam), luma=to_device(luma),
                  prev=torch.from_numpy(prev.view(np.int32)).cuda())]
    batch = B.Batch(items)
    batch.enqueue()
    torch.cuda.synchronize()
    res = batch.results()
    assert_same_result(res[0], ref, f"batch {name} prune {prune}")
    ref0 = orc.search(w, h, oracle_params(orc, items[1]["params"]), cost, f["s1"], f["s2"])
    assert_same_result(res[1], ref0, f"batch {name} unpruned")
    batch.close()


@pytest.mark.parametrize("name,N,C,R,K,lam,lo,prune", [("fhd", 4, 3, 3, 2, (0, 1), 1, 0),
                                                        ("fhd", 8, 6, 4, 4, (3, 10), 4, 2),
                                                        ("uhd", 8, 6, 4, 4, (1, 10), 6, 0),
                                                        ("uhd", 12, 6, 4, 4, (-1, 1), 9, 3),
                                                        ("small", 8, 3, 2, 2, (1, 10), 1, 0)])
def test_search_with_idle_threads_matches_oracle(orc, name, N, C, R, K, lam, lo, prune):
    """RS counts in [min_rs, N] (idle threads): the plan holds every RS count of the range;
    per-frame searches and a batch mixing it with the exact-N space equal the oracle.  The
    3 x 2 CTU frame has no partition into 8 RS, only into fewer."""
    import torch
    w, h = synth.SIZES[name] if name != "small" else (384, 256)
    frame = B.make_frame(w, h)
    gen = synth.SequenceGenerator(w, h, 60 + lo, 8.0)
    luma = gen.frame(1)
    f = orc.features(luma)
    W, H = B.ctu_dims(frame)
    prev = synth.ctu_times(orc.features(gen.frame(0))["tex"], synth.ar1_eps(W * H, 1, 7)[0])
    cost, _ = orc.cost_map(f["tex"], prev)
    params = B.make_params(N, C, R, K, lam=lam, prune=prune, min_rs=lo)
    ref = orc.search(w, h, oracle_params(orc, params), cost, f["s1"], f["s2"])
    assert lo <= ref["n_rs"] <= N
    gf = gpu_features(frame, to_device(luma))
    got = gpu_search(frame, params, cost, gf["s1"], gf["s2"])
    assert_same_result(got, ref, f"{name} N {N} min_rs {lo}")
    exact = B.make_params(N, C, R, K, lam=lam, prune=prune)
    if B.trs_space_size(frame, exact)[0] == 0:
        with pytest.raises(B.TrsError):
            gpu_search(frame, exact, cost, gf["s1"], gf["s2"])
        exact = params
    items = [dict(width=w, height=h, params=p, luma=to_device(luma),
                  prev=torch.from_numpy(prev.view(np.int32)).cuda()) for p in (params, exact)]
    batch = B.Batch(items)
    batch.enqueue()
    torch.cuda.synchronize()
    res = batch.results()
    batch.close()
    assert_same_result(res[0], ref, f"batch {name} min_rs {lo}")
    ref_exact = orc.search(w, h, oracle_params(orc, exact), cost, f["s1"], f["s2"])
    assert_same_result(res[1], ref_exact, f"batch {name} exact N")


@pytest.mark.parametrize("w,h,cs,N,C,R,K", [(8192, 8192, 128, 4, 3, 3, 2), (3840, 2160, 32, 4, 3, 3, 2),
                                             (100, 100, 128, 1, 1, 1, 1), (1920, 1080, 128, 1, 1, 1, 1)])
def test_full_path_extreme_sizes(orc, w, h, cs, N, C, R, K):
    """The largest frame (8192 x 8192) and a 121 x 69 CTU grid (prefix sums beyond LDS, wave
    scans), a single CTU and a single slice: the per-frame path equals the oracle's."""
    import torch
    luma = synth.make_frame(w, h, 21)
    W, H = (w + cs - 1) // cs, (h + cs - 1) // cs
    prev = synth.ctu_times(orc.features(luma, cs)["tex"], synth.ar1_eps(W * H, 1, 21)[0])
    params = B.make_params(N, C, R, K, lam=(1, 10))
    part = B.Partitioner(w, h, params, ctu_size=cs)
    part.enqueue(to_device(luma), torch.from_numpy(prev.view(np.int32)).cuda())
    got = B.read_result(part.out)
    ref = orc.partition(luma, prev, oracle_params(orc, params), cs=cs)
    assert_same_result(got, ref, f"{w}x{h} cs {cs} N {N}")
    if (W + 1) * (H + 1) > 2304:                         # the batched form keeps grids in LDS
        with pytest.raises(B.TrsError) as err:
            B.Batch([dict(width=w, height=h, ctu_size=cs, params=params, luma=to_device(luma),
                          prev=torch.from_numpy(prev.view(np.int32)).cuda())])
        assert err.value.status == B.TRS_ENOTIMPL
