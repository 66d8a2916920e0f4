"""GPU parity of the batched form: one launch sequence for many frames of mixed sizes and
thread budgets must give, for every frame, exactly the per-frame launch's result, which
must equal the oracle's."""
import numpy as np
import pytest

from helpers import assert_same_result, oracle_params, to_device
from paper_2012_14792_amd import binding as B
from paper_2012_14792_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    B.lib()


def _mixed_frames(orc, spec, seed=7):
    """spec: list of (size, N, lam); frames are consecutive frames of per-size sequences."""
    import torch
    gens, counts, out = {}, {}, []
    for name, N, lam in spec:
        w, h = synth.SIZES[name]
        if name not in gens:
            gens[name] = synth.SequenceGenerator(w, h, synth.batch_sequence_seed(name, seed), 8.0)
            counts[name] = 0
        f = counts[name]
        counts[name] += 1
        luma = gens[name].frame(f)
        tex = orc.features(gens[name].frame(max(f - 1, 0)))["tex"]
        prev = synth.ctu_times(tex, synth.ar1_eps(tex.size, 1, 100 + len(out))[0])
        C, R, K = synth.BOUNDS[N]
        out.append(dict(name=name, width=w, height=h, luma_np=luma, prev_np=prev,
                        params=B.make_params(N, C, R, K, lam=lam), luma=to_device(luma),
                        prev=torch.from_numpy(prev.view(np.int32)).cuda()))
    return out


SPEC = [("fhd", 4, (0, 1)), ("uhd", 8, (1, 10)), ("fhd", 16, (1, 10)), ("fhd", 8, (3, 10)),
        ("uhd", 4, (0, 1)), ("fhd", 4, (-1, 1)), ("uhd", 16, (1, 10)), ("fhd", 8, (0, 1))]


def test_batch_matches_per_frame_and_oracle(orc):
    import torch
    frames = _mixed_frames(orc, SPEC)
    batch = B.Batch(frames)
    batch.enqueue()
    torch.cuda.synchronize()
    got = batch.results()
    for i, fr in enumerate(frames):
        part = B.Partitioner(fr["width"], fr["height"], fr["params"])
        single = torch.empty(B.RESULT_BYTES, dtype=torch.uint8, device="cuda")
        part.enqueue(fr["luma"], fr["prev"], out=single)
        torch.cuda.synchronize()
        assert torch.equal(single, batch.out[i]), f"frame {i} differs from its per-frame launch"
        if fr["name"] == "fhd" or i == 1:
            ref = orc.partition(fr["luma_np"], fr["prev_np"], oracle_params(orc, fr["params"]))
            assert_same_result(got[i], ref, f"batch frame {i}")
    batch.close()


def test_batch_features_and_cost_in_workspace(orc):
    import torch
    frames = _mixed_frames(orc, SPEC[:3])
    batch = B.Batch(frames)
    batch.enqueue()
    torch.cuda.synchronize()
    for i, fr in enumerate(frames):
        feat, cost = batch.frame_arrays(i)
        W, H = (fr["width"] + 127) // 128, (fr["height"] + 127) // 128
        base = batch.ws.data_ptr()
        def view(ptr, n, dt):
            off = ptr - base
            return batch.ws[off:off + n * np.dtype(dt).itemsize].cpu().numpy().view(dt)
        o = orc.features(fr["luma_np"])
        for k in ("s1", "grad", "tex", "mean", "var"):
            assert np.array_equal(view(getattr(feat, k), W * H, np.uint32), o[k]), k
        assert np.array_equal(view(feat.s2, W * H, np.uint64), o["s2"])
        c, _ = orc.cost_map(o["tex"], fr["prev_np"])
        assert np.array_equal(view(cost, W * H, np.uint32), c)
    batch.close()


@pytest.mark.parametrize("block,wgs", [(64, 0), (128, 2), (512, 1), (256, 3)])
def test_batch_schedules_do_not_change_results(orc, block, wgs):
    import torch
    frames = _mixed_frames(orc, SPEC)
    ref = B.Batch(frames)
    ref.enqueue()
    other = B.Batch(frames, block=block, wgs_per_cu=wgs)
    other.enqueue()
    torch.cuda.synchronize()
    assert torch.equal(ref.out, other.out)
    ref.close()
    other.close()


def test_batch_graph_replays(orc):
    import torch
    frames = _mixed_frames(orc, SPEC)
    batch = B.Batch(frames)
    batch.enqueue()
    torch.cuda.synchronize()
    eager = batch.out.clone()
    g = batch.capture()
    for rep in range(3):
        batch.out.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(batch.out, eager), f"replay {rep}"
        batch.enqueue()                       # eager work between replays
        torch.cuda.synchronize()
    batch.close()


def test_batch_with_infeasible_frame(orc):
    import torch
    frames = _mixed_frames(orc, SPEC[:2])
    frames[0]["params"] = B.make_params(4, 3, 3, 2, area_k=1)     # nothing feasible
    batch = B.Batch(frames)
    batch.enqueue()
    torch.cuda.synchronize()
    got = batch.results()
    assert got[0]["status"] == 1
    for i, fr in enumerate(frames):
        ref = orc.partition(fr["luma_np"], fr["prev_np"], oracle_params(orc, fr["params"]))
        assert_same_result(got[i], ref, f"frame {i}")
    batch.close()


def test_batch_profile_events(orc):
    """Event timing around the six batch launches: one record per run, every stage timed,
    results unchanged by profiling."""
    import torch
    frames = _mixed_frames(orc, SPEC[:3])
    batch = B.Batch(frames)
    batch.enqueue()
    torch.cuda.synchronize()
    ref = batch.out.clone()
    B.trs_profile_read_batch()                       # drop anything recorded earlier
    B.trs_profile_enable(True)
    try:
        batch.enqueue()
        batch.enqueue()
    finally:
        B.trs_profile_enable(False)
    ms, runs = B.trs_profile_read_batch()
    assert runs == 2
    assert set(ms) == set(B.BATCH_STAGES)
    assert all(v > 0 for v in ms.values())
    assert torch.equal(batch.out, ref)
    assert B.trs_profile_read_batch() == ({k: 0.0 for k in B.BATCH_STAGES}, 0)
    batch.close()


def test_batch_fallback_kernels_match_oracle(orc):
    """A plan without compact record descriptors (one tile cut into 16 slices: k > 11) sends
    the whole batch through the per-(frame, item) search kernels; the same frames without it
    take the frame-inner kernels.  Both must give the per-frame launches' and the oracle's
    results.  CTU 64 frames, so the CTU-size paths other than 128 run too."""
    import torch
    w, h = 1920, 1080
    gen = synth.SequenceGenerator(w, h, 77, 8.0)
    W, H = (w + 63) // 64, (h + 63) // 64
    cases = [(16, 1, 1, 16, (1, 10)), (4, 3, 3, 2, (0, 1)), (8, 6, 4, 4, (1, 10)), (16, 1, 1, 16, (-1, 1))]
    frames = []
    for f, (N, C, R, K, lam) in enumerate(cases):
        luma = gen.frame(f)
        prev = synth.ctu_times(orc.features(gen.frame(f + 1), 64)["tex"], synth.ar1_eps(W * H, 1, 300 + f)[0])
        frames.append(dict(width=w, height=h, ctu_size=64, luma_np=luma, prev_np=prev,
                           params=B.make_params(N, C, R, K, lam=lam), luma=to_device(luma),
                           prev=torch.from_numpy(prev.view(np.int32)).cuda()))
    refs = [orc.partition(fr["luma_np"], fr["prev_np"], oracle_params(orc, fr["params"]), cs=64) for fr in frames]
    for subset in (frames, frames[1:3]):
        batch = B.Batch(subset)
        batch.enqueue()
        torch.cuda.synchronize()
        got = batch.results()
        for i, fr in enumerate(subset):
            part = B.Partitioner(w, h, fr["params"], ctu_size=64)
            single = torch.empty(B.RESULT_BYTES, dtype=torch.uint8, device="cuda")
            part.enqueue(fr["luma"], fr["prev"], out=single)
            torch.cuda.synchronize()
            assert torch.equal(single, batch.out[i]), f"frame {i} differs from its per-frame launch"
            ref = refs[next(j for j, x in enumerate(frames) if x is fr)]
            assert_same_result(got[i], ref, f"frame {i} of {len(subset)}")
        batch.close()


def test_batch_split_calls_pipelined_over_streams(orc):
    """trs_batch_features + trs_batch_search equal trs_batch_run, also when two batches are
    pipelined over two streams (the second batch's features run beside the first's search),
    eagerly and in a replayed graph; their profile events cover all six stages."""
    import torch
    frames = _mixed_frames(orc, SPEC[:4])
    whole = B.Batch(frames)
    whole.enqueue()
    torch.cuda.synchronize()
    halves = [B.Batch(frames[:2]), B.Batch(frames[2:])]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]

    def step():
        base = torch.cuda.current_stream()
        for st in streams:
            st.wait_stream(base)
        ev = None
        for bt, st in zip(halves, streams):
            if ev is not None:
                st.wait_event(ev)
            bt.enqueue_features(stream=st)
            ev = torch.cuda.Event()
            ev.record(st)
            bt.enqueue_search(stream=st)
        for st in streams:
            base.wait_stream(st)

    B.trs_profile_read_batch()
    B.trs_profile_enable(True)
    try:
        step()
        torch.cuda.synchronize()
    finally:
        B.trs_profile_enable(False)
    ms, runs = B.trs_profile_read_batch()
    assert runs == 2 and all(v > 0 for v in ms.values())
    assert torch.equal(torch.cat([h.out for h in halves]), whole.out)
    for h in halves:
        h.out.zero_()
    g = torch.cuda.CUDAGraph()
    cap = torch.cuda.Stream()
    cap.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(cap):
        with torch.cuda.graph(g, stream=cap):
            step()
    torch.cuda.current_stream().wait_stream(cap)
    for _ in range(3):
        for h in halves:
            h.out.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(torch.cat([h.out for h in halves]), whole.out)
    for bt in halves + [whole]:
        bt.close()


def test_batch_wide_and_narrow_time_totals(orc):
    """Frames whose predicted-time totals reach far beyond 2^32 (up to 2^31 - 1 per CTU) next to
    ordinary ones, in chunks of each kind and a mixed chunk: the batch matches the oracle frame
    by frame (record maxima and Eq. 4 bounds need the full 64 bits)."""
    import torch
    w, h = synth.SIZES["fhd"]
    gen = synth.SequenceGenerator(w, h, 91, 8.0)
    W, H = synth.ctu_grid(w, h)
    frames = []
    # chunks (8 frames each, in order): 0..7 all narrow, 8..15 narrow but for frame 12, 16..23 wide
    for f in range(24):
        luma = gen.frame(f)
        prev = synth.ctu_times(orc.features(gen.frame(f + 1))["tex"], synth.ar1_eps(W * H, 1, 600 + f)[0])
        if f >= 16:                                     # totals far above 2^32
            prev = np.minimum(prev.astype(np.uint64) * (40000 + 997 * f), 2**31 - 1).astype(np.uint32)
        if f == 12:
            prev = np.full(W * H, 2**31 - 1, np.uint32)
        frames.append(dict(width=w, height=h, luma_np=luma, prev_np=prev,
                           params=B.make_params(8, 6, 4, 4, lam=(3, 10)), luma=to_device(luma),
                           prev=torch.from_numpy(prev.view(np.int32)).cuda()))
    assert int(frames[16]["prev_np"].astype(np.uint64).sum()) >= 2**32
    assert int(frames[12]["prev_np"].astype(np.uint64).sum()) >= 2**32
    assert all(int(frames[f]["prev_np"].astype(np.uint64).sum()) < 2**31 for f in range(8))
    batch = B.Batch(frames)
    batch.enqueue()
    torch.cuda.synchronize()
    got = batch.results()
    for i, fr in enumerate(frames):
        ref = orc.partition(fr["luma_np"], fr["prev_np"], oracle_params(orc, fr["params"]))
        assert_same_result(got[i], ref, f"frame {i}")
    batch.close()
