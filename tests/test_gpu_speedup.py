"""The speed-up analog computed from the batched GPU path: its partitions equal the oracle's
on the same frames and time maps, so the sequence speed-ups agree exactly."""
import numpy as np
import pytest

import oracle
from paper_2012_14792_amd import speedup as SP
from paper_2012_14792_amd import synth

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("size,n", [("fhd", 4), ("fhd", 8), ("uhd", 8)])
def test_speedup_report_matches_oracle(size, n):
    res = SP.report(n_frames=3, sizes=(size,), threads=(n,), keep_decisions=True)[f"{size}_N{n}"]
    lumas, truth = res["inputs"]
    w, h = synth.SIZES[size]
    W, H = synth.ctu_grid(w, h)
    C, R, K = synth.BOUNDS[n]
    op = oracle.make_params(n, C, R, K, lam=synth.LAMBDA[(size, n)])
    rects = []
    for f in range(1, 4):
        luma = lumas[f].cpu().numpy().view(np.uint16)
        ref = oracle.partition(luma, truth[f - 1], op)
        got = res["decisions"][f - 1]
        assert [tuple(r) for r in got["rs"]] == [tuple(r) for r in ref["rs"]]
        assert got["rank"] == ref["rank"] and got["t_sel"] == ref["t_sel"]
        rects.append(ref["rs"])
    times = [truth[f].reshape(H, W).astype(np.int64) for f in range(1, 4)]
    assert res["sigma_proposed"] == SP.sequence_speedup(rects, times)
    assert res["sigma_proposed"] >= res["sigma_uniform"] * 0.9
    assert 1.0 < res["sigma_proposed_amdahl"] <= res["sigma_max"] <= n
