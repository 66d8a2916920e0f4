"""Random-access reference selection on the GPU path: every frame of a short RA sequence is
partitioned with the co-TL frame's and with the closest coded frame's times as the prediction,
and each batched GPU decision equals the oracle's on the same inputs."""
import numpy as np
import pytest

from helpers import assert_same_result, oracle_params
from paper_2012_14792_amd import binding as B
from paper_2012_14792_amd import ra, synth

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("size,N,gop,n", [("fhd", 4, 8, 17), ("fhd", 8, 16, 19)])
def test_ra_decisions_match_oracle(orc, size, N, gop, n):
    r = ra.report(size, N, gop, n, seed=71, keep_decisions=True)
    sched, lumas, times = r["inputs"]
    assert r["frames"] == sum(1 for p in range(n) if sched["cotl_ref"][p] >= 0)
    for name in ("cotl", "closest"):
        assert 0.0 <= r[name]["ctu_rel_err"] and 1.0 <= r[name]["sigma"] <= N
        for p, q, got in r[name]["decisions"]:
            assert q == sched[f"{name}_ref"][p]
            luma = lumas[p].cpu().numpy().view(np.uint16)
            lam = B.trs_lambda_policy(B.make_frame(luma.shape[1], luma.shape[0]), N)
            params = B.make_params(N, *synth.BOUNDS[N], lam=lam)
            ref = orc.partition(luma, times[q], oracle_params(orc, params))
            assert_same_result(got, ref, f"{name} frame {p} ref {q}")
