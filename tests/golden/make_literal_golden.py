"""Writes literal_uhd_n8.json: the oracle's exact literal-space decision for one 4K frame.

The input is frame 1 of the seeded drifting 4K sequence (generator seed 2, drift 8 px/frame)
with the previous frame's synthetic measured times as the prediction, N = 8, tiles <= 6 x 4,
<= 4 RS per tile, lambda = 1/10, every CTU boundary allowed.  Only oracle/ computes the result
(about a minute on one core).

    python tests/golden/make_literal_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as orc  # noqa: E402
from paper_2012_14792_amd import synth  # noqa: E402


def inputs():
    w, h = 3840, 2160
    gen = synth.SequenceGenerator(w, h, 2, 8.0)
    W, H = orc.ctu_dims(w, h)
    f0 = orc.features(gen.frame(0))
    luma = gen.frame(1)
    f = orc.features(luma)
    prev = synth.ctu_times(f0["tex"], synth.ar1_eps(W * H, 1, 2000)[0])
    cost, _ = orc.cost_map(f["tex"], prev)
    return w, h, luma, f, prev, cost


def main():
    w, h, luma, f, prev, cost = inputs()
    p = orc.make_params(8, 6, 4, 4, lam=(1, 10), dtile=-1, drs=-1)
    res = orc.literal_search(w, h, p, cost, f["s1"], f["s2"])
    res["rs"] = [list(r) for r in res["rs"]]
    with open(os.path.join(HERE, "literal_uhd_n8.json"), "w") as fh:
        json.dump({"source": "oracle.literal_search on frame 1 of synth.SequenceGenerator(3840, 2160, 2, 8.0); "
                             "prev = synth.ctu_times(tex of frame 0, synth.ar1_eps(510, 1, 2000)[0]); "
                             "N = 8, Cmax 6, Rmax 4, Kmax 4, lambda 1/10, area k 3, literal space",
                   "result": res}, fh, indent=1)


if __name__ == "__main__":
    main()
