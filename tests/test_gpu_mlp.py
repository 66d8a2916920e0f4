"""GPU parity of the learned CTU-time perceptron's kernels against the FP64 reference, and
of the search driven by its time map against the oracle.

Tolerances: the kernels compute in FP32 with sums of at most 64 products per layer and a
fixed-order reduction over samples; the reference is FP64.  Per output, the FP32 error is
bounded by a small multiple of 64 * 2^-24 times the sum of |terms|, so forward outputs are
checked to 2e-5 of the layer's scale and gradients (sums over thousands of samples) to
2e-4 of each tensor's norm.
"""
import warnings

import numpy as np
import pytest
import torch

import oracle
from oracle import mlp_ref
from paper_2012_14792_amd import binding as B
from paper_2012_14792_amd import synth
from paper_2012_14792_amd.mlp import TimeMLP, evaluate, training_pairs

from helpers import assert_same_result, gpu_features, oracle_params, to_device

pytestmark = pytest.mark.gpu

NAMES = ("w1", "b1", "w2", "b2", "w3", "b3")


def _weights(seed):
    rng = np.random.default_rng(seed)
    p = {"w1": rng.normal(0, 0.4, (64, 10)), "b1": rng.normal(0, 0.1, 64),
         "w2": rng.normal(0, 0.2, (64, 64)), "b2": rng.normal(0, 0.1, 64),
         "w3": rng.normal(0, 0.2, (1, 64)), "b3": rng.normal(0, 0.1, 1)}
    p32 = {k: v.astype(np.float32) for k, v in p.items()}
    return {k: v.astype(np.float64) for k, v in p32.items()}, [torch.from_numpy(p32[k]).cuda() for k in NAMES]


def _norm(seed):
    rng = np.random.default_rng(seed)
    mean = rng.normal(0, 0.2, 10).astype(np.float32)
    inv = rng.uniform(0.5, 2.0, 10).astype(np.float32)
    nm = B.MLPNorm()
    for i in range(10):
        nm.mean[i], nm.inv_std[i] = float(mean[i]), float(inv[i])
        nm.lo[i], nm.hi[i] = -1e30, 1e30
    return nm, mean.astype(np.float64), inv.astype(np.float64)


def _x(n, seed):
    return np.random.default_rng(seed).normal(0, 1.5, (n, 10)).astype(np.float32)


@pytest.mark.parametrize("wh", [(1920, 1080), (1000, 700), (128, 128), (3840, 2160)])
def test_inputs_match_reference(wh):
    w, h = wh
    frame = B.make_frame(w, h)
    luma = synth.make_frame(w, h, 11)
    f = gpu_features(frame, to_device(luma))
    W, H = B.ctu_dims(frame)
    prev = np.random.default_rng(1).integers(1, 200000, W * H).astype(np.uint32)
    x = torch.empty((W * H, 10), dtype=torch.float32, device="cuda")
    feats = {k: torch.from_numpy(v.view(np.int32) if v.dtype == np.uint32 else v.view(np.int64)).cuda()
             for k, v in f.items()}
    B.trs_mlp_inputs(frame, feats, torch.from_numpy(prev.view(np.int32)).cuda(), x)
    of = oracle.features(luma)
    ref = mlp_ref.inputs(w, h, 128, of["tex"], of["var"], of["mean"], prev)
    np.testing.assert_allclose(x.cpu().numpy(), ref, rtol=2e-7, atol=0)


@pytest.mark.parametrize("n", [1, 63, 64, 1000, 4099])
def test_forward_matches_fp64(n):
    p, ws = _weights(n)
    nm, mean, inv = _norm(n + 1)
    x = _x(n, n + 2)
    y = torch.empty(n, dtype=torch.float32, device="cuda")
    z1 = torch.empty((64, n), dtype=torch.float32, device="cuda")
    z2 = torch.empty((64, n), dtype=torch.float32, device="cuda")
    B.trs_mlp_forward(ws, nm, torch.from_numpy(x).cuda(), y, z1, z2)
    yr, (xn, zr1, _, zr2, _) = mlp_ref.forward(p, x.astype(np.float64), mean, inv)
    for got, ref in ((z1.cpu().numpy().T, zr1), (z2.cpu().numpy().T, zr2), (y.cpu().numpy(), yr)):
        scale = max(1.0, float(np.abs(ref).max()))
        assert np.abs(got - ref).max() <= 2e-5 * scale


def test_forward_without_preactivations_is_identical():
    _, ws = _weights(5)
    nm, _, _ = _norm(6)
    x = torch.from_numpy(_x(777, 7)).cuda()
    y1 = torch.empty(777, device="cuda")
    y2 = torch.empty(777, device="cuda")
    z1 = torch.empty((64, 777), device="cuda")
    z2 = torch.empty((64, 777), device="cuda")
    B.trs_mlp_forward(ws, nm, x, y1, z1, z2)
    B.trs_mlp_forward(ws, nm, x, y2)
    assert torch.equal(y1, y2)


@pytest.mark.parametrize("n", [1, 31, 2048, 40000])
def test_backward_matches_fp64(n):
    p, ws = _weights(100 + n)
    nm, mean, inv = _norm(n)
    x = _x(n, n + 3)
    dy = np.random.default_rng(n + 4).normal(0, 1, n).astype(np.float32)
    xd = torch.from_numpy(x).cuda()
    y = torch.empty(n, device="cuda")
    z1 = torch.empty((64, n), device="cuda")
    z2 = torch.empty((64, n), device="cuda")
    B.trs_mlp_forward(ws, nm, xd, y, z1, z2)
    grads = [torch.full_like(t, float("nan")) for t in ws]
    B.trs_mlp_backward(ws, nm, xd, z1, z2, torch.from_numpy(dy).cuda(), grads)
    _, cache = mlp_ref.forward(p, x.astype(np.float64), mean, inv)
    gr = mlp_ref.backward(p, cache, dy.astype(np.float64))
    for k, g in zip(NAMES, grads):
        got, ref = g.cpu().numpy().astype(np.float64), gr[k]
        assert got.shape == ref.shape, k
        assert np.linalg.norm(got - ref) <= 2e-4 * max(np.linalg.norm(ref), 1e-3), k
    # fixed summation order: a second call repeats every bit
    again = [torch.empty_like(t) for t in ws]
    B.trs_mlp_backward(ws, nm, xd, z1, z2, torch.from_numpy(dy).cuda(), again)
    for a, b in zip(grads, again):
        assert torch.equal(a, b)


def test_autograd_function_matches_direct_calls():
    torch.manual_seed(0)
    m = TimeMLP(seed=3)
    X = torch.randn(5000, 10, device="cuda") * 3 + 1
    T = torch.rand(5000, device="cuda") * 3
    m.fit_norm(X)
    y = m(X)
    loss = torch.mean((y - T) ** 2)
    loss.backward()
    dy = (2.0 / 5000) * (y.detach() - T)
    z1 = torch.empty((64, 5000), device="cuda")
    z2 = torch.empty((64, 5000), device="cuda")
    y2 = torch.empty(5000, device="cuda")
    ws = [t.detach() for t in m.parameters()]
    B.trs_mlp_forward(ws, m.norm, X, y2, z1, z2)
    assert torch.equal(y.detach(), y2)
    grads = [torch.empty_like(t) for t in ws]
    B.trs_mlp_backward(ws, m.norm, X, z1, z2, dy.contiguous(), grads)
    for p, g in zip(m.parameters(), grads):
        assert torch.allclose(p.grad, g, rtol=1e-5, atol=1e-7)


def _cost_expected(y, x, lo, hi, tex, prev, blend):
    """Host restatement of the time-map rule (single FP32 multiply, round half to even)."""
    a, b, wp = blend
    out = np.empty(y.size, dtype=np.uint32)
    nfb = 0
    for c in range(y.size):
        ok = np.isfinite(y[c]) and bool(np.all((x[c] >= lo) & (x[c] <= hi)))
        if ok:
            us = np.rint(np.float32(1000.0) * y[c])
            out[c] = 1 if us < 1 else (0x7FFFFFFF if us >= 2.0**31 else int(us))
            continue
        model = a + b * int(tex[c])
        v = model if prev is None else (int(prev[c]) if wp == 256 else (wp * int(prev[c]) + (256 - wp) * model + 128) >> 8)
        out[c] = min(v, 0x7FFFFFFF)
        nfb += 1
    return out, nfb


@pytest.mark.parametrize("blend", [(200, 3, 256), (150, 2, 96)])
def test_cost_rule_and_fallback(blend):
    n = 2000
    rng = np.random.default_rng(9)
    y = rng.uniform(-0.5, 4.0, n).astype(np.float32)
    y[::97] = np.nan
    y[5::101] = np.inf
    y[7::103] = 3.0e6
    y[11::89] = 0.0004999
    x = rng.uniform(0, 10, (n, 10)).astype(np.float32)
    x[3::53, 4] = 11.0
    x[4::59, 9] = -0.5
    lo = np.zeros(10, np.float32)
    hi = np.full(10, 10.0, np.float32)
    nm = B.MLPNorm()
    for i in range(10):
        nm.mean[i], nm.inv_std[i], nm.lo[i], nm.hi[i] = 0.0, 1.0, float(lo[i]), float(hi[i])
    tex = rng.integers(0, 5000, n).astype(np.uint32)
    prev = rng.integers(1, 100000, n).astype(np.uint32)
    frame = B.make_frame(128 * 50, 128 * 40)
    cost = torch.empty(n, dtype=torch.int32, device="cuda")
    nfb = torch.zeros(1, dtype=torch.int32, device="cuda")
    dev = lambda a: torch.from_numpy(a.view(np.int32) if a.dtype == np.uint32 else a).cuda()  # noqa: E731
    B.trs_mlp_cost(frame, dev(y), dev(x), nm, dev(tex), dev(prev), B.Blend(*blend), cost, nfb)
    exp, n_exp = _cost_expected(y, x, lo, hi, tex, prev, blend)
    np.testing.assert_array_equal(cost.cpu().numpy().view(np.uint32), exp)
    assert int(nfb.item()) == n_exp and n_exp > 0


@pytest.mark.parametrize("name", ["fhd_n4", "uhd_n8"])
def test_search_on_predicted_map_matches_oracle(name):
    """Search driven by a learned time map: the map is the FP64 reference's prediction,
    rounded by the library's time-map rule on the GPU; the oracle searches the host map
    built by the same rule."""
    cfg = synth.CONFIGS[name]
    w, h = cfg["width"], cfg["height"]
    frame = B.make_frame(w, h)
    gen = synth.SequenceGenerator(w, h, cfg["seed"], cfg["drift"])
    l0, l1 = gen.frame(0), gen.frame(1)
    f0, f1 = oracle.features(l0), oracle.features(l1)
    prev, _ = oracle.cost_map(f0["tex"], None)
    x = mlp_ref.inputs(w, h, 128, f1["tex"], f1["var"], f1["mean"], prev)
    rng = np.random.default_rng(2)
    p = {"w1": rng.normal(0, 0.3, (64, 10)), "b1": rng.normal(0, 0.1, 64),
         "w2": rng.normal(0, 0.15, (64, 64)), "b2": rng.normal(0, 0.1, 64),
         "w3": rng.normal(0, 0.1, (1, 64)), "b3": np.array([1.0])}
    mean, std = x.mean(0), x.std(0) + 1e-6
    y, _ = mlp_ref.forward(p, x, mean, 1.0 / std)
    y = np.abs(y).astype(np.float32) + np.float32(0.2)
    x32 = x.astype(np.float32)
    nm = B.MLPNorm()
    for i in range(10):
        nm.mean[i], nm.inv_std[i] = float(mean[i]), float(1 / std[i])
        nm.lo[i], nm.hi[i] = -1e30, 1e30
    n = y.size
    cost = torch.empty(n, dtype=torch.int32, device="cuda")
    dev = lambda a: torch.from_numpy(a.view(np.int32) if a.dtype == np.uint32 else a).cuda()  # noqa: E731
    B.trs_mlp_cost(frame, dev(y), dev(x32), nm, dev(f1["tex"]), dev(prev), B.Blend(200, 3, 256), cost)
    exp, _ = _cost_expected(y, x32, np.full(10, -1e30, np.float32), np.full(10, 1e30, np.float32),
                            f1["tex"], prev, (200, 3, 256))
    np.testing.assert_array_equal(cost.cpu().numpy().view(np.uint32), exp)
    params = B.make_params(cfg["n_threads"], cfg["max_tile_cols"], cfg["max_tile_rows"],
                           cfg["max_rs_per_tile"], lam=cfg["lam"])
    gf = gpu_features(frame, to_device(l1))
    ws = torch.empty(B.trs_search_workspace(frame, params), dtype=torch.uint8, device="cuda")
    out = torch.empty(B.RESULT_BYTES, dtype=torch.uint8, device="cuda")
    B.trs_search(frame, params, cost, dev(gf["s1"]), torch.from_numpy(gf["s2"].view(np.int64)).cuda(), ws, out)
    got = B.read_result(out)
    ref = oracle.search(w, h, oracle_params(oracle, params), exp, f1["s1"], f1["s2"])
    assert_same_result(got, ref, name)


def test_gradcheck_fp32():
    """torch.autograd.gradcheck of the Function (FP32 kernels, so central differences with
    a large step and loose tolerances)."""
    m = TimeMLP(seed=1)
    X = torch.randn(40, 10, device="cuda")
    m.fit_norm(X)
    fn = lambda *ws: _call(m, X, ws)  # noqa: E731
    ws = [p.detach().clone().requires_grad_() for p in m.parameters()]
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")     # gradcheck warns about non-double inputs
        assert torch.autograd.gradcheck(fn, ws, eps=1e-2, atol=2e-3, rtol=2e-2, fast_mode=True)


def _call(m, X, ws):
    from paper_2012_14792_amd.mlp import _MLPFunction
    return _MLPFunction.apply(X, m, *ws)


def test_nonfinite_weights_fall_back_to_plain_blend():
    w, h = 1920, 1080
    frame = B.make_frame(w, h)
    luma = synth.make_frame(w, h, 3)
    f = gpu_features(frame, to_device(luma))
    W, H = B.ctu_dims(frame)
    prev = np.random.default_rng(2).integers(100, 9000, W * H).astype(np.uint32)
    dev = lambda a: torch.from_numpy(a.view(np.int32)).cuda()  # noqa: E731
    feats = {k: torch.from_numpy(v.view(np.int32) if v.dtype == np.uint32 else v.view(np.int64)).cuda()
             for k, v in f.items()}
    m = TimeMLP(seed=0)
    with torch.no_grad():
        m.w2[3, 5] = float("nan")
    x = torch.empty((W * H, 10), device="cuda")
    B.trs_mlp_inputs(frame, feats, dev(prev), x)
    nfb = torch.zeros(1, dtype=torch.int32, device="cuda")
    for blend in [(200, 3, 256), (200, 3, 128)]:
        nfb.zero_()
        cost = m.cost_map(frame, x, dev(f["tex"]), dev(prev), blend, n_fallback=nfb)
        exp, _ = oracle.cost_map(oracle.features(luma)["tex"], prev, *blend)
        np.testing.assert_array_equal(cost.cpu().numpy().view(np.uint32), exp)
        assert int(nfb.item()) == W * H


@pytest.fixture(scope="module")
def trained():
    X, T = training_pairs(120_000, seed=5, frames_per_seq=40)
    m = TimeMLP(seed=0)
    m.fit_norm(X)
    hist = m.train(X, T, epochs=30, batch=2048, lr=3e-3)
    return m, hist


def test_training_reduces_loss(trained):
    _, hist = trained
    assert np.all(np.isfinite(hist))
    assert hist[-1] < 0.5 * hist[0]


def test_trained_predictor_beats_previous_frame_estimate(trained):
    """What the learned predictor gains over the method without it, on frames of sequences
    it was not trained on: a lower per-CTU squared error than the previous-frame estimate."""
    m, _ = trained
    s = evaluate(m, n_frames=17, seed=6, width=1920, height=1080, bounds=(4, 3, 3, 2))
    assert s["frames"] == 16
    assert s["per_ctu"]["mlp"]["ctu_mse_ms2"] < 0.97 * s["per_ctu"]["plain"]["ctu_mse_ms2"]
    assert 0 <= s["fallback_ctus"] < 16 * 135
    for lk in ("0/1", "1/10"):
        for k in ("plain", "mlp"):
            d = s["decisions"][lk][k]
            assert 0 <= d["makespan_err"] < 1 and 0 <= d["agree"] <= 1
        assert s["decisions"][lk]["mlp"]["regret"] >= -0.5
    # at lambda = 0 the regret is never negative: P* minimises the true makespan
    assert s["decisions"]["0/1"]["plain"]["regret"] >= 0 and s["decisions"]["0/1"]["mlp"]["regret"] >= 0
