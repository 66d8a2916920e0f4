"""Learned per-CTU time predictor on the library's HIP kernels.

The paper's estimator (Section 2.1) predicts a CTU's encoding time by the measured time of
the co-located CTU in the previous frame of the same temporal layer; its conclusion names a
better estimator as future work.  TimeMLP is such an estimator: a 10 -> 64 -> 64 -> 1
perceptron (exact GELU, FP32) over the CTU's own features (texture, variance, mean), its
neighbours' textures, its previous time, its neighbours' previous times and its area
fraction, predicting the current time in milliseconds.

Forward and backward run in the library's kernels (trs_mlp_forward / trs_mlp_backward),
wrapped as a torch.autograd.Function; the optimiser is torch's Adam.  Predictions become a
u32 time map through trs_mlp_cost, which falls back per CTU to the plain blend when a
prediction is not finite or an input lies outside the training range; the search then runs
unchanged on that map.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import binding as B
from . import synth

N_IN, N_HID = 10, 64


class _MLPFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, model, w1, b1, w2, b2, w3, b3):
        n = x.shape[0]
        y = torch.empty(n, dtype=torch.float32, device=x.device)
        z1 = torch.empty((N_HID, n), dtype=torch.float32, device=x.device)
        z2 = torch.empty((N_HID, n), dtype=torch.float32, device=x.device)
        ws = (w1, b1, w2, b2, w3, b3)
        B.trs_mlp_forward(ws, model.norm, x, y, z1, z2)
        ctx.save_for_backward(x, w1, b1, w2, b2, w3, b3, z1, z2)
        ctx.norm = model.norm
        return y

    @staticmethod
    def backward(ctx, dy):
        x, w1, b1, w2, b2, w3, b3, z1, z2 = ctx.saved_tensors
        ws = (w1, b1, w2, b2, w3, b3)
        grads = [torch.empty_like(t) for t in ws]
        B.trs_mlp_backward(ws, ctx.norm, x, z1, z2, dy.contiguous(), grads)
        return (None, None, *grads)


class TimeMLP:
    def __init__(self, seed: int = 0, device="cuda"):
        g = torch.Generator().manual_seed(seed)

        def dense(o, i, scale=1.0):
            return (torch.randn(o, i, generator=g, dtype=torch.float32) * scale * math.sqrt(2.0 / i)).to(device)

        self.w1 = dense(N_HID, N_IN).requires_grad_()
        self.b1 = torch.zeros(N_HID, device=device).requires_grad_()
        self.w2 = dense(N_HID, N_HID).requires_grad_()
        self.b2 = torch.zeros(N_HID, device=device).requires_grad_()
        self.w3 = dense(1, N_HID, 0.1).requires_grad_()
        self.b3 = torch.zeros(1, device=device).requires_grad_()
        self.norm = B.MLPNorm()
        for i in range(N_IN):
            self.norm.mean[i], self.norm.inv_std[i] = 0.0, 1.0
            self.norm.lo[i], self.norm.hi[i] = -float("inf"), float("inf")

    def parameters(self):
        return [self.w1, self.b1, self.w2, self.b2, self.w3, self.b3]

    def fit_norm(self, X: torch.Tensor) -> None:
        """Standardisation constants and the training range, from training inputs X [n][10]."""
        Xd = X.double()
        mean, std = Xd.mean(0), Xd.std(0).clamp_min(1e-6)
        lo, hi = X.min(0).values, X.max(0).values
        for i in range(N_IN):
            self.norm.mean[i] = float(mean[i])
            self.norm.inv_std[i] = float(1.0 / std[i])
            self.norm.lo[i] = float(lo[i])
            self.norm.hi[i] = float(hi[i])

    def __call__(self, x: torch.Tensor) -> torch.Tensor:
        return _MLPFunction.apply(x, self, *self.parameters())

    @torch.no_grad()
    def predict(self, x: torch.Tensor) -> torch.Tensor:
        y = torch.empty(x.shape[0], dtype=torch.float32, device=x.device)
        B.trs_mlp_forward(self.parameters(), self.norm, x, y)
        return y

    def train(self, X: torch.Tensor, T_ms: torch.Tensor, epochs: int = 4, batch: int = 8192,
              lr: float = 3e-3, seed: int = 0, log=None) -> list:
        """Adam on the mean squared error of the predicted times (milliseconds), with the
        learning rate decayed to zero on a cosine over all steps.  Returns the mean training
        loss of each epoch."""
        opt = torch.optim.Adam(self.parameters(), lr=lr, fused=X.is_cuda)
        n = X.shape[0]
        per_epoch = (n + batch - 1) // batch
        total = max(1, epochs * per_epoch)
        sched = torch.optim.lr_scheduler.LambdaLR(
            opt, lambda k: 0.5 * (1.0 + math.cos(math.pi * min(k, total) / total)))
        gen = torch.Generator(device=X.device).manual_seed(seed)
        hist = []
        for ep in range(epochs):
            perm = torch.randperm(n, generator=gen, device=X.device)
            tot = torch.zeros((), dtype=torch.float64, device=X.device)
            for s in range(0, n, batch):
                idx = perm[s:s + batch]
                y = self(X[idx].contiguous())
                loss = torch.mean((y - T_ms[idx]) ** 2)
                opt.zero_grad(set_to_none=True)
                loss.backward()
                opt.step()
                sched.step()
                tot += loss.detach().double() * idx.numel()
            hist.append(float(tot) / n)
            if log:
                log(f"epoch {ep}: mse {hist[-1]:.6f} ms^2")
        return hist

    @torch.no_grad()
    def cost_map(self, frame, x, tex, prev, blend=(200, 3, 256), cost=None, n_fallback=None):
        """u32 time map (as int32 tensor) from the prediction, with per-CTU fallback."""
        y = self.predict(x)
        if cost is None:
            cost = torch.empty(x.shape[0], dtype=torch.int32, device=x.device)
        B.trs_mlp_cost(frame, y, x, self.norm, tex, prev, B.Blend(*blend), cost, n_fallback)
        return cost

    def state_dict(self) -> dict:
        d = {k: getattr(self, k).detach().cpu() for k in ("w1", "b1", "w2", "b2", "w3", "b3")}
        for f in ("mean", "inv_std", "lo", "hi"):
            d[f] = torch.tensor(list(getattr(self.norm, f)), dtype=torch.float32)
        return d

    def load_state_dict(self, d: dict) -> None:
        with torch.no_grad():
            for k in ("w1", "b1", "w2", "b2", "w3", "b3"):
                getattr(self, k).copy_(d[k])
        for f in ("mean", "inv_std", "lo", "hi"):
            arr = getattr(self.norm, f)
            for i in range(N_IN):
                arr[i] = float(d[f][i])


def training_pairs(n_pairs: int, seed: int = 5, frames_per_seq: int = 58, device="cuda",
                   width: int = 1920, height: int = 1080, log=None):
    """(inputs, target ms) pairs: 1080p drifting sequences rendered on the device; features
    from the library's feature kernel; times from the synthetic AR(1) model; inputs from
    trs_mlp_inputs with the previous frame's times."""
    frame = B.make_frame(width, height)
    W, H = B.ctu_dims(frame)
    n_ctu = W * H
    feats = B.alloc_features(frame, device)
    X = torch.empty((n_pairs, N_IN), dtype=torch.float32, device=device)
    T = torch.empty(n_pairs, dtype=torch.float32, device=device)
    xb = torch.empty((n_ctu, N_IN), dtype=torch.float32, device=device)
    filled, s = 0, 0
    while filled < n_pairs:
        gen = synth.TorchSequenceGenerator(width, height, seed * 100000 + s, 8.0, device)
        eps = synth.ar1_eps(n_ctu, frames_per_seq, seed * 100000 + 50000 + s)
        prev = None
        for f in range(frames_per_seq):
            B.trs_features(frame, gen.frame(f), feats)
            tex = feats["tex"].cpu().numpy().view(np.uint32)
            tf = synth.ctu_times(tex, eps[f])
            if prev is not None and filled < n_pairs:
                B.trs_mlp_inputs(frame, feats, torch.from_numpy(prev.view(np.int32)).to(device), xb)
                k = min(n_ctu, n_pairs - filled)
                X[filled:filled + k] = xb[:k]
                T[filled:filled + k] = torch.from_numpy(tf[:k].astype(np.float32) / 1000.0).to(device)
                filled += k
            prev = tf
        s += 1
        if log and s % 32 == 0:
            log(f"training pairs: {filled}/{n_pairs}")
    return X, T


def _true_makespan(rects, truth_map: np.ndarray) -> int:
    return max(int(truth_map[y0:y1, x0:x1].sum()) for (x0, y0, x1, y1) in rects)


@torch.no_grad()
def evaluate(model: TimeMLP, n_frames: int = 64, seed: int = 6, width: int = 3840, height: int = 2160,
             bounds=(8, 6, 4, 4), lams=((0, 1), (1, 10)), blend=(200, 3, 256), device="cuda") -> dict:
    """Both estimators on new frames, each feeding the same search, at each lambda.

    For frames f = 1 .. n_frames - 1 with measured times T_f (synthetic truth), per lambda:
      makespan_err  |T~(P) - T_f(P)| / T_f(P) for the partition P the estimator leads to;
      regret        T_f(P) / T_f(P*) - 1, P* the partition the same search picks on T_f;
      agree         fraction of frames with rank(P) = rank(P*);
    and per estimator the per-CTU errors ctu_mae_ms and ctu_mse_ms2 (the training loss).
    lambda = 0 isolates the time estimate (step 1 alone decides); at lambda > 0 step 2's
    quality term picks among partitions within the bound.
    """
    N, C, R, K = bounds
    plist = {f"{a}/{b}": B.make_params(N, C, R, K, lam=(a, b)) for a, b in lams}
    frame = B.make_frame(width, height)
    W, H = B.ctu_dims(frame)
    gen = synth.TorchSequenceGenerator(width, height, seed, 8.0, device)
    eps = synth.ar1_eps(W * H, n_frames, seed * 1000 + 7)
    feats = B.alloc_features(frame, device)
    ws = torch.empty(max(B.trs_search_workspace(frame, p) for p in plist.values()),
                     dtype=torch.uint8, device=device)
    out = torch.empty(B.RESULT_BYTES, dtype=torch.uint8, device=device)
    x = torch.empty((W * H, N_IN), dtype=torch.float32, device=device)
    nfb = torch.zeros(1, dtype=torch.int32, device=device)
    est = ("plain", "mlp")
    per_ctu = {k: {"ctu_mae_ms": [], "ctu_mse_ms2": []} for k in est}
    dec = {lk: {k: {"makespan_err": [], "regret": [], "agree": []} for k in est} for lk in plist}
    prev = None
    for f in range(n_frames):
        B.trs_features(frame, gen.frame(f), feats)
        tex = feats["tex"].cpu().numpy().view(np.uint32)
        tf = synth.ctu_times(tex, eps[f])
        if prev is not None:
            prev_d = torch.from_numpy(prev.view(np.int32)).to(device)
            B.trs_mlp_inputs(frame, feats, prev_d, x)
            plain = B.trs_cost_map(frame, feats["tex"], prev_d, B.Blend(*blend), torch.empty_like(prev_d))
            maps = {"plain": plain, "mlp": model.cost_map(frame, x, feats["tex"], prev_d, blend, n_fallback=nfb),
                    "true": torch.from_numpy(tf.view(np.int32)).to(device)}
            for k in est:
                pred = maps[k].cpu().numpy().view(np.uint32).astype(np.float64)
                per_ctu[k]["ctu_mae_ms"].append(float(np.mean(np.abs(pred - tf))) / 1000.0)
                per_ctu[k]["ctu_mse_ms2"].append(float(np.mean((pred - tf) ** 2)) / 1e6)
            truth = tf.reshape(H, W).astype(np.int64)
            for lk, params in plist.items():
                res = {}
                for k, cmap in maps.items():
                    B.trs_search(frame, params, cmap, feats["s1"], feats["s2"], ws, out)
                    res[k] = B.read_result(out)
                t_star = _true_makespan(res["true"]["rs"], truth)
                for k in est:
                    t_true = _true_makespan(res[k]["rs"], truth)
                    dec[lk][k]["makespan_err"].append(abs(res[k]["t_sel"] - t_true) / t_true)
                    dec[lk][k]["regret"].append(t_true / t_star - 1.0)
                    dec[lk][k]["agree"].append(float(res[k]["rank"] == res["true"]["rank"]))
        prev = tf
    mean = lambda d: {m: float(np.mean(v)) for m, v in d.items()}  # noqa: E731
    summary = {"frames": n_frames - 1, "per_ctu": {k: mean(per_ctu[k]) for k in est},
               "decisions": {lk: {k: mean(dec[lk][k]) for k in est} for lk in plist},
               "fallback_ctus": int(nfb.item())}
    return summary

def main(argv=None):
    """Train on 1080p sequences and evaluate on new 4K frames against the plain blend:

        python -m paper_2012_14792_amd.mlp --pairs 2000000 --eval-frames 64 --save w.pt
    """
    import argparse
    import json
    import sys
    import time

    ap = argparse.ArgumentParser()
    ap.add_argument("--pairs", type=int, default=2_000_000)
    ap.add_argument("--epochs", type=int, default=8)
    ap.add_argument("--batch", type=int, default=8192)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--train-seed", type=int, default=5)
    ap.add_argument("--eval-frames", type=int, default=64)
    ap.add_argument("--eval-seed", type=int, default=6)
    ap.add_argument("--save", default=None)
    args = ap.parse_args(argv)
    log = lambda m: print(m, file=sys.stderr, flush=True)   # noqa: E731
    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    X, T = training_pairs(args.pairs, seed=args.train_seed, log=log)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    log(f"{args.pairs} pairs in {t1 - t0:.1f} s")
    m = TimeMLP(seed=0)
    m.fit_norm(X)
    hist = m.train(X, T, epochs=args.epochs, batch=args.batch, lr=args.lr, log=log)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    log(f"trained in {t2 - t1:.1f} s")
    if args.save:
        torch.save(m.state_dict(), args.save)
    res = evaluate(m, n_frames=args.eval_frames, seed=args.eval_seed)
    t3 = time.perf_counter()
    print(json.dumps({"pairs": args.pairs, "epochs": args.epochs, "batch": args.batch,
                      "train_loss": hist, "pairs_s": t1 - t0, "train_s": t2 - t1, "eval_s": t3 - t2,
                      "eval": res}))


if __name__ == "__main__":
    main()
