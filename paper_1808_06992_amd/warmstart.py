"""Learned ADMM warm start: training data from the method's own solves, GPU
training of the network, and evaluation against the cold start.

Every numerical step runs in libuoi kernels (Gram, ADMM solves, dataset
normalisation, network forward/backward/Adam); this module only sequences the
calls and shuffles mini-batches.  The network is not part of the paper (its
ADMM starts cold); it is judged by the ADMM iterations needed to reach the same
float64 KKT tolerance, with the cold start as the per-solve fallback.
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import _lib as api
from . import synth

__all__ = ["init_theta", "problem_pairs", "make_training_set", "train", "fit_network", "evaluate"]


def init_theta(n_in: int, hidden: int, n_out: int, seed: int = 0) -> torch.Tensor:
    """He-uniform weights, zero biases, in the flat order W1 b1 W2 b2 W3 b3
    (W stored [out][in]) that uoi_mlp_set_params takes."""
    rng = np.random.default_rng(seed)
    parts = []
    for fi, fo in ((n_in, hidden), (hidden, hidden), (hidden, n_out)):
        lim = np.sqrt(6.0 / fi)
        parts.append(rng.uniform(-lim, lim, size=fo * fi))
        parts.append(np.zeros(fo))
    return torch.as_tensor(np.concatenate(parts).astype(np.float32), device="cuda")


def problem_pairs(pr, seed: int, B1: int, kkt_tol: float = 1e-8):
    """(inputs, targets) of the B1 x q selection solves of one problem."""
    n, p = pr.X.shape
    X = torch.as_tensor(pr.X, device="cuda")
    y = torch.as_tensor(pr.y, device="cuda")
    rows = api.bootstrap_rows(seed, B1, n)
    G, c = api.gram(X, rows, y)
    c = c[:, :, 0].contiguous()
    res = api.lasso_solve_batch(G, c, pr.lambdas, kkt_tol=kkt_tol, max_iter=50000)
    return api.ws_dataset(c, pr.lambdas, res["z"])


def make_training_set(seeds, B1: int = 8, M: int = 64, kkt_tol: float = 1e-8, **gen_kw):
    """Solves of the workload distribution: for each design seed, M independent
    (beta, noise) draws (distinct supports) on B1 bootstraps at every lambda,
    solved by one batched multi-response ADMM sweep per design."""
    xs, ts = [], []
    for sd in seeds:
        Xn, Y, _, lam = synth.lasso_toeplitz_responses(sd, M, **gen_kw)
        n = Xn.shape[0]
        X = torch.as_tensor(Xn, device="cuda")
        Yd = torch.as_tensor(Y, device="cuda")
        rows = api.bootstrap_rows(sd, B1, n)
        G, Cm = api.gram(X, rows, Yd)
        res = api.lasso_solve_multi(G, Cm, lam, kkt_tol=kkt_tol, max_iter=50000)
        x, t = api.ws_dataset(Cm, lam, res["z"])
        xs.append(x)
        ts.append(t)
        del G, Cm, res
    return torch.cat(xs), torch.cat(ts)


def train(net: "api.MLP", X: torch.Tensor, T: torch.Tensor, *, epochs: int = 10, batch: int = 512,
          lr: float = 1e-3, seed: int = 0, log=None):
    """Adam on mini-batches of a shuffled order; returns the loss of the last
    mini-batch of every epoch (read back once per epoch, not per step)."""
    g = torch.Generator(device="cpu").manual_seed(seed)
    n = X.shape[0]
    hist = []
    for ep in range(epochs):
        perm = torch.randperm(n, generator=g).to(X.device)
        step_lr = lr * (0.5 ** (ep // max(1, epochs // 3)))
        starts = list(range(0, n, batch))
        last = None
        for s0 in starts:
            idx = perm[s0:s0 + batch]
            xb = X.index_select(0, idx).contiguous()
            tb = T.index_select(0, idx).contiguous()
            last = net.train_step(xb, tb, step_lr, want_loss=(s0 == starts[-1]))
        hist.append(last)
        if log:
            log(f"epoch {ep}: loss {hist[-1]:.4e}")
    return hist


def fit_network(seeds, *, B1: int = 8, M: int = 64, hidden: int = 512, epochs: int = 30,
                batch: int = 512, lr: float = 2e-3, init_seed: int = 7, log=None, **gen_kw):
    """Training set from the given design seeds, then a freshly initialised
    network trained on it.  Returns (net, loss history, number of training solves)."""
    X, T = make_training_set(seeds, B1=B1, M=M, **gen_kw)
    p = T.shape[1]
    net = api.MLP(p + 1, hidden, p)
    net.set_params(init_theta(p + 1, hidden, p, init_seed))
    hist = train(net, X, T, epochs=epochs, batch=batch, lr=lr, log=log)
    return net, hist, int(X.shape[0])


def evaluate(net, seeds, gen=synth.lasso_toeplitz, B1: int = 48, B2: int = 48, kkt_tol: float = 1e-6,
             precision: str = "mixed", check_every: int = 10, **gen_kw):
    """Cold versus network start on held-out problems: iterations, time, agreement.
    With check_every = 1 the iteration counts are exact (otherwise they are
    rounded up to the KKT check period); save_mean is the mean over solves of
    (cold - network) iterations, frac_saved / frac_worse the shares of solves
    that needed fewer / more iterations from the network start."""
    rows = []
    for sd in seeds:
        pr = gen(sd, **gen_kw)
        X = torch.as_tensor(pr.X, device="cuda")
        y = torch.as_tensor(pr.y, device="cuda")
        res = {}
        for name, kw in (("cold", {}), ("mlp", {"mlp": net})):
            api.lasso_fit(X, y, pr.lambdas, B1, B2, sd, kkt_tol=kkt_tol, precision=precision,
                          check_every=check_every, **kw)  # warm
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            out = api.lasso_fit(X, y, pr.lambdas, B1, B2, sd, kkt_tol=kkt_tol, precision=precision,
                                check_every=check_every, sel_beta=True, timing=True, **kw)
            torch.cuda.synchronize()
            out["wall_ms"] = 1000 * (time.perf_counter() - t0)
            res[name] = out
        it_c = res["cold"]["iters"].double()
        it_m = res["mlp"]["iters"].double()
        d = it_c - it_m
        sb_c = res["cold"]["sel_beta"]
        sb_m = res["mlp"]["sel_beta"]
        scale = sb_c.abs().amax(dim=-1, keepdim=True).clamp_min(1e-300)
        rows.append(dict(
            seed=sd,
            mean_iters_cold=float(it_c.mean()), mean_iters_mlp=float(it_m.mean()),
            save_mean=float(d.mean()), frac_saved=float((d > 0).double().mean()),
            frac_worse=float((d < 0).double().mean()),
            max_iters_cold=int(it_c.max()), max_iters_mlp=int(it_m.max()),
            admm_ms_cold=res["cold"]["stage_ms"]["admm"], admm_ms_mlp=res["mlp"]["stage_ms"]["admm"],
            fit_ms_cold=res["cold"]["wall_ms"], fit_ms_mlp=res["mlp"]["wall_ms"],
            warm_used=res["mlp"]["warm_used"], solves=int(it_c.numel()),
            unconverged_mlp=res["mlp"]["n_unconverged"],
            max_rel_diff=float(((sb_c - sb_m).abs() / scale).max()),
            same_supports=bool(torch.equal(res["cold"]["supports"], res["mlp"]["supports"])),
        ))
    return rows
