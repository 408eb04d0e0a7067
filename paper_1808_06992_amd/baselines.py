"""Non-learned accelerators of the selection sweep, measured as baselines for the
learned warm start.

* pathwise(): lambda continuation.  Each bootstrap's q lambdas (decreasing) run
  in `groups` consecutive blocks; block g starts every solve from the block
  g - 1 solution (z, u) at its smallest lambda, the nearest one.  Block 0 starts
  cold.  In the batched sweep every solve of a bootstrap shares one read of M
  per iteration, so a block costs as many iterations as its slowest solve, and
  the blocks run one after another.
* strong_rule(): the sequential strong rule (Tibshirani et al., 2012).  For
  bootstrap k and lambda_j it keeps feature i when i is in the support at
  lambda_{j-1} or |c_i - (G beta(lambda_{j-1}))_i| >= 2 lambda_j - lambda_{j-1}.
  It reports the kept-set sizes, the rule's violations (features the rule drops
  that are nonzero at lambda_j) and the per-iteration bytes that a reduced
  problem per solve would read, against the shared M of the batched sweep.

The solves run in libuoi kernels (Gram, factor, ADMM with warm starts); this
module sequences the calls, and the strong rule's bookkeeping on the solutions
is done on the host.  Run as
    python -m paper_1808_06992_amd.baselines [--groups 2 4 8] [--seed 0]
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np
import torch

from . import _lib as api
from . import synth

__all__ = ["pathwise", "strong_rule", "main"]


def _statistics(pr, seed: int, B1: int):
    n = pr.X.shape[0]
    X = torch.as_tensor(pr.X, device="cuda")
    y = torch.as_tensor(pr.y, device="cuda")
    rows = api.bootstrap_rows(seed, B1, n)
    G, c = api.gram(X, rows, y)
    return G, c[:, :, 0].contiguous()


def _timed(fn):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = fn()
    torch.cuda.synchronize()
    return out, 1000 * (time.perf_counter() - t0)


def pathwise(pr, seed: int = 0, B1: int = 48, groups=(2, 4, 8), kkt_tol: float = 1e-6,
             precision: str = "fp64", relax: float = 1.8, check_every: int = 1):
    """Cold start at every lambda against lambda continuation in blocks.
    Iteration counts are exact at check_every = 1.  Times are wall clock per
    solve_batch call minus one factorization each (every call factors G + rho I
    again; a continuation inside one fit would factor once)."""
    G, c = _statistics(pr, seed, B1)
    lam = np.asarray(pr.lambdas, dtype=np.float64)
    q = lam.size
    kw = dict(kkt_tol=kkt_tol, precision=precision, relax=relax, check_every=check_every, max_iter=50000)
    _, t_factor = _timed(lambda: api.spd_inverse(G, 1.0))
    _, t_factor = _timed(lambda: api.spd_inverse(G, 1.0))
    api.lasso_solve_batch(G, c, lam, **kw)  # warm-up of the shape
    cold, t_cold = _timed(lambda: api.lasso_solve_batch(G, c, lam, **kw))
    it_cold = cold["iters"].cpu().numpy()  # [B1, q]
    res = dict(config=dict(n=pr.X.shape[0], p=pr.X.shape[1], B1=B1, q=q, kkt_tol=kkt_tol, precision=precision,
                           relax=relax, check_every=check_every),
               factor_ms=t_factor,
               cold=dict(mean_iters=float(it_cold.mean()), sweep_iters=int(it_cold.max(axis=1).max()),
                         sum_block_max=int(it_cold.max(axis=1).max()), admm_ms=t_cold - t_factor),
               path={})
    z_cold = cold["z"]
    for ng in groups:
        bounds = np.linspace(0, q, ng + 1).round().astype(int)
        z_prev = u_prev = None
        its = np.zeros_like(it_cold)
        t_admm = 0.0
        block_max = []
        zs = []
        for g in range(ng):
            j0, j1 = bounds[g], bounds[g + 1]
            z0 = u0 = None
            if z_prev is not None:
                z0 = z_prev[:, -1:, :].expand(-1, j1 - j0, -1).contiguous()
                u0 = u_prev[:, -1:, :].expand(-1, j1 - j0, -1).contiguous()
            out, t = _timed(lambda: api.lasso_solve_batch(G, c, lam[j0:j1], z0=z0, u0=u0, **kw))
            t_admm += t - t_factor
            its[:, j0:j1] = out["iters"].cpu().numpy()
            block_max.append(int(out["iters"].max()))
            z_prev, u_prev = out["z"], out["u"]
            zs.append(out["z"])
        z_path = torch.cat(zs, dim=1)
        scale = z_cold.abs().amax(dim=-1, keepdim=True).clamp_min(1e-300)
        res["path"][ng] = dict(mean_iters=float(its.mean()), block_max=block_max, sum_block_max=int(sum(block_max)),
                               admm_ms=t_admm,
                               max_rel_diff=float(((z_path - z_cold).abs() / scale).max()))
    return res


def strong_rule(pr, seed: int = 0, B1: int = 48, kkt_tol: float = 1e-6, relax: float = 1.8):
    """Sequential strong rule on the cold solutions of every (bootstrap, lambda)."""
    G, c = _statistics(pr, seed, B1)
    lam = np.asarray(pr.lambdas, dtype=np.float64)
    out = api.lasso_solve_batch(G, c, lam, kkt_tol=kkt_tol, precision="fp64", relax=relax, max_iter=50000)
    Z = out["z"].cpu().numpy()          # [B1, q, p]
    Gh = G.cpu().numpy()
    ch = c.cpu().numpy()
    nb, q, p = Z.shape
    kept, viol, supp = [], 0, []
    for k in range(nb):
        grad = ch[k][None, :] - Z[k] @ Gh[k]   # [q, p]: c - G beta_j (G symmetric)
        for j in range(1, q):
            prev = Z[k, j - 1] != 0.0
            keep = prev | (np.abs(grad[j - 1]) >= 2 * lam[j] - lam[j - 1])
            now = Z[k, j] != 0.0
            viol += int(np.count_nonzero(now & ~keep))
            kept.append(int(keep.sum()))
            supp.append(int(now.sum()))
    kept = np.asarray(kept)
    # bytes read per iteration: the batched sweep reads each bootstrap's float32 M
    # once for all q solves; a reduced problem per solve reads its own |K| x |K| inverse
    shared = nb * p * p * 4
    reduced = float((kept.astype(np.float64) ** 2 * 4).sum())
    return dict(config=dict(n=pr.X.shape[0], p=p, B1=nb, q=q), solves_screened=int(kept.size),
                kept_mean=float(kept.mean()), kept_max=int(kept.max()), kept_min=int(kept.min()),
                support_mean=float(np.mean(supp)), violations=viol,
                bytes_per_iteration_shared=shared, bytes_per_iteration_reduced=reduced)


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(prog="python -m paper_1808_06992_amd.baselines", description=__doc__.split("\n")[0])
    ap.add_argument("--groups", type=int, nargs="+", default=[2, 4, 8])
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--small", action="store_true", help="the n200 p50 problem instead of n5000 p1000")
    ap.add_argument("--precision", choices=("fp64", "mixed"), default="fp64")
    a = ap.parse_args(argv)
    api.load()
    if not torch.cuda.is_available():
        raise SystemExit("no GPU: the solves run on the library's kernels only")
    pr = synth.lasso_small(a.seed) if a.small else synth.lasso_toeplitz(a.seed)
    B1 = pr.B1
    # exact iteration counts (a check every iteration), then times at the usual check period
    for ce in (1, 10):
        r = pathwise(pr, a.seed, B1, tuple(a.groups), precision=a.precision, check_every=ce)
        print(json.dumps(dict(pathwise=r), default=str), flush=True)
    print(json.dumps(dict(strong_rule=strong_rule(pr, a.seed, B1)), default=str), flush=True)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
