"""Reading real data for the fits, and a command-line front end.

    python -m paper_1808_06992_amd.ingest var   --series rec.npy --order 2 --intercept --out fit.npz
    python -m paper_1808_06992_amd.ingest lasso --X X.npy --y y.npy --out fit.npz

Arrays are read from .npy (never unpickled), .npz (one named array) or
delimited text (.csv / .txt), checked (shape, finite values) and handed to the
library on the current GPU; the lambda grid is log-spaced from lambda_max (the
largest absolute correlation of the design with the response, on centred
columns when an intercept is fitted) down to ratio * lambda_max.  The numbers
are computed by the library's kernels; this module only reads, checks and
writes files.
"""
from __future__ import annotations

import argparse
import os
import sys

import numpy as np

__all__ = ["load_array", "load_series", "lambda_grid", "main"]


def load_array(path: str, key: str | None = None) -> np.ndarray:
    """A float64 array from .npy, .npz (key, or the only array) or delimited text."""
    ext = os.path.splitext(path)[1].lower()
    if ext == ".npy":
        a = np.load(path, allow_pickle=False)
    elif ext == ".npz":
        with np.load(path, allow_pickle=False) as f:
            names = list(f.files)
            if key is None:
                if len(names) != 1:
                    raise ValueError(f"{path}: holds {names}; name the array to read")
                key = names[0]
            a = f[key]
    elif ext in (".csv", ".txt", ".tsv"):
        a = np.loadtxt(path, delimiter="," if ext == ".csv" else None, ndmin=2)
    else:
        raise ValueError(f"{path}: unsupported file type {ext!r} (.npy, .npz, .csv, .txt, .tsv)")
    a = np.asarray(a, dtype=np.float64)
    if not np.all(np.isfinite(a)):
        raise ValueError(f"{path}: contains NaN or Inf")
    return np.ascontiguousarray(a)


def load_series(path: str, key: str | None = None, *, order: int = 1, time_axis: int = 0) -> np.ndarray:
    """A T x p multivariate series (time along time_axis) with T >= order + 2."""
    s = load_array(path, key)
    if s.ndim == 1:
        s = s[:, None]
    if s.ndim != 2:
        raise ValueError(f"{path}: expected a 2-D series, got shape {s.shape}")
    if time_axis == 1:
        s = np.ascontiguousarray(s.T)
    if s.shape[0] < order + 2:
        raise ValueError(f"{path}: {s.shape[0]} time points are too few for order {order}")
    return s


def lambda_grid(lam_max: float, q: int, ratio: float) -> np.ndarray:
    if q == 1:
        return np.array([lam_max])
    return lam_max * np.power(ratio, np.arange(q, dtype=np.float64) / (q - 1))


def _var_lambda_max(s: np.ndarray, d: int, intercept: bool) -> float:
    T, p = s.shape
    N = T - d
    X = np.hstack([s[d - 1 - l: d - 1 - l + N] for l in range(d)])
    Y = s[d:]
    if intercept:
        X = X - X.mean(axis=0)
        Y = Y - Y.mean(axis=0)
    return float(np.max(np.abs(X.T @ Y))) / N


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(prog="python -m paper_1808_06992_amd.ingest", description=__doc__.split("\n")[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    for name in ("var", "lasso"):
        sp = sub.add_parser(name)
        sp.add_argument("--out", required=True, help="output .npz")
        sp.add_argument("--B1", type=int, default=30)
        sp.add_argument("--B2", type=int, default=30)
        sp.add_argument("--q", type=int, default=30, help="number of lambdas")
        sp.add_argument("--ratio", type=float, default=1e-3, help="smallest / largest lambda")
        sp.add_argument("--seed", type=int, default=0)
        sp.add_argument("--kkt-tol", type=float, default=1e-6)
        sp.add_argument("--precision", choices=("fp64", "mixed"), default="mixed")
        sp.add_argument("--relax", type=float, default=1.8)
        sp.add_argument("--rho", type=float, default=0.0,
                        help="ADMM penalty; 0 (default) scales it to the data (mean diagonal of the Grams)")
        if name == "var":
            sp.add_argument("--series", required=True)
            sp.add_argument("--key", default=None, help="array name inside an .npz")
            sp.add_argument("--order", type=int, default=1)
            sp.add_argument("--intercept", action="store_true")
            sp.add_argument("--per-equation", action="store_true")
            sp.add_argument("--time-axis", type=int, default=0, choices=(0, 1))
        else:
            sp.add_argument("--X", required=True)
            sp.add_argument("--y", required=True)
    a = ap.parse_args(argv)

    import torch

    from . import _lib as api
    api.load()
    if not torch.cuda.is_available():
        raise SystemExit("no GPU: the fits run on the library's kernels only")
    kw = dict(kkt_tol=a.kkt_tol, precision=a.precision, relax=a.relax, rho=a.rho)
    if a.cmd == "var":
        s = load_series(a.series, a.key, order=a.order, time_axis=a.time_axis)
        lam = lambda_grid(_var_lambda_max(s, a.order, a.intercept), a.q, a.ratio)
        out = api.var_fit(torch.as_tensor(s, device="cuda"), lam, a.B1, a.B2, a.seed, d=a.order,
                          intercept=a.intercept, per_equation=a.per_equation, **kw)
        A = out["A"].cpu().numpy().reshape(a.order, s.shape[1], s.shape[1])
        res = dict(A=A, mu=out["mu"].cpu().numpy(), supports=out["supports"].cpu().numpy().view(np.uint64),
                   jstar=out["jstar"].cpu().numpy(), losses=out["losses"].cpu().numpy(), lambdas=lam)
    else:
        X = load_array(a.X)
        y = load_array(a.y).reshape(-1)
        if X.ndim != 2 or X.shape[0] != y.size:
            raise ValueError(f"X {X.shape} and y {y.shape} do not match")
        lam = lambda_grid(float(np.max(np.abs(X.T @ y))) / X.shape[0], a.q, a.ratio)
        out = api.lasso_fit(torch.as_tensor(X, device="cuda"), torch.as_tensor(y, device="cuda"), lam, a.B1,
                            a.B2, a.seed, **kw)
        res = dict(beta=out["beta"].cpu().numpy(), supports=out["supports"].cpu().numpy().view(np.uint64),
                   jstar=out["jstar"].cpu().numpy(), losses=out["losses"].cpu().numpy(), lambdas=lam)
    res["status"] = np.int32(out["status"])
    np.savez(a.out, **res)
    print(f"{a.cmd}: status {out['status']}, unconverged {out['n_unconverged']}, wrote {a.out}")
    return 0 if out["status"] == 0 else 1


if __name__ == "__main__":
    sys.exit(main())
