"""Seeded synthetic inputs for UoI_LASSO and UoI_VAR.

This module only draws data: it holds none of the method's arithmetic and is
the one piece of code shared by the CPU oracle tests and the HIP path.  Every
array comes from ``numpy.random.default_rng(seed)`` in a fixed draw order, so
the same seed gives the same bytes on any machine running this numpy.

Workloads (sizes follow the synthetic setups the paper scales, Sec. IV and
Tables I-II, shrunk to one GPU):

* ``lasso_small``   -- linear model of Eq. (1): n=200, p=50, iid N(0,1) design,
                       10 nonzero coefficients ~ U[-3,3], noise sd 0.5.
* ``lasso_toeplitz`` -- n=5000, p=1000, rows ~ N(0, S) with S_ij = 0.5^|i-j|,
                       100 nonzero coefficients ~ N(0,1), noise variance set
                       so that b'Sb / sigma^2 = 5.
* ``var1``          -- VAR(1) series of Eq. (5) with d=1: sparse transition
                       matrix with a given fraction of N(0,1) entries rescaled
                       to a target spectral radius, unit Gaussian innovations,
                       a burn-in that is discarded.

The lambda grid is an input of both algorithms (Alg. 1 and Alg. 2 take the
vector lambda as an argument).  ``lambda_grid_lasso`` / ``lambda_grid_var``
build the grid used throughout: q values log-spaced from lambda_max down to
``ratio * lambda_max``, where lambda_max = max_i |x_i' y| / n on the full data
(the smallest penalty that zeroes every coefficient of the full-data problem
in the 1/(2n) scaling).  For VAR one grid serves all equations, since the
vectorised problem of Eq. (8) has a single penalty.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

__all__ = [
    "LassoProblem",
    "VarProblem",
    "lasso_small",
    "lasso_toeplitz",
    "lasso_random",
    "var1",
    "var_small",
    "lambda_grid_lasso",
    "lambda_grid_var",
    "CONFIGS",
]


@dataclass
class LassoProblem:
    X: np.ndarray          # n x p, float64, row-major
    y: np.ndarray          # n, float64
    beta_true: np.ndarray  # p, float64
    lambdas: np.ndarray    # q, float64, strictly decreasing
    B1: int
    B2: int
    seed: int
    name: str = ""


@dataclass
class VarProblem:
    series: np.ndarray     # T x p, float64, time ascending
    A_true: np.ndarray     # p x p (d = 1) or d x p x p (A_true[l] multiplies x_{t-l-1}), float64
    lambdas: np.ndarray    # q, float64, strictly decreasing
    B1: int
    B2: int
    seed: int
    name: str = ""
    d: int = 1             # autoregressive order
    intercept: bool = False
    mu_true: np.ndarray | None = None


def _log_grid(lam_max: float, q: int, ratio: float) -> np.ndarray:
    if q == 1:
        return np.array([lam_max], dtype=np.float64)
    expo = np.arange(q, dtype=np.float64) / (q - 1)
    return lam_max * np.power(ratio, expo)


def lambda_grid_lasso(X: np.ndarray, y: np.ndarray, q: int, ratio: float = 1e-3) -> np.ndarray:
    """Input grid: lambda_max = ||X'y||_inf / n, then log-spaced down to ratio*lambda_max."""
    n = X.shape[0]
    lam_max = float(np.max(np.abs(X.T @ y))) / n
    return _log_grid(lam_max, q, ratio)


def lambda_grid_var(series: np.ndarray, q: int, ratio: float = 1e-3) -> np.ndarray:
    """Input grid for the lag-1 regression: lambda_max = max_e ||X'Y_e||_inf / N'."""
    Xl = series[:-1]
    Yl = series[1:]
    lam_max = float(np.max(np.abs(Xl.T @ Yl))) / Xl.shape[0]
    return _log_grid(lam_max, q, ratio)


def lagged_design(series: np.ndarray, d: int):
    """Eq. (6)-(7): responses x_t (t = d .. T-1) and designs [x_{t-1}, ..., x_{t-d}] (lag 1 first)."""
    T, p = series.shape
    N = T - d
    Xl = np.hstack([series[d - 1 - l: d - 1 - l + N] for l in range(d)])
    return np.ascontiguousarray(Xl), np.ascontiguousarray(series[d:])


def lambda_grid_var_d(series: np.ndarray, d: int, intercept: bool, q: int,
                      ratio: float = 1e-3) -> np.ndarray:
    """lambda_max = max_e ||X'Y_e||_inf / N' over the lagged regression of order d,
    on centred columns when an intercept is fitted."""
    Xl, Yl = lagged_design(series, d)
    if intercept:
        Xl = Xl - Xl.mean(axis=0)
        Yl = Yl - Yl.mean(axis=0)
    lam_max = float(np.max(np.abs(Xl.T @ Yl))) / Xl.shape[0]
    return _log_grid(lam_max, q, ratio)


def var_d(p: int, T: int, d: int, frac: float, radius: float, seed: int, *, mu_scale: float = 0.0,
          intercept: bool = False, burn: int = 500, q: int = 30, B1: int = 30, B2: int = 30,
          ratio: float = 1e-3) -> VarProblem:
    """VAR(d): x_t = mu + sum_l A_l x_{t-l} + u_t, u_t ~ N(0, I), x = 0 before the
    burn-in.  Each A_l has round(frac p^2) nonzeros ~ N(0, 1) at random positions;
    A_l is then scaled by s^l so that the companion matrix has spectral radius
    `radius` (which scales every root of the characteristic polynomial by s).
    mu ~ N(0, mu_scale^2) per coordinate."""
    rng = np.random.default_rng(seed)
    nnz = int(round(frac * p * p))
    A = np.zeros((d, p, p))
    for l in range(d):
        pos = rng.choice(p * p, size=nnz, replace=False)
        A[l].reshape(-1)[pos] = rng.standard_normal(nnz)
    comp = np.zeros((d * p, d * p))
    comp[:p, :] = np.hstack(list(A))
    comp[p:, :-p] = np.eye((d - 1) * p)
    rad = float(np.max(np.abs(np.linalg.eigvals(comp)))) if nnz else 0.0
    if rad > 0:
        for l in range(d):
            A[l] *= (radius / rad) ** (l + 1)
    mu = mu_scale * rng.standard_normal(p)
    U = rng.standard_normal((T + burn, p))
    xs = np.zeros((T + burn + d, p))
    for t in range(d, T + burn + d):
        x = mu + U[t - d]
        for l in range(d):
            x = x + A[l] @ xs[t - 1 - l]
        xs[t] = x
    series = np.ascontiguousarray(xs[burn + d:])
    lam = lambda_grid_var_d(series, d, intercept, q, ratio)
    return VarProblem(series, A, lam, B1, B2, seed, f"var{d}_p{p}_T{T}", d=d, intercept=intercept,
                      mu_true=mu)


def lasso_random(n: int, p: int, k: int, seed: int, *, noise: float = 0.5, q: int = 16,
                 B1: int = 20, B2: int = 20, ratio: float = 1e-3) -> LassoProblem:
    """iid N(0,1) design, k coefficients ~ U[-3,3] on distinct random indices."""
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, p))
    beta = np.zeros(p)
    idx = rng.choice(p, size=min(k, p), replace=False)
    beta[idx] = rng.uniform(-3.0, 3.0, size=idx.size)
    y = X @ beta + noise * rng.standard_normal(n)
    lam = lambda_grid_lasso(X, y, q, ratio)
    return LassoProblem(np.ascontiguousarray(X), y, beta, lam, B1, B2, seed,
                        f"lasso_random_n{n}_p{p}")


def lasso_small(seed: int = 0) -> LassoProblem:
    """n=200, p=50, 10 nonzeros ~ U[-3,3], noise sd 0.5; B1=20, q=16, B2=20."""
    pr = lasso_random(200, 50, 10, seed, noise=0.5, q=16, B1=20, B2=20)
    pr.name = "lasso_n200_p50"
    return pr


def lasso_toeplitz(seed: int = 0, *, n: int = 5000, p: int = 1000, k: int = 100,
                   rho_x: float = 0.5, snr: float = 5.0, q: int = 48, B1: int = 48,
                   B2: int = 48, ratio: float = 1e-3) -> LassoProblem:
    """Rows ~ N(0, S), S_ij = rho_x^|i-j|, drawn as a stationary AR(1) across columns."""
    rng = np.random.default_rng(seed)
    E = rng.standard_normal((n, p))
    X = np.empty((n, p))
    X[:, 0] = E[:, 0]
    s = np.sqrt(1.0 - rho_x * rho_x)
    for j in range(1, p):
        X[:, j] = rho_x * X[:, j - 1] + s * E[:, j]
    beta = np.zeros(p)
    idx = rng.choice(p, size=k, replace=False)
    beta[idx] = rng.standard_normal(k)
    # population signal variance b' S b with S_ij = rho^|i-j|
    ii = np.arange(p)
    S = np.power(rho_x, np.abs(ii[:, None] - ii[None, :]))
    sig2 = float(beta @ S @ beta) / snr
    y = X @ beta + np.sqrt(sig2) * rng.standard_normal(n)
    lam = lambda_grid_lasso(X, y, q, ratio)
    return LassoProblem(np.ascontiguousarray(X), y, beta, lam, B1, B2, seed,
                        f"lasso_toeplitz_n{n}_p{p}")


def lasso_toeplitz_responses(seed: int, M: int, *, n: int = 5000, p: int = 1000, k: int = 100,
                             rho_x: float = 0.5, snr: float = 5.0, q: int = 48, ratio: float = 1e-3):
    """M independent (beta, noise) draws on one Toeplitz design: Y is n x M.

    Same distribution per column as ``lasso_toeplitz`` (a fresh support of k
    coefficients ~ N(0,1) and noise at the given SNR for every column); one
    lambda grid for all columns, from the largest lambda_max among them."""
    base = lasso_toeplitz(seed, n=n, p=p, k=k, rho_x=rho_x, snr=snr, q=q, ratio=ratio)
    rng = np.random.default_rng(seed + 7919)
    ii = np.arange(p)
    S = np.power(rho_x, np.abs(ii[:, None] - ii[None, :]))
    B = np.zeros((p, M))
    for m in range(M):
        idx = rng.choice(p, size=k, replace=False)
        B[idx, m] = rng.standard_normal(k)
    sig = np.sqrt(np.einsum("im,ij,jm->m", B, S, B) / snr)
    Y = base.X @ B + rng.standard_normal((n, M)) * sig[None, :]
    lam_max = float(np.max(np.abs(base.X.T @ Y))) / n
    return base.X, np.ascontiguousarray(Y), B, _log_grid(lam_max, q, ratio)


def var1(p: int, T: int, frac: float, radius: float, seed: int, *, burn: int = 500,
         q: int = 30, B1: int = 30, B2: int = 30, ratio: float = 1e-3) -> VarProblem:
    """VAR(1): x_t = A x_{t-1} + u_t, u_t ~ N(0, I), x_0 = 0, burn-in dropped."""
    rng = np.random.default_rng(seed)
    nnz = int(round(frac * p * p))
    pos = rng.choice(p * p, size=nnz, replace=False)
    A = np.zeros(p * p)
    A[pos] = rng.standard_normal(nnz)
    A = A.reshape(p, p)
    rad = float(np.max(np.abs(np.linalg.eigvals(A)))) if nnz else 0.0
    if rad > 0:
        A *= radius / rad
    U = rng.standard_normal((T + burn, p))
    xs = np.empty((T + burn, p))
    x = np.zeros(p)
    for t in range(T + burn):
        x = A @ x + U[t]
        xs[t] = x
    series = np.ascontiguousarray(xs[burn:])
    lam = lambda_grid_var(series, q, ratio)
    return VarProblem(series, A, lam, B1, B2, seed, f"var1_p{p}_T{T}")


def var_small(seed: int = 0, p: int = 192, T: int = 10000) -> VarProblem:
    """192-node VAR(1), 5% nonzero transition, spectral radius 0.9; B1=q=B2=30."""
    pr = var1(p, T, 0.05, 0.9, seed, q=30, B1=30, B2=30)
    pr.name = f"var1_p{p}_T{T}"
    return pr


def var_large(seed: int = 0) -> VarProblem:
    """1000-node VAR(1), 1% nonzero, spectral radius 0.95, T=20000; B1=q=B2=20."""
    pr = var1(1000, 20000, 0.01, 0.95, seed, q=20, B1=20, B2=20)
    pr.name = "var1_p1000_T20000"
    return pr


CONFIGS = {
    "lasso_n200_p50": lasso_small,
    "lasso_toeplitz_n5000_p1000": lasso_toeplitz,
    "var1_p192_T10000": var_small,
    "var1_p1000_T20000": var_large,
}
