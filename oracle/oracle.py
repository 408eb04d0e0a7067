"""ctypes front end of the C oracle (``uoi_oracle.c``) -- TEST INFRASTRUCTURE ONLY.

Each wrapper cites the passage of arXiv 1808.06992 the C routine follows.
The library is built with gcc (``build()``); nothing here touches a GPU.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "uoi_oracle.c")
_HDR = os.path.join(_HERE, "uoi_oracle.h")
_LIB = os.path.join(_HERE, "liboracle.so")

TAG_LASSO_BOOT, TAG_LASSO_SPLIT, TAG_VAR_BOOT, TAG_VAR_SPLIT = 1, 2, 3, 4

__all__ = [
    "build", "lib", "mix64", "key", "index", "boot_rows", "split_rows", "var_block_len",
    "var_boot_rows", "var_split_rows", "gram", "gram_var", "kkt", "lasso_cd", "lstsq_qr",
    "ols_normal", "uoi_lasso", "uoi_var", "uoi_var_d", "gram_multi", "decided_bits",
    "support_words",
]


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (plain -O2, OpenMP over independent solves)."""
    stale = (not os.path.exists(_LIB) or
             os.path.getmtime(_LIB) < max(os.path.getmtime(_SRC), os.path.getmtime(_HDR)))
    if force or stale:
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fopenmp",
                               "-o", tmp, _SRC, "-lm"], cwd=_HERE)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB)
        P = C.c_void_p
        i32, u32, u64, f64 = C.c_int32, C.c_uint32, C.c_uint64, C.c_double
        L.orc_mix64.restype = u64; L.orc_mix64.argtypes = [u64]
        L.orc_key.restype = u64; L.orc_key.argtypes = [u64, u32, u32, u32]
        L.orc_index.restype = u32; L.orc_index.argtypes = [u64, u32]
        L.orc_boot_rows.restype = None; L.orc_boot_rows.argtypes = [u64, i32, i32, P]
        L.orc_split_count.restype = i32; L.orc_split_count.argtypes = [i32, i32, i32]
        L.orc_split_rows.restype = None; L.orc_split_rows.argtypes = [u64, i32, i32, i32, i32, P, P]
        L.orc_var_block_len.restype = i32; L.orc_var_block_len.argtypes = [i32]
        L.orc_var_nblocks.restype = i32; L.orc_var_nblocks.argtypes = [i32, i32]
        L.orc_var_boot_rows.restype = None; L.orc_var_boot_rows.argtypes = [u64, i32, i32, i32, P]
        L.orc_var_split_rows.restype = None
        L.orc_var_split_rows.argtypes = [u64, i32, i32, i32, i32, i32, P, P, P, P]
        L.orc_gram.restype = None
        L.orc_gram.argtypes = [i32, P, i32, P, i32, i32, P, i32, P, P]
        L.orc_kkt.restype = f64; L.orc_kkt.argtypes = [i32, P, P, i32, f64, P]
        L.orc_lasso_cd.restype = i32; L.orc_lasso_cd.argtypes = [i32, P, P, i32, f64, f64, i32, P]
        L.orc_lstsq_qr.restype = i32; L.orc_lstsq_qr.argtypes = [i32, i32, P, P, P]
        L.orc_ols_normal.restype = i32; L.orc_ols_normal.argtypes = [i32, P, P, i32, i32, P, P, P]
        L.orc_uoi_lasso.restype = i32
        L.orc_uoi_lasso.argtypes = [i32, i32, P, P, i32, i32, i32, P, u64, i32, i32, f64, i32,
                                    P, P, P, P, P, P, P]
        L.orc_uoi_var.restype = i32
        L.orc_uoi_var.argtypes = [i32, i32, P, i32, i32, i32, i32, P, u64, i32, i32, f64, i32,
                                  P, P, P, P]
        L.orc_uoi_var_d.restype = i32
        L.orc_uoi_var_d.argtypes = [i32, i32, i32, i32, i32, P, i32, i32, i32, i32, P, u64, i32, i32,
                                    f64, i32, P, P, P, P, P]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# --- random indices (counter-based SplitMix64; the paper leaves the sampler open) ---

def mix64(x: int) -> int:
    return int(lib().orc_mix64(x))


def key(seed: int, tag: int, k: int, i: int) -> int:
    return int(lib().orc_key(seed, tag, k, i))


def index(r: int, m: int) -> int:
    return int(lib().orc_index(r, m))


def boot_rows(seed: int, k: int, n: int) -> np.ndarray:
    """Alg. 1 selection loop, the sample T^k: n rows drawn with replacement."""
    out = np.empty(n, np.int32)
    lib().orc_boot_rows(seed, k, n, _p(out))
    return out


def split_rows(seed: int, k: int, n: int, num: int = 4, den: int = 5):
    """Alg. 1 estimation loop: train/eval partition of the rows, each ascending."""
    ntr = int(lib().orc_split_count(n, num, den))
    tr = np.empty(max(ntr, 1), np.int32)
    ev = np.empty(max(n - ntr, 1), np.int32)
    lib().orc_split_rows(seed, k, n, num, den, _p(tr), _p(ev))
    return tr[:ntr], ev[: n - ntr]


def var_block_len(N: int) -> int:
    return int(lib().orc_var_block_len(N))


def var_boot_rows(seed: int, k: int, N: int, L: int) -> np.ndarray:
    """Alg. 2 block bootstrap (Sec. III-A.2): moving blocks of regression rows."""
    out = np.empty(N, np.int32)
    lib().orc_var_boot_rows(seed, k, N, L, _p(out))
    return out


def var_split_rows(seed: int, k: int, N: int, L: int, num: int = 4, den: int = 5):
    tr = np.empty(N, np.int32)
    ev = np.empty(N, np.int32)
    ntr = C.c_int(0)
    nev = C.c_int(0)
    lib().orc_var_split_rows(seed, k, N, L, num, den, _p(tr), C.byref(ntr), _p(ev), C.byref(nev))
    return tr[: ntr.value].copy(), ev[: nev.value].copy()


# --- statistics, LASSO, KKT, OLS ---

def gram(X: np.ndarray, y: np.ndarray, rows: np.ndarray):
    """G = X_r'X_r/m, c = X_r'y_r/m over the sampled rows (with multiplicity)."""
    X = _f64(X)
    y = _f64(y)
    rows = np.ascontiguousarray(rows, np.int32)
    n, p = X.shape
    G = np.empty((p, p))
    c = np.empty(p)
    lib().orc_gram(rows.size, _p(rows), p, _p(X), p, 1, _p(y), 1, _p(G), _p(c))
    return G, c


def gram_var(series: np.ndarray, rows: np.ndarray):
    """Lag-1 statistics of Eq. (6)-(7): row r uses x = series[r], y = series[r+1]."""
    s = _f64(series)
    rows = np.ascontiguousarray(rows, np.int32)
    T, p = s.shape
    G = np.empty((p, p))
    Cm = np.empty((p, p))
    lib().orc_gram(rows.size, _p(rows), p, _p(s), p, p, s[1:].ctypes.data, p, _p(G), _p(Cm))
    return G, Cm


def gram_multi(X: np.ndarray, Y: np.ndarray, rows: np.ndarray):
    """G = X_r'X_r/m and C = X_r'Y_r/m over the sampled rows, several response columns."""
    X = _f64(X); Y = _f64(Y)
    rows = np.ascontiguousarray(rows, np.int32)
    n, p = X.shape
    pe = Y.shape[1]
    G = np.empty((p, p))
    Cm = np.empty((p, pe))
    lib().orc_gram(rows.size, _p(rows), p, _p(X), p, pe, _p(Y), pe, _p(G), _p(Cm))
    return G, Cm


def kkt(G: np.ndarray, c: np.ndarray, lam: float, b: np.ndarray) -> float:
    """Relative KKT residual of the LASSO of Eq. (2) (1/(2m) scaling)."""
    G = _f64(G); c = _f64(c); b = _f64(b)
    return float(lib().orc_kkt(G.shape[0], _p(G), _p(c), 1, float(lam), _p(b)))


def lasso_cd(G: np.ndarray, c: np.ndarray, lam: float, tol: float = 1e-12,
             max_sweeps: int = 100000, b0: np.ndarray | None = None):
    """LASSO of Eq. (2) by cyclic coordinate descent; returns (beta, sweeps or -1)."""
    G = _f64(G); c = _f64(c)
    b = np.zeros(G.shape[0]) if b0 is None else _f64(b0).copy()
    st = int(lib().orc_lasso_cd(G.shape[0], _p(G), _p(c), 1, float(lam), float(tol),
                                int(max_sweeps), _p(b)))
    return b, st


def lstsq_qr(A: np.ndarray, yv: np.ndarray) -> np.ndarray:
    """Householder-QR least squares (independent of the normal equations)."""
    m, s = A.shape
    Af = np.asfortranarray(A, dtype=np.float64).copy(order="F")
    yy = _f64(yv).copy()
    b = np.empty(max(s, 1))
    if lib().orc_lstsq_qr(m, s, Af.ctypes.data, _p(yy), _p(b)) != 0:
        raise np.linalg.LinAlgError("singular")
    return b[:s]


def ols_normal(G: np.ndarray, c: np.ndarray, idx) -> np.ndarray:
    """OLS on columns idx from the normal equations G[S,S] b = c[S] (Cholesky)."""
    G = _f64(G); c = _f64(c)
    idx = np.ascontiguousarray(idx, np.int32)
    s = idx.size
    b = np.empty(max(s, 1))
    work = np.empty(max(s * s, 1))
    if lib().orc_ols_normal(G.shape[0], _p(G), _p(c), 1, s, _p(idx), _p(b), _p(work)) != 0:
        raise np.linalg.LinAlgError("not positive definite")
    return b[:s]


def support_words(b: np.ndarray) -> np.ndarray:
    """Bitmask of the nonzero entries: bit i of word i//64."""
    p = b.shape[-1]
    W = (p + 63) // 64
    out = np.zeros(b.shape[:-1] + (W,), np.uint64)
    nz = b != 0
    for i in range(p):
        out[..., i // 64] |= nz[..., i].astype(np.uint64) << np.uint64(i % 64)
    return out


def decided_bits(G, c, lam, b, tau=1e-6):
    """Support bits whose value is decided by a margin above tau.

    Active bits: |b_i| / ||b||_inf > tau.  Inactive bits: (lam - |g_i|) / ||c||_inf > tau
    with g = c - G b.  Bits inside the margin may legitimately differ between two
    solvers that both meet a KKT tolerance near tau."""
    g = c - G @ b
    cn = max(np.max(np.abs(c)), 1e-300)
    bn = max(np.max(np.abs(b)), 1e-300)
    act = (b != 0) & (np.abs(b) / bn > tau)
    inact = (b == 0) & ((lam - np.abs(g)) / cn > tau)
    return act | inact


# --- Algorithm 1 and Algorithm 2 ---

def uoi_lasso(X, y, lambdas, B1, B2, seed, *, num=4, den=5, tol=1e-12, max_sweeps=100000,
              keep_selection=False, keep_ols=False):
    """Algorithm 1 (UoI_LASSO).  Returns a dict of all intermediate results."""
    X = _f64(X); y = _f64(y); lam = _f64(lambdas)
    n, p = X.shape
    q = lam.size
    W = (p + 63) // 64
    beta = np.empty(p)
    supp = np.empty((q, W), np.uint64)
    jstar = np.empty(B2, np.int32)
    losses = np.empty((B2, q))
    sel = np.empty((B1, q, p)) if keep_selection else None
    skkt = np.empty((B1, q)) if keep_selection else None
    ols = np.empty((B2, q, p)) if keep_ols else None
    st = lib().orc_uoi_lasso(n, p, _p(X), _p(y), B1, B2, q, _p(lam), seed, num, den, tol,
                             max_sweeps, _p(beta), _p(supp), _p(jstar), _p(losses),
                             _p(sel), _p(skkt), _p(ols))
    return dict(status=int(st), beta=beta, supports=supp, jstar=jstar, losses=losses,
                sel_beta=sel, sel_kkt=skkt, ols_beta=ols)


def uoi_var(series, lambdas, B1, B2, seed, *, block_len=0, num=4, den=5, tol=1e-12,
            max_sweeps=100000):
    """Algorithm 2 (UoI_VAR) with d = 1.  A[e, l] = coefficient of x_{t-1,l} in equation e."""
    s = _f64(series); lam = _f64(lambdas)
    T, p = s.shape
    q = lam.size
    W = (p + 63) // 64
    A = np.empty((p, p))
    supp = np.empty((q, p, W), np.uint64)
    jstar = np.empty(B2, np.int32)
    losses = np.empty((B2, q))
    st = lib().orc_uoi_var(T, p, _p(s), block_len, B1, B2, q, _p(lam), seed, num, den, tol,
                           max_sweeps, _p(A), _p(supp), _p(jstar), _p(losses))
    return dict(status=int(st), A=A, supports=supp, jstar=jstar, losses=losses)


def uoi_var_d(series, lambdas, B1, B2, seed, *, d=1, intercept=False, per_equation=False, block_len=0,
              num=4, den=5, tol=1e-12, max_sweeps=100000):
    """Algorithm 2 for VAR(d) (Eq. (5)-(8)), optionally with an unpenalised intercept.
    A[l, e, m] = coefficient of x_{t-l-1, m} in equation e; mu [p]; supports [q][p][W]
    with bit l*p + m of equation e (Eq. (7) column order), W = ceil(d*p/64).
    per_equation: every equation picks its own support index per split (jstar
    [B2][p], losses [B2][q][p]) instead of one from the summed loss."""
    s = _f64(series); lam = _f64(lambdas)
    T, p = s.shape
    q = lam.size
    W = (d * p + 63) // 64
    A = np.empty((d, p, p))
    mu = np.empty(p)
    supp = np.empty((q, p, W), np.uint64)
    jstar = np.empty((B2, p) if per_equation else B2, np.int32)
    losses = np.empty((B2, q, p) if per_equation else (B2, q))
    st = lib().orc_uoi_var_d(T, p, d, 1 if intercept else 0, 1 if per_equation else 0, _p(s), block_len,
                             B1, B2, q, _p(lam), seed, num, den, tol, max_sweeps, _p(A), _p(mu), _p(supp),
                             _p(jstar), _p(losses))
    return dict(status=int(st), A=A, mu=mu, supports=supp, jstar=jstar, losses=losses)
