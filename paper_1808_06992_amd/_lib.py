"""ctypes binding of libuoi.so (include/uoi.h).

Argument marshalling only: device buffers are torch CUDA (HIP) tensors, the
stream is torch's current stream, and every step of the computation runs in
the library's kernels.  There is no fallback: if the library is not built or
a call fails, an exception is raised.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libuoi.so")

UOI_OK, UOI_EINVAL, UOI_ENOMEM, UOI_EHIP, UOI_ENOCONV = 0, -1, -2, -3, -4
UOI_FP64, UOI_MIXED = 0, 1
UOI_COLD, UOI_MLP = 0, 1
UOI_SOLVER_BATCHED, UOI_SOLVER_PLAIN = 0, 1
UOI_FLAG_TIMING = 1
UOI_FLAG_INTERCEPT = 2
UOI_FLAG_EAGER = 4
UOI_FLAG_NO_TUNE = 8
UOI_FLAG_PER_EQUATION = 16

PRECISIONS = {"fp64": UOI_FP64, "mixed": UOI_MIXED}
SOLVERS = {"batched": UOI_SOLVER_BATCHED, "plain": UOI_SOLVER_PLAIN}
WARM = {"cold": UOI_COLD, "mlp": UOI_MLP}
STAGES = ("index+gram", "factor", "admm", "verify", "support", "estimation-gram", "ols",
          "loss+average")


class UoiError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"uoi error {code}: {msg}")
        self.code = code


class Opts(C.Structure):
    _fields_ = [
        ("B1", C.c_int32), ("B2", C.c_int32), ("q", C.c_int32),
        ("lambdas", C.POINTER(C.c_double)), ("seed", C.c_uint64),
        ("rho", C.c_double), ("kkt_tol", C.c_double),
        ("max_iter", C.c_int32), ("check_every", C.c_int32),
        ("train_num", C.c_int32), ("train_den", C.c_int32),
        ("precision", C.c_int32), ("warm_start", C.c_int32), ("solver", C.c_int32),
        ("flags", C.c_uint32), ("stream", C.c_void_p), ("mlp", C.c_void_p),
        ("relax", C.c_double), ("cg_max_iter", C.c_int32),
    ]


class KStat(C.Structure):
    _fields_ = [("ms", C.c_double), ("bytes", C.c_double), ("flops", C.c_double),
                ("launches", C.c_int64)]


KSTATS = ("admm64", "admm32", "plain", "gram")


class Diag(C.Structure):
    _fields_ = [
        ("iters", C.c_void_p), ("kkt", C.c_void_p), ("sel_beta", C.c_void_p),
        ("losses", C.c_void_p), ("n_solves", C.c_int64), ("n_unconverged", C.c_int64),
        ("max_iters", C.c_int32), ("warm_used", C.c_int64), ("stage_ms", C.c_float * 8),
        ("kstat", KStat * 4), ("n_refit_unconverged", C.c_int64),
    ]


def kstats(d: Diag) -> dict:
    return {name: dict(ms=d.kstat[i].ms, bytes=d.kstat[i].bytes, flops=d.kstat[i].flops,
                       launches=int(d.kstat[i].launches)) for i, name in enumerate(KSTATS)}


EXPORTS = (
    "uoi_default_opts", "uoi_lasso_fit", "uoi_var_fit", "uoi_lasso_solve_batch", "uoi_gram",
    "uoi_bootstrap_rows", "uoi_split_rows", "uoi_var_boot_rows", "uoi_var_split_rows",
    "uoi_spd_inverse", "uoi_release_workspace", "uoi_last_error", "uoi_version",
    "uoi_mlp_create", "uoi_mlp_destroy", "uoi_mlp_num_params", "uoi_mlp_set_params",
    "uoi_mlp_get_params", "uoi_mlp_forward", "uoi_mlp_loss_grad", "uoi_mlp_train_step",
    "uoi_ws_dataset", "uoi_lasso_solve_multi", "uoi_lasso_solve_batch_noalloc", "uoi_tune_reset",
)

_lib = None


def load():
    """Load libuoi.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_1808_06992_amd/build.py")
    L = C.CDLL(LIB_PATH)
    P, i32, u64, f64 = C.c_void_p, C.c_int32, C.c_uint64, C.c_double
    L.uoi_default_opts.restype = None
    L.uoi_default_opts.argtypes = [C.POINTER(Opts)]
    L.uoi_lasso_fit.restype = i32
    L.uoi_lasso_fit.argtypes = [i32, i32, P, P, C.POINTER(Opts), P, P, P, C.POINTER(Diag)]
    L.uoi_var_fit.restype = i32
    L.uoi_var_fit.argtypes = [i32, i32, i32, P, i32, C.POINTER(Opts), P, P, P, P, C.POINTER(Diag)]
    L.uoi_lasso_solve_batch.restype = i32
    L.uoi_lasso_solve_batch.argtypes = [i32, i32, P, P, C.POINTER(Opts), P, P, P, P, P, P]
    L.uoi_lasso_solve_batch_noalloc.restype = i32
    L.uoi_lasso_solve_batch_noalloc.argtypes = [i32, i32, P, P, C.POINTER(Opts), P, P, P, P, P, P]
    L.uoi_gram.restype = i32
    L.uoi_gram.argtypes = [i32, i32, P, i32, P, i32, i32, P, i32, P, P, P]
    L.uoi_bootstrap_rows.restype = i32
    L.uoi_bootstrap_rows.argtypes = [u64, i32, i32, P, P]
    L.uoi_split_rows.restype = i32
    L.uoi_split_rows.argtypes = [u64, i32, i32, i32, i32, P, P, P]
    L.uoi_var_boot_rows.restype = i32
    L.uoi_var_boot_rows.argtypes = [u64, i32, i32, i32, P, P]
    L.uoi_var_split_rows.restype = i32
    L.uoi_var_split_rows.argtypes = [u64, i32, i32, i32, i32, i32, P, P, P, P, P]
    L.uoi_spd_inverse.restype = i32
    L.uoi_spd_inverse.argtypes = [i32, i32, P, f64, P, P]
    L.uoi_release_workspace.restype = None
    L.uoi_release_workspace.argtypes = []
    L.uoi_tune_reset.restype = None
    L.uoi_tune_reset.argtypes = []
    L.uoi_last_error.restype = C.c_char_p
    L.uoi_last_error.argtypes = []
    L.uoi_version.restype = C.c_char_p
    L.uoi_version.argtypes = []
    L.uoi_mlp_create.restype = i32
    L.uoi_mlp_create.argtypes = [i32, i32, i32, C.POINTER(C.c_void_p)]
    L.uoi_mlp_destroy.restype = None
    L.uoi_mlp_destroy.argtypes = [P]
    L.uoi_mlp_num_params.restype = C.c_int64
    L.uoi_mlp_num_params.argtypes = [P]
    L.uoi_mlp_set_params.restype = i32
    L.uoi_mlp_set_params.argtypes = [P, P, P]
    L.uoi_mlp_get_params.restype = i32
    L.uoi_mlp_get_params.argtypes = [P, P, P]
    L.uoi_mlp_forward.restype = i32
    L.uoi_mlp_forward.argtypes = [P, i32, P, P, P]
    L.uoi_mlp_loss_grad.restype = i32
    L.uoi_mlp_loss_grad.argtypes = [P, i32, P, P, P, C.POINTER(C.c_double), P]
    L.uoi_mlp_train_step.restype = i32
    L.uoi_mlp_train_step.argtypes = [P, i32, P, P, C.c_float, C.POINTER(C.c_double), P]
    L.uoi_ws_dataset.restype = i32
    L.uoi_ws_dataset.argtypes = [i32, i32, i32, i32, P, P, P, P, P, P]
    L.uoi_lasso_solve_multi.restype = i32
    L.uoi_lasso_solve_multi.argtypes = [i32, i32, i32, P, P, C.POINTER(Opts), P, P, P]
    _lib = L
    return L


def _check(code: int, allow_noconv: bool = True) -> int:
    if code == UOI_OK or (allow_noconv and code == UOI_ENOCONV):
        return code
    raise UoiError(code, load().uoi_last_error().decode())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t: torch.Tensor, dtype=torch.float64) -> torch.Tensor:
    if not (t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise ValueError(f"expected a contiguous {dtype} tensor on the GPU")
    return t


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def make_opts(lambdas, *, B1=1, B2=1, seed=0, rho=1.0, kkt_tol=1e-6, max_iter=20000,
              check_every=10, train=(4, 5), precision="fp64", solver="batched",
              warm_start="cold", timing=False, stream="current", mlp=None, relax=1.0,
              cg_max_iter=4000, eager=False, tune=True):
    lam = np.ascontiguousarray(np.asarray(lambdas, dtype=np.float64))
    o = Opts()
    load().uoi_default_opts(C.byref(o))
    o.B1, o.B2, o.q = int(B1), int(B2), int(lam.size)
    o.lambdas = lam.ctypes.data_as(C.POINTER(C.c_double))
    o.seed = int(seed)
    o.rho, o.kkt_tol = float(rho), float(kkt_tol)
    o.max_iter, o.check_every = int(max_iter), int(check_every)
    o.train_num, o.train_den = int(train[0]), int(train[1])
    o.precision = PRECISIONS[precision]
    o.solver = SOLVERS[solver]
    o.warm_start = WARM[warm_start]
    o.flags = ((UOI_FLAG_TIMING if timing else 0) | (UOI_FLAG_EAGER if eager else 0)
               | (0 if tune else UOI_FLAG_NO_TUNE))
    o.relax = float(relax)
    o.cg_max_iter = int(cg_max_iter)
    o.stream = _stream() if stream == "current" else C.c_void_p(stream)
    if mlp is not None:
        o.mlp = mlp.handle
        o.warm_start = UOI_MLP
    return o, lam  # keep lam alive with the struct


def lasso_fit(X: torch.Tensor, y: torch.Tensor, lambdas, B1: int, B2: int, seed: int = 0, *,
              diag: bool = True, sel_beta: bool = False, **kw):
    """UoI_LASSO (Alg. 1) on device tensors; returns a dict of device tensors."""
    L = load()
    X = _dev(X); y = _dev(y)
    n, p = X.shape
    o, lam = make_opts(lambdas, B1=B1, B2=B2, seed=seed, **kw)
    q = lam.size
    W = (p + 63) // 64
    dev = X.device
    beta = torch.empty(p, dtype=torch.float64, device=dev)
    supp = torch.empty((q, W), dtype=torch.int64, device=dev)
    jstar = torch.empty(B2, dtype=torch.int32, device=dev)
    out = dict(beta=beta, supports=supp, jstar=jstar)
    d = Diag()
    if diag:
        out["iters"] = torch.empty((B1, q), dtype=torch.int32, device=dev)
        out["kkt"] = torch.empty((B1, q), dtype=torch.float64, device=dev)
        out["losses"] = torch.empty((B2, q), dtype=torch.float64, device=dev)
        d.iters, d.kkt, d.losses = out["iters"].data_ptr(), out["kkt"].data_ptr(), out["losses"].data_ptr()
        if sel_beta:
            out["sel_beta"] = torch.empty((B1, q, p), dtype=torch.float64, device=dev)
            d.sel_beta = out["sel_beta"].data_ptr()
    code = _check(L.uoi_lasso_fit(n, p, _ptr(X), _ptr(y), C.byref(o), _ptr(beta), _ptr(supp),
                                  _ptr(jstar), C.byref(d)))
    out["status"] = code
    out["n_unconverged"] = int(d.n_unconverged)
    out["n_refit_unconverged"] = int(d.n_refit_unconverged)
    out["max_iters"] = int(d.max_iters)
    out["warm_used"] = int(d.warm_used)
    out["stage_ms"] = dict(zip(STAGES, list(d.stage_ms)))
    out["kstat"] = kstats(d)
    return out


def var_fit(series: torch.Tensor, lambdas, B1: int, B2: int, seed: int = 0, *, d: int = 1,
            intercept: bool = False, per_equation: bool = False, block_len: int = 0, diag: bool = True,
            sel_beta: bool = False, **kw):
    """UoI_VAR (Alg. 2) of order d on a device series.  A[l, i, m] = coefficient of
    x_{t-l-1, m} in equation i (returned as [p, p] when d = 1), mu [p] (zeros unless
    intercept), supports [q, p, ceil(d p / 64)] with bit l*p + m for A[l, i, m].
    per_equation: jstar [B2, p] and losses [B2, q, p] (one choice per equation)."""
    L = load()
    series = _dev(series)
    T, p = series.shape
    o, lam = make_opts(lambdas, B1=B1, B2=B2, seed=seed, **kw)
    if intercept:
        o.flags |= UOI_FLAG_INTERCEPT
    if per_equation:
        o.flags |= UOI_FLAG_PER_EQUATION
    q = lam.size
    P = d * p
    W = (P + 63) // 64
    dev = series.device
    A = torch.empty((d, p, p), dtype=torch.float64, device=dev)
    mu = torch.empty(p, dtype=torch.float64, device=dev)
    supp = torch.empty((q, p, W), dtype=torch.int64, device=dev)
    jstar = torch.empty((B2, p) if per_equation else B2, dtype=torch.int32, device=dev)
    out = dict(A=A[0] if d == 1 else A, mu=mu, supports=supp, jstar=jstar)
    dg = Diag()
    if diag:
        out["iters"] = torch.empty((B1, q, p), dtype=torch.int32, device=dev)
        out["kkt"] = torch.empty((B1, q, p), dtype=torch.float64, device=dev)
        out["losses"] = torch.empty((B2, q, p) if per_equation else (B2, q), dtype=torch.float64, device=dev)
        dg.iters, dg.kkt, dg.losses = out["iters"].data_ptr(), out["kkt"].data_ptr(), out["losses"].data_ptr()
        if sel_beta:
            out["sel_beta"] = torch.empty((B1, q, p, P), dtype=torch.float64, device=dev)
            dg.sel_beta = out["sel_beta"].data_ptr()
    code = _check(L.uoi_var_fit(T, p, d, _ptr(series), int(block_len), C.byref(o), _ptr(A), _ptr(mu),
                                _ptr(supp), _ptr(jstar), C.byref(dg)))
    out["status"] = code
    out["n_unconverged"] = int(dg.n_unconverged)
    out["n_refit_unconverged"] = int(dg.n_refit_unconverged)
    out["max_iters"] = int(dg.max_iters)
    out["stage_ms"] = dict(zip(STAGES, list(dg.stage_ms)))
    out["kstat"] = kstats(dg)
    return out


def lasso_solve_batch(G: torch.Tensor, c: torch.Tensor, lambdas, *, z0=None, u0=None,
                      no_alloc: bool = False, **kw):
    """ADMM solves of nb LASSOs (G, c) at all lambdas; returns z, u [nb, q, p], iters, kkt.
    no_alloc: through uoi_lasso_solve_batch_noalloc (static scratch, no allocation)."""
    L = load()
    G = _dev(G); c = _dev(c)
    nb, p, _ = G.shape
    o, lam = make_opts(lambdas, **kw)
    q = lam.size
    dev = G.device
    z = torch.empty((nb, q, p), dtype=torch.float64, device=dev)
    u = torch.empty((nb, q, p), dtype=torch.float64, device=dev)
    its = torch.empty((nb, q), dtype=torch.int32, device=dev)
    kkt = torch.empty((nb, q), dtype=torch.float64, device=dev)
    fn = L.uoi_lasso_solve_batch_noalloc if no_alloc else L.uoi_lasso_solve_batch
    code = _check(fn(nb, p, _ptr(G), _ptr(c), C.byref(o),
                     _ptr(None if z0 is None else _dev(z0)),
                     _ptr(None if u0 is None else _dev(u0)),
                     _ptr(z), _ptr(u), _ptr(its), _ptr(kkt)))
    return dict(z=z, u=u, iters=its, kkt=kkt, status=code)


def gram(X: torch.Tensor, rows: torch.Tensor, Y: torch.Tensor | None = None, *, ldx=None, ldy=None):
    """G_b = X_r'X_r/m, C_b = X_r'Y_r/m for row lists rows[b] (int32 [nb, m])."""
    L = load()
    X = _dev(X)
    rows = _dev(rows, torch.int32)
    nb, m = rows.shape
    p = X.shape[1] if ldx is None else X.shape[-1]
    ldx = X.shape[1] if ldx is None else ldx
    G = torch.empty((nb, p, p), dtype=torch.float64, device=X.device)
    if Y is not None:
        Y = _dev(Y)
        pe = 1 if Y.dim() == 1 else Y.shape[1]
        ldy = pe if ldy is None else ldy
        Cm = torch.empty((nb, p, pe), dtype=torch.float64, device=X.device)
    else:
        pe, ldy, Cm = 0, 0, None
    _check(L.uoi_gram(nb, m, _ptr(rows), p, _ptr(X), ldx, pe, _ptr(Y), ldy, _ptr(G), _ptr(Cm),
                      _stream()), allow_noconv=False)
    return G, Cm


def gram_var(series: torch.Tensor, rows: torch.Tensor):
    """Lag-1 statistics: row r uses x = series[r], y = series[r+1]."""
    L = load()
    s = _dev(series)
    rows = _dev(rows, torch.int32)
    nb, m = rows.shape
    T, p = s.shape
    G = torch.empty((nb, p, p), dtype=torch.float64, device=s.device)
    Cm = torch.empty((nb, p, p), dtype=torch.float64, device=s.device)
    ysrc = C.c_void_p(s.data_ptr() + 8 * p)
    _check(L.uoi_gram(nb, m, _ptr(rows), p, _ptr(s), p, p, ysrc, p, _ptr(G), _ptr(Cm), _stream()),
           allow_noconv=False)
    return G, Cm


def bootstrap_rows(seed: int, nb: int, n: int, device="cuda"):
    rows = torch.empty((nb, n), dtype=torch.int32, device=device)
    _check(load().uoi_bootstrap_rows(seed, nb, n, _ptr(rows), _stream()), allow_noconv=False)
    return rows


def split_rows(seed: int, nb: int, n: int, num: int = 4, den: int = 5, device="cuda"):
    ntr = (n * num) // den
    tr = torch.empty((nb, ntr), dtype=torch.int32, device=device)
    ev = torch.empty((nb, n - ntr), dtype=torch.int32, device=device)
    _check(load().uoi_split_rows(seed, nb, n, num, den, _ptr(tr), _ptr(ev), _stream()),
           allow_noconv=False)
    return tr, ev


def var_boot_rows(seed: int, nb: int, N: int, L: int, device="cuda"):
    rows = torch.empty((nb, N), dtype=torch.int32, device=device)
    _check(load().uoi_var_boot_rows(seed, nb, N, L, _ptr(rows), _stream()), allow_noconv=False)
    return rows


def var_split_rows(seed: int, nb: int, N: int, L: int, num: int = 4, den: int = 5, device="cuda"):
    tr = torch.empty((nb, N), dtype=torch.int32, device=device)
    ev = torch.empty((nb, N), dtype=torch.int32, device=device)
    ntr = (C.c_int32 * nb)()
    nev = (C.c_int32 * nb)()
    _check(load().uoi_var_split_rows(seed, nb, N, L, num, den, _ptr(tr), _ptr(ev), ntr, nev,
                                     _stream()), allow_noconv=False)
    return [tr[k, : ntr[k]] for k in range(nb)], [ev[k, : nev[k]] for k in range(nb)]


def spd_inverse(G: torch.Tensor, rho: float):
    L = load()
    G = _dev(G)
    nb, p, _ = G.shape
    M = torch.empty_like(G)
    _check(L.uoi_spd_inverse(nb, p, _ptr(G), float(rho), _ptr(M), _stream()), allow_noconv=False)
    return M


def release_workspace():
    load().uoi_release_workspace()


def tune_reset():
    """Forget the autotuner's recorded launch shapes (UOI_TUNE_FILE is read again)."""
    load().uoi_tune_reset()


def version() -> str:
    return load().uoi_version().decode()


class MLP:
    """Warm-start network living on the GPU (uoi_mlp_* functions)."""

    def __init__(self, n_in: int, hidden: int, n_out: int):
        L = load()
        h = C.c_void_p()
        _check(L.uoi_mlp_create(n_in, hidden, n_out, C.byref(h)), allow_noconv=False)
        self.handle = h
        self.n_in, self.hidden, self.n_out = n_in, hidden, n_out
        self.nparam = int(L.uoi_mlp_num_params(h))

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.uoi_mlp_destroy(self.handle)
            self.handle = None

    def set_params(self, theta: torch.Tensor):
        theta = _dev(theta, torch.float32)
        assert theta.numel() == self.nparam
        _check(load().uoi_mlp_set_params(self.handle, _ptr(theta), _stream()), allow_noconv=False)

    def get_params(self) -> torch.Tensor:
        t = torch.empty(self.nparam, dtype=torch.float32, device="cuda")
        _check(load().uoi_mlp_get_params(self.handle, _ptr(t), _stream()), allow_noconv=False)
        return t

    def forward(self, X: torch.Tensor) -> torch.Tensor:
        X = _dev(X, torch.float32)
        Y = torch.empty((X.shape[0], self.n_out), dtype=torch.float32, device=X.device)
        _check(load().uoi_mlp_forward(self.handle, X.shape[0], _ptr(X), _ptr(Y), _stream()),
               allow_noconv=False)
        return Y

    def loss_grad(self, X: torch.Tensor, T: torch.Tensor):
        X = _dev(X, torch.float32); T = _dev(T, torch.float32)
        g = torch.empty(self.nparam, dtype=torch.float32, device=X.device)
        loss = C.c_double()
        _check(load().uoi_mlp_loss_grad(self.handle, X.shape[0], _ptr(X), _ptr(T), _ptr(g),
                                        C.byref(loss), _stream()), allow_noconv=False)
        return loss.value, g

    def train_step(self, X: torch.Tensor, T: torch.Tensor, lr: float, want_loss: bool = True):
        """One Adam step; returns the batch loss (a synchronisation) or None."""
        loss = C.c_double()
        _check(load().uoi_mlp_train_step(self.handle, X.shape[0], _ptr(X), _ptr(T), float(lr),
                                         C.byref(loss) if want_loss else None, _stream()),
               allow_noconv=False)
        return loss.value if want_loss else None


def ws_dataset(c: torch.Tensor, lambdas, z: torch.Tensor):
    """Network inputs / targets from solved problems: c [nb, p] or [nb, p, pe],
    z [nb, q, p] or [nb, q, pe, p]."""
    c = _dev(c.contiguous()); z = _dev(z.contiguous())
    if c.dim() == 2:
        c = c.unsqueeze(-1).contiguous()
    nb, p, pe = c.shape
    lam = np.ascontiguousarray(np.asarray(lambdas, dtype=np.float64))
    q = lam.size
    X = torch.empty((nb * q * pe, p + 1), dtype=torch.float32, device=c.device)
    T = torch.empty((nb * q * pe, p), dtype=torch.float32, device=c.device)
    _check(load().uoi_ws_dataset(nb, p, q, pe, _ptr(c), lam.ctypes.data_as(C.c_void_p), _ptr(z), _ptr(X),
                                 _ptr(T), _stream()), allow_noconv=False)
    return X, T


def lasso_solve_multi(G: torch.Tensor, Cm: torch.Tensor, lambdas, **kw):
    """Solves sharing each Gram: G [nb, p, p], Cm [nb, p, pe]; z [nb, q, pe, p]."""
    G = _dev(G); Cm = _dev(Cm.contiguous())
    nb, p, pe = Cm.shape
    o, lam = make_opts(lambdas, **kw)
    q = lam.size
    z = torch.empty((nb, q, pe, p), dtype=torch.float64, device=G.device)
    its = torch.empty((nb, q, pe), dtype=torch.int32, device=G.device)
    kkt = torch.empty((nb, q, pe), dtype=torch.float64, device=G.device)
    code = _check(load().uoi_lasso_solve_multi(nb, p, pe, _ptr(G), _ptr(Cm), C.byref(o), _ptr(z), _ptr(its),
                                               _ptr(kkt)))
    return dict(z=z, iters=its, kkt=kkt, status=code)
