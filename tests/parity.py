"""Shared checks of the estimation step (Alg. 1 / Alg. 2 estimation loops)
against the oracle.

Several results are correct when a support bit lies inside the oracle's margin
or two supports tie in loss, so the GPU's discrete choices (its intersection
supports and its chosen support per split) are checked for validity and every
continuous result is then compared, unconditionally, with oracle refits taken
on those choices: Householder-QR least squares on the training rows for
UoI_LASSO, the oracle's normal-equation Cholesky on the training Gram for the
per-equation VAR refits.  When the GPU's choices coincide with the oracle's own,
the results are also compared with the oracle's end-to-end values."""
from __future__ import annotations

import numpy as np


def words_to_bool(w, p):
    """Support bitmasks (64-bit words, bit i of word i // 64) as booleans [..., p]."""
    w = np.ascontiguousarray(np.asarray(w).view(np.uint64))
    bits = np.unpackbits(w.view(np.uint8), axis=-1, bitorder="little")
    return bits[..., :p].astype(bool)


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def check_jstar(losses_ref, jstar_ref, jstar_gpu, gap=1e-9):
    """Every split picks the reference choice, or one whose reference loss ties within gap."""
    for k, (a, b) in enumerate(zip(jstar_ref, jstar_gpu)):
        if a == b:
            continue
        L = losses_ref[k]
        g = abs(L[b] - L[a]) / max(abs(L[a]), 1e-300)
        assert g <= gap, f"split {k}: reference j*={a}, GPU j*={b}, loss gap {g}"


# --------------------------------------------------------------------------- LASSO

def lasso_refit(orc, X, y, seed, k, S, num=4, den=5):
    """Refit of support S on split k's training rows (QR) and its evaluation loss."""
    n, p = X.shape
    tr, ev = orc.split_rows(seed, k, n, num, den)
    b = np.zeros(p)
    if S.size:
        b[S] = orc.lstsq_qr(X[np.ix_(tr, S)], y[tr])
    r = y[ev] - X[ev] @ b
    return b, float(r @ r / ev.size)


def check_lasso_estimation(orc, X, y, seed, out, ref=None, js_all=True, rtol=1e-9):
    """Losses, chosen supports and beta* of a GPU UoI_LASSO fit.

    js_all: refit every (split, support) for the loss comparison; otherwise only
    the supports that differ from the oracle's (ref required) are refitted and the
    others are compared with ref["losses"].  beta* is always compared with the
    average of the refits on the GPU's chosen supports."""
    p = X.shape[1]
    bits = words_to_bool(out["supports"].cpu().numpy(), p)          # [q][p]
    js = out["jstar"].cpu().numpy()
    lg = out["losses"].cpu().numpy()
    B2, q = lg.shape
    # the chosen support is the first minimiser of the reported losses
    assert np.array_equal(js, np.argmin(lg, axis=1)), (js, np.argmin(lg, axis=1))
    same = np.zeros(q, bool)
    if ref is not None:
        same = np.all(bits == words_to_bool(ref["supports"], p), axis=1)
    want = np.empty((B2, q))
    for j in range(q):
        if not js_all and same[j]:
            want[:, j] = ref["losses"][:, j]
            continue
        S = np.flatnonzero(bits[j])
        for k in range(B2):
            want[k, j] = lasso_refit(orc, X, y, seed, k, S)[1]
    np.testing.assert_allclose(lg, want, rtol=rtol, atol=0)
    check_jstar(want, np.argmin(want, axis=1), js)
    acc = np.zeros(p)
    for k in range(B2):
        acc += lasso_refit(orc, X, y, seed, k, np.flatnonzero(bits[js[k]]))[0]
    bstar = acc / B2
    b = out["beta"].cpu().numpy()
    assert rel(b, bstar) <= rtol if np.abs(bstar).max() > 0 else not np.any(b)
    assert not np.any(b[~bits[np.unique(js)].any(0)])               # zero off the union
    if ref is not None:
        if same.all():
            np.testing.assert_allclose(lg, ref["losses"], rtol=rtol, atol=0)
            check_jstar(ref["losses"], ref["jstar"], js)
        if same.all() and np.array_equal(js, ref["jstar"]):
            assert rel(b, ref["beta"]) <= 1e-6
    return dict(same=same, bits=bits)


# --------------------------------------------------------------------------- VAR

def lagged(series, d):
    """Eq. (6)-(7) written out: responses x_t (t = d .. T-1), designs [x_{t-1} .. x_{t-d}]."""
    T, p = series.shape
    N = T - d
    Xl = np.hstack([series[d - 1 - l: d - 1 - l + N] for l in range(d)])
    return np.ascontiguousarray(Xl), np.ascontiguousarray(series[d:])


def var_split_stats(orc, series, seed, k, d=1, intercept=False, num=4, den=5):
    """Training statistics of split k (oracle Gram over the training rows, centred
    by the training means when an intercept is fitted), the training means and
    the evaluation rows."""
    T, p = series.shape
    N = T - d
    L = orc.var_block_len(N)
    tr, ev = orc.var_split_rows(seed, k, N, L, num, den)
    Xl, Yl = lagged(series, d)
    Xt, Yt = Xl[tr], Yl[tr]
    xm = Xt.mean(axis=0) if intercept else np.zeros(Xl.shape[1])
    ym = Yt.mean(axis=0) if intercept else np.zeros(p)
    G, Cm = orc.gram_multi(Xt - xm, Yt - ym, np.arange(tr.size, dtype=np.int32))
    return G, Cm, xm, ym, Xl[ev], Yl[ev]


def var_refits(orc, series, stats, bits_j):
    """Per-equation refits of supports bits_j [p][d p] (Eq. (7) column order) from a
    split's training statistics (normal-equation Cholesky), their intercepts
    ybar_T - xbar_T' b, and the evaluation loss summed over equations.
    Returns (coefficients [p][d p], intercepts [p], loss)."""
    G, Cm, xm, ym, Xe, Ye = stats
    p, P = bits_j.shape
    F = np.zeros((p, P))
    for e in range(p):
        S = np.flatnonzero(bits_j[e])
        if S.size:
            F[e, S] = orc.ols_normal(G, Cm[:, e], S)
    mu = ym - F @ xm
    Rm = Ye - mu - Xe @ F.T
    per_eq = np.sum(Rm * Rm, axis=0) / Xe.shape[0]
    return F, mu, float(per_eq.sum()), per_eq


def check_var_estimation(orc, series, seed, out, ref=None, d=1, intercept=False, rtol=1e-9):
    """Losses of supports that differ from the oracle's, chosen supports, A and mu of
    a GPU UoI_VAR fit, against refits conditional on the GPU's supports."""
    T, p = series.shape
    P = d * p
    bits = words_to_bool(out["supports"].cpu().numpy(), P)          # [q][p][d p]
    js = out["jstar"].cpu().numpy()
    lg = out["losses"].cpu().numpy()
    B2, q = lg.shape
    assert np.array_equal(js, np.argmin(lg, axis=1))
    same = np.zeros(q, bool)
    if ref is not None:
        same = np.all(bits == words_to_bool(ref["supports"], P), axis=(1, 2))
    want = np.empty((B2, q))
    fits, stats = {}, {}

    def st(k):
        if k not in stats:
            stats[k] = var_split_stats(orc, series, seed, k, d, intercept)
        return stats[k]

    for j in range(q):
        if ref is not None and same[j]:
            want[:, j] = ref["losses"][:, j]
            continue
        for k in range(B2):
            fits[(k, j)] = var_refits(orc, series, st(k), bits[j])
            want[k, j] = fits[(k, j)][2]
    np.testing.assert_allclose(lg, want, rtol=rtol, atol=0)
    check_jstar(want, np.argmin(want, axis=1), js)
    accA = np.zeros((p, P))
    accm = np.zeros(p)
    for k in range(B2):
        f = fits.get((k, js[k])) or var_refits(orc, series, st(k), bits[js[k]])
        accA += f[0]
        accm += f[1]
    Astar = (accA / B2).reshape(p, d, p).transpose(1, 0, 2)        # A[l][e][m] = F[e][l p + m]
    A = out["A"].cpu().numpy().reshape(d, p, p)
    assert rel(A, Astar) <= rtol if np.abs(Astar).max() > 0 else not np.any(A)
    mu = out["mu"].cpu().numpy()
    if intercept:
        np.testing.assert_allclose(mu, accm / B2, rtol=rtol, atol=rtol * max(np.abs(accm).max() / B2, 1.0))
    else:
        assert np.all(mu == 0.0)
    if ref is not None and same.all():
        check_jstar(ref["losses"], ref["jstar"], js)
        if np.array_equal(js, ref["jstar"]):
            assert rel(A, np.asarray(ref["A"]).reshape(d, p, p)) <= 1e-6
            if intercept:
                np.testing.assert_allclose(mu, ref["mu"], rtol=1e-6, atol=1e-6 * np.abs(ref["mu"]).max())
    return dict(same=same, bits=bits)


def check_var_per_equation(orc, series, seed, out, ref, d=1, intercept=False, rtol=1e-9):
    """As check_var_estimation for the per-equation choice: losses [B2][q][p] against
    oracle refits on the GPU's supports, each equation's j* an argmin of its own
    losses, A and mu from the refits each equation chose."""
    T, p = series.shape
    P = d * p
    bits = words_to_bool(out["supports"].cpu().numpy(), P)          # [q][p][d p]
    js = out["jstar"].cpu().numpy()                                 # [B2][p]
    lg = out["losses"].cpu().numpy()                                # [B2][q][p]
    B2, q = lg.shape[:2]
    assert np.array_equal(js, np.argmin(lg, axis=1))
    want = np.empty((B2, q, p))
    F = {}
    for k in range(B2):
        stats = var_split_stats(orc, series, seed, k, d, intercept)
        for j in range(q):
            F[(k, j)] = var_refits(orc, series, stats, bits[j])
            want[k, j] = F[(k, j)][3]
    np.testing.assert_allclose(lg, want, rtol=rtol, atol=0)
    accA, accm = np.zeros((p, P)), np.zeros(p)
    for k in range(B2):
        for e in range(p):
            check_jstar(want[:, :, e], np.argmin(want[:, :, e], axis=1), js[:, e])
            f = F[(k, js[k, e])]
            accA[e] += f[0][e]
            accm[e] += f[1][e]
    Astar = (accA / B2).reshape(p, d, p).transpose(1, 0, 2)
    A = out["A"].cpu().numpy().reshape(d, p, p)
    assert rel(A, Astar) <= rtol
    mu = out["mu"].cpu().numpy()
    if intercept:
        np.testing.assert_allclose(mu, accm / B2, rtol=rtol, atol=rtol * max(np.abs(accm).max() / B2, 1.0))
    if np.array_equal(bits, words_to_bool(ref["supports"], P)) and np.array_equal(js, ref["jstar"]):
        assert rel(A, np.asarray(ref["A"]).reshape(d, p, p)) <= 1e-6
