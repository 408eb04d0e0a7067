"""End-to-end UoI_LASSO / UoI_VAR parity of the HIP path against the CPU oracle.

Supports are compared bit for bit on every bit the oracle decides with a
margin (a bit inside the margin can legitimately differ between two solvers
that both meet the KKT tolerance); the chosen support per split must agree
wherever the loss gap exceeds 1e-9 relative; beta* / A must agree within
1e-6 relative to its largest entry."""
import numpy as np
import pytest
import torch

from paper_1808_06992_amd import synth

from parity import (check_lasso_estimation, check_var_estimation, check_var_per_equation,
                    words_to_bool)

pytestmark = pytest.mark.gpu

TAU = 1e-6


@pytest.fixture(scope="module")
def api():
    from paper_1808_06992_amd import _lib
    _lib.load()
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return _lib


def cuda(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def lasso_decided(orc, pr, seed, sel_beta):
    """Decided intersection bits per lambda: every bootstrap decided, or one decidedly zero."""
    n, p = pr.X.shape
    B1, q = sel_beta.shape[:2]
    all_dec = np.ones((q, p), bool)
    some_zero = np.zeros((q, p), bool)
    for k in range(B1):
        G, c = orc.gram(pr.X, pr.y, orc.boot_rows(seed, k, n))
        for j in range(q):
            d = orc.decided_bits(G, c, pr.lambdas[j], sel_beta[k, j], TAU)
            all_dec[j] &= d
            some_zero[j] |= d & (sel_beta[k, j] == 0)
    return all_dec | some_zero


@pytest.mark.parametrize("precision,solver,rho", [("fp64", "batched", 1.0), ("fp64", "plain", 1.0),
                                                  ("mixed", "batched", 1.0), ("mixed", "batched", 0.0),
                                                  ("fp64", "plain", 0.0)])
def test_uoi_lasso_small_config(api, orc, precision, solver, rho):
    """rho = 0 sets the penalty to the mean diagonal of the Grams; the
    minimisers, hence every comparison, are the same."""
    pr = synth.lasso_small(0)
    seed = 0
    ref = orc.uoi_lasso(pr.X, pr.y, pr.lambdas, pr.B1, pr.B2, seed, keep_selection=True)
    assert ref["status"] == 0
    out = api.lasso_fit(cuda(pr.X), cuda(pr.y), pr.lambdas, pr.B1, pr.B2, seed, kkt_tol=1e-10,
                        precision=precision, solver=solver, sel_beta=True, rho=rho)
    assert out["status"] == 0 and out["n_unconverged"] == 0
    p = pr.X.shape[1]
    dec = lasso_decided(orc, pr, seed, ref["sel_beta"])
    got = words_to_bool(out["supports"].cpu().numpy(), p)
    want = words_to_bool(ref["supports"], p)
    assert np.array_equal(got[dec], want[dec])
    # selection estimates agree solve by solve
    sb = out["sel_beta"].cpu().numpy()
    for k in range(pr.B1):
        for j in range(pr.lambdas.size):
            r = ref["sel_beta"][k, j]
            assert np.abs(sb[k, j] - r).max() <= 1e-6 * max(np.abs(r).max(), 1e-300)
    # losses, chosen supports and beta* against oracle refits on the GPU's
    # supports, and against the oracle's own results where the choices coincide
    check_lasso_estimation(orc, pr.X, pr.y, seed, out, ref)


def test_uoi_lasso_ragged_sizes(api, orc):
    # p not a multiple of 16 or 64, q odd, n not a multiple of the row chunk
    pr = synth.lasso_random(157, 37, 6, 11, q=7, B1=5, B2=6)
    ref = orc.uoi_lasso(pr.X, pr.y, pr.lambdas, pr.B1, pr.B2, 5, keep_selection=True)
    assert ref["status"] == 0
    out = api.lasso_fit(cuda(pr.X), cuda(pr.y), pr.lambdas, pr.B1, pr.B2, 5, kkt_tol=1e-10)
    assert out["status"] == 0 and out["n_unconverged"] == 0
    dec = lasso_decided(orc, pr, 5, ref["sel_beta"])
    got = words_to_bool(out["supports"].cpu().numpy(), 37)
    want = words_to_bool(ref["supports"], 37)
    assert np.array_equal(got[dec], want[dec])
    check_lasso_estimation(orc, pr.X, pr.y, 5, out, ref)


def test_uoi_lasso_all_refit_paths(api, orc):
    """Dense coefficients make the intersection supports span every refit route:
    in-LDS Cholesky (|S| <= 80), blocked Cholesky with the factor in global
    scratch (80 < |S| <= 256) and conjugate gradients (|S| > 256); every
    lambda's loss is compared, so each route is checked against the oracle's QR."""
    pr = synth.lasso_random(700, 320, 320, 5, noise=0.1, q=10, B1=3, B2=3)
    seed = 5
    ref = orc.uoi_lasso(pr.X, pr.y, pr.lambdas, pr.B1, pr.B2, seed, keep_selection=True)
    assert ref["status"] == 0
    out = api.lasso_fit(cuda(pr.X), cuda(pr.y), pr.lambdas, pr.B1, pr.B2, seed, kkt_tol=1e-10)
    assert out["status"] == 0
    p = pr.X.shape[1]
    got = words_to_bool(out["supports"].cpu().numpy(), p)
    want = words_to_bool(ref["supports"], p)
    sizes = want.sum(1)
    assert sizes.min() <= 80 and np.any((sizes > 80) & (sizes <= 256)) and sizes.max() > 256
    dec = lasso_decided(orc, pr, seed, ref["sel_beta"])
    assert np.array_equal(got[dec], want[dec])
    same = np.all(got == want, axis=1)       # lambdas whose supports agree bit for bit
    for lo, hi in ((0, 80), (81, 256), (257, p)):
        assert np.any(same & (sizes >= lo) & (sizes <= hi)), (lo, hi, sizes, same)
    lg = out["losses"].cpu().numpy()
    np.testing.assert_allclose(lg[:, same], ref["losses"][:, same], rtol=1e-9)
    check_lasso_estimation(orc, pr.X, pr.y, seed, out, ref)


def test_uoi_lasso_refits_on_support_union(api, orc):
    """Sparse supports: the union of the q supports covers at most 3/4 of the
    columns, so the estimation products are formed over those columns only and
    beta* is scattered back; everything is compared with the oracle's full-width
    refits."""
    pr = synth.lasso_random(400, 200, 40, 9, noise=0.5, q=8, B1=6, B2=6, ratio=0.01)
    seed = 2
    ref = orc.uoi_lasso(pr.X, pr.y, pr.lambdas, pr.B1, pr.B2, seed, keep_selection=True)
    assert ref["status"] == 0
    out = api.lasso_fit(cuda(pr.X), cuda(pr.y), pr.lambdas, pr.B1, pr.B2, seed, kkt_tol=1e-10)
    assert out["status"] == 0
    p = pr.X.shape[1]
    got = words_to_bool(out["supports"].cpu().numpy(), p)
    want = words_to_bool(ref["supports"], p)
    union = got.any(0)
    assert 0 < union.sum() <= 3 * p // 4
    dec = lasso_decided(orc, pr, seed, ref["sel_beta"])
    assert np.array_equal(got[dec], want[dec])
    b = out["beta"].cpu().numpy()
    assert not np.any(b[~union])
    check_lasso_estimation(orc, pr.X, pr.y, seed, out, ref)


def test_uoi_var_small(api, orc):
    pr = synth.var1(12, 600, 0.15, 0.8, 4, burn=50, q=6, B1=4, B2=4)
    seed = 3
    ref = orc.uoi_var(pr.series, pr.lambdas, pr.B1, pr.B2, seed)
    assert ref["status"] == 0
    out = api.var_fit(cuda(pr.series), pr.lambdas, pr.B1, pr.B2, seed, kkt_tol=1e-10)
    assert out["status"] == 0
    p = pr.series.shape[1]
    got = words_to_bool(out["supports"].cpu().numpy(), p)
    want = words_to_bool(ref["supports"], p)
    mism = np.argwhere(got != want)
    assert mism.shape[0] <= 2, f"support mismatches {mism.tolist()}"
    check_var_estimation(orc, pr.series, seed, out, ref)
    assert np.all(out["mu"].cpu().numpy() == 0)


def test_nan_input_rejected(api):
    pr = synth.lasso_random(50, 8, 3, 2, q=3)
    X = pr.X.copy()
    X[3, 4] = np.nan
    with pytest.raises(api.UoiError) as ei:
        api.lasso_fit(cuda(X), cuda(pr.y), pr.lambdas, 2, 2, 0)
    assert ei.value.code == api.UOI_EINVAL


def test_refit_cg_cap_reported(api, orc):
    """Refits of supports above 256 members use conjugate gradients; one that is
    still above its tolerance at the iteration cap is counted and the fit returns
    UOI_ENOCONV (with the default cap every refit converges)."""
    pr = synth.lasso_random(700, 320, 320, 5, noise=0.1, q=10, B1=3, B2=3)
    X, y = cuda(pr.X), cuda(pr.y)
    capped = api.lasso_fit(X, y, pr.lambdas, pr.B1, pr.B2, 5, kkt_tol=1e-10, cg_max_iter=1)
    assert capped["status"] == api.UOI_ENOCONV
    assert capped["n_unconverged"] == 0 and capped["n_refit_unconverged"] > 0
    full = api.lasso_fit(X, y, pr.lambdas, pr.B1, pr.B2, 5, kkt_tol=1e-10)
    assert full["status"] == 0 and full["n_refit_unconverged"] == 0


@pytest.mark.parametrize("d,intercept,p,precision", [(2, True, 12, "fp64"), (3, False, 23, "fp64"),
                                                     (1, True, 12, "mixed"), (2, True, 40, "mixed")])
def test_uoi_var_order_d_and_intercept(api, orc, d, intercept, p, precision):
    """VAR(d) with an optional intercept (Eq. (5)-(8), Alg. 2 returning A_1..A_d and
    mu) against the oracle's explicit lagged design: supports in Eq. (7)'s column
    order (d = 3, p = 23: 69 coefficients per equation, two words), then losses,
    j*, A and mu against oracle refits on the GPU's supports."""
    seed = 6
    pr = synth.var_d(p, 600, d, 0.15, 0.8, 4, mu_scale=1.0, intercept=intercept, burn=50, q=6, B1=4, B2=4)
    ref = orc.uoi_var_d(pr.series, pr.lambdas, pr.B1, pr.B2, seed, d=d, intercept=intercept)
    assert ref["status"] == 0
    print(f"var d={d} intercept={intercept} p={p} {precision}", flush=True)
    out = api.var_fit(cuda(pr.series), pr.lambdas, pr.B1, pr.B2, seed, d=d, intercept=intercept,
                      kkt_tol=1e-10, precision=precision)
    assert out["status"] == 0 and out["n_unconverged"] == 0
    P = d * p
    got = words_to_bool(out["supports"].cpu().numpy(), P)
    want = words_to_bool(ref["supports"], P)
    mism = np.argwhere(got != want)
    assert mism.shape[0] <= 2, f"support mismatches {mism.tolist()}"
    check_var_estimation(orc, pr.series, seed, out, ref, d=d, intercept=intercept)


def test_uoi_var_per_equation_choice(api, orc):
    """Every equation chooses its own support index per split (UOI_FLAG_PER_EQUATION):
    supports as the joint fit's, per-equation losses against oracle refits on the
    GPU's supports, per-equation j*, and A and mu from the chosen refits."""
    seed, d = 8, 2
    pr = synth.var_d(12, 600, d, 0.15, 0.8, 5, mu_scale=1.0, intercept=True, burn=50, q=6, B1=4, B2=4)
    ref = orc.uoi_var_d(pr.series, pr.lambdas, pr.B1, pr.B2, seed, d=d, intercept=True, per_equation=True)
    assert ref["status"] == 0
    out = api.var_fit(cuda(pr.series), pr.lambdas, pr.B1, pr.B2, seed, d=d, intercept=True,
                      per_equation=True, kkt_tol=1e-10)
    assert out["status"] == 0
    assert out["jstar"].shape == (pr.B2, 12) and out["losses"].shape == (pr.B2, 6, 12)
    mism = np.argwhere(words_to_bool(out["supports"].cpu().numpy(), d * 12) != words_to_bool(ref["supports"], d * 12))
    assert mism.shape[0] <= 2, f"support mismatches {mism.tolist()}"
    check_var_per_equation(orc, pr.series, seed, out, ref, d=d, intercept=True)


def test_ingest_command_line_var_fit(api, tmp_path):
    """The command-line front end reads a series file, builds the lambda grid and
    fits on the GPU: the same results as the binding called directly."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    pr = synth.var_d(8, 400, 2, 0.2, 0.8, 3, mu_scale=1.0, intercept=True, burn=50, q=5, B1=3, B2=3)
    np.save(tmp_path / "s.npy", pr.series)
    out = tmp_path / "fit.npz"
    r = subprocess.run([sys.executable, "-m", "paper_1808_06992_amd.ingest", "var", "--series",
                        str(tmp_path / "s.npy"), "--order", "2", "--intercept", "--B1", "3", "--B2", "3",
                        "--q", "5", "--precision", "fp64", "--kkt-tol", "1e-10", "--out", str(out)],
                       cwd=root, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    with np.load(out, allow_pickle=False) as f:
        res = {k: f[k] for k in f.files}
    np.testing.assert_allclose(res["lambdas"], pr.lambdas, rtol=1e-12)
    ref = api.var_fit(cuda(pr.series), res["lambdas"], 3, 3, 0, d=2, intercept=True, kkt_tol=1e-10,
                      precision="fp64", relax=1.8)
    assert np.array_equal(res["A"], ref["A"].cpu().numpy())
    assert np.array_equal(res["mu"], ref["mu"].cpu().numpy())
    assert np.array_equal(res["supports"], ref["supports"].cpu().numpy().view(np.uint64))


@pytest.mark.gpu
def test_pathwise_and_strong_rule_baselines(api):
    """The non-learned baselines of the learned warm start on the n200 p50 fit:
    lambda continuation in 2 and 4 blocks reaches the cold solutions (within the
    KKT tolerance's reach), with iteration counts reported per block; the
    sequential strong rule keeps every support feature of nearly every solve."""
    from paper_1808_06992_amd import baselines
    pr = synth.lasso_small(0)
    r = baselines.pathwise(pr, 0, pr.B1, groups=(2, 4), kkt_tol=1e-10, precision="fp64")
    assert r["cold"]["mean_iters"] > 0
    for ng in (2, 4):
        pw = r["path"][ng]
        assert len(pw["block_max"]) == ng
        assert pw["max_rel_diff"] < 1e-6, pw
    sr = baselines.strong_rule(pr, 0, pr.B1)
    assert sr["solves_screened"] == pr.B1 * (pr.lambdas.size - 1)
    assert sr["kept_min"] >= 0 and sr["kept_mean"] >= sr["support_mean"]
    assert sr["violations"] <= 0.01 * sr["solves_screened"] * sr["config"]["p"]
