"""GPU parity of the individual steps against the CPU oracle (MI355X only).

Index streams are compared bit for bit; float64 statistics, inverses and ADMM
solutions are compared with the tolerances stated in each test."""
import numpy as np
import pytest
import torch

from paper_1808_06992_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    from paper_1808_06992_amd import _lib
    _lib.load()
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return _lib


def cuda(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


# --------------------------------------------------------------------------- indices

@pytest.mark.parametrize("n", [1, 7, 200, 1001, 5000])
def test_bootstrap_rows_bit_identical(api, orc, n):
    rows = api.bootstrap_rows(12345, 5, n).cpu().numpy()
    for k in range(5):
        assert np.array_equal(rows[k], orc.boot_rows(12345, k, n))


@pytest.mark.parametrize("n", [2, 5, 200, 1001, 5000])
def test_split_rows_bit_identical(api, orc, n):
    tr, ev = api.split_rows(99, 4, n)
    tr, ev = tr.cpu().numpy(), ev.cpu().numpy()
    for k in range(4):
        t, e = orc.split_rows(99, k, n)
        assert np.array_equal(tr[k], t) and np.array_equal(ev[k], e)


@pytest.mark.parametrize("N,L", [(9999, 22), (19999, 28), (103, 5), (10, 10)])
def test_var_rows_bit_identical(api, orc, N, L):
    rows = api.var_boot_rows(7, 3, N, L).cpu().numpy()
    for k in range(3):
        assert np.array_equal(rows[k], orc.var_boot_rows(7, k, N, L))
    if (N + L - 1) // L >= 2:
        trs, evs = api.var_split_rows(7, 3, N, L)
        for k in range(3):
            t, e = orc.var_split_rows(7, k, N, L)
            assert np.array_equal(trs[k].cpu().numpy(), t)
            assert np.array_equal(evs[k].cpu().numpy(), e)


# --------------------------------------------------------------------------- Gram

@pytest.mark.parametrize("n,p,m", [(37, 5, 37), (517, 133, 601), (300, 64, 17), (1000, 200, 1000)])
def test_gram_parity(api, orc, n, p, m):
    rng = np.random.default_rng(n + p)
    X = rng.standard_normal((n, p))
    y = rng.standard_normal(n)
    rows = rng.integers(0, n, size=(3, m)).astype(np.int32)
    G, c = api.gram(cuda(X), cuda(rows, torch.int32), cuda(y))
    G, c = G.cpu().numpy(), c.cpu().numpy()
    for b in range(3):
        Go, co = orc.gram(X, y, rows[b])
        np.testing.assert_allclose(G[b], Go, rtol=1e-12, atol=1e-13)
        np.testing.assert_allclose(c[b, :, 0], co, rtol=1e-12, atol=1e-13)
        assert np.array_equal(G[b], G[b].T)


@pytest.mark.parametrize("p,nb", [(100, 200), (100, 530), (300, 100)])
def test_gram_parity_split_and_full_rounds(api, orc, p, nb):
    """On a 256-CU part with two Gram workgroups per CU (512 slots): 200
    single-tile products are each split in two over their rows (the cases above
    split into four), 530 fill more than a round and run unsplit.  At p = 300
    (600 tiles) the unsplit launch also holds tiles off the diagonal and a ragged
    last tile row.  Every product matches the oracle and stays symmetric."""
    rng = np.random.default_rng(11)
    n, m = 400, 300
    X = rng.standard_normal((n, p))
    y = rng.standard_normal(n)
    rows = rng.integers(0, n, size=(nb, m)).astype(np.int32)
    G, c = api.gram(cuda(X), cuda(rows, torch.int32), cuda(y))
    G, c = G.cpu().numpy(), c.cpu().numpy()
    for b in range(nb):
        Go, co = orc.gram(X, y, rows[b])
        np.testing.assert_allclose(G[b], Go, rtol=1e-12, atol=1e-13)
        np.testing.assert_allclose(c[b, :, 0], co, rtol=1e-12, atol=1e-13)
        assert np.array_equal(G[b], G[b].T)


def test_gram_var_parity(api, orc):
    pr = synth.var1(70, 400, 0.1, 0.8, 3, burn=20)
    N = pr.series.shape[0] - 1
    rows = np.stack([orc.var_boot_rows(3, k, N, 8) for k in range(2)])
    G, Cm = api.gram_var(cuda(pr.series), cuda(rows, torch.int32))
    for b in range(2):
        Go, Co = orc.gram_var(pr.series, rows[b])
        np.testing.assert_allclose(G[b].cpu().numpy(), Go, rtol=1e-12, atol=1e-13)
        np.testing.assert_allclose(Cm[b].cpu().numpy(), Co, rtol=1e-12, atol=1e-13)


# --------------------------------------------------------------------------- inverse

@pytest.mark.parametrize("p,nb", [(1, 2), (7, 2), (50, 2), (88, 2), (89, 2), (130, 2), (192, 2), (200, 2),
                                  (257, 11), (300, 3), (384, 2)])
def test_spd_inverse_parity(api, orc, p, nb):
    """Blocked sweeps of 64-wide pivot blocks with a ragged last block (p = 89,
    130, 200, 257, 300: 25, 2, 8, 1 and 44 columns), blocks that end on p (192,
    384), and a batch that is not a multiple of the 8 XCDs."""
    rng = np.random.default_rng(p)
    n = 3 * p + 10
    X = rng.standard_normal((n, p))
    G = np.stack([orc.gram(X, X[:, 0], orc.boot_rows(1, k, n))[0] for k in range(nb)])
    M = api.spd_inverse(cuda(G), 1.0).cpu().numpy()
    for b in range(nb):
        ref = np.linalg.inv(G[b] + np.eye(p))
        np.testing.assert_allclose(M[b], ref, rtol=1e-11, atol=1e-13 * np.abs(ref).max())
        if p > 88:  # blocked sweeps: the upper triangle is stored as the mirror of the lower one
            assert np.array_equal(M[b], M[b].T)


@pytest.mark.parametrize("p,nb", [(1000, 7), (700, 48)])
def test_spd_inverse_parity_many_tiles(api, p, nb):
    """More tiles per block step than workgroups resident at once; an odd batch,
    and ragged last pivot blocks of 40 (p = 1000) and 60 (p = 700) columns."""
    rng = np.random.default_rng(p + nb)
    n = 2 * p
    G = np.empty((nb, p, p))
    for b in range(nb):
        X = rng.standard_normal((n, p))
        G[b] = X.T @ X / n
    M = api.spd_inverse(cuda(G), 1.0).cpu().numpy()
    for b in sorted({0, nb // 2, nb - 1}):
        ref = np.linalg.inv(G[b] + np.eye(p))
        np.testing.assert_allclose(M[b], ref, rtol=1e-11, atol=1e-13 * np.abs(ref).max())
        assert np.array_equal(M[b], M[b].T)
    # every matrix: residual of (G + I) M = I
    R = np.einsum("bij,bjk->bik", G + np.eye(p), M) - np.eye(p)
    assert np.abs(R).max() < 1e-11


# --------------------------------------------------------------------------- ADMM

def _oracle_solutions(orc, G, c, lams):
    out = []
    b = None
    for lam in lams:
        b, st = orc.lasso_cd(G, c, lam, tol=1e-13, b0=b)
        assert st >= 0
        out.append(b.copy())
    return np.array(out)


@pytest.mark.parametrize("solver,precision,relax", [("batched", "fp64", 1.0), ("plain", "fp64", 1.0),
                                                    ("batched", "mixed", 1.0), ("batched", "fp64", 1.6),
                                                    ("plain", "fp64", 1.7), ("batched", "mixed", 1.6)])
@pytest.mark.parametrize("n,p,q", [(200, 50, 16), (400, 130, 9)])
def test_admm_matches_oracle(api, orc, solver, precision, relax, n, p, q):
    pr = synth.lasso_random(n, p, 10, 5, q=q)
    Gs, cs = [], []
    for k in range(3):
        G, c = orc.gram(pr.X, pr.y, orc.boot_rows(0, k, n))
        Gs.append(G)
        cs.append(c)
    Gs, cs = np.array(Gs), np.array(cs)
    res = api.lasso_solve_batch(cuda(Gs), cuda(cs), pr.lambdas, kkt_tol=1e-10, solver=solver,
                                precision=precision, max_iter=50000, relax=relax)
    z = res["z"].cpu().numpy()
    assert res["status"] == 0
    assert np.all(res["iters"].cpu().numpy() >= 0)
    for k in range(3):
        ref = _oracle_solutions(orc, Gs[k], cs[k], pr.lambdas)
        for j in range(q):
            # the GPU estimate meets the KKT bound when checked by the oracle
            assert orc.kkt(Gs[k], cs[k], pr.lambdas[j], z[k, j]) <= 1e-8
            scale = max(np.abs(ref[j]).max(), 1e-300)
            assert np.abs(z[k, j] - ref[j]).max() <= 1e-6 * scale
            dec = orc.decided_bits(Gs[k], cs[k], pr.lambdas[j], ref[j])
            assert np.array_equal((z[k, j] != 0)[dec], (ref[j] != 0)[dec])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_admm_cold_start_zero_solutions(api, orc, precision):
    """lambda >= ||c||_inf: z = 0 is the solution, and a cold start meets the KKT
    bound at iteration 0 (its first check needs no product: the gradient at z = 0
    is c).  The other lambdas converge to the oracle's solutions."""
    pr = synth.lasso_random(300, 70, 8, 3, q=6)
    Gs, cs = [], []
    for k in range(2):
        G, c = orc.gram(pr.X, pr.y, orc.boot_rows(0, k, 300))
        Gs.append(G)
        cs.append(c)
    Gs, cs = np.array(Gs), np.array(cs)
    cmax = np.abs(cs).max(axis=1)
    lams = np.array([2.0 * cmax.max(), 1.0 * cmax.max() + 1e-9, 0.5 * cmax.min(), 0.2 * cmax.min()])
    res = api.lasso_solve_batch(cuda(Gs), cuda(cs), lams, kkt_tol=1e-9, precision=precision)
    assert res["status"] == 0
    z, its, kkt = (res[k].cpu().numpy() for k in ("z", "iters", "kkt"))
    for k in range(2):
        for j, lam in enumerate(lams):
            if lam >= cmax[k]:
                assert its[k, j] == 0 and np.all(z[k, j] == 0.0)
                assert kkt[k, j] == 0.0
            else:
                assert its[k, j] > 0
                assert orc.kkt(Gs[k], cs[k], lam, z[k, j]) <= 1e-8
                ref, st = orc.lasso_cd(Gs[k], cs[k], lam, tol=1e-13)
                assert st >= 0
                assert np.abs(z[k, j] - ref).max() <= 1e-6 * max(np.abs(ref).max(), 1e-300)


def test_admm_reports_nonconvergence(api, orc):
    pr = synth.lasso_random(200, 50, 10, 1, q=4)
    G, c = orc.gram(pr.X, pr.y, np.arange(200, dtype=np.int32))
    res = api.lasso_solve_batch(cuda(G[None]), cuda(c[None]), pr.lambdas, kkt_tol=1e-12,
                                max_iter=1, check_every=1)
    assert res["status"] == api.UOI_ENOCONV
    its = res["iters"].cpu().numpy()
    assert np.any(its < 0)


def _three_bootstraps(orc, pr, n):
    Gs, cs = [], []
    for k in range(3):
        G, c = orc.gram(pr.X, pr.y, orc.boot_rows(0, k, n))
        Gs.append(G)
        cs.append(c)
    return np.array(Gs), np.array(cs)


@pytest.mark.parametrize("relax", [1.0, 1.6])
def test_mixed_tight_tolerance_iterations(api, orc, relax):
    """A tolerance below what the float32 iteration resolves (1e-10): solves park
    at the float32 floor and the float64 finish converges them, so the mixed
    path's iteration counts stay close to the float64 path's (the float32 phase
    does not run on to the iteration cap)."""
    pr = synth.lasso_random(200, 50, 10, 5, q=16)
    Gs, cs = _three_bootstraps(orc, pr, 200)
    kw = dict(kkt_tol=1e-10, max_iter=50000, relax=relax)
    r64 = api.lasso_solve_batch(cuda(Gs), cuda(cs), pr.lambdas, precision="fp64", **kw)
    r32 = api.lasso_solve_batch(cuda(Gs), cuda(cs), pr.lambdas, precision="mixed", **kw)
    assert r64["status"] == 0 and r32["status"] == 0
    i64 = r64["iters"].cpu().numpy().astype(float)
    i32 = r32["iters"].cpu().numpy().astype(float)
    assert i64.min() >= 0 and i32.min() >= 0
    print(f"relax {relax}: float64 mean {i64.mean():.1f} max {i64.max():.0f}; "
          f"mixed mean {i32.mean():.1f} max {i32.max():.0f}")
    assert i32.max() <= 1.5 * i64.max() + 30
    assert i32.mean() <= 1.3 * i64.mean() + 15
    z = r32["z"].cpu().numpy()
    for k in range(3):
        for j in range(pr.lambdas.size):
            assert orc.kkt(Gs[k], cs[k], pr.lambdas[j], z[k, j]) <= 1e-8


def test_mixed_iteration_cap_bounds_both_phases(api, orc):
    """max_iter bounds the float32 phase and the float64 finish together: no
    converged solve reports more than max_iter iterations, the others are flagged."""
    pr = synth.lasso_random(200, 50, 10, 5, q=16)
    Gs, cs = _three_bootstraps(orc, pr, 200)
    cap = 40
    res = api.lasso_solve_batch(cuda(Gs), cuda(cs), pr.lambdas, kkt_tol=1e-10, max_iter=cap,
                                precision="mixed")
    its = res["iters"].cpu().numpy()
    assert res["status"] == api.UOI_ENOCONV
    assert np.any(its < 0)
    assert its.max() <= cap
    assert np.all((its == -1) | (its >= 0))


@pytest.mark.parametrize("precision,relax", [("fp64", 1.0), ("mixed", 1.6)])
def test_graph_replay_matches_eager_launches(api, orc, precision, relax):
    """Chunks of ADMM iterations replayed as captured graphs give exactly the
    results of launching every iteration eagerly: several replays of the cached
    graphs (within a sweep and across calls), with eager work and
    synchronisations between them, each compared with the eager result."""
    pr = synth.lasso_random(400, 130, 10, 5, q=9)
    Gs, cs = _three_bootstraps(orc, pr, 400)
    G, c = cuda(Gs), cuda(cs)
    kw = dict(kkt_tol=1e-10, precision=precision, relax=relax, max_iter=50000)
    ref = api.lasso_solve_batch(G, c, pr.lambdas, eager=True, **kw)
    assert ref["status"] == 0
    pr2 = synth.lasso_random(200, 50, 10, 6, q=5)
    G2, c2 = _three_bootstraps(orc, pr2, 200)
    for rep in range(3):
        got = api.lasso_solve_batch(G, c, pr.lambdas, **kw)
        torch.cuda.synchronize()
        for key in ("z", "u", "iters", "kkt"):
            assert torch.equal(got[key], ref[key]), (rep, key)
        # eager work of another shape between the replays
        other = api.lasso_solve_batch(cuda(G2), cuda(c2), pr2.lambdas, eager=True, kkt_tol=1e-8)
        assert other["status"] == 0
        torch.cuda.synchronize()


def test_graph_replay_whole_fit_matches_eager(api, orc):
    pr = synth.lasso_small(0)
    X, y = cuda(pr.X), cuda(pr.y)
    a = api.lasso_fit(X, y, pr.lambdas, pr.B1, pr.B2, 0, kkt_tol=1e-8, precision="mixed", relax=1.8,
                      eager=True, sel_beta=True)
    for rep in range(2):
        b = api.lasso_fit(X, y, pr.lambdas, pr.B1, pr.B2, 0, kkt_tol=1e-8, precision="mixed", relax=1.8,
                          sel_beta=True)
        for key in ("beta", "supports", "jstar", "iters", "kkt", "sel_beta", "losses"):
            assert torch.equal(a[key], b[key]), (rep, key)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_autotuner_candidates_give_identical_results(api, orc, precision, tmp_path, monkeypatch):
    """Every candidate launch shape the autotuner chooses among -- column-tile width
    FN = 1..4 of the ADMM products (all four are candidates at R = q pe = 192
    solves per Gram), each with one or two row blocks per wave (candidates 0..3
    and 4..7, float32 and float64 products alike), and 1..3 passes of the factor
    over the batch of 16 Grams -- gives exactly the default's results: each is
    forced through a tune file and compared.  Then the tuner times the
    candidates itself and records its choices."""
    n, p, nb, pe, q = 400, 130, 16, 16, 12
    rng = np.random.default_rng(7)
    X = rng.standard_normal((n, p))
    B = np.zeros((p, pe))
    for e in range(pe):
        B[rng.choice(p, 8, replace=False), e] = rng.uniform(-2, 2, 8)
    Y = X @ B + 0.5 * rng.standard_normal((n, pe))
    Gs, Cs = [], []
    for k in range(nb):
        G, Cm = orc.gram_multi(X, Y, orc.boot_rows(0, k, n))
        Gs.append(G)
        Cs.append(Cm)
    G, Cm = cuda(np.array(Gs)), cuda(np.array(Cs))
    lam = np.abs(X.T @ Y).max() / n * np.logspace(0, -2.5, q)
    path = tmp_path / "tune.txt"
    path.write_text("")
    monkeypatch.setenv("UOI_TUNE_FILE", str(path))
    kw = dict(kkt_tol=1e-9, precision=precision, relax=1.6)
    api.tune_reset()
    ref = api.lasso_solve_multi(G, Cm, lam, tune=False, **kw)   # defaults (empty file)
    assert ref["status"] == 0
    R = q * pe
    keys = [f"admm64_fn/nb{nb}/p{p}/R{R}", f"admm32_fn/nb{nb}/p{p}/R{R}", f"spd_passes/nb{nb}/p{p}"]
    for fn in range(8):
        for passes in range(3):
            path.write_text(f"{keys[0]} {fn}\n{keys[1]} {fn}\n{keys[2]} {passes}\n")
            api.tune_reset()
            got = api.lasso_solve_multi(G, Cm, lam, tune=False, **kw)
            for key in ("z", "iters", "kkt"):
                assert torch.equal(got[key], ref[key]), (fn, passes, key)
    path.write_text("")
    api.tune_reset()
    tuned = api.lasso_solve_multi(G, Cm, lam, **kw)
    for key in ("z", "iters", "kkt"):
        assert torch.equal(tuned[key], ref[key]), key
    rec = dict(line.split() for line in path.read_text().splitlines())
    assert 0 <= int(rec[keys[2]]) <= 2 and 0 <= int(rec[keys[0]]) <= 7
    if precision == "mixed":
        assert 0 <= int(rec[keys[1]]) <= 7
    monkeypatch.delenv("UOI_TUNE_FILE")
    api.tune_reset()
