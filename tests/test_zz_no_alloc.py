"""The allocation-free entry point (uoi_lasso_solve_batch_noalloc) against
uoi_lasso_solve_batch: the same kernels on the same inputs, so every output must
be identical, on two calls in a row (the second smaller, so it runs on what the
first left in the shared static scratch)."""
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


def _problem(orc, n, p, nb, q, seed):
    pr = synth.lasso_random(n, p, max(2, p // 8), seed, q=q)
    Gs, cs = [], []
    for k in range(nb):
        G, c = orc.gram(pr.X, pr.y, orc.boot_rows(seed, k, n))
        Gs.append(G)
        cs.append(c)
    return (torch.as_tensor(np.array(Gs), device="cuda"), torch.as_tensor(np.array(cs), device="cuda"),
            pr.lambdas)


@pytest.mark.parametrize("precision,relax", [("fp64", 1.0), ("mixed", 1.6)])
def test_no_alloc_matches_allocating_entry_point(api, orc, precision, relax):
    kw = dict(kkt_tol=1e-9, precision=precision, relax=relax, max_iter=20000)
    for n, p, nb, q, seed in ((400, 130, 3, 9, 1), (200, 50, 2, 6, 2)):   # second call smaller
        G, c, lam = _problem(orc, n, p, nb, q, seed)
        print(f"no-alloc {precision} nb={nb} p={p} q={q}", flush=True)
        ref = api.lasso_solve_batch(G, c, lam, **kw)
        got = api.lasso_solve_batch(G, c, lam, no_alloc=True, **kw)
        assert ref["status"] == 0 and got["status"] == 0
        for key in ("z", "u", "iters", "kkt"):
            assert torch.equal(got[key], ref[key]), key
        z = got["z"].cpu().numpy()
        Gn, cn = G.cpu().numpy(), c.cpu().numpy()
        for k in range(nb):
            for j in range(q):
                assert orc.kkt(Gn[k], cn[k], lam[j], z[k, j]) <= 1e-8


def test_no_alloc_warm_start_and_reuse(api, orc):
    """A warm start (z0 given) through the static scratch, after a cold call."""
    G, c, lam = _problem(orc, 300, 70, 2, 5, 4)
    cold = api.lasso_solve_batch(G, c, lam, kkt_tol=1e-10, no_alloc=True)
    z0 = cold["z"].clone()
    ref = api.lasso_solve_batch(G, c, lam, kkt_tol=1e-10, z0=z0)
    got = api.lasso_solve_batch(G, c, lam, kkt_tol=1e-10, z0=z0, no_alloc=True)
    for key in ("z", "u", "iters", "kkt"):
        assert torch.equal(got[key], ref[key]), key


def test_no_alloc_rejects_oversize(api):
    """A problem whose scratch exceeds the static array fails with UOI_EINVAL and
    a message naming the sizes, before any device work."""
    nb, p = 40, 1000  # M alone needs 320 MB
    G = torch.zeros((nb, p, p), dtype=torch.float64, device="cuda")
    c = torch.zeros((nb, p), dtype=torch.float64, device="cuda")
    with pytest.raises(api.UoiError) as ei:
        api.lasso_solve_batch(G, c, [1.0, 0.5], no_alloc=True)
    assert ei.value.code == api.UOI_EINVAL
    assert "static buffer" in str(ei.value)
