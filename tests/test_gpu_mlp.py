"""Warm-start network on the GPU: forward and gradients against the FP64 oracle
(which rounds the same GEMM operands to bfloat16), training, and the gain of
the trained network over the cold start."""
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


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("n_in,hid,n_out,n", [(37, 40, 21, 67), (201, 64, 200, 130)])
def test_forward_and_gradients_match_oracle(api, n_in, hid, n_out, n):
    from oracle import mlp as omlp
    rng = np.random.default_rng(n)
    ps = omlp.init_params(n_in, hid, n_out, seed=3)
    ps[1] += 0.05; ps[3] += 0.05; ps[5] += 0.1
    theta = omlp.flat(ps).astype(np.float32)
    X = rng.standard_normal((n, n_in)).astype(np.float32)
    T = rng.standard_normal((n, n_out)).astype(np.float32)
    net = api.MLP(n_in, hid, n_out)
    assert net.nparam == theta.size
    net.set_params(torch.as_tensor(theta, device="cuda"))
    Y = net.forward(torch.as_tensor(X, device="cuda")).cpu().numpy()
    ps64 = omlp.unflat(theta.astype(np.float64), n_in, hid, n_out)
    yo, _ = omlp.forward(ps64, X.astype(np.float64), bf16=True)
    assert _rel(Y, yo) <= 1e-2
    loss, g = net.loss_grad(torch.as_tensor(X, device="cuda"), torch.as_tensor(T, device="cuda"))
    lo, go = omlp.loss_and_grads(ps64, X.astype(np.float64), T.astype(np.float64), bf16=True)
    assert abs(loss - lo) <= 1e-3 * lo
    gg = omlp.unflat(g.cpu().numpy().astype(np.float64), n_in, hid, n_out)
    for a, b in zip(gg, go):
        assert _rel(a, b) <= 3e-2
    # round trip of the parameters
    assert np.array_equal(net.get_params().cpu().numpy(), theta)


def test_training_reduces_loss(api):
    rng = np.random.default_rng(0)
    n_in, hid, n_out, n = 16, 64, 8, 256
    W = rng.standard_normal((n_in, n_out)) / 4
    X = rng.standard_normal((n, n_in)).astype(np.float32)
    T = np.maximum(X @ W, 0).astype(np.float32)
    from oracle import mlp as omlp
    net = api.MLP(n_in, hid, n_out)
    net.set_params(torch.as_tensor(omlp.flat(omlp.init_params(n_in, hid, n_out, 1)).astype(np.float32),
                                   device="cuda"))
    Xd, Td = torch.as_tensor(X, device="cuda"), torch.as_tensor(T, device="cuda")
    l0 = net.loss_grad(Xd, Td)[0]
    for _ in range(150):
        l = net.train_step(Xd, Td, 3e-3)
    assert l < 0.1 * l0


def test_warm_start_gains_over_cold_start(api):
    """Network trained on solves of the workload distribution (p = 200 for test
    time), evaluated on held-out designs with exact iteration counts (a KKT
    check after every iteration): the warm-started fits reach the same
    solutions, most solves start from the network, and they need strictly fewer
    ADMM iterations than from the cold start.  Measured: 1.6 - 2.1 of about 87
    iterations saved per solve (2 %), 58 - 63 % of the solves faster, 17 %
    slower.  (At p = 1000, the benchmark's size, the held-out starts are
    rejected by the objective gate and the gain is zero; the benchmark reports
    that variant separately.)"""
    from oracle import mlp as omlp
    from paper_1808_06992_amd import warmstart as ws
    kw = dict(n=1000, p=200, k=20, q=16)
    X, T = ws.make_training_set(range(1000, 1060), B1=4, M=64, **kw)
    p = 200
    net = api.MLP(p + 1, 512, p)
    net.set_params(torch.as_tensor(omlp.flat(omlp.init_params(p + 1, 512, p, 7)).astype(np.float32),
                                   device="cuda"))
    hist = ws.train(net, X, T, epochs=30, batch=512, lr=2e-3)
    print("training loss by epoch:", [f"{h:.3e}" for h in hist])
    assert hist[-1] < 0.5 * hist[0]
    rows = ws.evaluate(net, [2000, 2001], B1=16, B2=8, kkt_tol=1e-8, precision="fp64", check_every=1, **kw)
    print("warm-start rows:", rows)
    for r in rows:
        assert r["unconverged_mlp"] == 0
        assert r["max_rel_diff"] <= 1e-5          # the same LASSO solutions
        assert r["warm_used"] > r["solves"] // 2  # most solves start from the network
        assert r["save_mean"] >= 1.0              # at least one ADMM iteration saved per solve
        assert r["frac_saved"] > 2 * r["frac_worse"]
