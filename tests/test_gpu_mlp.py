"""Learned diagonal B_0 network on the GPU (features, forward, gradient, Adam) against
the float64 oracle evaluated on the same bfloat16-rounded weights."""
import numpy as np
import pytest
import torch

from oracle import mlp as omlp

pytestmark = pytest.mark.gpu


def params(seed):
    rng = np.random.default_rng(seed + 50)
    return omlp.init_params(seed) + 0.05 * rng.standard_normal(omlp.NPARAM)


def inputs(N, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((N, 8)).astype(np.float32)
    t = (np.log(1.0 / (np.exp(X[:, 0]) + 0.5)) + 0.1 * X[:, 3]).astype(np.float32)
    return X, t


def test_features_match_oracle():
    import paper_2009_12663_amd as P
    for nx, nz in [(37, 11), (1, 1), (5, 1), (300, 70)]:
        rng = np.random.default_rng(nx * 100 + nz)
        logD = rng.standard_normal(3 * nx * nz).astype(np.float32)
        gabs = np.abs(rng.standard_normal(3 * nx * nz)).astype(np.float32)
        X = P.Mlp.features(torch.from_numpy(logD), torch.from_numpy(gabs), nx, nz, 0.8).cpu().numpy()
        want = omlp.features(logD.astype(np.float64), gabs.astype(np.float64), nx, nz, 0.8)
        np.testing.assert_allclose(X, want, rtol=1e-7, atol=0)


@pytest.mark.parametrize("N", [1, 63, 5000, 70001])
def test_forward_matches_oracle(N):
    import paper_2009_12663_amd as P
    p = params(1).astype(np.float32)
    X, _ = inputs(N, N)
    net = P.Mlp(torch.from_numpy(p))
    out = net.forward(torch.from_numpy(X)).double().cpu().numpy()
    h0 = net.forward(torch.from_numpy(X), exp_out=True).double().cpu().numpy()
    want = omlp.forward(omlp.round_bf16(p), X.astype(np.float64))
    err = np.abs(out - want).max() / max(np.abs(want).max(), 1.0)
    herr = np.abs(h0 / np.exp(want) - 1).max()
    print(f"\n[mlp fwd] N={N} max err {err:.2e} h0 rel {herr:.2e}", flush=True)
    assert err <= 1e-5 and herr <= 1e-5
    net.close()


@pytest.mark.parametrize("N", [1, 777, 40000])
def test_gradient_matches_oracle(N):
    import paper_2009_12663_amd as P
    p = params(2).astype(np.float32)
    X, t = inputs(N, N + 1)
    net = P.Mlp(torch.from_numpy(p))
    g, loss = net.grad(torch.from_numpy(X), torch.from_numpy(t))
    g, loss = g.double().cpu().numpy(), float(loss.item())
    lw, gw = omlp.loss_and_grad(omlp.round_bf16(p), X.astype(np.float64), t.astype(np.float64))
    gerr = np.linalg.norm(g - gw) / np.linalg.norm(gw)
    print(f"\n[mlp grad] N={N} loss {loss:.6e} vs {lw:.6e}; grad rel_F {gerr:.2e}", flush=True)
    assert abs(loss - lw) <= 1e-5 * lw
    assert gerr <= 1e-5
    # deterministic: the fixed-order reduction gives the same bits twice
    g2, loss2 = net.grad(torch.from_numpy(X), torch.from_numpy(t))
    assert np.array_equal(g, g2.double().cpu().numpy()) and loss == float(loss2.item())
    net.close()


def test_adam_steps_match_oracle():
    """Three Adam steps on the float32 master weights; entries whose gradient is of the
    size of the gradient's own rounding error may legitimately take the other sign, so
    they are held only to a bound on the size of Adam's steps."""
    import paper_2009_12663_amd as P
    lr = 1e-3
    p = params(3).astype(np.float32)
    X, t = inputs(3000, 9)
    net = P.Mlp(torch.from_numpy(p))
    Xg, tg = torch.from_numpy(X).cuda(), torch.from_numpy(t).cuda()
    loss = torch.empty(1, device="cuda")
    opt = omlp.Adam(omlp.NPARAM, lr=lr)
    ref = p.astype(np.float64)
    for step in range(3):
        l_ref, g_ref = omlp.loss_and_grad(omlp.round_bf16(ref), X.astype(np.float64), t.astype(np.float64))
        ref = opt.step(ref, g_ref)
        net.train_step(Xg, tg, lr, loss)
        got = net.get_params().double().cpu().numpy()
        assert abs(float(loss.item()) - l_ref) <= 1e-4 * l_ref
        big = np.abs(g_ref) > 1e-2 * np.abs(g_ref).max()
        err = np.abs(got - ref)[big].max()
        print(f"\n[adam] step {step + 1}: max |dp| on {big.sum()} entries {err:.2e}", flush=True)
        assert err <= 1e-3 * lr * (step + 1) + 1e-6
        assert np.abs(got - ref).max() <= 8 * lr * (step + 1)
    net.close()


def test_training_reduces_loss():
    import paper_2009_12663_amd as P
    X, t = inputs(20000, 11)
    net = P.Mlp(torch.from_numpy(omlp.init_params(0).astype(np.float32)))
    Xg, tg = torch.from_numpy(X).cuda(), torch.from_numpy(t).cuda()
    loss = torch.empty(1, device="cuda")
    net.train_step(Xg, tg, 3e-3, loss)
    l0 = float(loss.item())
    for _ in range(300):
        net.train_step(Xg, tg, 3e-3, loss)
    l1 = float(loss.item())
    print(f"\n[mlp train] loss {l0:.4e} -> {l1:.4e}", flush=True)
    assert l1 < 0.05 * l0
    net.close()


def test_argument_errors():
    import paper_2009_12663_amd as P
    net = P.Mlp(torch.zeros(omlp.NPARAM))
    with pytest.raises(P.BfgsError):
        net.forward(torch.zeros((0, 8)))
    with pytest.raises(P.BfgsError):
        net.train_step(torch.zeros((4, 8), device="cuda"), torch.zeros(4, device="cuda"), -1.0,
                       torch.empty(1, device="cuda"))
    net.close()
