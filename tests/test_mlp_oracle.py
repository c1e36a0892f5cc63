"""Pins for the FP64 MLP oracle: forward against torch.nn layers, backprop
against central finite differences and torch autograd, Adam against
torch.optim.Adam (all CPU, float64)."""
import numpy as np
import pytest
import torch

from oracle import mlp as M


def _params(seed, scale=0.5):
    rng = np.random.default_rng(seed)
    p = rng.normal(0, scale, M.BLOB)
    p[4545:4549] = rng.normal(1.0, 0.3, 4)       # means
    p[4549:4553] = rng.uniform(0.5, 2.0, 4)      # stds
    return p


def _feats(seed, n):
    rng = np.random.default_rng(seed)
    return rng.integers(0, 5000, size=(n, 4)).astype(np.int64)


def _torch_net(p):
    d = M.unpack(p)
    l1 = torch.nn.Linear(4, 64).double()
    l2 = torch.nn.Linear(64, 64).double()
    l3 = torch.nn.Linear(64, 1).double()
    with torch.no_grad():
        l1.weight.copy_(torch.from_numpy(d["W1"]))
        l1.bias.copy_(torch.from_numpy(d["b1"]))
        l2.weight.copy_(torch.from_numpy(d["W2"]))
        l2.bias.copy_(torch.from_numpy(d["b2"]))
        l3.weight.copy_(torch.from_numpy(d["w3"][None, :]))
        l3.bias.copy_(torch.tensor([d["b3"]], dtype=torch.float64))
    return torch.nn.Sequential(l1, torch.nn.ReLU(), l2, torch.nn.ReLU(), l3), (l1, l2, l3)


@pytest.mark.parametrize("seed", range(3))
def test_forward_matches_torch_layers(seed):
    p = _params(seed)
    F = _feats(seed, 200)
    y, _ = M.forward(p, F)
    net, _ = _torch_net(p)
    X = torch.from_numpy(M.inputs(p, F))
    ref = net(X).detach().numpy()[:, 0]
    assert np.allclose(y, ref, rtol=1e-12, atol=1e-12)
    # the normaliser is (log1p(f) - mean) / std
    d = M.unpack(p)
    assert np.allclose(M.inputs(p, F), (np.log1p(F) - d["mean"]) / d["std"])


@pytest.mark.parametrize("seed", range(3))
def test_gradient_matches_autograd(seed):
    p = _params(10 + seed)
    F = _feats(seed, 300)
    T = np.random.default_rng(seed).normal(2.0, 1.0, 300)
    loss, g, _ = M.loss_grad(p, F, T)
    net, (l1, l2, l3) = _torch_net(p)
    X = torch.from_numpy(M.inputs(p, F))
    out = net(X)[:, 0]
    L = torch.mean((out - torch.from_numpy(T)) ** 2)
    L.backward()
    ref = np.concatenate([l1.weight.grad.numpy().ravel(), l1.bias.grad.numpy(), l2.weight.grad.numpy().ravel(),
                          l2.bias.grad.numpy(), l3.weight.grad.numpy().ravel(), l3.bias.grad.numpy()])
    assert abs(loss - float(L)) < 1e-12
    assert np.allclose(g, ref, rtol=1e-10, atol=1e-12)


def test_gradient_matches_finite_differences():
    """Central differences (h = 1e-5) on inputs with no pre-activation near 0."""
    rng = np.random.default_rng(5)
    p = _params(5)
    F = _feats(5, 40)
    T = rng.normal(0, 1, 40)
    _, (X, Z1, H1, Z2, H2) = M.forward(p, F)
    keep = (np.abs(Z1).min(1) > 1e-3) & (np.abs(Z2).min(1) > 1e-3)
    F, T = F[keep], T[keep]
    assert len(T) >= 10
    _, g, _ = M.loss_grad(p, F, T)
    idx = np.concatenate([rng.choice(256, 20, replace=False), 256 + rng.choice(64, 10, replace=False),
                          320 + rng.choice(4096, 40, replace=False), 4416 + rng.choice(64, 10, replace=False),
                          4480 + rng.choice(64, 10, replace=False), [4544]])
    h = 1e-5
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (M.loss_grad(pp, F, T)[0] - M.loss_grad(pm, F, T)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), i


def test_adam_matches_torch_optim():
    rng = np.random.default_rng(3)
    p = _params(3)
    w = torch.nn.Parameter(torch.from_numpy(p[:M.NET].copy()))
    opt = torch.optim.Adam([w], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    m = np.zeros(M.NET)
    v = np.zeros(M.NET)
    cur = p.copy()
    for t in range(1, 6):
        g = rng.normal(0, 1, M.NET)
        w.grad = torch.from_numpy(g.copy())
        opt.step()
        cur, m, v = M.adam(cur, g, m, v, t, 1e-3)
    assert np.allclose(cur[:M.NET], w.detach().numpy(), rtol=1e-12, atol=1e-14)
    assert np.array_equal(cur[M.NET:], p[M.NET:])  # the normaliser is not trained
