"""Pins of the warm-start network oracle against torch CPU float64 (a library
used only here), central finite differences and torch's Adam."""
import numpy as np
import pytest
import torch

import oracle

torch.set_default_dtype(torch.float64)


def to_nchw(x):
    return torch.from_numpy(np.ascontiguousarray(np.transpose(x, (0, 3, 1, 2))))


def w_to_torch(w):       # [co, ky, kx, ci] -> [co, ci, ky, kx]
    return torch.from_numpy(np.ascontiguousarray(np.transpose(w, (0, 3, 1, 2))))


@pytest.fixture
def rng():
    return np.random.default_rng(7)


@pytest.mark.parametrize("shape", [(2, 5, 6, 3, 4), (1, 1, 1, 2, 2), (3, 4, 3, 5, 2)])
def test_conv_forward_matches_torch(rng, shape):
    B, H, W, Ci, Co = shape
    x = rng.normal(size=(B, H, W, Ci))
    w = rng.normal(size=(Co, 3, 3, Ci))
    b = rng.normal(size=Co)
    z = oracle.wn_conv_fwd(x, w, b)
    ref = torch.nn.functional.conv2d(to_nchw(x), w_to_torch(w), torch.from_numpy(b), padding=1)
    np.testing.assert_allclose(z, ref.permute(0, 2, 3, 1).numpy(), rtol=1e-12, atol=1e-12)


def test_conv_backward_matches_autograd(rng):
    B, H, W, Ci, Co = 2, 5, 4, 3, 4
    x = rng.normal(size=(B, H, W, Ci))
    w = rng.normal(size=(Co, 3, 3, Ci))
    dz = rng.normal(size=(B, H, W, Co))
    xt = to_nchw(x).requires_grad_(True)
    wt = w_to_torch(w).requires_grad_(True)
    bt = torch.zeros(Co, requires_grad=True)
    out = torch.nn.functional.conv2d(xt, wt, bt, padding=1)
    out.backward(to_nchw(dz))
    dx = oracle.wn_conv_bwd_data(dz, w, Ci)
    dw, db = oracle.wn_conv_bwd_weight(x, dz)
    np.testing.assert_allclose(dx, xt.grad.permute(0, 2, 3, 1).numpy(), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(dw, wt.grad.permute(0, 2, 3, 1).numpy(), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(db, bt.grad.numpy(), rtol=1e-12, atol=1e-12)


def torch_net(params, x, L, C):
    h = to_nchw(x)
    off = 0
    for l in range(L):
        w = params[off:off + C * 9 * C].reshape(C, 3, 3, C).permute(0, 3, 1, 2)
        b = params[off + C * 9 * C: off + C * 9 * C + C]
        off += C * 9 * C + C
        h = torch.nn.functional.conv2d(h, w, b, padding=1)
        h = torch.relu(h) if l + 1 < L else torch.nn.functional.softplus(h)
    return h.permute(0, 2, 3, 1)


@pytest.mark.parametrize("L,C", [(6, 4), (2, 3)])
def test_network_loss_and_gradient_match_autograd(rng, L, C):
    B, H, W = 2, 5, 6
    n = oracle.wn_n_params(C, L)
    params = rng.normal(scale=0.4, size=n)
    x = rng.uniform(0, 2, size=(B, H, W, C))
    t = rng.uniform(0, 2, size=(B, H, W, C))
    out = oracle.wn_forward(params, x, L)
    loss, g = oracle.wn_loss_grad(params, x, t, L)
    pt = torch.from_numpy(params).requires_grad_(True)
    o = torch_net(pt, x, L, C)
    lt = torch.mean((o - torch.from_numpy(t)) ** 2)
    lt.backward()
    np.testing.assert_allclose(out, o.detach().numpy(), rtol=1e-12, atol=1e-13)
    assert loss == pytest.approx(lt.item(), rel=1e-12)
    np.testing.assert_allclose(g, pt.grad.numpy(), rtol=1e-9, atol=1e-13)
    assert np.all(out > 0)


def test_network_gradient_by_finite_differences(rng):
    L, C, B, H, W = 3, 2, 1, 4, 4
    n = oracle.wn_n_params(C, L)
    params = rng.normal(scale=0.5, size=n)
    x = rng.uniform(0, 2, size=(B, H, W, C))
    t = rng.uniform(0, 2, size=(B, H, W, C))
    _, g = oracle.wn_loss_grad(params, x, t, L)
    h = 1e-6
    for k in rng.choice(n, size=15, replace=False):
        e = np.zeros(n)
        e[k] = h
        fd = (oracle.wn_loss_grad(params + e, x, t, L)[0] - oracle.wn_loss_grad(params - e, x, t, L)[0]) / (2 * h)
        assert fd == pytest.approx(g[k], rel=1e-6, abs=1e-9)


def test_adam_matches_torch(rng):
    n = 50
    p = rng.normal(size=n)
    m = np.zeros(n)
    v = np.zeros(n)
    pt = torch.from_numpy(p.copy()).requires_grad_(True)
    opt = torch.optim.Adam([pt], lr=3e-3, betas=(0.9, 0.999), eps=1e-8)
    for t in range(1, 6):
        g = rng.normal(size=n)
        oracle.wn_adam(p, g, m, v, t, lr=3e-3)
        opt.zero_grad()
        pt.grad = torch.from_numpy(g.copy())
        opt.step()
        np.testing.assert_allclose(p, pt.detach().numpy(), rtol=1e-12, atol=1e-14)
