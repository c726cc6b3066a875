"""Warm-start network kernels against the FP64 oracle.

One layer isolates the convolution: the GPU rounds input and weights to
bfloat16 and accumulates in FP32, so the oracle fed the same rounded values
must agree to FP32 accumulation error.  The six-layer network also rounds
every hidden activation and every activation gradient to bfloat16 (relative
error 2^-9 each), so it is compared with the unrounded FP64 oracle at 2e-2.
"""
import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sg():
    assert torch.cuda.is_available()
    from paper_1601_08201_amd import sgtv
    sgtv.lib()
    return sgtv


def bf16(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(torch.bfloat16).to(torch.float64).numpy()


def rel(a, b):
    a, b = np.asarray(a, np.float64).ravel(), np.asarray(b, np.float64).ravel()
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def data(seed, B=2, H=8, C=64, scale=1.0):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0, scale, size=(B, H, 64, C)).astype(np.float32)
    t = rng.uniform(0, scale, size=(B, H, 64, C)).astype(np.float32)
    return x, t


def layer_params(sg, L, seed):
    return sg.init_params(L, 64, seed) + np.float32(0.01) * np.random.default_rng(seed + 1).normal(
        size=sg.wsnet_param_count(L, 64)).astype(np.float32)


def rounded_params(p, L):
    """weights rounded to bfloat16 as the GPU multiplies them; biases kept FP32."""
    q = p.astype(np.float64).copy()
    per = 64 * 9 * 64 + 64
    for l in range(L):
        q[l * per: l * per + 64 * 9 * 64] = bf16(p[l * per: l * per + 64 * 9 * 64])
    return q


def test_one_layer_forward_tight(sg):
    x, _ = data(1)
    p = layer_params(sg, 1, 3)
    N = sg.WarmStartNet(layers=1, height=8, max_batch=4).set_params(p)
    out = N.forward(x)
    ref = oracle.wn_forward(rounded_params(p, 1), bf16(x), L=1)
    err = rel(out, ref)
    print("one-layer forward rel L2", err, flush=True)
    assert err <= 1e-5


@pytest.mark.parametrize("H", [8, 6, 12])
def test_one_layer_gradient(sg, H):
    x, t = data(2, H=H)
    p = layer_params(sg, 1, 4)
    N = sg.WarmStartNet(layers=1, height=H, max_batch=4).set_params(p)
    g = np.empty(p.size, np.float32)
    loss = N.backward(x, t, g)
    loss_o, g_o = oracle.wn_loss_grad(rounded_params(p, 1), bf16(x), t, L=1)
    print("one-layer loss", loss, loss_o, "grad rel L2", rel(g, g_o), flush=True)
    assert loss == pytest.approx(loss_o, rel=1e-5)
    assert rel(g, g_o) <= 5e-3


def test_six_layer_network_against_fp64(sg):
    x, t = data(3, B=3, H=16)
    p = layer_params(sg, 6, 5)
    N = sg.WarmStartNet(layers=6, height=16, max_batch=4).set_params(p)
    out = N.forward(x)
    g = np.empty(p.size, np.float32)
    loss = N.backward(x, t, g)
    out_o = oracle.wn_forward(p, x, L=6)
    loss_o, g_o = oracle.wn_loss_grad(p, x, t, L=6)
    print("six-layer out rel", rel(out, out_o), "loss", loss, loss_o, "grad rel", rel(g, g_o), flush=True)
    assert rel(out, out_o) <= 2e-2
    assert loss == pytest.approx(loss_o, rel=2e-2)
    assert rel(g, g_o) <= 2e-2
    # per layer as well
    per = 64 * 9 * 64 + 64
    for l in range(6):
        assert rel(g[l * per:(l + 1) * per], g_o[l * per:(l + 1) * per]) <= 5e-2


def test_backward_is_deterministic(sg):
    x, t = data(4)
    p = layer_params(sg, 6, 6)
    N = sg.WarmStartNet(layers=6, height=8, max_batch=4).set_params(p)
    g1, g2 = np.empty(p.size, np.float32), np.empty(p.size, np.float32)
    l1 = N.backward(x, t, g1)
    l2 = N.backward(x, t, g2)
    assert l1 == l2
    np.testing.assert_array_equal(g1, g2)


def test_adam_first_step_follows_gradient_signs(sg):
    """After one step Adam moves every parameter by -lr * g / (|g| + eps'),
    i.e. about -lr sign(g); signs agree with the oracle's FP64 gradient
    wherever that gradient is not tiny."""
    x, t = data(5)
    p = layer_params(sg, 2, 7)
    N = sg.WarmStartNet(layers=2, height=8, max_batch=4).set_params(p)
    N.backward(x, t)
    lr = 1e-3
    N.adam_step(lr=lr)
    step = (N.params().astype(np.float64) - p) / lr
    _, g_o = oracle.wn_loss_grad(p, x, t, L=2)
    m = np.zeros_like(g_o)
    v = np.zeros_like(g_o)
    q = p.astype(np.float64).copy()
    oracle.wn_adam(q, g_o, m, v, 1, lr=lr)
    big = np.abs(g_o) > 1e-2 * np.abs(g_o).max()
    np.testing.assert_allclose(step[big], ((q - p) / lr)[big], atol=2e-3)


def test_adam_five_steps_against_fp64(sg):
    """Five Adam steps on the GPU's own gradients: after each step every
    parameter equals the FP64 oracle's Adam (Kingma and Ba) fed the same
    gradients, to FP32 rounding of the parameters and moments."""
    x, t = data(9)
    p = layer_params(sg, 2, 10)
    N = sg.WarmStartNet(layers=2, height=8, max_batch=4).set_params(p)
    q = p.astype(np.float64).copy()
    m = np.zeros_like(q)
    v = np.zeros_like(q)
    g = np.empty(p.size, np.float32)
    lrs = [1e-3, 2e-3, 5e-4, 1e-3, 3e-3]
    for step, lr in enumerate(lrs, start=1):
        N.backward(x, t, g)
        N.adam_step(lr=lr)
        oracle.wn_adam(q, g.astype(np.float64), m, v, step, lr=lr)
        got = N.params().astype(np.float64)
        err = np.abs(got - q)
        print("adam step", step, "max abs error", err.max(), "moved", np.abs(q - p).max(), flush=True)
        np.testing.assert_allclose(got, q, rtol=1e-6, atol=1e-8)
    # the parameters moved by many times the tolerance
    assert np.median(np.abs(q - p)) > 1e-4


def test_training_lowers_the_loss(sg):
    x, _ = data(6, B=4)
    t = np.sqrt(x).astype(np.float32)
    p = layer_params(sg, 6, 8)
    N = sg.WarmStartNet(layers=6, height=8, max_batch=4).set_params(p)
    first = N.backward(x, t)
    for _ in range(40):
        N.adam_step(lr=2e-3)
        last = N.backward(x, t)
    print("loss", first, "->", last, flush=True)
    assert last < 0.5 * first


def test_invalid_network_arguments(sg):
    with pytest.raises(sg.SgtvError):
        sg.WarmStartNet(channels=32)
    with pytest.raises(sg.SgtvError):
        sg.WarmStartNet(width=32)
    with pytest.raises(sg.SgtvError):
        sg.WarmStartNet(height=7)
    N = sg.WarmStartNet(layers=2, height=8, max_batch=2)
    x, t = data(7, B=3)
    with pytest.raises(sg.SgtvError):
        N.forward(x)              # no parameters yet
    N.set_params(layer_params(sg, 2, 1))
    with pytest.raises(sg.SgtvError):
        N.forward(x)              # batch above max_batch
    with pytest.raises(sg.SgtvError):
        N.adam_step()             # no gradient yet


@pytest.mark.parametrize("floor", [0.0, 0.3])
@pytest.mark.parametrize("mode", ["ratio", "direct"])
def test_start_images_against_fp64(sg, mode, floor):
    """wsnet_start: the network sees f / mean(f) and the start image is
    c_out * s * f (ratio) or c_out * s * mean(f) (direct), raised to at least
    floor * c_out * mean(f) when floor > 0."""
    rng = np.random.default_rng(11)
    f = rng.gamma(2.0, 1.5, size=(3, 8, 64, 64)).astype(np.float32)
    f[1] *= np.float32(40.0)
    f[2, :4] = 0.0
    p = layer_params(sg, 1, 5)
    N = sg.WarmStartNet(layers=1, height=8, max_batch=4).set_params(p)
    c_out = 1.75
    x0 = N.start(f, mode, c_out, floor=floor)
    m = f.reshape(3, -1).astype(np.float64).mean(axis=1)[:, None, None, None]
    xin = bf16((f.astype(np.float64) / m).astype(np.float32))
    s = oracle.wn_forward(rounded_params(p, 1), xin, L=1)
    ref = c_out * s * (f.astype(np.float64) if mode == "ratio" else m)
    if floor > 0:
        lo = floor * c_out * m * np.ones_like(ref)
        assert np.mean(ref < lo) > 0.01     # the floor acts on this input
        ref = np.maximum(ref, lo)
        assert np.all(x0 >= np.float32(0.999) * lo.astype(np.float32))
    err = rel(x0, ref)
    print("start", mode, "floor", floor, "rel L2", err, flush=True)
    assert err <= 1e-5
    assert np.all(x0 >= 0)
    # power-of-two scaling of an image is exact through the mean and the
    # network input, so the start image scales bit for bit
    x4 = N.start(np.float32(4.0) * f, mode, c_out, floor=floor)
    np.testing.assert_array_equal(x4, np.float32(4.0) * x0)


def test_start_image_of_zero_image(sg):
    p = layer_params(sg, 1, 6)
    N = sg.WarmStartNet(layers=1, height=8, max_batch=2).set_params(p)
    z = np.zeros((1, 8, 64, 64), np.float32)
    assert np.all(N.start(z, "ratio", 2.0) == 0.0)
    s = N.forward(z)
    np.testing.assert_allclose(N.start(z, "direct", 2.0), 2.0 * s, rtol=1e-6)


def test_start_rejects_bad_arguments(sg):
    p = layer_params(sg, 1, 7)
    N = sg.WarmStartNet(layers=1, height=8, max_batch=2).set_params(p)
    f = np.ones((1, 8, 64, 64), np.float32)
    with pytest.raises(sg.SgtvError):
        sg.wsnet_start(N._n, f, 1, 7, 1.0, np.empty_like(f))
    with pytest.raises(sg.SgtvError):
        N.start(f, "ratio", 0.0)
    with pytest.raises(sg.SgtvError):
        N.start(f, "direct", 1.0, floor=-0.1)
    with pytest.raises(sg.SgtvError):
        N.start(f, "direct", 1.0, floor=float("inf"))
    with pytest.raises(sg.SgtvError):
        N.start(f, "ratio", float("nan"))
    with pytest.raises(sg.SgtvError):
        N.start(np.ones((3, 8, 64, 64), np.float32), "ratio", 1.0)


def test_save_and_load_round_trip(sg, tmp_path):
    p = layer_params(sg, 2, 9)
    N = sg.WarmStartNet(layers=2, height=8, max_batch=2).set_params(p)
    path = tmp_path / "net.bin"
    N.save(path)
    assert path.stat().st_size == 24 + 4 * p.size
    M = sg.WarmStartNet(layers=2, height=8, max_batch=2)
    M.load(path)
    np.testing.assert_array_equal(M.params(), p)
    x, _ = data(12, B=2)
    np.testing.assert_array_equal(M.forward(x), N.forward(x))
    with pytest.raises(sg.SgtvError):
        sg.WarmStartNet(layers=3, height=8, max_batch=2).load(path)     # other shape
    bad = tmp_path / "bad.bin"
    bad.write_bytes(b"not a network")
    with pytest.raises(sg.SgtvError):
        M.load(bad)


def test_train_step_equals_backward_and_adam(sg):
    """wsnet_train_step (no wait for the device, the loss summed on it) leaves
    parameters bit for bit where backward + adam_step leave them, and its loss
    sum equals the sum of the losses backward returns, in the same order."""
    import torch
    p = layer_params(sg, 2, 11)
    A = sg.WarmStartNet(layers=2, height=8, max_batch=4).set_params(p)
    B = sg.WarmStartNet(layers=2, height=8, max_batch=4).set_params(p)
    losses = []
    for k in range(6):
        x, t = data(20 + k, B=3 if k % 2 else 4, H=8)
        lr = 1e-3 * (1.0 - 0.1 * k)
        losses.append(A.backward(x, t))
        A.adam_step(lr=lr)
        xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
        B.train_step(xd, td, lr=lr)
    s, n = B.loss_sum(reset=True)
    assert n == 6
    tot = 0.0
    for l in losses:
        tot += l
    assert s == tot
    np.testing.assert_array_equal(B.params(), A.params())
    assert B.loss_sum() == (0.0, 0)
    with pytest.raises(RuntimeError):
        B.train_step(xd, td, lr=-1.0)
    A.close()
    B.close()
