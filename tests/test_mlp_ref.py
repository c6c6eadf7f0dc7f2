"""Pins of the fp64 MLP reference: finite differences, an independent
automatic-differentiation library (torch, CPU, float64) and closed forms."""
import numpy as np
import pytest

from oracle import mlp_ref as R


def setup(seed=0, B=37):
    rng = np.random.default_rng(seed)
    p = rng.normal(0, 0.3, R.NPARAM)
    X = rng.normal(2.0, 3.0, (B, R.IN))
    T = rng.normal(-1.0, 2.0, (B, R.OUT))
    norm = np.concatenate([X.mean(0), X.std(0), T.mean(0), T.std(0)])
    return p, norm, X, T


def test_layout_size():
    assert R.NPARAM == 16 * 64 + 64 + 64 * 64 + 64 + 2 * 64 + 2 == 5378
    assert R.NNORM == 36


def test_gradient_finite_differences():
    p, norm, X, T = setup()
    loss, g = R.loss_and_grad(p, norm, X, T)
    rng = np.random.default_rng(1)
    idx = rng.choice(R.NPARAM, 60, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros(R.NPARAM)
        e[i] = h
        fd = (R.loss_and_grad(p + e, norm, X, T)[0] - R.loss_and_grad(p - e, norm, X, T)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 + 1e-5 * abs(fd), (i, fd, g[i])


def test_gradient_matches_autograd():
    torch = pytest.importorskip("torch")
    p, norm, X, T = setup(2)
    loss, g = R.loss_and_grad(p, norm, X, T)
    pt = torch.tensor(p, dtype=torch.float64, requires_grad=True)
    w, o = {}, 0
    for name, shape in R.SIZES:
        n = int(np.prod(shape))
        w[name] = pt[o:o + n].reshape(shape)
        o += n
    mx, sx, my, sy = [torch.tensor(a) for a in R.split_norm(norm)]
    xn = (torch.tensor(X) - mx) / sx
    h1 = torch.relu(torch.nn.functional.linear(xn, w["W1"], w["b1"]))
    h2 = torch.relu(torch.nn.functional.linear(h1, w["W2"], w["b2"]))
    y = torch.nn.functional.linear(h2, w["W3"], w["b3"])
    lt = torch.nn.functional.mse_loss(y, (torch.tensor(T) - my) / sy)
    lt.backward()
    assert abs(lt.item() - loss) < 1e-12
    np.testing.assert_allclose(pt.grad.numpy(), g, rtol=1e-10, atol=1e-12)
    yref, _ = R.forward(p, norm, X)
    np.testing.assert_allclose(yref, y.detach().numpy() * sy.numpy() + my.numpy(), rtol=1e-12)


def test_zero_output_layer_closed_form():
    # W3 = 0, b3 = c: output is c everywhere; dL/db3 = 2 mean(c - tn), dL/dW1 = 0
    p, norm, X, T = setup(3)
    w = R.unpack(p)
    w["W3"][:] = 0.0
    w["b3"][:] = [0.5, -0.25]
    q = R.pack(w)
    mx, sx, my, sy = R.split_norm(norm)
    yref, _ = R.forward(q, norm, X)
    np.testing.assert_allclose(yref, np.tile(np.array([0.5, -0.25]) * sy + my, (len(X), 1)))
    loss, g = R.loss_and_grad(q, norm, X, T)
    tn = (T - my) / sy
    gb3 = 2 * (np.array([0.5, -0.25]) - tn).mean(0) / R.OUT
    np.testing.assert_allclose(R.unpack(g)["b3"], gb3, rtol=1e-12)
    assert np.all(R.unpack(g)["W1"] == 0) and np.all(R.unpack(g)["W2"] == 0)


def test_adam_first_step_is_signed_lr():
    # with bias correction the first Adam step moves each parameter by
    # -lr * g / (|g| + eps)
    rng = np.random.default_rng(4)
    p = rng.normal(size=10)
    g = rng.normal(size=10)
    q, m, v = R.adam_step(p, g, np.zeros(10), np.zeros(10), 1, 0.01, eps=1e-8)
    np.testing.assert_allclose(q, p - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_training_reduces_loss():
    p, norm, X, T = setup(5, B=64)
    m = np.zeros(R.NPARAM)
    v = np.zeros(R.NPARAM)
    l0 = R.loss_and_grad(p, norm, X, T)[0]
    for s in range(1, 201):
        _, g = R.loss_and_grad(p, norm, X, T)
        p, m, v = R.adam_step(p, g, m, v, s, 1e-3)
    assert R.loss_and_grad(p, norm, X, T)[0] < 0.5 * l0
