"""Pins of the oracle's control-variate network: gradients by finite differences,
Adam against its textbook first step, and a fit that actually learns."""
import numpy as np
import pytest

from oracle import mlp
from paper_2301_05780_amd import workloads


def _data(n=64, seed=0):
    rng = np.random.default_rng(seed)
    X = rng.uniform(0, 1, size=(n, 2))
    T = np.sin(3 * X[:, 0]) + X[:, 1] ** 2
    return X, T


def test_param_count_and_layout():
    theta = workloads.mlp_init(0)
    assert theta.size == mlp.N_PARAMS == workloads.MLP_PARAMS == 4417
    W1, b1, W2, b2, w3, b3 = mlp.unpack(theta)
    assert W1.shape == (64, 2) and W2.shape == (64, 64) and w3.shape == (64,)
    assert np.array_equal(mlp.pack(W1, b1, W2, b2, w3, b3), theta)


def test_loss_gradient_finite_differences():
    rng = np.random.default_rng(1)
    theta = workloads.mlp_init(3) + rng.normal(0, 0.05, mlp.N_PARAMS)
    X, T = _data()
    _, g = mlp.loss_and_grad(theta, X, T)
    idx = rng.choice(mlp.N_PARAMS, 200, replace=False)
    idx = np.concatenate([idx, [0, 1, 128, 192, 4288, 4416]])
    e = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += e
        tm[i] -= e
        fd = (mlp.loss_and_grad(tp, X, T)[0] - mlp.loss_and_grad(tm, X, T)[0]) / (2 * e)
        assert g[i] == pytest.approx(fd, rel=1e-6, abs=1e-10)


def test_input_gradient_finite_differences():
    theta = workloads.mlp_init(4)
    X, _ = _data(32, 2)
    gx = mlp.grad_input(theta, X)
    e = 1e-6
    for d in range(2):
        Xp, Xm = X.copy(), X.copy()
        Xp[:, d] += e
        Xm[:, d] -= e
        fd = (mlp.forward(theta, Xp)[0] - mlp.forward(theta, Xm)[0]) / (2 * e)
        assert np.allclose(gx[:, d], fd, rtol=1e-6, atol=1e-10)


def test_adam_first_step():
    """Bias correction makes the first step lr * g / (|g| + eps) per coordinate."""
    theta = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    new, m, s = mlp.adam_step(theta, g, np.zeros(3), np.zeros(3), 1, 0.01)
    assert np.allclose(new, theta - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    assert np.allclose(m, 0.1 * g) and np.allclose(s, 0.001 * g * g)


def test_training_reduces_loss():
    X, T = _data(512, 3)
    theta0 = workloads.mlp_init(0)
    order = workloads.minibatch_order(512, 40, seed=1)
    theta, losses = mlp.train(theta0, X, T, order, batch=64, lr=3e-3)
    assert losses[-20:].mean() < 0.05 * losses[:5].mean()


def test_grad_table_reproduces_bilinear_fields():
    """Bilinear interpolation is exact for fields a + b x + c y + d x y, so a
    table sampled from such a field returns it exactly at any point."""
    n = 17
    dom = (-0.5, 1.5, 0.25, 2.25)
    xs = dom[0] + np.arange(n) * (dom[1] - dom[0]) / (n - 1)
    ys = dom[2] + np.arange(n) * (dom[3] - dom[2]) / (n - 1)
    X, Y = np.meshgrid(xs, ys)
    f0 = lambda x, y: 0.5 + 2.0 * x - 1.0 * y + 0.25 * x * y
    f1 = lambda x, y: -1.0 + 0.5 * x * y
    tab = np.stack([f0(X, Y), f1(X, Y)], axis=-1).astype(np.float32)
    cv = mlp.GradLutCV(tab, dom)
    rng = np.random.default_rng(3)
    x, y = rng.uniform(dom[0], dom[1], 500), rng.uniform(dom[2], dom[3], 500)
    gx, gy = cv.grad(x, y)
    # the float32 table rounds the node values: compare at float32 resolution
    assert np.allclose(gx, f0(x, y), atol=1e-6) and np.allclose(gy, f1(x, y), atol=1e-6)
    # outside the domain the position is clamped to the boundary
    gx2, _ = cv.grad(np.array([dom[1] + 1.0]), np.array([dom[2]]))
    assert np.isclose(gx2[0], f0(dom[1], dom[2]), atol=1e-6)


def test_network_cv_on_a_non_unit_domain():
    """The control variate's network sees the domain's unit coordinates:
    NetworkCV.grad equals finite differences, in the domain's coordinates,
    of v at the mapped point; on the unit square the map is the identity."""
    from oracle.mlp import NetworkCV, forward
    rng = np.random.default_rng(8)
    theta = rng.normal(0.0, 0.3, 4417)
    dom = (-100.0, 100.0, -60.0, 40.0)
    cvn = NetworkCV(theta, dom)
    x, y = rng.uniform(-90, 90, 20), rng.uniform(-50, 30, 20)
    v = lambda a, b: forward(theta, np.stack([(a - dom[0]) / 200.0, (b - dom[2]) / 100.0], axis=1))[0]
    e = 1e-3
    gx, gy = cvn.grad(x, y)
    assert np.allclose(gx, (v(x + e, y) - v(x - e, y)) / (2 * e), rtol=1e-5, atol=1e-9)
    assert np.allclose(gy, (v(x, y + e) - v(x, y - e)) / (2 * e), rtol=1e-5, atol=1e-9)
    u = rng.uniform(0, 1, (20, 2))
    a = NetworkCV(theta).grad(u[:, 0], u[:, 1])
    b = NetworkCV(theta, (0.0, 1.0, 0.0, 1.0)).grad(u[:, 0], u[:, 1])
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
