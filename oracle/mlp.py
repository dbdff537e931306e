"""The learned control variate network v: R^2 -> R, in float64.

The paper's variance reduction (Sec. 2.3, eq. 11; Sec. 4.2, eqs. 37-38) uses
F = sigma^T grad u0 with u0 a coarse approximation of the solution: any F
keeps the mean, and F = sigma^T grad u (with the sign convention of eq. 37)
removes the variance.  Here u0 is a small network

    v(x) = w3 . tanh(W2 tanh(W1 x + b1) + b2) + b3,   widths 2 -> 64 -> 64 -> 1

fitted by least squares to pathwise estimates of u that the method itself
produces.  This module holds the network's forward pass, its input gradient
grad v (what the path integral of eq. 37 needs), the gradient of the
mean-squared loss with respect to all parameters (reverse mode written out by
hand) and the Adam update (Kingma and Ba, 2015), all in float64.

Parameter vector layout (P = 4417 entries):
  W1[64, 2] row-major, b1[64], W2[64, 64] row-major (out, in), b2[64], w3[64], b3[1]
"""
import numpy as np

WIDTH = 64
N_PARAMS = WIDTH * 2 + WIDTH + WIDTH * WIDTH + WIDTH + WIDTH + 1


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    assert theta.size == N_PARAMS
    o = 0
    W1 = theta[o:o + 2 * WIDTH].reshape(WIDTH, 2); o += 2 * WIDTH
    b1 = theta[o:o + WIDTH]; o += WIDTH
    W2 = theta[o:o + WIDTH * WIDTH].reshape(WIDTH, WIDTH); o += WIDTH * WIDTH
    b2 = theta[o:o + WIDTH]; o += WIDTH
    w3 = theta[o:o + WIDTH]; o += WIDTH
    b3 = theta[o]
    return W1, b1, W2, b2, w3, b3


def pack(W1, b1, W2, b2, w3, b3):
    return np.concatenate([np.ravel(W1), b1, np.ravel(W2), b2, w3, [b3]]).astype(np.float64)


def forward(theta, X):
    """v at the rows of X (B x 2); returns (v, cache)."""
    W1, b1, W2, b2, w3, b3 = unpack(theta)
    X = np.asarray(X, dtype=np.float64)
    h1 = np.tanh(X @ W1.T + b1)
    h2 = np.tanh(h1 @ W2.T + b2)
    v = h2 @ w3 + b3
    return v, (X, h1, h2)


def grad_input(theta, X):
    """grad_x v at the rows of X: W1^T [(1 - h1^2) * (W2^T [(1 - h2^2) * w3])]."""
    W1, b1, W2, b2, w3, b3 = unpack(theta)
    _, (X, h1, h2) = forward(theta, X)
    g2 = (1.0 - h2 * h2) * w3
    g1 = (1.0 - h1 * h1) * (g2 @ W2)
    return g1 @ W1


def loss_and_grad(theta, X, T):
    """Loss L = mean_i (v(x_i) - t_i)^2 / 2 and dL/dtheta (reverse mode by hand)."""
    W1, b1, W2, b2, w3, b3 = unpack(theta)
    v, (X, h1, h2) = forward(theta, X)
    B = X.shape[0]
    r = v - np.asarray(T, dtype=np.float64)
    loss = 0.5 * np.mean(r * r)
    dv = r / B
    gw3 = h2.T @ dv
    gb3 = dv.sum()
    dz2 = np.outer(dv, w3) * (1.0 - h2 * h2)
    gW2 = dz2.T @ h1
    gb2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2) * (1.0 - h1 * h1)
    gW1 = dz1.T @ X
    gb1 = dz1.sum(axis=0)
    return loss, pack(gW1, gb1, gW2, gb2, gw3, gb3)


def adam_step(theta, grad, m, s, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (bias-corrected); returns new (theta, m, s).  step counts from 1."""
    m = beta1 * m + (1.0 - beta1) * grad
    s = beta2 * s + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** step)
    shat = s / (1.0 - beta2 ** step)
    return theta - lr * mhat / (np.sqrt(shat) + eps), m, s


def train(theta, X, T, order, batch, lr):
    """Adam over the minibatches given by ``order`` (a flat index array, consumed
    ``batch`` at a time, remainder dropped).  Returns (theta, losses)."""
    theta = np.array(theta, dtype=np.float64)
    m = np.zeros_like(theta)
    s = np.zeros_like(theta)
    losses = []
    nb = len(order) // batch
    for i in range(nb):
        sel = order[i * batch:(i + 1) * batch]
        loss, g = loss_and_grad(theta, X[sel], T[sel])
        theta, m, s = adam_step(theta, g, m, s, i + 1, lr)
        losses.append(loss)
    return theta, np.array(losses)


class NetworkCV:
    """Adapter giving the assembly oracle grad v at path points.  The
    network's input is the point in the domain's unit coordinates
    ((x - x0) / (x1 - x0), (y - y0) / (y1 - y0)); the gradient is taken with
    respect to the domain's coordinates (chain rule)."""

    def __init__(self, theta, domain=(0.0, 1.0, 0.0, 1.0)):
        self.theta = np.asarray(theta, dtype=np.float64)
        self.x0, x1, self.y0, y1 = (float(v) for v in domain)
        self.sx, self.sy = 1.0 / (x1 - self.x0), 1.0 / (y1 - self.y0)

    def grad(self, x, y):
        u = np.stack([(x - self.x0) * self.sx, (y - self.y0) * self.sy], axis=1)
        g = grad_input(self.theta, u)
        return g[:, 0] * self.sx, g[:, 1] * self.sy


class GradLutCV:
    """grad v read by bilinear interpolation from a float32 table [n, n, 2] on the
    node-centred grid of the domain (the paper stores F on a look-up table,
    Sec. 4.2); the table is an input, its values promoted to float64."""

    def __init__(self, table, domain):
        self.t = np.asarray(table, dtype=np.float32).astype(np.float64)
        self.n = self.t.shape[0]
        self.domain = tuple(float(v) for v in domain)

    def grad(self, x, y):
        n = self.n
        x0, x1, y0, y1 = self.domain
        fx = np.clip((x - x0) / (x1 - x0) * (n - 1), 0.0, n - 1)
        fy = np.clip((y - y0) / (y1 - y0) * (n - 1), 0.0, n - 1)
        i = np.minimum(np.floor(fx), n - 2).astype(np.int64)
        j = np.minimum(np.floor(fy), n - 2).astype(np.int64)
        tx = (fx - i)[..., None]
        ty = (fy - j)[..., None]
        t = self.t
        v = (1.0 - ty) * ((1.0 - tx) * t[j, i] + tx * t[j, i + 1]) + ty * ((1.0 - tx) * t[j + 1, i] + tx * t[j + 1, i + 1])
        return v[..., 0], v[..., 1]


class ExactGradientCV:
    """F built from the exact solution's gradient: the zero-variance choice of eq. (11)."""

    def __init__(self, coef):
        self.coef = coef

    def grad(self, x, y):
        return self.coef.grad_exact(x, y)
