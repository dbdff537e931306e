"""Seeded synthetic inputs shared by the HIP path's tests/benchmark and the oracle.

This module holds input definitions and input generators only: problem
parameters, seeded draws of batched instances, tabulated coefficient fields,
initial network weights and minibatch orders.  It holds none of the
assembly's arithmetic (no paths, exits, interpolation or tallies), so both
sides of every parity check read identical inputs without sharing method code.

Workloads (all formula-defined manufactured problems, so no dataset is needed;
the paper's own experiment in Sec. 5 is formula-defined too, eq. 43):

  poisson_small   Poisson on [0,1]^2, 2 x 2 subdomains, knots every 1/16
                  (29 knots, 449 structural nonzeros), N = 1000, h = 1e-3,
                  float64, seed 0
  varcoef         variable sigma, drift and reaction on [0,1]^2, 8 x 8
                  subdomains, knot spacing 1/128 (1729 knots), N = 1e4,
                  h = 1e-4; float32 paths, float64 accumulation
  batched         64 instances of the amplitude family: a ~ U(0, 0.8), grid
                  H in {4, 6, 8, 12, 16}, knot spacing log-uniform in
                  [1/256, 1/64] (m = round(1 / (H s))), N ~ U[2e3, 2e4]
  cv_small        poisson_small plus the 2-64-64-1 tanh control-variate network
  large_lut       poisson coefficients tabulated on a 4096^2 float32 grid,
                  32 x 32 subdomains, knot spacing 1/1024 (62465 knots),
                  N = 1e4, h = 1e-5
"""
import numpy as np

KIND_CODES = {"poisson": 0, "varcoef": 1, "amplitude": 2, "lut": 3, "constsol": 4, "exittime": 5}
LUT_STRIDE = 8
MLP_WIDTH = 64
MLP_PARAMS = MLP_WIDTH * 2 + MLP_WIDTH + MLP_WIDTH * MLP_WIDTH + MLP_WIDTH + MLP_WIDTH + 1


def poisson_small(exit_rule="gm"):
    return dict(name="poisson_small", kind="poisson", param=(), domain=(0.0, 1.0, 0.0, 1.0),
                H=2, m=8, ext=4, n_paths=1000, h=1e-3, seed=0, precision="fp64",
                exit_rule=exit_rule)


def varcoef(exit_rule="gm"):
    return dict(name="varcoef", kind="varcoef", param=(), domain=(0.0, 1.0, 0.0, 1.0),
                H=8, m=16, ext=8, n_paths=10000, h=1e-4, seed=0, precision="fp32",
                exit_rule=exit_rule)


def large_lut(exit_rule="gm"):
    return dict(name="large_lut", kind="lut", param=(), domain=(0.0, 1.0, 0.0, 1.0),
                H=32, m=32, ext=16, n_paths=10000, h=1e-5, seed=0, precision="fp32",
                exit_rule=exit_rule, lut_n=4096)


def sec5(exit_rule="gm"):
    """The numerical experiment of Sec. 5 at one-GPU scale: Lap u = f on
    [-100, 100]^2 with the solution of eq. 43, 10 x 10 subdomains, 64 knots
    per interface counted with the two crossings (63 lattice intervals per
    subdomain side), side stencils widened by half a segment (32 lattice
    units) each way, RBF interpolation with the shape parameter at condition
    number 1e10 for the longest stencil; Phase I with h0 = 0.08 and
    N0 = 1000, target precision eps = 0.01, N_job = 200."""
    return dict(name="sec5", kind="eq43", param=(), domain=(-100.0, 100.0, -100.0, 100.0),
                H=10, m=63, ext=32, n_paths=1000, h=0.08, seed=0, precision="fp32",
                exit_rule=exit_rule, interp="rbf", rbf_condition=1e10, eps=0.01, n_job=200)


def batched(seed=0, n_instances=64):
    """Instance draws of the batched workload (NumPy PCG64, ``seed``)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(n_instances):
        a = float(rng.uniform(0.0, 0.8))
        H = int(rng.choice([4, 6, 8, 12, 16]))
        s = float(np.exp(rng.uniform(np.log(1 / 256), np.log(1 / 64))))
        m = max(2, int(round(1.0 / (H * s))))
        N = int(rng.integers(2000, 20001))
        out.append(dict(name=f"batched[{i}]", kind="amplitude", param=(a,),
                        domain=(0.0, 1.0, 0.0, 1.0), H=H, m=m, ext=m // 2,
                        n_paths=N, h=1e-4, seed=0, instance=i, precision="fp32",
                        exit_rule="gm"))
    return out


def poisson_lut(n=4096, domain=(0.0, 1.0, 0.0, 1.0)):
    """The poisson coefficient fields tabulated on an n x n node-centred grid.

    Layout: float32 [n (y nodes)][n (x nodes)][8] with fields
    (sxx, sxy, syy, dx, dy, c, f, 0); node (i, j) sits at
    (x0 + i (x1 - x0)/(n - 1), y0 + j (y1 - y0)/(n - 1)).
    This tabulates the problem data (sigma = sqrt 2 I, d = 0, c = 0,
    f = Laplacian of sin(pi x) sin(pi y) + x^2 y); it is an input, not part
    of the method.
    """
    x0, x1, y0, y1 = domain
    xs = x0 + np.arange(n) * ((x1 - x0) / (n - 1))
    ys = y0 + np.arange(n) * ((y1 - y0) / (n - 1))
    tab = np.zeros((n, n, LUT_STRIDE), dtype=np.float32)
    tab[..., 0] = np.sqrt(2.0)
    tab[..., 2] = np.sqrt(2.0)
    # f[j, i] = -2 pi^2 sin(pi x_i) sin(pi y_j) + 2 y_j, formed as an outer product
    a = -2.0 * np.pi ** 2 * np.sin(np.pi * xs)
    tab[..., 6] = a[None, :] * np.sin(np.pi * ys)[:, None] + 2.0 * ys[:, None]
    return tab


def varied_lut(n=65, domain=(0.0, 1.0, 0.0, 1.0)):
    """A tabulated problem whose every field varies, sigma with an off-diagonal
    entry (same layout as ``poisson_lut``):

      sxx = 1.3 + 0.25 sin(2 pi x) cos(pi y)     sxy = 0.2 sin(pi (x + 2 y))
      syy = 1.2 + 0.3 cos(2 pi y) sin(pi x)      d = (0.5 sin 2 pi y, -0.4 cos 2 pi x)
      c = -(0.5 + x y)                           f = cos 3x + y

    det sigma >= 1.05 * 0.9 - 0.04 > 0, so A = sigma sigma^T is uniformly
    elliptic.  No manufactured solution: it serves the parity checks.
    """
    x0, x1, y0, y1 = domain
    xs = x0 + np.arange(n) * ((x1 - x0) / (n - 1))
    ys = y0 + np.arange(n) * ((y1 - y0) / (n - 1))
    X, Y = np.meshgrid(xs, ys)
    tab = np.zeros((n, n, LUT_STRIDE), dtype=np.float32)
    tab[..., 0] = 1.3 + 0.25 * np.sin(2 * np.pi * X) * np.cos(np.pi * Y)
    tab[..., 1] = 0.2 * np.sin(np.pi * (X + 2 * Y))
    tab[..., 2] = 1.2 + 0.3 * np.cos(2 * np.pi * Y) * np.sin(np.pi * X)
    tab[..., 3] = 0.5 * np.sin(2 * np.pi * Y)
    tab[..., 4] = -0.4 * np.cos(2 * np.pi * X)
    tab[..., 5] = -(0.5 + X * Y)
    tab[..., 6] = np.cos(3 * X) + Y
    return tab


def mlp_init(seed=0):
    """Initial parameters of the 2-64-64-1 network (Glorot-uniform weights, zero biases).

    Layout: W1[64,2], b1[64], W2[64,64] (out, in), b2[64], w3[64], b3.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    w = MLP_WIDTH

    def glorot(fan_out, fan_in):
        lim = np.sqrt(6.0 / (fan_in + fan_out))
        return rng.uniform(-lim, lim, size=(fan_out, fan_in))

    W1 = glorot(w, 2)
    W2 = glorot(w, w)
    w3 = glorot(1, w).ravel()
    return np.concatenate([W1.ravel(), np.zeros(w), W2.ravel(), np.zeros(w), w3, [0.0]])


def minibatch_order(n_samples, epochs, seed=0):
    """Concatenated per-epoch permutations of range(n_samples) (int32)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.concatenate([rng.permutation(n_samples) for _ in range(epochs)]).astype(np.int32)
