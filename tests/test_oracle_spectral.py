"""Pins of the pseudospectral subdomain solves (Sec. 3.3, Sec. 5.1) of the
oracle: closed forms of the Chebyshev differentiation matrix, exactness on
polynomial solutions of an anisotropic operator with drift and reaction,
spectral convergence on a smooth solution, exact reproduction of a bilinear
harmonic solution through the knots and the hat interpolation, the RBF
cardinal property of the side values, exact polynomial interpolation of the
global u0 and its gradient, and agreement with the independent Feynman-Kac
point evaluation (eq. 8) within its standard error."""
import numpy as np
import pytest

from oracle import spectral as sp
from oracle.coeffs import Coefficients
from oracle.evaluate import evaluate
from oracle.geometry import Geometry
from oracle.rbf import shape_for_condition


class ConstCoef:
    """Constant symmetric sigma, drift and reaction, f = L u* and g = u* for a
    cubic u* (test-local, written out by hand)."""
    S = np.array([[1.2, 0.3], [0.3, 0.8]])
    d = (0.5, -0.7)
    c = -1.5

    @staticmethod
    def u(x, y):
        return 1.0 + x - 2.0 * y + x * x * y - 3.0 * x * y * y + x ** 3

    def sigma(self, x, y):
        one = np.ones_like(x)
        return self.S[0, 0] * one, self.S[0, 1] * one, self.S[1, 1] * one

    def drift(self, x, y):
        return self.d[0] * np.ones_like(x), self.d[1] * np.ones_like(x)

    def reaction(self, x, y):
        return self.c * np.ones_like(x)

    def source(self, x, y):
        A = self.S @ self.S.T
        ux = 1.0 + 2.0 * x * y - 3.0 * y * y + 3.0 * x * x
        uy = -2.0 + x * x - 6.0 * x * y
        uxx, uxy, uyy = 2.0 * y + 6.0 * x, 2.0 * x - 6.0 * y, -6.0 * x
        return (0.5 * A[0, 0] * uxx + A[0, 1] * uxy + 0.5 * A[1, 1] * uyy + self.d[0] * ux + self.d[1] * uy
                + self.c * self.u(x, y))

    def boundary(self, x, y):
        return self.u(x, y)


class BilinearHarmonic:
    """Poisson (sigma = sqrt 2 I) with u* = 2 + x/2 - 3y/10 + 7xy/10: harmonic,
    and linear along every grid line, so hat interpolation of its knot values
    is exact on every side."""

    @staticmethod
    def u(x, y):
        return 2.0 + 0.5 * x - 0.3 * y + 0.7 * x * y

    def sigma(self, x, y):
        s = np.full_like(x, np.sqrt(2.0))
        return s, np.zeros_like(x), s.copy()

    def drift(self, x, y):
        return np.zeros_like(x), np.zeros_like(x)

    def reaction(self, x, y):
        return np.zeros_like(x)

    def source(self, x, y):
        return np.zeros_like(x)

    def boundary(self, x, y):
        return self.u(x, y)


def test_differentiation_matrix_closed_forms():
    for p in (2, 5, 16):
        t = sp.cheb_nodes(p)
        D = sp.diff_matrix(p)
        assert np.all(np.diff(t) > 0) and t[0] == -1.0 and abs(t[-1] - 1.0) < 1e-15
        # exact on every polynomial of degree <= p
        for k in range(p + 1):
            ref = k * t ** (k - 1) if k else np.zeros_like(t)
            assert np.allclose(D @ t ** k, ref, atol=1e-10 * p * p), (p, k)
        # the classical corner entries (2 p^2 + 1) / 6 at the end points (with
        # ascending nodes the lower end carries the minus sign)
        assert np.isclose(D[-1, -1], (2 * p * p + 1) / 6.0, rtol=1e-12)
        assert np.isclose(D[0, 0], -(2 * p * p + 1) / 6.0, rtol=1e-12)


@pytest.mark.parametrize("p", [3, 6])
def test_collocation_is_exact_for_a_cubic(p):
    """Anisotropic sigma with an off-diagonal entry, drift and reaction on a
    rectangle with unequal sides: a wrong Kronecker order, scale or sign
    breaks the exact reproduction."""
    c = ConstCoef()
    box = (0.25, 0.75, -0.5, 0.5)
    U = sp.solve_square(c, box, p, lambda s, x, y: c.u(x, y))
    x, y = sp.square_grid(box, p)
    X, Y = np.meshgrid(x, y, indexing="ij")
    assert np.max(np.abs(U - c.u(X, Y))) < 1e-11


def test_spectral_convergence():
    """Smooth Poisson solution, boundary values from u*: the error falls
    geometrically with p."""
    c = Coefficients("poisson")
    box = (0.0, 0.5, 0.5, 1.0)
    errs = []
    for p in (4, 6, 8, 12):
        U = sp.solve_square(c, box, p, lambda s, x, y: c.exact(x, y))
        x, y = sp.square_grid(box, p)
        X, Y = np.meshgrid(x, y, indexing="ij")
        errs.append(np.max(np.abs(U - c.exact(X, Y))))
    # about two orders per two degrees until rounding (amplified ~p^4) takes over
    assert errs[1] < 2e-2 * errs[0] and errs[2] < 2e-2 * errs[1]
    assert errs[3] < 1e-10


@pytest.mark.parametrize("ext", [0, 2])
def test_subdomains_reproduce_a_bilinear_harmonic_solution(ext):
    """Knot values of u*, hat interpolation along the lines, g on the domain
    boundary: every square's grid values equal u* (3 x 3 squares, so there are
    corner, edge and floating squares)."""
    c = BilinearHarmonic()
    g = Geometry((0.0, 1.5, -0.5, 1.0), 3, 4, ext)
    p = 7
    U = sp.solve_subdomains(g, c, c.u(g.x, g.y), p)
    assert U.shape == (9, p + 1, p + 1)
    s = 0.5
    for a in range(3):
        for cc in range(3):
            box = (a * s, (a + 1) * s, -0.5 + cc * s, -0.5 + (cc + 1) * s)
            x, y = sp.square_grid(box, p)
            X, Y = np.meshgrid(x, y, indexing="ij")
            assert np.max(np.abs(U[a + 3 * cc] - c.u(X, Y))) < 1e-11, (a, cc)


def test_rbf_side_values_interpolate_the_lattice():
    """RBF side values at the line's lattice points are the lattice values
    (the cardinal property, eq. 5), boundary lattice points carrying g."""
    c = Coefficients("poisson")
    g = Geometry((0.0, 1.0, 0.0, 1.0), 2, 8, 4)
    rng = np.random.default_rng(3)
    u = rng.normal(size=g.n)
    cc = shape_for_condition(2 * 4 + 8 + 1, g.dx, 1e8)
    at = 8                                                   # the line x = 1/2
    q = np.arange(0, 13)                                     # side [0, 8] widened by 4
    vals = sp.line_values(g, c, u, True, at, 0, 8, g.lattice_y(q), interp=("rbf", cc))
    ref = np.where(q == 0, c.boundary(np.full(13, 0.5), np.zeros(13)), 0.0)
    ref[1:] = u[g.index[at, q[1:]]]
    assert np.allclose(vals, ref, atol=1e-6 * np.abs(ref).max())
    hat = sp.line_values(g, c, u, True, at, 0, 8, g.lattice_y(q))
    assert np.allclose(hat, ref, atol=1e-14)


def test_interpolation_and_gradients_are_exact_for_polynomials():
    """Grid values of a degree-p polynomial on every square: the barycentric
    interpolant and its grid derivatives give the polynomial and its gradient
    at any point; the gradient table holds grad u at its nodes."""
    g = Geometry((-1.0, 1.0, 0.0, 2.0), 2, 4, 2)
    p = 5

    def u(x, y):
        return 0.3 + x ** 5 - 2.0 * x ** 2 * y ** 3 + y ** 4 - x * y

    def grad(x, y):
        return 5 * x ** 4 - 4.0 * x * y ** 3 - y, -6.0 * x * x * y * y + 4 * y ** 3 - x

    U = []
    for (xlo, xhi, ylo, yhi) in sp.subdomain_boxes(g):
        x, y = sp.square_grid((g.lattice_x(xlo), g.lattice_x(xhi), g.lattice_y(ylo), g.lattice_y(yhi)), p)
        X, Y = np.meshgrid(x, y, indexing="ij")
        U.append(u(X, Y))
    U = np.array(U)
    gx, gy = sp.grid_gradients(g, U, p)
    rng = np.random.default_rng(5)
    pts = np.concatenate([rng.uniform([-1.0, 0.0], [1.0, 2.0], size=(40, 2)), [[0.0, 1.0], [-1.0, 2.0], [1.0, 0.0]]])
    v = sp.interpolate(g, [U, gx, gy], p, pts)
    ex = grad(pts[:, 0], pts[:, 1])
    assert np.allclose(v[0], u(pts[:, 0], pts[:, 1]), atol=1e-11)
    assert np.allclose(v[1], ex[0], atol=1e-9) and np.allclose(v[2], ex[1], atol=1e-9)
    tab = sp.grad_table(g, U, p, 9)
    xs = -1.0 + 2.0 * np.arange(9) / 8
    ys = 2.0 * np.arange(9) / 8
    X, Y = np.meshgrid(xs, ys)
    gxr, gyr = grad(X, Y)
    assert np.allclose(tab[..., 0], gxr, atol=1e-9) and np.allclose(tab[..., 1], gyr, atol=1e-9)


def test_agrees_with_the_feynman_kac_point_values():
    """Knot values of u* on a fine lattice (hat interpolation then adds
    error below 1e-4): the spectral u0 and the Feynman-Kac point values of the
    same Dirichlet problems agree within four standard errors plus the
    time-step bias, and the spectral values are within 2e-4 of u*."""
    c = Coefficients("poisson")
    g = Geometry((0.0, 1.0, 0.0, 1.0), 2, 64, 0)
    p = 20
    U = sp.solve_subdomains(g, c, c.exact(g.x, g.y), p)
    pts = np.array([[0.2, 0.3], [0.71, 0.77], [0.33, 0.62], [0.9, 0.15]])
    u_sp = sp.interpolate(g, [U], p, pts)[0]
    ue = c.exact(pts[:, 0], pts[:, 1])
    assert np.max(np.abs(u_sp - ue)) < 2e-4
    u_fk, se, _ = evaluate(g, c, c.exact(g.x, g.y), pts, 6000, 1e-4, seed=5)
    assert np.all(np.abs(u_fk - u_sp) <= 4.0 * se + 2e-3), (u_fk - u_sp, se)


@pytest.mark.parametrize("kind", ["poisson", "amplitude", "lut", "varcoef", "eq43"])
def test_exact_gradients_by_finite_differences(kind):
    """grad u* of every family with a closed form against central differences."""
    if kind == "lut":
        from paper_2301_05780_amd import workloads
        c = Coefficients("lut", lut=workloads.poisson_lut(17), lut_n=17)
        dom = (0.0, 1.0)
    elif kind == "eq43":
        c = Coefficients("eq43")
        dom = (-100.0, 100.0)
    else:
        c = Coefficients(kind, (0.4,) if kind == "amplitude" else ())
        dom = (0.0, 1.0)
    rng = np.random.default_rng(7)
    x, y = rng.uniform(*dom, size=(2, 25))
    e = 1e-6 * (dom[1] - dom[0])
    gx, gy = c.grad_exact(x, y)
    fx = (c.exact(x + e, y) - c.exact(x - e, y)) / (2 * e)
    fy = (c.exact(x, y + e) - c.exact(x, y - e)) / (2 * e)
    scale = max(np.abs(gx).max(), np.abs(gy).max())
    assert np.allclose(gx, fx, atol=1e-7 * scale) and np.allclose(gy, fy, atol=1e-7 * scale)
