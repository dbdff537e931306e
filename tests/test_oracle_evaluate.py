"""Pins of the oracle's point evaluation inside the subdomains (eq. 8 on each
square with the knot values as interface data, Sec. 3.3)."""
import numpy as np
import pytest

from closed_forms import mean_exit_time_rectangle
from oracle.geometry import Geometry
from oracle.coeffs import Coefficients
from oracle.evaluate import evaluate, line_value


def test_constant_solution_is_reproduced_exactly():
    """u = 1 solves the constsol problem; with every knot value 1 each path's
    score Z_K + Y_K u(exit) telescopes to 1 (Euler form of Y), so the mean is
    1 to rounding and the standard error vanishes."""
    g = Geometry((0, 1, 0, 1), 3, 6, 3)
    c = Coefficients("constsol")
    pts = np.array([[0.1, 0.15], [0.5, 0.52], [0.9, 0.07], [0.4, 0.95]])
    u, se, steps = evaluate(g, c, np.ones(g.n), pts, 300, 1e-3, seed=3)
    assert np.allclose(u, 1.0, rtol=0, atol=1e-12)
    assert np.all(se < 1e-10) and np.all(steps >= 300)


def test_mean_exit_time_of_the_domain():
    """exittime family: u is the mean exit time of the unit square, a double
    sine series.  Interface data = that series at the knots; the value at an
    interior point of a square agrees with the series within 3 SE plus the
    hat-interpolation error (d^2/8 max|u''| <= 2e-5 at d = 1/64) and the
    O(h) bias of the Gobet-Menozzi rule."""
    g = Geometry((0, 1, 0, 1), 2, 32, 16)
    c = Coefficients("exittime")
    uk = np.array([mean_exit_time_rectangle(x, y, 1.0, 1.0) for x, y in zip(g.x, g.y)])
    pts = np.array([[0.3, 0.2], [0.75, 0.6]])
    u, se, _ = evaluate(g, c, uk, pts, 4000, 2e-5, seed=1)
    for (x, y), ui, si in zip(pts, u, se):
        exact = mean_exit_time_rectangle(x, y, 1.0, 1.0)
        assert abs(ui - exact) <= 3 * si + 1e-4, (x, y, ui, exact, si)


def test_manufactured_poisson_in_a_corner_square():
    """poisson family in a square with two boundary sides: g on those, u* at
    the knots of the two interface sides; the value matches u*."""
    g = Geometry((0, 1, 0, 1), 4, 16, 8)
    c = Coefficients("poisson")
    uk = c.exact(g.x, g.y)
    pts = np.array([[0.08, 0.17], [0.2, 0.04]])
    u, se, _ = evaluate(g, c, uk, pts, 4000, 2e-5, seed=2)
    exact = c.exact(pts[:, 0], pts[:, 1])
    assert np.all(np.abs(u - exact) <= 3 * se + 2e-4), (u, exact, se)


def test_points_on_grid_lines_take_the_line_value():
    """A point on its square's boundary needs no paths: at a knot it returns
    the knot value, between knots the hat interpolation, on the domain
    boundary g."""
    g = Geometry((0, 1, 0, 1), 2, 8, 4)
    c = Coefficients("poisson")
    rng = np.random.default_rng(0)
    uk = rng.uniform(-1, 1, g.n)
    k = int(g.index[8, 3])              # knot (1/2, 3/16)
    mid = 0.5 * (3 + 4) / 16            # halfway between lattice points 3 and 4 on x = 1/2
    pts = np.array([[g.x[k], g.y[k]], [0.5, mid], [0.0, 0.3], [0.7, 1.0]])
    u, se, steps = evaluate(g, c, uk, pts, 50, 1e-3, seed=0)
    k4 = int(g.index[8, 4])
    assert u[0] == uk[k]
    assert u[1] == pytest.approx(0.5 * uk[k] + 0.5 * uk[k4], abs=1e-15)
    assert u[2] == pytest.approx(c.exact(np.array([0.0]), np.array([0.3]))[0], abs=1e-15)
    assert u[3] == pytest.approx(c.exact(np.array([0.7]), np.array([1.0]))[0], abs=1e-15)
    assert np.all(se == 0) and np.all(steps == 0)
    # the interpolation helper: lattice ends on the boundary take g
    v = line_value(g, c, uk, True, 8, 0.5 / 16, 0, 8)   # between (1/2, 0) and knot (1/2, 1/16)
    k1 = int(g.index[8, 1])
    assert v == pytest.approx(0.5 * c.exact(np.array([0.5]), np.array([0.0]))[0] + 0.5 * uk[k1], abs=1e-15)
