"""Pins of the oracle's tabulated-coefficient family: bilinear reads, and the
Gobet-Menozzi shift taken at the projection when sigma varies along a side."""
import numpy as np
import pytest

from oracle.geometry import Geometry
from oracle.coeffs import Coefficients, LUT_STRIDE
from oracle.assemble import exit_flags, C_GM
from paper_2301_05780_amd import workloads


def _table(fields, n, domain):
    x0, x1, y0, y1 = domain
    xs = x0 + np.arange(n) * ((x1 - x0) / (n - 1))
    ys = y0 + np.arange(n) * ((y1 - y0) / (n - 1))
    X, Y = np.meshgrid(xs, ys)
    tab = np.zeros((n, n, LUT_STRIDE), dtype=np.float32)
    for q, f in enumerate(fields):
        tab[..., q] = f(X, Y)
    return tab


def test_bilinear_fields_are_reproduced_exactly():
    """Bilinear interpolation is exact for a + b x + c y + d x y: a table sampled
    from such fields (dyadic coefficients, so float32 holds the nodes exactly)
    returns them at any point, on a domain that is not the unit square."""
    dom = (-0.5, 1.5, 0.25, 2.25)
    fields = [lambda x, y: 1.5 + 0.25 * x * y, lambda x, y: 0.125 * x - 0.25 * y,
              lambda x, y: 2.0 + 0.5 * y, lambda x, y: x - y, lambda x, y: 0.75 * x * y,
              lambda x, y: -1.0 - 0.5 * x, lambda x, y: 3.0 * y - 2.0 * x * y]
    c = Coefficients("lut", lut=_table(fields, 17, dom), lut_n=17, domain=dom)
    rng = np.random.default_rng(0)
    x, y = rng.uniform(dom[0], dom[1], 400), rng.uniform(dom[2], dom[3], 400)
    sxx, sxy, syy = c.sigma(x, y)
    dx, dy = c.drift(x, y)
    got = [sxx, sxy, syy, dx, dy, c.reaction(x, y), c.source(x, y)]
    for q, f in enumerate(fields):
        assert np.allclose(got[q], f(x, y), rtol=0, atol=1e-13), q
    # outside the domain the point is clamped to the nearest boundary point
    assert c.reaction(np.array([dom[1] + 3.0]), np.array([dom[2] - 1.0]))[0] == pytest.approx(
        fields[5](dom[1], dom[2]), abs=1e-13)
    # the Dirichlet datum stays the poisson solution
    assert c.boundary(np.array([0.3]), np.array([0.7]))[0] == pytest.approx(
        np.sin(np.pi * 0.3) * np.sin(np.pi * 0.7) + 0.09 * 0.7, rel=1e-15)


def test_node_values_are_returned_at_nodes():
    tab = workloads.varied_lut(9)
    c = Coefficients("lut", lut=tab, lut_n=9)
    i, j = np.meshgrid(np.arange(9), np.arange(9))
    x, y = i.ravel() / 8.0, j.ravel() / 8.0
    sxx, sxy, syy = c.sigma(x, y)
    assert np.array_equal(sxx, tab[j.ravel(), i.ravel(), 0].astype(np.float64))
    assert np.array_equal(sxy, tab[j.ravel(), i.ravel(), 1].astype(np.float64))
    assert np.array_equal(c.source(x, y), tab[j.ravel(), i.ravel(), 6].astype(np.float64))


def test_gm_shift_uses_sigma_at_the_projection():
    """sxx = 1 + y, sxy = 1/4, syy = 3/2 + x/2 (bilinear, so the table holds them
    exactly).  On the E side x = xhi the normal diffusion is
    a_nn = (1 + yc)^2 + 1/16 with yc the point's y clamped to the side, on the
    N side a_nn = 1/16 + (3/2 + xc/2)^2; the flag switches at the line shifted
    by c_GM sqrt(a_nn) sqrt(h), not at a shift taken at the knot."""
    fields = [lambda x, y: 1.0 + y, lambda x, y: 0.25 + 0 * x, lambda x, y: 1.5 + 0.5 * x]
    c = Coefficients("lut", lut=_table(fields + [lambda x, y: 0 * x] * 4, 9, (0, 1, 0, 1)), lut_n=9)
    g = Geometry((0, 1, 0, 1), 2, 4, 2)
    k = int(g.index[4, 2])               # index[ix, iy]: knot (1/2, 1/4) on x = 1/2, patch [0, 1] x [0, 1/2]
    xlo, xhi, ylo, yhi = g.box[k]
    assert (xlo, xhi, ylo, yhi) == (0.0, 1.0, 0.0, 0.5)
    h = 1e-2
    for y in [0.05, 0.2, 0.45, 0.49]:    # inside the side's range
        d = C_GM * np.sqrt((1 + y) ** 2 + 1 / 16) * np.sqrt(h)
        for fac, expect in [(1 - 1e-6, True), (1 + 1e-6, False)]:
            fE, fN, fW, fS = exit_flags(c, g, k, np.array([xhi - fac * d]), np.array([y]), h, "gm")
            assert bool(fE[0]) == expect and not fW[0], (y, fac)
    # beyond the side's end the projection is clamped to the corner (yc = yhi)
    d = C_GM * np.sqrt((1 + yhi) ** 2 + 1 / 16) * np.sqrt(h)
    assert exit_flags(c, g, k, np.array([xhi - 0.999 * d]), np.array([0.7]), h, "gm")[0][0]
    assert not exit_flags(c, g, k, np.array([xhi - 1.001 * d]), np.array([0.7]), h, "gm")[0][0]
    # N side at y = 1/2: a_nn = 1/16 + (3/2 + x/2)^2 at the point's x
    for x in [0.1, 0.6, 0.9]:
        d = C_GM * np.sqrt(1 / 16 + (1.5 + 0.5 * x) ** 2) * np.sqrt(h)
        assert exit_flags(c, g, k, np.array([x]), np.array([yhi - 0.999 * d]), h, "gm")[1][0]
        assert not exit_flags(c, g, k, np.array([x]), np.array([yhi - 1.001 * d]), h, "gm")[1][0]
    # W side: a_nn = (1 + y)^2 + 1/16, shifted inwards from x = 0
    d = C_GM * np.sqrt((1 + 0.3) ** 2 + 1 / 16) * np.sqrt(h)
    assert exit_flags(c, g, k, np.array([0.999 * d]), np.array([0.3]), h, "gm")[2][0]
    assert not exit_flags(c, g, k, np.array([1.001 * d]), np.array([0.3]), h, "gm")[2][0]
    # the naive rule ignores sigma
    fE = exit_flags(c, g, k, np.array([xhi - 1e-9, xhi + 1e-9]), np.array([0.2, 0.2]), h, "naive")[0]
    assert list(fE) == [False, True]


def test_varied_table_is_uniformly_elliptic():
    tab = workloads.varied_lut(65).astype(np.float64)
    det = tab[..., 0] * tab[..., 2] - tab[..., 1] ** 2
    assert det.min() > 0.9
