"""Pins of the oracle's RBF cardinal interpolation (Sec. 2.1, eqs. 1-5) and of
its use in the assembly (eq. 21), against an independent library routine,
the properties the paper states and brute force on kept paths."""
import numpy as np
import pytest
from scipy.interpolate import RBFInterpolator

from oracle.geometry import Geometry
from oracle.coeffs import Coefficients
from oracle.assemble import assemble
from oracle.rbf import cardinal, condition, shape_for_condition, interpolation_matrix

SMALL = Geometry((0, 1, 0, 1), 2, 8, 4)


def _scipy_cardinal(nodes, z, c):
    """Cardinal functions through scipy's inverse multiquadric interpolant.
    scipy's kernel is 1/sqrt(1 + (eps r)^2) = c phi_c(r) with eps = 1/c, and
    cardinal functions do not change when the basis is scaled."""
    ip = RBFInterpolator(np.asarray(nodes)[:, None], np.eye(len(nodes)), kernel="inverse_multiquadric",
                         epsilon=1.0 / c, degree=-1)
    return ip(np.atleast_1d(z)[:, None]).T


def test_cardinal_matches_an_independent_solver():
    rng = np.random.default_rng(0)
    for S, d, cf in ((5, 0.1, 1.0), (17, 1 / 64, 2.0), (33, 1 / 128, 3.0)):
        nodes = np.arange(S) * d
        z = rng.uniform(0, nodes[-1], 9)
        c = cf * d
        assert np.abs(cardinal(nodes, z, c) - _scipy_cardinal(nodes, z, c)).max() < 1e-9


def test_cardinal_property():
    """H_j(z_i) = delta_ij (Sec. 2.1), to the conditioning of Phi."""
    S, d = 33, 1 / 128
    nodes = np.arange(S) * d
    for cf in (1.0, 3.0, 5.0):
        c = cf * d
        H = cardinal(nodes, nodes, c)
        assert np.abs(H - np.eye(S)).max() < 1e-15 * condition(nodes, c) * S


def test_interpolant_reproduces_the_basis():
    """A combination of the basis functions is interpolated exactly."""
    S, d = 21, 0.05
    nodes = np.arange(S) * d
    c = 2.5 * d
    rng = np.random.default_rng(1)
    alpha = rng.normal(size=S)
    u = lambda z: (alpha[:, None] / np.sqrt((np.atleast_1d(z)[None, :] - nodes[:, None]) ** 2 + c * c)).sum(0)
    z = rng.uniform(0, nodes[-1], 50)
    assert np.abs(u(nodes) @ cardinal(nodes, z, c) - u(z)).max() < 1e-9


def test_more_accurate_than_hat_inside_an_extended_stencil():
    """In the middle half of a stencil (where the patch side lies once the
    stencil is extended by half a segment on each end, Sec. 5.1) the RBF
    interpolant of a smooth function beats the hat interpolant by far."""
    S, d = 33, 1 / 32
    nodes = np.arange(S) * d
    u = lambda z: np.sin(3 * z) + np.cos(5 * z)
    z = np.linspace(0.25, 0.75, 401)
    c = shape_for_condition(S, d, 1e8)
    e_rbf = np.abs(u(nodes) @ cardinal(nodes, z, c) - u(z)).max()
    e_hat = np.abs(np.interp(z, nodes, u(nodes)) - u(z)).max()
    assert e_rbf < 1e-2 * e_hat


def test_cardinal_functions_tend_to_sinc():
    """On an equispaced pointset the cardinal functions approach sinc as the
    shape parameter grows (Sec. 2.1)."""
    S = 121
    nodes = np.arange(S) * 1.0
    z = np.linspace(55, 65, 101)
    dev = [np.abs(cardinal(nodes, z, c)[60] - np.sinc(z - 60)).max() for c in (2.0, 4.0, 8.0)]
    assert dev[0] > dev[1] > dev[2] and dev[2] < 1e-2


def test_shape_for_condition():
    """c is found where cond(Phi) reaches the target; cond grows with c."""
    for S, d in ((33, 1 / 128), (65, 1 / 1024), (17, 0.5)):
        c = shape_for_condition(S, d, 1e10)
        nodes = np.arange(S) * d
        assert condition(nodes, c) == pytest.approx(1e10, rel=1e-3)
        assert condition(nodes, 0.9 * c) < 1e10 < condition(nodes, 1.1 * c)
        ev = np.linalg.eigvalsh(interpolation_matrix(nodes, c))
        assert ev[0] > 0                       # positive definite


def _retally(geom, coef, k, paths, c, N):
    """Row k of G and b recomputed from kept path records with scipy's weights."""
    cols = geom.col_idx[geom.row_ptr[k]:geom.row_ptr[k + 1]]
    pos = {int(j): i for i, j in enumerate(cols)}
    g = np.zeros(cols.size)
    b = 0.0
    for p in range(N):
        Y = paths["Y"][p]
        b += paths["Z"][p] + paths["Xi"][p]
        o = int(paths["side"][p])
        s = geom.side(k, "ENWS"[o])
        if s["boundary"]:
            b += Y * paths["g_side"][p]
            continue
        vert = s["line"] == "x"
        along = paths["y"][p] if vert else paths["x"][p]
        a0, da = (geom.y0, geom.dy) if vert else (geom.x0, geom.dx)
        t = min(max((along - a0) / da, s["clo"]), s["chi"])
        qs = np.arange(s["clo"], s["chi"] + 1)
        H = _scipy_cardinal(qs * da, [t * da], c)[:, 0]
        for q, w in zip(qs, H):
            if q == 0 or q == geom.L:
                px, py = (geom.lattice_x(s["at"]), geom.lattice_y(q)) if vert else (geom.lattice_x(q), geom.lattice_y(s["at"]))
                b += Y * w * coef.boundary(np.array([px]), np.array([py]))[0]
            else:
                j = int(geom.index[s["at"], q] if vert else geom.index[q, s["at"]])
                g[pos[j]] -= Y * w
    g /= N
    g[pos[k]] = 1.0
    return g, b / N


@pytest.mark.parametrize("kind", ["poisson", "varcoef"])
def test_assembled_rbf_rows_by_brute_force(kind):
    coef = Coefficients(kind, ())
    c = 2.0 * SMALL.dx
    N = 200
    ks = [int(SMALL.index[8, 3]), int(SMALL.index[8, 8]), int(SMALL.index[1, 8])]
    out = assemble(SMALL, coef, N, 1e-3, 11, knots=ks, keep_paths=True, interp=("rbf", c))
    for k in ks:
        g, b = _retally(SMALL, coef, k, out["paths"][k], c, N)
        r = out["rows"][k]
        assert np.abs(r["val"] - g).max() < 1e-9 and abs(r["b"] - b) < 1e-9
        # the same paths as the hat assembly: step totals and exit sides agree
        hat = assemble(SMALL, coef, N, 1e-3, 11, knots=[k])["rows"][k]
        assert np.array_equal(hat["diag"][:6], r["diag"][:6])


def test_rbf_row_close_to_hat_row_in_the_mean():
    """Both interpolations estimate the same patch problem: the exact
    solution satisfies either row up to a small multiple of the row's Monte
    Carlo standard error (the interpolation and time-step biases are below
    it at this path count)."""
    coef = Coefficients("varcoef", ())
    geom = Geometry((0, 1, 0, 1), 2, 8, 4)
    ks = [int(geom.index[8, 3]), int(geom.index[5, 8])]
    c = shape_for_condition(17, geom.dx, 1e8)
    for k in ks:
        res = []
        for interp in (None, ("rbf", c)):
            r = assemble(geom, coef, 4000, 1e-4, 3, knots=[k], interp=interp)["rows"][k]
            cols = r["cols"]
            u = coef.exact(geom.x[cols], geom.y[cols])
            res.append(abs(r["val"] @ u - r["b"]) / (3 * np.sqrt(np.sum(r["se_val"] ** 2 * u * u)) + 3 * r["se_b"]))
        assert res[0] < 1.5 and res[1] < 1.5
