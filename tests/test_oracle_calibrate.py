"""Pins of the Phase II calibration oracle (mixed GM/EM paths, eqs. 32-41)."""
import numpy as np

from oracle.geometry import Geometry
from oracle.coeffs import Coefficients
from oracle.assemble import integrate_knot, exit_points
from oracle.calibrate import mixed_paths, path_scores, calibrate_knot, plan, STATS_WIDTH


def _small():
    return Geometry((0.0, 1.0, 0.0, 1.0), 3, 4, 2)


def test_mixed_records_are_the_gm_and_the_naive_paths():
    """The path does not change when it passes its GM exit, so the GM record
    equals the Gobet-Menozzi run and the EM record the naive run of the same
    stream, path by path (two independent integrators)."""
    g, c = _small(), Coefficients("varcoef")
    for k in (0, g.n // 2, g.n - 1):
        gm, em = mixed_paths(c, g.box[k], (g.x[k], g.y[k]), k, 3, 200, 2e-3, 11)
        ref_gm = integrate_knot(g, c, k, 200, 2e-3, 11, 3, "gm")
        ref_em = integrate_knot(g, c, k, 200, 2e-3, 11, 3, "naive")
        for key in ("K", "x", "y", "Y", "Z", "Xi", "flags"):
            assert np.array_equal(gm[key], ref_gm[key]), (k, key)
            assert np.array_equal(em[key], ref_em[key]), (k, key)
        assert np.all(gm["K"] <= em["K"])


def test_constant_solution_gives_zero_bias_and_variance():
    """u = 1 (f = c, g = 1) with u0 = 1: Z_K + Y_K = 1 along every path, so
    both scores are 1, the bias bound and the variance vanish, h_i = h0 and
    N_i is the minimum of one job."""
    g, c = _small(), Coefficients("constsol")
    u0 = np.ones(g.n)
    stats = np.array([calibrate_knot(g, c, k, u0, 300, 2e-3, 5) for k in range(g.n)])
    assert np.all(np.abs(stats[:, 0]) < 1e-10)
    assert np.allclose(stats[:, 1], 300.0, rtol=0, atol=1e-10)
    pl = plan(stats, 300, 2e-3, 0.01, 50)
    assert np.all(pl["var"] < 1e-20) and np.all(pl["bias"] < 1e-12)
    assert np.all(pl["h"] == 2e-3) and np.all(pl["n_paths"] == 50)


def test_scores_use_u0_on_interfaces_and_g_on_the_boundary():
    """With u0 the exact solution at the knots, the EM score of a long run
    matches u*(x_k) to within its Monte Carlo error and the discretisation
    bias (poisson family, h small)."""
    g, c = _small(), Coefficients("poisson")
    u0 = c.exact(g.x, g.y)
    k = g.n // 2
    gm, em = mixed_paths(c, g.box[k], (g.x[k], g.y[k]), k, 0, 4000, 2e-4, 2)
    phi = path_scores(g, c, k, em, u0)
    se = phi.std() / np.sqrt(phi.size)
    assert abs(phi.mean() - u0[k]) < 4 * se + 5e-3


def test_plan_formulas_on_a_hand_example():
    # one knot: 100 paths, mean difference 0.002, mean phi 1, E[phi^2] 1.04 (var 0.04),
    # xi with var 0.01 and cov -0.016 (rho^2 = 0.64)
    N = 100
    s = np.zeros(STATS_WIDTH)
    s[0] = 0.002 * N
    s[1] = 1.0 * N
    s[2] = 1.04 * N
    s[3] = 0.0
    s[4] = 0.01 * N
    s[5] = -0.016 * N
    pl = plan(s[None, :], N, 1e-3, 0.01, 100)
    assert np.isclose(pl["bias"][0], 0.001)
    assert np.isclose(pl["var"][0], 0.04)
    assert np.isclose(pl["rho2"][0], 0.64)
    # eq. 40: min(h0, 2 h0 eps / (3 * 0.002)) = min(1e-3, 3.33e-3) = 1e-3
    assert pl["h"][0] == 1e-3
    # eq. 41: 9 * 0.04 * 0.36 / 1e-4 = 1296 -> closest multiple of 100 is 1300
    assert pl["n_paths"][0] == 1300
    # a large bias shrinks the step: mean difference 0.02 -> 2e-3 * 0.01 / 0.06
    s2 = s.copy()
    s2[0] = 0.02 * N
    assert np.isclose(plan(s2[None, :], N, 1e-3, 0.01, 100)["h"][0], 2e-3 * 0.01 / 0.06)


def test_rbf_scores_by_an_independent_interpolant():
    """With the RBF interpolation, each exit's u0 value equals scipy's
    inverse-multiquadric interpolant of the side's stencil values (knot
    values, g at the boundary lattice points) at the clamped exit point."""
    from scipy.interpolate import RBFInterpolator
    g, c = _small(), Coefficients("varcoef")
    u0 = c.exact(g.x, g.y) + np.random.default_rng(4).normal(0.0, 0.01, g.n)
    cc = 1.5 * g.dx
    for k in (1, g.n // 2):
        gm, em = mixed_paths(c, g.box[k], (g.x[k], g.y[k]), k, 0, 60, 2e-3, 9)
        phi = path_scores(g, c, k, em, u0, ("rbf", cc))
        ex = exit_points(g, c, k, em)
        for p in range(60):
            o = int(ex["side"][p])
            s = g.side(k, "ENWS"[o])
            if s["boundary"]:
                assert phi[p] == em["Z"][p] + em["Y"][p] * ex["g_side"][p]
                continue
            vert = s["line"] == "x"
            along = em["y"][p] if vert else em["x"][p]
            a0, da = (g.y0, g.dy) if vert else (g.x0, g.dx)
            t = min(max((along - a0) / da, s["clo"]), s["chi"])
            qs = np.arange(s["clo"], s["chi"] + 1)
            vals = []
            for q in qs:
                if q == 0 or q == g.L:
                    px, py = (g.lattice_x(s["at"]), g.lattice_y(q)) if vert else (g.lattice_x(q), g.lattice_y(s["at"]))
                    vals.append(c.boundary(np.array([px]), np.array([py]))[0])
                else:
                    vals.append(u0[g.index[s["at"], q] if vert else g.index[q, s["at"]]])
            ip = RBFInterpolator((qs * da)[:, None], np.array(vals), kernel="inverse_multiquadric",
                                 epsilon=1.0 / cc, degree=-1)
            ref = em["Z"][p] + em["Y"][p] * ip(np.array([[t * da]]))[0]
            assert abs(phi[p] - ref) < 1e-9, (k, p)
