"""Pins of the oracle's paths, exits and rows against closed forms and invariants."""
import math

import numpy as np
import pytest
from scipy import special

from closed_forms import mean_exit_time_rectangle, harmonic_measure_top
from oracle.geometry import Geometry
from oracle.coeffs import Coefficients
from oracle.assemble import assemble, integrate_knot, exit_points, C_GM, to_csr
from oracle.philox import normals_for_draw
from oracle.solve import solve, rmse
from oracle.mlp import ExactGradientCV

SMALL = Geometry((0, 1, 0, 1), 2, 8, 4)
K_LOW = int(SMALL.index[8, 3])          # knot (1/2, 3/16), patch [0,1] x [0,1/2]
K_CROSS = int(SMALL.index[8, 8])        # crossing knot, patch = whole domain


def test_gobet_menozzi_constant():
    """c_GM = -zeta(1/2)/sqrt(2 pi); the paper prints it as 0.5826 (Sec. 2.3)."""
    assert C_GM == pytest.approx(-special.zeta(0.5) / math.sqrt(2 * math.pi), rel=1e-15)
    assert round(C_GM, 4) == 0.5826


@pytest.mark.parametrize("kind,param", [("poisson", ()), ("varcoef", ()), ("amplitude", (0.37,))])
def test_source_is_operator_of_exact_solution(kind, param):
    """f = L u* of problem (6), checked by central differences of u*."""
    c = Coefficients(kind, param)
    rng = np.random.default_rng(5)
    x, y = rng.uniform(0.05, 0.95, 50), rng.uniform(0.05, 0.95, 50)
    e = 1e-4
    u = c.exact
    uxx = (u(x + e, y) - 2 * u(x, y) + u(x - e, y)) / e ** 2
    uyy = (u(x, y + e) - 2 * u(x, y) + u(x, y - e)) / e ** 2
    uxy = (u(x + e, y + e) - u(x + e, y - e) - u(x - e, y + e) + u(x - e, y - e)) / (4 * e * e)
    ux = (u(x + e, y) - u(x - e, y)) / (2 * e)
    uy = (u(x, y + e) - u(x, y - e)) / (2 * e)
    sxx, sxy, syy = c.sigma(x, y)
    axx, axy, ayy = sxx * sxx + sxy * sxy, sxx * sxy + sxy * syy, sxy * sxy + syy * syy
    dx, dy = c.drift(x, y)
    Lu = 0.5 * axx * uxx + axy * uxy + 0.5 * ayy * uyy + dx * ux + dy * uy + c.reaction(x, y) * u(x, y)
    assert np.allclose(c.source(x, y), Lu, rtol=1e-5, atol=1e-5)


def test_eq43_source_and_gradient_by_finite_differences():
    """The Sec. 5 problem: f = Lap u* (eq. 42) and grad u* by central
    differences of eq. 43 over the domain [-100, 100]^2."""
    c = Coefficients("eq43")
    rng = np.random.default_rng(6)
    x, y = rng.uniform(-100, 100, 200), rng.uniform(-100, 100, 200)
    e = 1e-2
    u = c.exact
    lap = (u(x + e, y) + u(x - e, y) + u(x, y + e) + u(x, y - e) - 4 * u(x, y)) / e ** 2
    assert np.allclose(c.source(x, y), lap, rtol=0, atol=2e-7)
    gx, gy = c.grad_exact(x, y)
    assert np.allclose(gx, (u(x + e, y) - u(x - e, y)) / (2 * e), atol=2e-7)
    assert np.allclose(gy, (u(x, y + e) - u(x, y - e)) / (2 * e), atol=2e-7)
    # the generator of sigma = sqrt(2) I is the Laplacian: eq. 42 as written
    sxx, sxy, syy = c.sigma(x, y)
    assert np.allclose(0.5 * sxx * sxx, 1.0) and np.all(sxy == 0) and np.allclose(0.5 * syy * syy, 1.0)
    assert np.all(c.boundary(x, y) == u(x, y)) and np.all((u(x, y) > 2.3) & (u(x, y) < 3.7))


def test_mean_exit_time_series_and_gm_order():
    """h E[K] -> E[tau] of eq. (26).  With the exit-time family, b_k = h E[K]
    exactly (f = -1, g = 0).  Gobet-Menozzi (first order) sits within 3 SE
    plus O(h); the naive rule overshoots by O(sqrt h), far outside."""
    c = Coefficients("exittime")
    h, N = 1e-3, 16000
    ref = mean_exit_time_rectangle(0.5, 3 / 16, 1.0, 0.5)
    gm = assemble(SMALL, c, N, h, seed=1, exit_rule="gm", knots=[K_LOW])["rows"][K_LOW]
    nv = assemble(SMALL, c, N, h, seed=1, exit_rule="naive", knots=[K_LOW])["rows"][K_LOW]
    assert gm["b"] == pytest.approx(gm["diag"][0] * h / N, rel=1e-12)
    assert abs(gm["b"] - ref) < 3 * gm["se_b"] + 2 * h * ref
    assert nv["b"] - ref > 8 * nv["se_b"]


def test_mean_exit_time_scales_with_area():
    """Scaling the domain by 2 multiplies E[tau] by 4 (Sec. 3.3 after eq. 26)."""
    c = Coefficients("exittime")
    big = Geometry((0, 2, 0, 2), 2, 8, 4)
    h, N = 1e-3, 8000
    r1 = assemble(SMALL, c, N, h, seed=2, knots=[K_CROSS])["rows"][K_CROSS]
    r4 = assemble(big, c, N, 4 * h, seed=2, knots=[K_CROSS])["rows"][K_CROSS]
    # same random numbers, time step scaled with the area: identical paths up to scale
    assert r4["b"] == pytest.approx(4 * r1["b"], rel=1e-9)
    ref = mean_exit_time_rectangle(0.5, 0.5, 1, 1)
    assert abs(r1["b"] - ref) < 3 * r1["se_b"] + 2 * h * ref


def test_exit_side_probabilities_harmonic_measure():
    c = Coefficients("exittime")
    N = 16000
    r = assemble(SMALL, c, N, 1e-4, seed=3, knots=[K_LOW])["rows"][K_LOW]
    p_top = r["diag"][3] / N
    ref = harmonic_measure_top(0.5, 3 / 16, 1.0, 0.5)
    se = math.sqrt(ref * (1 - ref) / N)
    assert abs(p_top - ref) < 4 * se + 0.01
    # east and west sides are symmetric
    assert abs(r["diag"][2] - r["diag"][4]) / N < 4 * math.sqrt(0.1 / N)


def test_pdd_special_case_crossing_knot():
    """A patch equal to the whole domain reduces PDDSparse to plain PDD: the
    row is the identity and b is the Feynman-Kac estimate of u(x_k) (eq. 8)."""
    c = Coefficients("poisson")
    r = assemble(SMALL, c, 8000, 1e-3, seed=4, knots=[K_CROSS])["rows"][K_CROSS]
    assert list(r["cols"]) == [K_CROSS] and r["val"][0] == 1.0
    assert abs(r["b"] - 1.125) < 3 * r["se_b"] + 0.01


def test_row_sum_is_mass_sent_to_boundary():
    """With c = 0 (Y = 1) every path hands total weight 1 to knots or data, so
    sum_j G_kj equals the mean weight that reaches boundary data."""
    c = Coefficients("poisson")
    out = assemble(SMALL, c, 500, 1e-3, seed=5, keep_paths=True)
    for k, row in out["rows"].items():
        p = out["paths"][k]
        to_bdry = p["boundary"].astype(float)
        for side in range(4):
            sel = (~p["boundary"]) & (p["side"] == side)
            if not sel.any():
                continue
            name = "ENWS"[side]
            # lattice endpoints 0 and L on an interface line are boundary points
            for q, w in ((p["q0"], p["w0"]), (p["q0"] + 1, p["w1"])):
                on_b = sel & ((q == 0) | (q == SMALL.L))
                to_bdry = to_bdry + np.where(on_b, w, 0.0)
        assert row["val"].sum() == pytest.approx(to_bdry.mean(), abs=1e-13)


def test_constant_solution_identity():
    """u = 1 solves the problem with f = c, g = 1.  With Y_{n+1} = Y_n (1 + c h),
    Z telescopes to 1 - Y_K along every path, so G 1 = b holds path by path."""
    g = Geometry((0, 1, 0, 1), 4, 4, 2)
    c = Coefficients("constsol")
    R = to_csr(g, assemble(g, c, 300, 1e-3, seed=6)["rows"])
    rowsum = np.add.reduceat(R["val"], g.row_ptr[:-1])
    assert np.allclose(rowsum, R["b"], rtol=0, atol=1e-12 * R["mass"].max())
    # and the reaction makes Y < 1, so the identity is not trivial
    assert np.all(R["b"] < 1.0 - 1e-3)


def test_interpolation_weights_are_hat_functions():
    """Exit weights equal the hat functions max(0, 1 - |t - q|) on the line
    lattice and reproduce linear data exactly (eq. 21 with linear interpolation)."""
    c = Coefficients("poisson")
    k = K_LOW
    rng = np.random.default_rng(7)
    n = 2000
    x = rng.uniform(-0.2, 1.2, n)
    y = np.full(n, 0.5) + rng.uniform(0.0, 0.05, n)     # above the north side y = 1/2
    flags = np.zeros((n, 4), dtype=bool)
    flags[:, 1] = True
    rec = dict(x=x, y=y, flags=flags)
    ex = exit_points(SMALL, c, k, rec)
    assert np.all(ex["side"] == 1) and not ex["boundary"].any()
    t = np.clip(x / SMALL.dx, 0, SMALL.L)                # clamp range of the side is [0, L]
    for q_off, wname in ((0, "w0"), (1, "w1")):
        q = ex["q0"] + q_off
        assert np.allclose(ex[wname], np.maximum(0.0, 1.0 - np.abs(t - q)), atol=1e-12)
    lin = lambda q: 3.0 - 2.0 * q
    assert np.allclose(ex["w0"] * lin(ex["q0"]) + ex["w1"] * lin(ex["q0"] + 1), lin(t), atol=1e-12)


def test_corner_overshoot_goes_to_closest_line():
    """A diagonal overshoot is projected onto the closest side line (Sec. 3.3, Fig. 3)."""
    c = Coefficients("poisson")
    k = K_LOW                                          # patch [0,1] x [0,1/2]
    x = np.array([0.52, 0.51, 1.01])
    y = np.array([0.51, 0.53, 0.502])
    flags = np.array([[False, True, False, False]] * 2 + [[True, True, False, False]])
    ex = exit_points(SMALL, c, k, dict(x=x, y=y, flags=flags))
    assert list(ex["side"]) == [1, 1, 1]               # north is closer for the last one
    assert not ex["boundary"][2] and ex["q0"][2] == SMALL.L - 1 and ex["w1"][2] == 1.0
    flags2 = np.array([[True, True, False, False]])
    ex2 = exit_points(SMALL, c, k, dict(x=np.array([1.002]), y=np.array([0.51]), flags=flags2))
    assert ex2["side"][0] == 0 and ex2["boundary"][0]  # east (the domain boundary) is closer
    assert ex2["g_side"][0] == pytest.approx(c.boundary(np.array([1.0]), np.array([0.51]))[0])


def test_scalar_replay_of_paths():
    """A scalar, one-path-at-a-time replay of the step loop reproduces the
    vectorised paths bit for bit (exit step, exit iterate, Y, Z)."""
    c = Coefficients("varcoef")
    g = Geometry((0, 1, 0, 1), 3, 4, 2)
    k, h, seed, inst = 5, 1e-3, 11, 3
    rec = integrate_knot(g, c, k, 40, h, seed, inst, "gm")
    xlo, xhi, ylo, yhi = g.box[k]
    sq = math.sqrt(h)
    for p in range(40):
        x, y, Y, Z, n = g.x[k], g.y[k], 1.0, 0.0, 0
        while True:
            (a, b) = normals_for_draw(n // 2, np.array([p], dtype=np.uint64), k, inst, seed)
            nx, ny = (a if n % 2 == 0 else b)
            X1, Y1 = np.array([x]), np.array([y])
            sxx, sxy, syy = (v[0] for v in c.sigma(X1, Y1))
            dx, dy = (v[0] for v in c.drift(X1, Y1))
            cr, fs = c.reaction(X1, Y1)[0], c.source(X1, Y1)[0]
            dWx, dWy = sq * nx[0], sq * ny[0]
            x, y, Y, Z = (x + dx * h + (sxx * dWx + sxy * dWy),
                          y + dy * h + (sxy * dWx + syy * dWy),
                          Y * (1.0 + cr * h), Z - fs * Y * h)
            n += 1
            sh = lambda xx, yy, line: C_GM * math.sqrt(c.normal_diffusion(np.array([xx]), np.array([yy]), line)[0]) * sq
            yc, xc = min(max(y, ylo), yhi), min(max(x, xlo), xhi)
            if (x >= xhi - sh(xhi, yc, "x") or x <= xlo + sh(xlo, yc, "x")
                    or y >= yhi - sh(xc, yhi, "y") or y <= ylo + sh(xc, ylo, "y")):
                break
        assert rec["K"][p] == n
        assert (rec["x"][p], rec["y"][p], rec["Y"][p], rec["Z"][p]) == (x, y, Y, Z)


def test_manufactured_solution_poisson_small():
    """Interface error of the solved system (eq. 10: bias + statistical error).
    GM at h = 1e-3 with N = 1000 has RMSE near 0.02; the naive rule's O(sqrt h)
    bias is visibly larger."""
    c = Coefficients("poisson")
    ue = c.exact(SMALL.x, SMALL.y)
    res = {}
    for rule in ("gm", "naive"):
        R = to_csr(SMALL, assemble(SMALL, c, 1000, 1e-3, seed=0, exit_rule=rule)["rows"])
        u = solve(SMALL.row_ptr, SMALL.col_idx, R["val"], R["b"])
        res[rule] = rmse(u, ue)
    assert res["gm"] < 0.04
    assert res["naive"] > res["gm"]


def test_exact_gradient_control_variate():
    """F = sigma^T grad u* (eq. 37 with u0 = u*) keeps the mean (eq. 38) and
    collapses the score variance (eq. 11)."""
    c = Coefficients("poisson")
    k = K_LOW
    ue = c.exact(SMALL.x, SMALL.y)
    plain = assemble(SMALL, c, 2000, 1e-4, seed=8, knots=[k], u_ref=ue, keep_paths=True)
    cv = assemble(SMALL, c, 2000, 1e-4, seed=8, knots=[k], u_ref=ue, keep_paths=True,
                  cv=ExactGradientCV(c))
    rp, rc = plain["rows"][k], cv["rows"][k]
    # same paths: G identical, b shifted by mean(Xi)
    assert np.array_equal(rp["val"], rc["val"])
    xi = cv["paths"][k]["Xi"]
    assert rc["b"] - rp["b"] == pytest.approx(xi.mean(), abs=1e-12)
    assert abs(xi.mean()) < 4 * xi.std() / math.sqrt(xi.size)
    var_p, var_c = np.var(rp["score"]), np.var(rc["score"])
    assert var_p / var_c > 50
