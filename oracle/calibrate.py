"""Phase II calibration of PDDSparse (Sec. 4.1-4.2, eqs. 32-41), in float64.

Test infrastructure only: the plain, slow definition the GPU calibration is
checked against.

Mixed Gobet-Menozzi / Euler-Maruyama trajectories (Sec. 4.1).  Every path of
knot x_i starts at x_i and is advanced by the Euler-Maruyama scheme of
``assemble`` (same stream, same step).  The first step at which the iterate is
no longer strictly inside the Gobet-Menozzi-shrunk patch gives the GM exit;
the path then simply continues until it leaves the closed patch, which gives
the naive (EM) exit.  Both exits are resolved as in the assembly (side choice,
projection, hat weights) and scored with the warm-up solution u0 as Dirichlet
data on the patch boundary: interpolated knot values on interface sides, g on
the domain boundary,

    phi = Z_K + Y_K u0(P_K),

and the control variate xi = Xi at the GM exit (eq. 37).  Per knot:

    bias bound     beta_i = |mean(phi_EM - phi_GM)| / 2                  (35, 36)
    variance       V_i = mean(phi_GM^2) - mean(phi_GM)^2
    correlation    rho_i^2 = cov(phi_GM, xi)^2 / (var(phi_GM) var(xi))   (39)
    time step      h_i = min(h0, 2 h0 eps / (3 |mean(phi_GM - phi_EM)|))  (40)
    paths          N_i = 9 V_i (1 - rho_i^2) / eps^2, rounded to the closest
                   multiple k N_job, k >= 1                               (41)

With interp=("rbf", c) the exit values of u0 use the cardinal functions of
the side's stencil, as the assembly's interpolation (eq. 21).

Readings: eq. 41 is read as 2 eps / 3 = 2 sqrt(V (1 - rho^2) / N_i); the
variance is the population variance of the N0 scores; rho^2 = 0 when either
variance is 0; h_i = h0 when the mean difference is 0.
"""
import numpy as np

from .assemble import exit_flags_box, exit_points, _lattice_target
from .philox import normals_for_draw

STATS_WIDTH = 8      # sum(phi_EM - phi_GM), sum phi_GM, sum phi_GM^2, sum xi, sum xi^2, sum phi_GM xi, sum K_GM, sum K_EM


def mixed_paths(coef, box, start, word2, instance, n_paths, h, seed, cv=None):
    """Integrate n_paths paths from ``start`` until they leave the closed
    rectangle box, recording on the way the state at the first
    Gobet-Menozzi exit.  Path p draws from the stream with counter
    (draw, p, word2, instance).  Returns (gm, em): two dicts of per-path
    arrays K, x, y, Y, Z, Xi, flags in the format of integrate_paths."""
    N = int(n_paths)
    sq = np.sqrt(h)
    path = np.arange(N, dtype=np.uint64)
    x = np.full(N, float(start[0]))
    y = np.full(N, float(start[1]))
    Y = np.ones(N)
    Z = np.zeros(N)
    Xi = np.zeros(N)
    K = np.zeros(N, dtype=np.int64)
    gm = {key: np.zeros(N) for key in ("x", "y", "Y", "Z", "Xi")}
    gm["K"] = np.zeros(N, dtype=np.int64)
    gm["flags"] = np.zeros((N, 4), dtype=bool)
    em = {key: np.zeros(N) for key in ("x", "y", "Y", "Z", "Xi")}
    em["K"] = np.zeros(N, dtype=np.int64)
    em["flags"] = np.zeros((N, 4), dtype=bool)
    gm_done = np.zeros(N, dtype=bool)
    alive = np.arange(N)
    j = 0
    while alive.size:
        normals = normals_for_draw(j, path[alive], word2, instance, seed)
        pos = np.arange(alive.size)          # positions of the running paths within this draw
        for half in range(2):
            idx = alive[pos]
            nx, ny = normals[half][0][pos], normals[half][1][pos]
            xa, ya, Ya = x[idx], y[idx], Y[idx]
            sxx, sxy, syy = coef.sigma(xa, ya)
            ddx, ddy = coef.drift(xa, ya)
            cr = coef.reaction(xa, ya)
            fs = coef.source(xa, ya)
            dWx, dWy = sq * nx, sq * ny
            if cv is not None:
                gx, gy = cv.grad(xa, ya)
                Xi[idx] = Xi[idx] - Ya * ((sxx * gx + sxy * gy) * dWx + (sxy * gx + syy * gy) * dWy)
            x[idx] = xa + ddx * h + (sxx * dWx + sxy * dWy)
            y[idx] = ya + ddy * h + (sxy * dWx + syy * dWy)
            Y[idx] = Ya * (1.0 + cr * h)
            Z[idx] = Z[idx] - fs * Ya * h
            K[idx] += 1
            # first Gobet-Menozzi exit (recorded once)
            fresh = ~gm_done[idx]
            if fresh.any():
                fE, fN, fW, fS = exit_flags_box(coef, box, x[idx], y[idx], h, "gm")
                hit = fresh & (fE | fN | fW | fS)
                hi = idx[hit]
                for key, arr in (("x", x), ("y", y), ("Y", Y), ("Z", Z), ("Xi", Xi), ("K", K)):
                    gm[key][hi] = arr[hi]
                gm["flags"][hi] = np.stack([fE[hit], fN[hit], fW[hit], fS[hit]], axis=1)
                gm_done[hi] = True
            # naive exit: the path ends
            fE, fN, fW, fS = exit_flags_box(coef, box, x[idx], y[idx], h, "naive")
            out = fE | fN | fW | fS
            oi = idx[out]
            for key, arr in (("x", x), ("y", y), ("Y", Y), ("Z", Z), ("Xi", Xi), ("K", K)):
                em[key][oi] = arr[oi]
            em["flags"][oi] = np.stack([fE[out], fN[out], fW[out], fS[out]], axis=1)
            pos = pos[~out]
            if pos.size == 0:
                break
        alive = alive[pos]
        j += 1
    return gm, em


def path_scores(geom, coef, k, rec, u0, interp=None):
    """phi = Z_K + Y_K u0(P_K) per path, with P_K the resolved exit point of
    ``rec`` (exit_points) and u0 the interpolated knot values u0[j] on
    interface sides (g at boundary lattice points), g on boundary sides.
    interp: None for the hat weights, ("rbf", c) for the cardinal functions
    of the side's stencil (the assembly's interpolation, eq. 21)."""
    ex = exit_points(geom, coef, k, rec, interp)
    uex = np.where(ex["boundary"], ex["g_side"], 0.0)
    for p in np.nonzero(~ex["boundary"])[0]:
        side = int(ex["side"][p])
        s = geom.side(k, ("E", "N", "W", "S")[side])
        if interp is not None:
            pairs = ex["contribs"][p]
        else:
            q0 = int(ex["q0"][p])
            pairs = ((q0, ex["w0"][p]), (q0 + 1, ex["w1"][p]))
        val = 0.0
        for q, w in pairs:
            j = _lattice_target(geom, k, side, q)
            if j < 0:
                if s["line"] == "x":
                    px, py = geom.lattice_x(s["at"]), geom.lattice_y(q)
                else:
                    px, py = geom.lattice_x(q), geom.lattice_y(s["at"])
                val += w * float(coef.boundary(np.array([px]), np.array([py]))[0])
            else:
                val += w * float(u0[j])
        uex[p] = val
    return rec["Z"] + rec["Y"] * uex


def calibrate_knot(geom, coef, k, u0, n_paths, h, seed, instance=0, cv=None, interp=None):
    """STATS_WIDTH sums of knot k from n_paths mixed trajectories."""
    gm, em = mixed_paths(coef, geom.box[k], (geom.x[k], geom.y[k]), k, instance, n_paths, h, seed, cv)
    phi_gm = path_scores(geom, coef, k, gm, u0, interp)
    phi_em = path_scores(geom, coef, k, em, u0, interp)
    xi = gm["Xi"]
    return np.array([np.sum(phi_em - phi_gm), np.sum(phi_gm), np.sum(phi_gm * phi_gm), np.sum(xi),
                     np.sum(xi * xi), np.sum(phi_gm * xi), float(gm["K"].sum()), float(em["K"].sum())])


def calibrate(geom, coef, u0, n_paths, h, seed, instance=0, cv=None, knots=None, interp=None):
    """Per-knot STATS_WIDTH sums (rows in knot order; only ``knots`` if given)."""
    ks = range(geom.n) if knots is None else knots
    return {int(k): calibrate_knot(geom, coef, int(k), u0, n_paths, h, seed, instance, cv, interp) for k in ks}


def plan(stats, n_paths, h0, eps, n_job, h0_cal=None):
    """Eqs. 35-41 from the sums: (h_i, N_i, bias bound, variance, rho^2) per
    knot.  stats: array [n, STATS_WIDTH].  h0_cal is the calibration step h0'
    of the sums (eq. 40's numerator; default h0, as in the Sec. 4.3
    pseudocode), h0 the cap of eq. 40."""
    h0_cal = h0 if h0_cal is None else h0_cal
    stats = np.asarray(stats, dtype=np.float64).reshape(-1, STATS_WIDTH)
    N = float(n_paths)
    mdiff = stats[:, 0] / N
    mphi = stats[:, 1] / N
    var = np.maximum(stats[:, 2] / N - mphi * mphi, 0.0)
    mxi = stats[:, 3] / N
    varxi = np.maximum(stats[:, 4] / N - mxi * mxi, 0.0)
    cov = stats[:, 5] / N - mphi * mxi
    denom = var * varxi
    rho2 = np.where(denom > 0.0, np.minimum(cov * cov / np.where(denom > 0.0, denom, 1.0), 1.0), 0.0)
    bias = 0.5 * np.abs(mdiff)
    with np.errstate(divide="ignore"):
        h = np.where(mdiff != 0.0, np.minimum(h0, 2.0 * h0_cal * eps / (3.0 * np.abs(mdiff))), h0)
    n_raw = 9.0 * var * (1.0 - rho2) / (eps * eps)
    k = np.maximum(np.floor(n_raw / n_job + 0.5), 1.0)
    return dict(h=h, n_paths=(k * n_job).astype(np.int64), bias=bias, var=var, rho2=rho2)
