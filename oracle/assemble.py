"""Monte Carlo assembly of the PDDSparse rows (eqs. 8-9, 20-25), in float64.

For every knot x_k, N_k paths of the diffusion of (9) start at x_k and are
advanced by the Euler-Maruyama scheme (Sec. 2.3) until they first leave the
knot's patch (eq. 15).  With coefficients frozen at the left point X_n and
Brownian increment dW_n = sqrt(h) xi_n (xi_n from the stream of ``philox``):

    X_{n+1}  = X_n + d(X_n) h + sigma(X_n) dW_n
    Y_{n+1}  = Y_n (1 + c(X_n) h)
    Z_{n+1}  = Z_n - f(X_n) Y_n h
    Xi_{n+1} = Xi_n - Y_n F(X_n) . dW_n,     F = sigma^T grad v   (eq. 37)

The exit test is applied to X_{n+1}, never to the start point, so every path
takes at least one step.  Readings taken where the paper is terse:

* Naive rule (Sec. 2.3): exit when X_{n+1} is strictly outside the closed
  patch.  Gobet-Menozzi rule (Sec. 2.3): exit when X_{n+1} is not strictly
  inside the patch shrunk, side by side, by c_GM sqrt(a_nn(P_O)) sqrt(h), with
  a_nn = N^T A N the normal diffusion of side O evaluated at the projection P_O
  of X_{n+1} onto the side (its along-side coordinate clamped to the side) and
  c_GM = -zeta(1/2)/sqrt(2 pi) = 0.5825971579390106 (the paper prints 0.5826).
* Exit side: among the sides that the test flags, the one whose grid line is
  closest to X_{n+1}; ties go to the first in the order E, N, W, S.  The exit
  point is the normal projection onto that line, its along-line coordinate
  clamped to the extended stencil range (Sec. 3.3, Fig. 3).
* Interpolation (eq. 21 with the linear scheme footnote 8 allows): hat
  functions on the line's knot lattice.  With t the along-line lattice
  coordinate of the exit point, i0 = min(floor t, chi - 1) and w = t - i0; the
  lattice points i0 and i0 + 1 receive 1 - w and w.  Interior lattice points
  are unknowns (row entries of G); lattice points on the boundary contribute
  Y w g(point) to b.
* RBF interpolation (eq. 21 with the cardinal functions of eq. 5, the scheme
  of Sec. 2.1 and 5.1), selected by interp=("rbf", c): every lattice point
  clo..chi of the side's extended stencil receives its cardinal weight
  H_q(z) at the clamped exit point z (``rbf.cardinal``), with the same split
  into unknowns and boundary data as the hat weights.
* Score split (eqs. 24-25): b_k collects Z_K + Xi_K and Y_K times every
  boundary datum reached; G_kj = -mean(Y_K w_j); G_kk = 1; contributions of
  one column through two sides are summed.  The control variate adds to b only.
"""
import numpy as np

from .philox import normals_for_draw
from .rbf import cardinal

C_GM = 0.5825971579390106          # -zeta(1/2) / sqrt(2 pi), Gobet-Menozzi constant
SIDE_CODE = {"E": 0, "N": 1, "W": 2, "S": 3}
DIAG_WIDTH = 8                      # sum K, N, exits E/N/W/S, sum s, sum s^2


def _gm_shifts(coef, box, x, y, h):
    """Per-path inward shifts (dE, dN, dW, dS) of the Gobet-Menozzi rule for the
    rectangle box = (xlo, xhi, ylo, yhi)."""
    xlo, xhi, ylo, yhi = box
    yc = np.minimum(np.maximum(y, ylo), yhi)
    xc = np.minimum(np.maximum(x, xlo), xhi)
    sh = np.sqrt(h)
    dE = C_GM * np.sqrt(coef.normal_diffusion(np.full_like(y, xhi), yc, "x")) * sh
    dW = C_GM * np.sqrt(coef.normal_diffusion(np.full_like(y, xlo), yc, "x")) * sh
    dN = C_GM * np.sqrt(coef.normal_diffusion(xc, np.full_like(x, yhi), "y")) * sh
    dS = C_GM * np.sqrt(coef.normal_diffusion(xc, np.full_like(x, ylo), "y")) * sh
    return dE, dN, dW, dS


def exit_flags_box(coef, box, x, y, h, exit_rule):
    """Boolean flags (E, N, W, S) of the sides of box = (xlo, xhi, ylo, yhi)
    that the exit test trips on."""
    xlo, xhi, ylo, yhi = box
    if exit_rule == "naive":
        return x > xhi, y > yhi, x < xlo, y < ylo
    dE, dN, dW, dS = _gm_shifts(coef, box, x, y, h)
    return x >= xhi - dE, y >= yhi - dN, x <= xlo + dW, y <= ylo + dS


def exit_flags(coef, geom, k, x, y, h, exit_rule):
    """Boolean flags (E, N, W, S) of the sides of knot k's patch the exit test trips on."""
    return exit_flags_box(coef, geom.box[k], x, y, h, exit_rule)


def integrate_paths(coef, box, start, word2, instance, n_paths, h, seed, exit_rule, cv=None):
    """Run n_paths paths from ``start`` to their first exit from the rectangle
    box = (xlo, xhi, ylo, yhi).  Path p draws from the stream with counter
    (draw, p, word2, instance).

    Returns a dict of per-path arrays: K (steps, exit step included), x, y
    (the exit iterate X_K before projection), Y, Z, Xi, and flags (N x 4 bool,
    sides tripped at the exit step).
    """
    N = int(n_paths)
    sq = np.sqrt(h)
    path = np.arange(N, dtype=np.uint64)
    x = np.full(N, float(start[0]))
    y = np.full(N, float(start[1]))
    Y = np.ones(N)
    Z = np.zeros(N)
    Xi = np.zeros(N)
    K = np.zeros(N, dtype=np.int64)
    flags = np.zeros((N, 4), dtype=bool)
    alive = np.arange(N)
    j = 0
    while alive.size:
        first, second = normals_for_draw(j, path[alive], word2, instance, seed)
        idx = alive
        for half, (nx, ny) in enumerate((first, second)):
            if half == 1:
                nx, ny = nx[keep], ny[keep]
            xa, ya, Ya = x[idx], y[idx], Y[idx]
            sxx, sxy, syy = coef.sigma(xa, ya)
            ddx, ddy = coef.drift(xa, ya)
            cr = coef.reaction(xa, ya)
            fs = coef.source(xa, ya)
            dWx, dWy = sq * nx, sq * ny
            if cv is not None:
                gx, gy = cv.grad(xa, ya)
                Fx = sxx * gx + sxy * gy
                Fy = sxy * gx + syy * gy
                Xi[idx] = Xi[idx] - Ya * (Fx * dWx + Fy * dWy)
            x[idx] = xa + ddx * h + (sxx * dWx + sxy * dWy)
            y[idx] = ya + ddy * h + (sxy * dWx + syy * dWy)
            Y[idx] = Ya * (1.0 + cr * h)
            Z[idx] = Z[idx] - fs * Ya * h
            K[idx] += 1
            fE, fN, fW, fS = exit_flags_box(coef, box, x[idx], y[idx], h, exit_rule)
            out = fE | fN | fW | fS
            flags[idx[out]] = np.stack([fE[out], fN[out], fW[out], fS[out]], axis=1)
            keep = ~out
            idx = idx[keep]
            if idx.size == 0:
                break
        alive = idx
        j += 1
    return dict(K=K, x=x, y=y, Y=Y, Z=Z, Xi=Xi, flags=flags)


def integrate_knot(geom, coef, k, n_paths, h, seed, instance, exit_rule, cv=None):
    """Run n_paths paths from knot k to their first exit from its patch
    (stream counter (draw, path, k, instance))."""
    return integrate_paths(coef, geom.box[k], (geom.x[k], geom.y[k]), k, instance, n_paths, h, seed,
                           exit_rule, cv)


def exit_points(geom, coef, k, rec, interp=None):
    """Side choice, projection and interpolation weights for every path.

    Returns dict(side (0..3 for E, N, W, S), boundary (bool), g_side (g at
    the projected point on a boundary side, else 0), and two interface lattice
    contributions (q0, w0), (q1, w1): along-line lattice coordinates and
    weights (w0 = w1 = 0 on boundary sides).  With interp=("rbf", c) it also
    holds ``contribs``: per path the list of (q, H_q) over the side stencil
    (empty on boundary sides), which then replaces the hat pair.
    """
    xlo, xhi, ylo, yhi = geom.box[k]
    x, y, fl = rec["x"], rec["y"], rec["flags"]
    dist = np.stack([np.abs(x - xhi), np.abs(y - yhi), np.abs(x - xlo), np.abs(y - ylo)], axis=1)
    dist = np.where(fl, dist, np.inf)
    side = np.argmin(dist, axis=1)                   # first minimum: order E, N, W, S
    N = x.size
    boundary = np.zeros(N, dtype=bool)
    g_side = np.zeros(N)
    q0 = np.zeros(N, dtype=np.int64)
    w0 = np.zeros(N)
    w1 = np.zeros(N)
    line_pos = np.zeros(N)                           # physical coordinate of the side line
    along = np.zeros(N)                              # physical along-line coordinate
    clo = np.zeros(N)
    chi = np.zeros(N)
    for o, name in enumerate(("E", "N", "W", "S")):
        sel = side == o
        if not sel.any():
            continue
        s = geom.side(k, name)
        if s["line"] == "x":
            line_pos[sel] = geom.lattice_x(s["at"])
            along[sel] = y[sel]
        else:
            line_pos[sel] = geom.lattice_y(s["at"])
            along[sel] = x[sel]
        boundary[sel] = s["boundary"]
        clo[sel] = s["clo"]
        chi[sel] = s["chi"]
    ex_line = (side == 0) | (side == 2)              # E/W sides: line x = const, along = y
    a0 = np.where(ex_line, geom.y0, geom.x0)
    a1 = np.where(ex_line, geom.y1, geom.x1)
    da = np.where(ex_line, geom.dy, geom.dx)
    # boundary sides: g at the projection, clamped to the domain
    pb = np.minimum(np.maximum(along, a0), a1)
    gx = np.where(ex_line, line_pos, pb)
    gy = np.where(ex_line, pb, line_pos)
    if boundary.any():
        g_side[boundary] = coef.boundary(gx[boundary], gy[boundary])
    # interface sides: lattice coordinate, clamp, hat weights
    t = (along - a0) / da
    t = np.minimum(np.maximum(t, clo), chi)
    i0 = np.minimum(np.floor(t), chi - 1.0)
    w = t - i0
    iface = ~boundary
    q0[iface] = i0[iface].astype(np.int64)
    w0[iface] = 1.0 - w[iface]
    w1[iface] = w[iface]
    out = dict(side=side, boundary=boundary, g_side=g_side, q0=q0, w0=w0, w1=w1,
               line_pos=line_pos, ex_line=ex_line)
    if interp is not None:
        kind, c = interp
        if kind != "rbf":
            raise ValueError(kind)
        contribs = []
        for p in range(N):
            if boundary[p]:
                contribs.append([])
                continue
            qs = np.arange(int(clo[p]), int(chi[p]) + 1)
            # nodes and exit point measured from the stencil's first point
            H = cardinal((qs - clo[p]) * da[p], [(t[p] - clo[p]) * da[p]], c)[:, 0]
            contribs.append(list(zip(qs.tolist(), H.tolist())))
        out["contribs"] = contribs
    return out


def _pairs(ex, p):
    """The (lattice coordinate, weight) contributions of interface path p."""
    if "contribs" in ex:
        return ex["contribs"][p]
    q0 = int(ex["q0"][p])
    return ((q0, ex["w0"][p]), (q0 + 1, ex["w1"][p]))


def _lattice_target(geom, k, side, q):
    """Knot index of lattice point q on the line of ``side`` of knot k's patch,
    or -1 when the point lies on the domain boundary."""
    s = geom.side(k, ("E", "N", "W", "S")[side])
    if q <= 0 or q >= geom.L:
        return -1
    if s["line"] == "x":
        return int(geom.index[s["at"], q])
    return int(geom.index[q, s["at"]])


def knot_row(geom, coef, k, rec, ex, u_ref=None):
    """Turn the exit records of one knot into its row of G and its b entry.

    Returns dict(cols, val, se_val, b, se_b, mass, diag) with cols the pattern
    columns of row k (ascending), val the entries (diagonal exactly 1),
    se_* the Monte Carlo standard errors of the entries, mass the mean absolute
    contribution per path (scale of the rounding tolerance) and diag the
    DIAG_WIDTH diagnostics.
    """
    N = rec["K"].size
    Yk = rec["Y"]
    bpath = rec["Z"] + rec["Xi"] + Yk * ex["g_side"]   # per-path b contribution
    abs_path = np.abs(rec["Z"]) + np.abs(rec["Xi"]) + np.abs(Yk * ex["g_side"])
    cols = geom.col_idx[geom.row_ptr[k]:geom.row_ptr[k + 1]]
    pos_of = {int(c): i for i, c in enumerate(cols)}
    gsum = np.zeros(cols.size)
    gsq = np.zeros(cols.size)
    uref_part = np.zeros(N)
    for p in range(N):
        if ex["boundary"][p]:
            continue
        side = int(ex["side"][p])
        s = geom.side(k, ("E", "N", "W", "S")[side])
        for q, w in _pairs(ex, p):
            contrib = Yk[p] * w
            j = _lattice_target(geom, k, side, q)
            if j < 0:
                if s["line"] == "x":
                    px, py = geom.lattice_x(s["at"]), geom.lattice_y(q)
                else:
                    px, py = geom.lattice_x(q), geom.lattice_y(s["at"])
                gval = float(coef.boundary(np.array([px]), np.array([py]))[0])
                bpath[p] += contrib * gval
                abs_path[p] += abs(contrib * gval)
            else:
                i = pos_of[j]
                gsum[i] -= contrib
                gsq[i] += contrib * contrib
                abs_path[p] += abs(contrib)
                if u_ref is not None:
                    uref_part[p] += contrib * u_ref[j]
    val = gsum / N
    se_val = np.sqrt(np.maximum(gsq / N - val * val, 0.0) / N)
    kk = pos_of[k]
    val[kk] = 1.0
    se_val[kk] = 0.0
    b = bpath.sum() / N
    se_b = np.sqrt(max(np.mean(bpath * bpath) - b * b, 0.0) / N)
    s = bpath + uref_part
    diag = np.zeros(DIAG_WIDTH)
    diag[0] = rec["K"].sum()
    diag[1] = N
    for o in range(4):
        diag[2 + o] = np.count_nonzero(ex["side"] == o)
    diag[6] = s.sum()
    diag[7] = (s * s).sum()
    return dict(cols=cols, val=val, se_val=se_val, b=b, se_b=se_b,
                mass=abs_path.mean(), diag=diag, score=s)


def assemble(geom, coef, n_paths, h, seed, instance=0, exit_rule="gm", cv=None,
             u_ref=None, knots=None, keep_paths=False, interp=None):
    """Assemble the rows of G and entries of b for the given knots (all by default).

    n_paths: int, or per-knot array of length geom.n; h likewise (the knot's
    own time step h_i of eq. 40).  interp: None for the hat weights,
    ("rbf", c) for the inverse-multiquadric cardinal weights.
    Returns dict(rows={k: knot_row(...)}, and the per-path records if keep_paths).
    """
    if exit_rule not in ("naive", "gm"):
        raise ValueError(exit_rule)
    ks = range(geom.n) if knots is None else [int(k) for k in knots]
    npk = np.broadcast_to(np.asarray(n_paths, dtype=np.int64), (geom.n,))
    hk = np.broadcast_to(np.asarray(h, dtype=np.float64), (geom.n,))
    rows, paths = {}, {}
    for k in ks:
        rec = integrate_knot(geom, coef, k, npk[k], float(hk[k]), seed, instance, exit_rule, cv)
        ex = exit_points(geom, coef, k, rec, interp)
        rows[k] = knot_row(geom, coef, k, rec, ex, u_ref)
        if keep_paths:
            rec.update(ex)
            paths[k] = rec
    out = dict(rows=rows)
    if keep_paths:
        out["paths"] = paths
    return out


def to_csr(geom, rows):
    """Full CSR value array and b vector from a dict of all rows."""
    val = np.empty(geom.nnz)
    b = np.empty(geom.n)
    se_val = np.empty(geom.nnz)
    se_b = np.empty(geom.n)
    mass = np.empty(geom.n)
    diag = np.empty((geom.n, DIAG_WIDTH))
    for k in range(geom.n):
        r = rows[k]
        a, e = geom.row_ptr[k], geom.row_ptr[k + 1]
        val[a:e] = r["val"]
        se_val[a:e] = r["se_val"]
        b[k], se_b[k], mass[k] = r["b"], r["se_b"], r["mass"]
        diag[k] = r["diag"]
    return dict(val=val, b=b, se_val=se_val, se_b=se_b, mass=mass, diag=diag)
