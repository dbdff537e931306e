"""Point values inside the subdomains once the interfacial values are known, in float64.

After G u = b is solved, every subdomain square is an independent Dirichlet
problem for (6): its sides carry u, known on the interfaces from the knot
values (interpolated along each grid line) and g on the domain boundary
(Sec. 3.3).  The paper solves these problems pseudospectrally; the minimal
version here applies the Feynman-Kac formula (eq. 8, Sec. 2.2) to the square
itself:

    u(x) = E[ Z_tau + Y_tau u(X_tau) ],   tau = first exit from the square,

with the same Euler-Maruyama step, exit rules and side choice as the
assembly (the square plays the role of the patch; see ``assemble``).  The
exit point P is the projection onto the chosen side, its along-side
coordinate clamped to the side; u(P) is g(P) on a boundary side and, on an
interface side, the hat-function interpolation of the lattice values of the
side's line (lattice points on the domain boundary take g).

Which square: point (x, y) belongs to the square with lower-left corner
(x0 + a s, y0 + c s), s = (x1 - x0) / H, a = min(floor((x - x0) / s), H - 1)
(likewise c).  A point on a grid line lies on its square's boundary: its
value is the line interpolation itself, with no paths.

Stream: path p of point i draws from the counter (draw, p, i, instance + 2^31)
so point streams never coincide with the knot streams of an assembly whose
instance is below 2^31.
"""
import numpy as np

from .assemble import integrate_paths

POINT_STREAM = 1 << 31


def _square(geom, x, y):
    """Lattice box (xlo, xhi, ylo, yhi) of the square holding (x, y)."""
    m, H = geom.m, geom.H
    a = min(int(np.floor((x - geom.x0) / (geom.dx * m))), H - 1)
    c = min(int(np.floor((y - geom.y0) / (geom.dy * m))), H - 1)
    a, c = max(a, 0), max(c, 0)
    return a * m, (a + 1) * m, c * m, (c + 1) * m


def line_value(geom, coef, u_knots, vertical, at, along, lo, hi):
    """u at the point of the grid line (x = lattice at if vertical, else
    y = lattice at) with physical along-line coordinate ``along``: g on a
    boundary line; otherwise hat interpolation between the lattice points
    i0 and i0 + 1, t = lattice coordinate clamped to [lo, hi],
    i0 = min(floor t, hi - 1), w = t - i0."""
    L = geom.L
    if vertical:
        lpos, a0, d = geom.lattice_x(at), geom.y0, geom.dy
    else:
        lpos, a0, d = geom.lattice_y(at), geom.x0, geom.dx
    if at == 0 or at == L:
        a_lo = geom.lattice_y(lo) if vertical else geom.lattice_x(lo)
        a_hi = geom.lattice_y(hi) if vertical else geom.lattice_x(hi)
        pa = min(max(along, a_lo), a_hi)
        px, py = (lpos, pa) if vertical else (pa, lpos)
        return float(coef.boundary(np.array([px]), np.array([py]))[0])
    t = min(max((along - a0) / d, float(lo)), float(hi))
    i0 = min(np.floor(t), hi - 1.0)
    w = t - i0
    vals = []
    for q in (int(i0), int(i0) + 1):
        if q == 0 or q == L:
            qc = geom.lattice_y(q) if vertical else geom.lattice_x(q)
            px, py = (lpos, qc) if vertical else (qc, lpos)
            vals.append(float(coef.boundary(np.array([px]), np.array([py]))[0]))
        else:
            j = geom.index[at, q] if vertical else geom.index[q, at]
            vals.append(float(u_knots[j]))
    return (1.0 - w) * vals[0] + w * vals[1]


def evaluate(geom, coef, u_knots, points, n_paths, h, seed, instance=0, exit_rule="gm"):
    """u and its Monte Carlo standard error at each row of ``points`` (P x 2).

    Returns (u, se, K) with K the total path-steps per point."""
    pts = np.asarray(points, dtype=np.float64).reshape(-1, 2)
    P = pts.shape[0]
    u = np.empty(P)
    se = np.empty(P)
    steps = np.zeros(P, dtype=np.int64)
    for i in range(P):
        x, y = pts[i]
        xlo, xhi, ylo, yhi = _square(geom, x, y)
        box = (geom.lattice_x(xlo), geom.lattice_x(xhi), geom.lattice_y(ylo), geom.lattice_y(yhi))
        on_v = x in (box[0], box[1])
        on_h = y in (box[2], box[3])
        if on_v or on_h:
            if on_v:
                at = xlo if x == box[0] else xhi
                u[i] = line_value(geom, coef, u_knots, True, at, y, ylo, yhi)
            else:
                at = ylo if y == box[2] else yhi
                u[i] = line_value(geom, coef, u_knots, False, at, x, xlo, xhi)
            se[i] = 0.0
            continue
        rec = integrate_paths(coef, box, (x, y), i, instance + POINT_STREAM, n_paths, h, seed, exit_rule)
        steps[i] = rec["K"].sum()
        ex, ey, fl = rec["x"], rec["y"], rec["flags"]
        dist = np.stack([np.abs(ex - box[1]), np.abs(ey - box[3]), np.abs(ex - box[0]), np.abs(ey - box[2])],
                        axis=1)
        side = np.argmin(np.where(fl, dist, np.inf), axis=1)     # first minimum: E, N, W, S
        s = np.empty(ex.size)
        for p in range(ex.size):
            o = int(side[p])
            if o in (0, 2):
                val = line_value(geom, coef, u_knots, True, xhi if o == 0 else xlo, ey[p], ylo, yhi)
            else:
                val = line_value(geom, coef, u_knots, False, yhi if o == 1 else ylo, ex[p], xlo, xhi)
            s[p] = rec["Z"][p] + rec["Y"][p] * val
        N = s.size
        u[i] = s.sum() / N
        se[i] = np.sqrt(max(np.mean(s * s) - u[i] * u[i], 0.0) / N)
    return u, se, steps
