"""Pseudospectral solves inside the subdomains and the global u0(x), in float64.

Test infrastructure only: the plain definition the GPU subdomain solves are
checked against.  Nothing outside tests/ and the benchmark's CPU baseline
imports it.

Once the knot values are known (the solve of G u = b), every subdomain square
is an independent Dirichlet problem for (6): its sides carry u, interpolated
along the grid lines from the knot values on interfaces, and g on the domain
boundary (Sec. 3.3).  The paper solves these problems with the pseudospectral
method (Sec. 3.3, Sec. 5.1) and uses the resulting global solution u0(x) for
the pathwise control variate F = sigma^T grad u0 kept on a look-up table
(Sec. 4.2, eq. 37; Sec. 4.3, Phase I).

Discretisation (Chebyshev collocation):

* On each square, the tensor grid of the p + 1 Chebyshev-Gauss-Lobatto points
  per direction, t_j = -cos(pi j / p), j = 0..p (ascending), mapped affinely
  onto the square's sides.  Grid values U[i, j] = u(x_i, y_j).
* Differentiation: D_ij = (w_j / w_i) / (t_i - t_j) for i != j and
  D_ii = -sum_{j != i} D_ij, with the barycentric weights w_j = (-1)^j,
  halved at both ends (the Chebyshev differentiation matrix in barycentric
  form); on a side of length S the first derivative is (2 / S) D, the second
  its square.
* Collocation: at every interior grid point the operator of (6),
  1/2 a_xx u_xx + a_xy u_xy + 1/2 a_yy u_yy + d . grad u + c u = f with
  A = sigma sigma^T and the coefficients at that point; at every boundary
  grid point u equals the side value.  The (p + 1)^2 linear system is solved
  directly (LAPACK).

Side values (readings, stated in the library's header too):

* A side on the domain boundary takes g at its grid points.
* An interface side takes its line's lattice values (knot values; g at the
  two lattice points on the domain boundary) interpolated to its grid points
  over the stencil of the side: the line's lattice points from the side's
  lower end minus ``ext`` to its upper end plus ``ext``, clipped to the domain
  (the extended side stencils of Sec. 3.3 and 5.1).  Interpolation: hat
  functions on the lattice (i0 = min(floor t, chi - 1), w = t - i0) or the
  inverse-multiquadric cardinal functions of that stencil (eqs. 1-5,
  ``rbf.cardinal``).
* The four corner points of a square take the value of its lower and upper
  (horizontal) sides.

The global solution: u0 at a point is the 2-D barycentric Chebyshev
interpolant of its square's grid values (the square of a point is the one
with lower-left corner index min(floor((x - x0) / S), H - 1) per direction,
as for the point evaluation in ``evaluate``); grad u0 interpolates the grid
derivatives (2/S) D U and U ((2/S) D)^T the same way.
"""
import numpy as np

from .rbf import cardinal


def cheb_nodes(p):
    """Chebyshev-Gauss-Lobatto points on [-1, 1], ascending."""
    return -np.cos(np.pi * np.arange(p + 1) / p)


def bary_weights(p):
    """Barycentric weights of the Chebyshev-Gauss-Lobatto points."""
    w = (-1.0) ** np.arange(p + 1)
    w[0] *= 0.5
    w[-1] *= 0.5
    return w


def diff_matrix(p):
    """First-derivative collocation matrix on [-1, 1] (barycentric form, the
    diagonal from the negative row sum)."""
    t = cheb_nodes(p)
    w = bary_weights(p)
    dt = t[:, None] - t[None, :]
    np.fill_diagonal(dt, 1.0)
    D = (w[None, :] / w[:, None]) / dt
    np.fill_diagonal(D, 0.0)
    np.fill_diagonal(D, -D.sum(axis=1))
    return D


def square_grid(box, p):
    """Grid coordinates (x_i, y_j) of the square box = (xa, xb, ya, yb)."""
    xa, xb, ya, yb = box
    t = cheb_nodes(p)
    return xa + (xb - xa) * (t + 1.0) / 2.0, ya + (yb - ya) * (t + 1.0) / 2.0


def solve_square(coef, box, p, side_value):
    """Collocation solve of (6) on the square box with Dirichlet data.

    side_value(side, x, y) returns the boundary values at the points (x, y) of
    side 'S', 'N' (horizontal, all p + 1 points) or 'W', 'E' (vertical,
    interior points only).  Returns the grid values U[i, j]."""
    xa, xb, ya, yb = box
    x, y = square_grid(box, p)
    D = diff_matrix(p)
    Dx = (2.0 / (xb - xa)) * D
    Dy = (2.0 / (yb - ya)) * D
    I = np.eye(p + 1)
    X, Y = np.meshgrid(x, y, indexing="ij")            # X[i, j] = x_i, Y[i, j] = y_j
    xf, yf = X.ravel(), Y.ravel()                      # flat index i (p + 1) + j
    sxx, sxy, syy = coef.sigma(xf, yf)
    axx = sxx * sxx + sxy * sxy
    axy = sxx * sxy + sxy * syy
    ayy = sxy * sxy + syy * syy
    ddx, ddy = coef.drift(xf, yf)
    cr = coef.reaction(xf, yf)
    Dxx, Dyy = np.kron(Dx @ Dx, I), np.kron(I, Dy @ Dy)
    Dxk, Dyk = np.kron(Dx, I), np.kron(I, Dy)
    A = (0.5 * axx[:, None] * Dxx + axy[:, None] * np.kron(Dx, Dy) + 0.5 * ayy[:, None] * Dyy
         + ddx[:, None] * Dxk + ddy[:, None] * Dyk + np.diag(cr))
    rhs = coef.source(xf, yf).astype(np.float64)
    bnd = np.zeros((p + 1, p + 1), dtype=bool)
    bnd[0, :] = bnd[-1, :] = bnd[:, 0] = bnd[:, -1] = True
    val = np.zeros((p + 1, p + 1))
    val[:, 0] = side_value("S", x, np.full(p + 1, ya))
    val[:, -1] = side_value("N", x, np.full(p + 1, yb))
    val[0, 1:-1] = side_value("W", np.full(p - 1, xa), y[1:-1])
    val[-1, 1:-1] = side_value("E", np.full(p - 1, xb), y[1:-1])
    b = bnd.ravel()
    A[b, :] = 0.0
    A[b, b] = 1.0
    rhs[b] = val.ravel()[b]
    return np.linalg.solve(A, rhs).reshape(p + 1, p + 1)


def line_values(geom, coef, u_knots, vertical, at, lo, hi, along, interp=None):
    """u at physical along-line coordinates ``along`` of the grid line at
    lattice coordinate ``at`` (x = const if vertical), interpolated over the
    stencil [max(lo - ext, 0), min(hi + ext, L)] of the side [lo, hi]."""
    L, e = geom.L, geom.ext
    clo, chi = max(0, lo - e), min(L, hi + e)
    q = np.arange(clo, chi + 1)
    if vertical:
        px, py = np.full(q.size, geom.lattice_x(at)), geom.lattice_y(q)
        a0, d = geom.y0, geom.dy
    else:
        px, py = geom.lattice_x(q), np.full(q.size, geom.lattice_y(at))
        a0, d = geom.x0, geom.dx
    vals = np.empty(q.size)
    edge = (q == 0) | (q == L)
    vals[edge] = coef.boundary(px[edge], py[edge])
    inner = ~edge
    idx = geom.index[at, q[inner]] if vertical else geom.index[q[inner], at]
    vals[inner] = np.asarray(u_knots, dtype=np.float64)[idx]
    along = np.asarray(along, dtype=np.float64)
    if interp is not None and interp[0] == "rbf":
        nodes = a0 + q * d
        return cardinal(nodes, along, interp[1]).T @ vals
    t = np.clip((along - a0) / d, clo, chi)
    i0 = np.minimum(np.floor(t), chi - 1.0)
    w = t - i0
    k = (i0 - clo).astype(np.int64)
    return (1.0 - w) * vals[k] + w * vals[k + 1]


def subdomain_boxes(geom):
    """Lattice boxes (xlo, xhi, ylo, yhi) of the H x H squares, index a + H c."""
    m, H = geom.m, geom.H
    return [(a * m, (a + 1) * m, c * m, (c + 1) * m) for c in range(H) for a in range(H)]


def solve_subdomains(geom, coef, u_knots, p, interp=None):
    """Grid values of every square: array [H^2, p + 1, p + 1], square a + H c
    (a along x, c along y)."""
    L = geom.L
    out = []
    for (xlo, xhi, ylo, yhi) in subdomain_boxes(geom):
        box = (geom.lattice_x(xlo), geom.lattice_x(xhi), geom.lattice_y(ylo), geom.lattice_y(yhi))

        def side_value(s, x, y, xlo=xlo, xhi=xhi, ylo=ylo, yhi=yhi):
            if s in ("S", "N"):
                at = ylo if s == "S" else yhi
                if at == 0 or at == L:
                    return coef.boundary(x, y)
                return line_values(geom, coef, u_knots, False, at, xlo, xhi, x, interp)
            at = xlo if s == "W" else xhi
            if at == 0 or at == L:
                return coef.boundary(x, y)
            return line_values(geom, coef, u_knots, True, at, ylo, yhi, y, interp)

        out.append(solve_square(coef, box, p, side_value))
    return np.array(out)


def grid_gradients(geom, U, p):
    """(dU/dx, dU/dy) on every square's grid: (2/S) D U and U ((2/S) D)^T."""
    D = diff_matrix(p)
    sx = (geom.x1 - geom.x0) / geom.H
    sy = (geom.y1 - geom.y0) / geom.H
    gx = np.einsum("ik,skj->sij", (2.0 / sx) * D, U)
    gy = np.einsum("sik,jk->sij", U, (2.0 / sy) * D)
    return gx, gy


def _lagrange_row(t, w, z):
    """Barycentric Lagrange basis l_i(z) of the nodes t, exact at a node."""
    diff = z - t
    hit = np.flatnonzero(diff == 0.0)
    if hit.size:
        out = np.zeros(t.size)
        out[hit[0]] = 1.0
        return out
    r = w / diff
    return r / r.sum()


def interpolate(geom, fields, p, points):
    """Values of grid fields (each [H^2, p + 1, p + 1]) at the rows of
    ``points`` (P x 2) by 2-D barycentric interpolation on the square of each
    point.  Returns an array [len(fields), P]."""
    pts = np.asarray(points, dtype=np.float64).reshape(-1, 2)
    t = cheb_nodes(p)
    w = bary_weights(p)
    H = geom.H
    sx = (geom.x1 - geom.x0) / H
    sy = (geom.y1 - geom.y0) / H
    out = np.empty((len(fields), pts.shape[0]))
    for k, (x, y) in enumerate(pts):
        a = min(max(int(np.floor((x - geom.x0) / sx)), 0), H - 1)
        c = min(max(int(np.floor((y - geom.y0) / sy)), 0), H - 1)
        xa = geom.x0 + a * sx
        ya = geom.y0 + c * sy
        lx = _lagrange_row(t, w, 2.0 * (x - xa) / sx - 1.0)
        ly = _lagrange_row(t, w, 2.0 * (y - ya) / sy - 1.0)
        for f, F in enumerate(fields):
            out[f, k] = lx @ F[a + H * c] @ ly
    return out


def grad_table(geom, U, p, n):
    """grad u0 on the n x n node grid of the domain, [n, n, 2] indexed
    [j, i] (node (x0 + i (x1 - x0) / (n - 1), y0 + j (y1 - y0) / (n - 1))),
    the table the gradient-table control variate reads."""
    gx, gy = grid_gradients(geom, U, p)
    xs = geom.x0 + (geom.x1 - geom.x0) * np.arange(n) / (n - 1)
    ys = geom.y0 + (geom.y1 - geom.y0) * np.arange(n) / (n - 1)
    X, Y = np.meshgrid(xs, ys)                         # X[j, i]
    v = interpolate(geom, [gx, gy], p, np.stack([X.ravel(), Y.ravel()], axis=1))
    return np.stack([v[0], v[1]], axis=1).reshape(n, n, 2)
