"""PDDSparse discretisation of a grid-aligned square domain (Sec. 3.1).

Omega = [x0, x1] x [y0, y1] is cut into H x H open squares (the subdomains of
eq. 12).  Every square side carries m lattice intervals, so the knot lattice
has spacing dx = (x1 - x0) / (H m), dy = (y1 - y0) / (H m) and integer
coordinates (ix, iy) in [0, H m]^2.

Knots sit on the grid lines, crossings included (Sec. 3.1, "Knots").  Reading
taken: only lattice points inside Omega are unknowns; lattice points on the
boundary take the Dirichlet datum g and enter b, not the unknown vector.
Canonical order of the unknowns: lexicographic in (iy, ix).

Slab (eq. 13): union of the closed squares whose boundary holds the knot, i.e.
two squares for a knot between crossings and four at a crossing.  For the
grid-aligned square the slab lies inside the closed domain, so the patch of
eq. 15 equals the slab.

Sides E, N, W, S (eq. 14) are the four sides of the patch rectangle.  A side
lying on the domain boundary is a boundary side (exit datum g); otherwise it
is an interface segment with a stencil (eq. 17): the knots on the side's grid
line whose along-line lattice coordinate lies in the side's range widened by
``ext`` lattice units at both ends (the paper widens stencils by half a
segment where possible, Sec. 5.1, and beyond corners, Sec. 3.3, Fig. 3),
clipped to the domain.  The knot stencil (eq. 18) is the union over sides; the
sparsity pattern of row k is {k} united with that stencil (support of eq. 24),
kept whether or not a sampled entry turns out to be zero.
"""
import numpy as np

SIDES = ("E", "N", "W", "S")


class Geometry:
    """Knots, patches, sides and CSR pattern of one partition.

    Parameters: domain (x0, x1, y0, y1), H subdomains per direction,
    m lattice intervals per subdomain side, ext stencil extension in lattice
    units.
    """

    def __init__(self, domain, H, m, ext):
        self.x0, self.x1, self.y0, self.y1 = (float(v) for v in domain)
        self.H, self.m, self.ext = int(H), int(m), int(ext)
        if self.H < 2 or self.m < 1 or self.ext < 0:
            raise ValueError("need H >= 2, m >= 1, ext >= 0")
        self.L = self.H * self.m                      # lattice intervals per direction
        self.dx = (self.x1 - self.x0) / self.L
        self.dy = (self.y1 - self.y0) / self.L
        self._build_knots()
        self._build_patches()
        self._build_pattern()

    # --- knots -----------------------------------------------------------
    def _build_knots(self):
        L, m = self.L, self.m
        ixs, iys = [], []
        for iy in range(1, L):
            for ix in range(1, L):
                if ix % m == 0 or iy % m == 0:
                    ixs.append(ix)
                    iys.append(iy)
        self.ix = np.array(ixs, dtype=np.int64)
        self.iy = np.array(iys, dtype=np.int64)
        self.n = self.ix.size
        self.index = -np.ones((L + 1, L + 1), dtype=np.int64)   # index[ix, iy]
        self.index[self.ix, self.iy] = np.arange(self.n)
        self.x = self.x0 + self.ix * self.dx
        self.y = self.y0 + self.iy * self.dy

    def lattice_x(self, i):
        return self.x0 + np.asarray(i, dtype=np.float64) * self.dx

    def lattice_y(self, i):
        return self.y0 + np.asarray(i, dtype=np.float64) * self.dy

    # --- slabs / patches (eqs. 13-15) ------------------------------------
    def _build_patches(self):
        m = self.m
        ix, iy = self.ix, self.iy
        on_v = ix % m == 0
        on_h = iy % m == 0
        xlo = np.where(on_v, ix - m, (ix // m) * m)
        xhi = np.where(on_v, ix + m, (ix // m) * m + m)
        ylo = np.where(on_h, iy - m, (iy // m) * m)
        yhi = np.where(on_h, iy + m, (iy // m) * m + m)
        self.box_i = np.stack([xlo, xhi, ylo, yhi], axis=1)          # lattice units
        self.box = np.stack([self.lattice_x(xlo), self.lattice_x(xhi),
                             self.lattice_y(ylo), self.lattice_y(yhi)], axis=1)

    def side(self, k, o):
        """Description of side o of knot k's patch.

        Returns dict(line='x'|'y' (the coordinate that is constant on the side),
        at=lattice coordinate of the line, lo/hi=side range along the line,
        boundary=bool, clo/chi=clamp range along the line).
        """
        xlo, xhi, ylo, yhi = (int(v) for v in self.box_i[k])
        L, e = self.L, self.ext
        if o == "E":
            line, at, lo, hi = "x", xhi, ylo, yhi
        elif o == "W":
            line, at, lo, hi = "x", xlo, ylo, yhi
        elif o == "N":
            line, at, lo, hi = "y", yhi, xlo, xhi
        else:
            line, at, lo, hi = "y", ylo, xlo, xhi
        boundary = at == 0 or at == L
        if boundary:
            clo, chi = 0, L
        else:
            clo, chi = max(0, lo - e), min(L, hi + e)
        return dict(line=line, at=at, lo=lo, hi=hi, boundary=boundary, clo=clo, chi=chi)

    def stencil(self, k, o):
        """Knot indices of the stencil of side o (eq. 17), ordered along the line."""
        s = self.side(k, o)
        if s["boundary"]:
            return np.zeros(0, dtype=np.int64)
        t = np.arange(max(1, s["clo"]), min(self.L - 1, s["chi"]) + 1)
        if s["line"] == "x":
            idx = self.index[s["at"], t]
        else:
            idx = self.index[t, s["at"]]
        assert np.all(idx >= 0), "every interior lattice point of a grid line is a knot"
        return idx

    # --- CSR pattern (eq. 24 support) -------------------------------------
    def _build_pattern(self):
        row_ptr = np.zeros(self.n + 1, dtype=np.int64)
        cols = []
        for k in range(self.n):
            parts = [np.array([k], dtype=np.int64)] + [self.stencil(k, o) for o in SIDES]
            c = np.unique(np.concatenate(parts))
            cols.append(c)
            row_ptr[k + 1] = row_ptr[k] + c.size
        self.row_ptr = row_ptr
        self.col_idx = np.concatenate(cols) if cols else np.zeros(0, dtype=np.int64)
        self.nnz = int(row_ptr[-1])

    def csr_position(self, k, j):
        """Position of column j in row k of the pattern (KeyError if absent)."""
        a, b = self.row_ptr[k], self.row_ptr[k + 1]
        pos = a + np.searchsorted(self.col_idx[a:b], j)
        if pos >= b or self.col_idx[pos] != j:
            raise KeyError((k, j))
        return int(pos)


def knot_count(H, m):
    """Closed form of the number of unknown knots: 2 (H-1)(H m - 1) - (H-1)^2."""
    return 2 * (H - 1) * (H * m - 1) - (H - 1) ** 2
