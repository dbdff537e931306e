"""Pins of the oracle's discretisation (Sec. 3.1): knots, patches, stencils, pattern."""
import numpy as np
import pytest

from oracle.geometry import Geometry, knot_count, SIDES


@pytest.mark.parametrize("H,m", [(2, 8), (3, 4), (4, 6), (8, 16)])
def test_knot_count_closed_form(H, m):
    g = Geometry((0, 1, 0, 1), H, m, m // 2)
    # brute force over the lattice: interior points on a grid line
    L = H * m
    brute = sum(1 for ix in range(1, L) for iy in range(1, L) if ix % m == 0 or iy % m == 0)
    assert g.n == brute == knot_count(H, m)


def test_canonical_order_is_lexicographic_in_y_then_x():
    g = Geometry((0, 1, 0, 1), 3, 4, 2)
    key = g.iy * 10_000 + g.ix
    assert np.all(np.diff(key) > 0)


def test_poisson_small_rows_by_hand():
    """2 x 2 subdomains, 8 intervals per side: a knot between crossings has a
    two-square patch with one interface side spanning wall to wall (15 knots
    on the other line) -> 16 entries; the crossing knot's patch is the whole
    domain -> only the diagonal."""
    g = Geometry((0, 1, 0, 1), 2, 8, 4)
    counts = np.diff(g.row_ptr)
    assert g.n == 29 and g.nnz == 449
    crossing = g.index[8, 8]
    assert counts[crossing] == 1
    assert np.all(np.delete(counts, crossing) == 16)
    k = g.index[8, 3]                          # on x = 1/2, below the crossing
    assert tuple(g.box[k]) == (0.0, 1.0, 0.0, 0.5)
    cols = g.col_idx[g.row_ptr[k]:g.row_ptr[k + 1]]
    expect = sorted([k] + [g.index[ix, 8] for ix in range(1, 16)])
    assert list(cols) == expect


def _brute_stencil(g, k):
    """Stencil by geometry in physical coordinates: knots lying on a side line
    of the patch, within the side widened by ext spacings, that is not part
    of the domain boundary."""
    xlo, xhi, ylo, yhi = g.box[k]
    e = g.ext
    tol = 1e-9
    out = set()
    for j in range(g.n):
        xj, yj = g.x[j], g.y[j]
        for xline in (xlo, xhi):
            if abs(xline - g.x0) < tol or abs(xline - g.x1) < tol:
                continue
            if abs(xj - xline) < tol and ylo - e * g.dy - tol <= yj <= yhi + e * g.dy + tol:
                out.add(j)
        for yline in (ylo, yhi):
            if abs(yline - g.y0) < tol or abs(yline - g.y1) < tol:
                continue
            if abs(yj - yline) < tol and xlo - e * g.dx - tol <= xj <= xhi + e * g.dx + tol:
                out.add(j)
    return out


@pytest.mark.parametrize("H,m,ext", [(3, 4, 2), (4, 4, 2), (4, 6, 3), (3, 5, 0)])
def test_pattern_matches_brute_force(H, m, ext):
    g = Geometry((-1.0, 2.0, 0.5, 3.5), H, m, ext)
    for k in range(g.n):
        cols = set(int(c) for c in g.col_idx[g.row_ptr[k]:g.row_ptr[k + 1]])
        assert cols == _brute_stencil(g, k) | {k}


def test_patch_contains_knot_and_matches_slab():
    g = Geometry((0, 1, 0, 1), 4, 6, 3)
    for k in range(g.n):
        xlo, xhi, ylo, yhi = g.box[k]
        assert xlo < g.x[k] < xhi and ylo < g.y[k] < yhi
        area_squares = (xhi - xlo) * (yhi - ylo) / (g.m * g.dx) ** 2
        crossing = g.ix[k] % g.m == 0 and g.iy[k] % g.m == 0
        assert round(area_squares) == (4 if crossing else 2)


def test_side_types():
    g = Geometry((0, 1, 0, 1), 4, 4, 2)
    for k in range(g.n):
        for o in SIDES:
            s = g.side(k, o)
            assert s["boundary"] == (s["at"] in (0, g.L))
            assert 0 <= s["clo"] <= s["lo"] < s["hi"] <= s["chi"] <= g.L


def test_sec5_discretisation_counts():
    """The Sec. 5 partition: 10 x 10 subdomains with 64 knots per interface
    counted with both crossings (63 lattice intervals per side).  Interior
    knots only gives 11,241 unknowns; the paper's n = 11,277 also counts the
    36 ends of the 18 interior grid lines on the boundary.  Stencils widened
    by 32 lattice units reach 191 points at crossing knots."""
    from paper_2301_05780_amd import workloads
    w = workloads.sec5()
    g = Geometry(w["domain"], w["H"], w["m"], w["ext"])
    assert g.n == 11241 and g.n + 2 * 18 == 11277
    lengths = [g.side(k, o)["chi"] - g.side(k, o)["clo"] + 1 for k in range(0, g.n, 97) for o in "ENWS"
               if not g.side(k, o)["boundary"]]
    assert max(lengths) == 191
