"""One-dimensional RBF cardinal interpolation on a side stencil (Sec. 2.1,
eqs. 1-5; used on patch sides by eq. 21), in float64.

Test infrastructure only: the plain definition the GPU interpolation is
checked against.

The basis is the inverse multiquadric with shape parameter c.  Eq. 3 prints
the square root of r^2 - c^2, which is imaginary for r < c and not positive
definite; the reading taken is the usual inverse multiquadric

    phi_c(r) = 1 / sqrt(r^2 + c^2).

The interpolation matrix Phi_ij = phi_c(|z_i - z_j|) (eq. 2) is symmetric
positive definite, so the cardinal functions of eq. 5 are the entries of

    H(z) = Phi^{-1} [phi_c(|z - z_1|), ..., phi_c(|z - z_m|)]^T,

solved here with a dense LU solve per evaluation point.  Sec. 5.1 picks c so
that the spectral condition number of Phi is about 1e10; ``shape_for_condition``
finds that c for a given stencil by bisection on log c (the condition number
grows monotonically with c for a fixed equispaced stencil).
"""
import numpy as np


def imq(r, c):
    """Inverse multiquadric phi_c(r) = 1 / sqrt(r^2 + c^2) (eq. 3, sign read as +)."""
    r = np.asarray(r, dtype=np.float64)
    return 1.0 / np.sqrt(r * r + float(c) * float(c))


def interpolation_matrix(nodes, c):
    """Phi of eq. 2 for the collinear pointset ``nodes``."""
    z = np.asarray(nodes, dtype=np.float64)
    return imq(np.abs(z[:, None] - z[None, :]), c)


def cardinal(nodes, z, c):
    """Cardinal functions H_j(z) of eq. 5: array [len(nodes), len(z)]."""
    zn = np.asarray(nodes, dtype=np.float64)
    zz = np.atleast_1d(np.asarray(z, dtype=np.float64))
    rhs = imq(np.abs(zz[None, :] - zn[:, None]), c)
    return np.linalg.solve(interpolation_matrix(zn, c), rhs)


def condition(nodes, c):
    """Spectral (2-norm) condition number of Phi (inf once the smallest
    eigenvalue is lost to rounding)."""
    ev = np.linalg.eigvalsh(interpolation_matrix(nodes, c))
    return float(ev[-1] / ev[0]) if ev[0] > 0 else float("inf")


def shape_for_condition(n_nodes, spacing, target):
    """Shape parameter c at which Phi of n_nodes equispaced points (spacing
    ``spacing``) has condition number ``target`` (Sec. 5.1 chooses about 1e10)."""
    nodes = np.arange(int(n_nodes)) * float(spacing)
    lo, hi = 1e-3 * spacing, 1e3 * spacing
    if not condition(nodes, lo) < target < condition(nodes, hi):
        raise ValueError("target condition number out of reach")
    for _ in range(200):
        mid = np.sqrt(lo * hi)
        if condition(nodes, mid) < target:
            lo = mid
        else:
            hi = mid
        if hi / lo - 1.0 < 1e-12:
            break
    return float(np.sqrt(lo * hi))
