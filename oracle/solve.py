"""Solution of the assembled system G u = b (eq. 23) and interface error measures.

The paper solves the system with a direct library solver on one core
(Sec. 4.3); the oracle does the same with LAPACK through NumPy (dense LU) or
SciPy's sparse LU for larger systems.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def csr_matrix(row_ptr, col_idx, val, n):
    return sp.csr_matrix((np.asarray(val, dtype=np.float64),
                          np.asarray(col_idx), np.asarray(row_ptr)), shape=(n, n))


def solve(row_ptr, col_idx, val, b):
    """u with G u = b; dense LU up to n = 4000, sparse LU above."""
    n = len(b)
    G = csr_matrix(row_ptr, col_idx, val, n)
    if n <= 4000:
        return np.linalg.solve(G.toarray(), np.asarray(b, dtype=np.float64))
    return spla.spsolve(G.tocsc(), np.asarray(b, dtype=np.float64))


def relative_residual(row_ptr, col_idx, val, b, u):
    """||b - G u||_2 / ||b||_2 in float64."""
    G = csr_matrix(row_ptr, col_idx, val, len(b))
    r = np.asarray(b) - G @ np.asarray(u)
    return float(np.linalg.norm(r) / np.linalg.norm(b))


def rmse(u, u_exact):
    """Root mean square interface error (Sec. 5.2.1 uses it next to the max error)."""
    d = np.asarray(u) - np.asarray(u_exact)
    return float(np.sqrt(np.mean(d * d)))
