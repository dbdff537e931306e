"""Coefficient families of the elliptic Dirichlet problem (6) used by the oracle.

Problem (6): 1/2 a_xx u_xx + a_xy u_xy + 1/2 a_yy u_yy + d . grad u + c u = f in
Omega, u = g on the boundary, with A = sigma sigma^T (eq. 7) and c <= 0.
Each family returns, at arrays of points, the diffusion matrix sigma (taken
symmetric: sxx, sxy, syy), the drift d, the reaction c, the source f, the
boundary datum g and, for manufactured problems, the exact solution u*.

Families (all on the unit square in the workloads that use them):
  poisson    sigma = sqrt(2) I, d = 0, c = 0, u* = sin(pi x) sin(pi y) + x^2 y, f = Lap u*
  varcoef    sigma = diag(sqrt(2(1 + sin(2 pi x)/2)), sqrt(2(1 + cos(2 pi y)/2))),
             d = (sin 2 pi y, cos 2 pi x), c = -(1 + x^2), u* = e^x cos 2y, f = L u*
  amplitude  sigma = diag(sqrt(2(1 + a sin 2 pi x)), sqrt(2(1 + a cos 2 pi y))),
             d = 0, c = 0, u* as in poisson, f = L u*
  lut        the seven fields (sxx, sxy, syy, dx, dy, c, f) tabulated in float32 on
             an n x n node-centred grid, read by bilinear interpolation; g is the
             poisson u*
  constsol   sigma, d, c of varcoef, f = c, g = 1, so that u = 1 solves (6)
  exittime   sigma = sqrt(2) I, d = 0, c = 0, f = -1, g = 0: u is the mean exit
             time of eq. (26)
  eq43       the Poisson problem of the Sec. 5 experiment (eq. 42, Lap u = f):
             sigma = sqrt(2) I, d = 0, c = 0, u* of eq. 43, f = Lap u*, g = u*

f = L u* is written out by hand for each manufactured family; the tests check
it against finite differences of u* through the operator of (6).
"""
import numpy as np

PI = np.pi

LUT_FIELDS = ("sxx", "sxy", "syy", "dx", "dy", "c", "f")
LUT_STRIDE = 8          # float32 per node (seven fields, one pad word)


def _u_poisson(x, y):
    return np.sin(PI * x) * np.sin(PI * y) + x * x * y


def _u_eq43(x, y):
    """Eq. 43: 3 + sin(sqrt(1 + x^2/100 + y^2/50))/3 + tanh(sin(3x/25 + y/20) + sin(x/20 - 3y/25))/3."""
    r = np.sqrt(1.0 + x * x / 100.0 + y * y / 50.0)
    s = np.sin(3.0 * x / 25.0 + y / 20.0) + np.sin(x / 20.0 - 3.0 * y / 25.0)
    return 3.0 + np.sin(r) / 3.0 + np.tanh(s) / 3.0


def _grad_eq43(x, y):
    r = np.sqrt(1.0 + x * x / 100.0 + y * y / 50.0)
    a, b = 3.0 * x / 25.0 + y / 20.0, x / 20.0 - 3.0 * y / 25.0
    sech2 = 1.0 - np.tanh(np.sin(a) + np.sin(b)) ** 2
    ux = np.cos(r) * x / (100.0 * r) + sech2 * (3.0 / 25.0 * np.cos(a) + np.cos(b) / 20.0)
    uy = np.cos(r) * y / (50.0 * r) + sech2 * (np.cos(a) / 20.0 - 3.0 / 25.0 * np.cos(b))
    return ux / 3.0, uy / 3.0


def _lap_eq43(x, y):
    """Laplacian of eq. 43, differentiated by hand term by term."""
    r = np.sqrt(1.0 + x * x / 100.0 + y * y / 50.0)
    rx, ry = x / (100.0 * r), y / (50.0 * r)
    # d2 r/dx2 + d2 r/dy2
    rxx = 1.0 / (100.0 * r) - x * x / (100.0 ** 2 * r ** 3)
    ryy = 1.0 / (50.0 * r) - y * y / (50.0 ** 2 * r ** 3)
    lap_sin_r = np.cos(r) * (rxx + ryy) - np.sin(r) * (rx * rx + ry * ry)
    a, b = 3.0 * x / 25.0 + y / 20.0, x / 20.0 - 3.0 * y / 25.0
    s = np.sin(a) + np.sin(b)
    sx = 3.0 / 25.0 * np.cos(a) + np.cos(b) / 20.0
    sy = np.cos(a) / 20.0 - 3.0 / 25.0 * np.cos(b)
    sxx = -(3.0 / 25.0) ** 2 * np.sin(a) - (1.0 / 20.0) ** 2 * np.sin(b)
    syy = -(1.0 / 20.0) ** 2 * np.sin(a) - (3.0 / 25.0) ** 2 * np.sin(b)
    t = np.tanh(s)
    lap_tanh_s = (1.0 - t * t) * (sxx + syy) - 2.0 * t * (1.0 - t * t) * (sx * sx + sy * sy)
    return (lap_sin_r + lap_tanh_s) / 3.0


class Coefficients:
    """Pointwise coefficients of one BVP instance, float64 in and out."""

    def __init__(self, kind, param=(), lut=None, lut_n=0, domain=(0.0, 1.0, 0.0, 1.0)):
        self.kind = kind
        self.param = tuple(float(p) for p in param)
        self.domain = tuple(float(v) for v in domain)
        if kind == "lut":
            tab = np.asarray(lut, dtype=np.float32).reshape(lut_n, lut_n, LUT_STRIDE)
            self.lut = tab.astype(np.float64)        # float32 table promoted to float64
            self.lut_n = int(lut_n)
        elif kind not in ("poisson", "varcoef", "amplitude", "constsol", "exittime", "eq43"):
            raise ValueError(kind)

    # --- bilinear read of the node-centred table ---------------------------
    def _lut(self, x, y):
        n = self.lut_n
        x0, x1, y0, y1 = self.domain
        fx = np.clip((x - x0) / (x1 - x0) * (n - 1), 0.0, n - 1)
        fy = np.clip((y - y0) / (y1 - y0) * (n - 1), 0.0, n - 1)
        i = np.minimum(np.floor(fx), n - 2).astype(np.int64)
        j = np.minimum(np.floor(fy), n - 2).astype(np.int64)
        tx = (fx - i)[..., None]
        ty = (fy - j)[..., None]
        t = self.lut
        v00, v10 = t[j, i], t[j, i + 1]
        v01, v11 = t[j + 1, i], t[j + 1, i + 1]
        return (1.0 - ty) * ((1.0 - tx) * v00 + tx * v10) + ty * ((1.0 - tx) * v01 + tx * v11)

    # --- coefficients -------------------------------------------------------
    def sigma(self, x, y):
        """Symmetric diffusion matrix entries (sxx, sxy, syy)."""
        z = np.zeros_like(x)
        if self.kind in ("poisson", "exittime", "eq43"):
            s = np.full_like(x, np.sqrt(2.0))
            return s, z, s.copy()
        if self.kind in ("varcoef", "constsol"):
            return (np.sqrt(2.0 * (1.0 + 0.5 * np.sin(2 * PI * x))), z,
                    np.sqrt(2.0 * (1.0 + 0.5 * np.cos(2 * PI * y))))
        if self.kind == "amplitude":
            a = self.param[0]
            return (np.sqrt(2.0 * (1.0 + a * np.sin(2 * PI * x))), z,
                    np.sqrt(2.0 * (1.0 + a * np.cos(2 * PI * y))))
        v = self._lut(x, y)
        return v[..., 0], v[..., 1], v[..., 2]

    def drift(self, x, y):
        if self.kind in ("varcoef", "constsol"):
            return np.sin(2 * PI * y), np.cos(2 * PI * x)
        if self.kind == "lut":
            v = self._lut(x, y)
            return v[..., 3], v[..., 4]
        return np.zeros_like(x), np.zeros_like(x)

    def reaction(self, x, y):
        if self.kind in ("varcoef", "constsol"):
            return -(1.0 + x * x)
        if self.kind == "lut":
            return self._lut(x, y)[..., 5]
        return np.zeros_like(x)

    def source(self, x, y):
        k = self.kind
        if k == "poisson":
            return -2.0 * PI * PI * np.sin(PI * x) * np.sin(PI * y) + 2.0 * y
        if k == "varcoef":
            ex, c2y, s2y = np.exp(x), np.cos(2 * y), np.sin(2 * y)
            return ex * ((1.0 + 0.5 * np.sin(2 * PI * x)) * c2y
                         - 4.0 * (1.0 + 0.5 * np.cos(2 * PI * y)) * c2y
                         + np.sin(2 * PI * y) * c2y
                         - 2.0 * np.cos(2 * PI * x) * s2y
                         - (1.0 + x * x) * c2y)
        if k == "amplitude":
            a = self.param[0]
            ss = np.sin(PI * x) * np.sin(PI * y)
            return ((1.0 + a * np.sin(2 * PI * x)) * (-PI * PI * ss + 2.0 * y)
                    + (1.0 + a * np.cos(2 * PI * y)) * (-PI * PI * ss))
        if k == "constsol":
            return -(1.0 + x * x)
        if k == "exittime":
            return np.full_like(x, -1.0)
        if k == "eq43":
            return _lap_eq43(x, y)
        return self._lut(x, y)[..., 6]

    def boundary(self, x, y):
        """Dirichlet datum g."""
        if self.kind == "constsol":
            return np.ones_like(x)
        if self.kind == "exittime":
            return np.zeros_like(x)
        return self.exact(x, y)

    def exact(self, x, y):
        """Manufactured solution u* (None where the family has no closed form)."""
        if self.kind in ("poisson", "amplitude", "lut"):
            return _u_poisson(x, y)
        if self.kind == "varcoef":
            return np.exp(x) * np.cos(2 * y)
        if self.kind == "constsol":
            return np.ones_like(x)
        if self.kind == "eq43":
            return _u_eq43(x, y)
        return None

    def grad_exact(self, x, y):
        """Gradient of u* (used by the exact-gradient control variate test)."""
        if self.kind in ("poisson", "amplitude", "lut"):
            return (PI * np.cos(PI * x) * np.sin(PI * y) + 2 * x * y,
                    PI * np.sin(PI * x) * np.cos(PI * y) + x * x)
        if self.kind == "varcoef":
            return np.exp(x) * np.cos(2 * y), -2 * np.exp(x) * np.sin(2 * y)
        if self.kind == "eq43":
            return _grad_eq43(x, y)
        return np.zeros_like(x), np.zeros_like(x)

    def normal_diffusion(self, x, y, line):
        """a_nn = N^T A N for a side whose normal is the x axis (line 'x') or the y axis."""
        sxx, sxy, syy = self.sigma(x, y)
        if line == "x":
            return sxx * sxx + sxy * sxy
        return sxy * sxy + syy * syy
