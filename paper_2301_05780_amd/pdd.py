"""Thin ctypes binding of libpdd (include/pdd.h): argument marshalling only.

Every computation runs in the HIP library; this module converts Python
values and torch tensors into the C structures and device pointers of the
ABI and raises ``PddError`` on any non-OK status.  There is no fallback:
if libpdd.so is missing the import of the library fails loudly.
"""
import ctypes as C
import functools
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpdd.so")

OK, EINVAL, ENOMEM, EDEVICE, ENOTCONV, EUNSUPPORTED = range(6)
KIND = {"poisson": 0, "varcoef": 1, "amplitude": 2, "lut": 3, "constsol": 4, "exittime": 5, "eq43": 6}
PRECISION = {"fp64": 0, "fp32": 1}
EXIT = {"naive": 0, "gm": 1}
CV_MODE = {"none": 0, "network": 1, "grad_lut": 2}
DIAG_WIDTH = 8
DUMP_WIDTH = 8
MLP_PARAMS = 4417
CAL_WIDTH = 8
COLLECT_STREAM = 0x40000000          # added to the instance word by pdd_collect_training
INTERP = {"hat": 0, "rbf": 1}


class PddError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"pdd status {status}: {msg}")
        self.status = status


class Coeffs(C.Structure):
    _fields_ = [("kind", C.c_int32), ("lut_n", C.c_int32), ("param", C.c_double * 4),
                ("lut", C.c_void_p)]


class Partition(C.Structure):
    _fields_ = [("x0", C.c_double), ("x1", C.c_double), ("y0", C.c_double), ("y1", C.c_double),
                ("H", C.c_int32), ("_pad", C.c_int32)]


class Knots(C.Structure):
    _fields_ = [("m", C.c_int32), ("ext", C.c_int32)]


class CV(C.Structure):
    _fields_ = [("mode", C.c_int32), ("lut_n", C.c_int32), ("params", C.c_void_p),
                ("grad_lut", C.c_void_p)]


class CVSpec:
    """Control variate for pdd_assemble: mode 'network' (params: float32 device
    tensor of MLP_PARAMS) or 'grad_lut' (table: float32 device tensor
    [n, n, 2] over the domain)."""

    def __init__(self, mode, params=None, table=None):
        self.mode, self.params, self.table = mode, params, table

    def struct(self):
        n = int(self.table.shape[0]) if self.table is not None else 0
        return CV(CV_MODE[self.mode], n, _ptr(self.params), _ptr(self.table))


class Run(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("instance", C.c_uint32), ("precision", C.c_int32),
                ("exit_rule", C.c_int32), ("dump_paths", C.c_int32), ("n_paths", C.c_int64),
                ("n_paths_per_knot", C.c_void_p), ("h", C.c_double), ("cv", C.c_void_p),
                ("u_ref", C.c_void_p), ("dump", C.c_void_p), ("interp", C.c_int32), ("rbf_c", C.c_double),
                ("h_per_knot", C.c_void_p)]


class Instance(C.Structure):
    _fields_ = [("coeffs", Coeffs), ("part", Partition), ("knots", Knots), ("run", Run),
                ("row_ptr", C.c_void_p), ("col_idx", C.c_void_p), ("val", C.c_void_p), ("b", C.c_void_p),
                ("diag", C.c_void_p)]


_lib = None


def lib():
    """The loaded libpdd.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2301_05780_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, f64 = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        sig = {
            "pdd_create": [C.POINTER(vp), i32, vp],
            "pdd_destroy": [vp],
            "pdd_set_stream": [vp, vp],
            "pdd_sync": [vp],
            "pdd_last_error": [vp],
            "pdd_pattern": [C.POINTER(Partition), C.POINTER(Knots), C.POINTER(i64), C.POINTER(i64), vp, vp],
            "pdd_knot_xy": [C.POINTER(Partition), C.POINTER(Knots), vp],
            "pdd_assemble": [vp, C.POINTER(Coeffs), C.POINTER(Partition), C.POINTER(Knots),
                             C.POINTER(Run), vp, vp, vp, vp, vp],
            "pdd_set_launch": [vp, i32, i32, i32, i32],
            "pdd_set_refill": [vp, i32],
            "pdd_calibrate": [vp, C.POINTER(Coeffs), C.POINTER(Partition), C.POINTER(Knots), C.POINTER(Run), vp, vp],
            "pdd_calibration_plan": [i64, vp, i64, f64, f64, f64, i32, vp, vp, vp, vp, vp],
            "pdd_rbf_shape": [i32, f64, f64, C.POINTER(f64)],
            "pdd_plan_tickets": [C.POINTER(Partition), C.POINTER(Knots), vp, i32, i32, i32, C.POINTER(i64), vp, vp,
                                 vp],
            "pdd_get_refill": [vp, C.POINTER(i32)],
            "pdd_set_spare_rows": [vp, i32],
            "pdd_get_spare_rows": [vp, C.POINTER(i32)],
            "pdd_set_table_read": [vp, i32],
            "pdd_table_fields": [vp, C.POINTER(C.c_uint32), C.POINTER(i32)],
            "pdd_solve": [vp, i64, vp, vp, vp, vp, vp, f64, i32, C.POINTER(i32), C.POINTER(f64)],
            "pdd_solve_noalloc": [vp, i64, vp, vp, vp, vp, vp, f64, i32, C.POINTER(i32), C.POINTER(f64)],
            "pdd_mlp_init": [vp, vp, C.c_uint64],
            "pdd_mlp_eval": [vp, vp, i64, vp, vp, vp],
            "pdd_mlp_grad_bf16": [vp, vp, i64, vp, vp],
            "pdd_spectral_solve": [vp, C.POINTER(Coeffs), C.POINTER(Partition), C.POINTER(Knots), i32, i32, f64, vp,
                                   vp],
            "pdd_spectral_eval": [vp, C.POINTER(Partition), i32, vp, i64, vp, vp, vp],
            "pdd_spectral_grad_lut": [vp, C.POINTER(Partition), i32, vp, i32, vp],
            "pdd_spectral_tables": [i32, C.POINTER(f64), C.POINTER(f64)],
            "pdd_assemble_batch": [vp, i32, vp],
            "pdd_graph_begin": [vp],
            "pdd_graph_end": [vp, C.POINTER(i32)],
            "pdd_graph_launch": [vp],
            "pdd_autotune": [vp, i32, vp, i32, C.POINTER(f64), C.c_char_p, i32],
            "pdd_mlp_grad": [vp, vp, i64, vp, vp, vp, vp],
            "pdd_mlp_train": [vp, vp, vp, vp, i64, vp, vp, vp, i64, i32, i32, i32, C.c_float, vp],
            "pdd_mlp_bake_grad_lut": [vp, vp, C.POINTER(Partition), i32, vp],
            "pdd_collect_training": [vp, C.POINTER(Coeffs), C.POINTER(Partition), C.POINTER(Knots), C.POINTER(Run),
                                     vp, i32, i32, vp, vp],
            "pdd_eval_subdomain": [vp, C.POINTER(Coeffs), C.POINTER(Partition), C.POINTER(Knots), vp, i64, vp,
                                   C.POINTER(Run), vp, vp],
            "pdd_last_launch": [vp, C.POINTER(i32), C.POINTER(i32), C.POINTER(i64)],
            "pdd_set_timing": [vp, i32],
            "pdd_kernel_ms": [vp, C.POINTER(f64), C.POINTER(i32)],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = None if name == "pdd_destroy" else (C.c_char_p if name == "pdd_last_error" else C.c_int)
        _lib = L
    return _lib


def _ptr(t):
    """Device (or host) data pointer of a tensor / array, None for None."""
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        return t.ctypes.data
    return t.data_ptr()


def _check(status, ctx=None):
    if status != OK:
        msg = lib().pdd_last_error(ctx)
        raise PddError(status, msg.decode() if msg else "")


def partition_of(w):
    x0, x1, y0, y1 = w["domain"]
    return Partition(x0, x1, y0, y1, int(w["H"]), 0)


def knots_of(w):
    return Knots(int(w["m"]), int(w["ext"]))


def pattern(w):
    """(n, nnz, row_ptr, col_idx) of the workload's system, computed on the host
    (cached per discretisation; the arrays are shared, read them only)."""
    d = tuple(float(v) for v in w["domain"])
    return _pattern(d, int(w["H"]), int(w["m"]), int(w["ext"]))


@functools.lru_cache(maxsize=8)
def _pattern(domain, H, m, ext):
    w = dict(domain=domain, H=H, m=m, ext=ext)
    part, kn = partition_of(w), knots_of(w)
    n, nnz = C.c_int64(), C.c_int64()
    _check(lib().pdd_pattern(C.byref(part), C.byref(kn), C.byref(n), C.byref(nnz), None, None))
    rp = np.empty(n.value + 1, dtype=np.int32)
    ci = np.empty(max(nnz.value, 1), dtype=np.int32)
    _check(lib().pdd_pattern(C.byref(part), C.byref(kn), C.byref(n), C.byref(nnz),
                             rp.ctypes.data, ci.ctypes.data))
    rp.setflags(write=False)
    ci.setflags(write=False)
    return n.value, nnz.value, rp, ci[:nnz.value]


def plan_tickets(w, paths_per_ticket, spatial=False, grid=0):
    """The work decomposition of a single-instance assembly of w (host only):
    (tickets int32[T, 3] = knot, first path, end path; claim order int32[T];
    XCD split int32[9] of the order, or None unless spatial and grid >= 8)."""
    part, kn = partition_of(w), knots_of(w)
    n = pattern(w)[0]
    npk = w.get("n_paths_per_knot")
    npk = np.full(n, int(w["n_paths"]), dtype=np.int32) if npk is None else np.ascontiguousarray(npk, dtype=np.int32)
    T = C.c_int64()
    args = (C.byref(part), C.byref(kn), npk.ctypes.data, int(paths_per_ticket), 1 if spatial else 0, int(grid),
            C.byref(T))
    _check(lib().pdd_plan_tickets(*args, None, None, None))
    tickets = np.empty((max(T.value, 1), 3), dtype=np.int32)
    order = np.empty(max(T.value, 1), dtype=np.int32)
    xb = np.empty(9, dtype=np.int32) if (spatial and grid >= 8) else None
    _check(lib().pdd_plan_tickets(*args, tickets.ctypes.data, order.ctypes.data,
                                  None if xb is None else xb.ctypes.data))
    return tickets[:T.value], order[:T.value], xb


def calibration_plan(stats, n_paths, h0, eps, n_job, h0_cal=None):
    """Per-knot h_i, N_i, bias bound, variance and rho^2 from calibration sums
    (host; stats: array [n, CAL_WIDTH]); h0_cal is the calibration step h0'
    (default h0), h0 the production cap."""
    st = np.ascontiguousarray(stats, dtype=np.float64).reshape(-1, CAL_WIDTH)
    n = st.shape[0]
    h = np.empty(n)
    paths = np.empty(n, dtype=np.int32)
    bias, var, rho2 = np.empty(n), np.empty(n), np.empty(n)
    _check(lib().pdd_calibration_plan(n, st.ctypes.data, int(n_paths), float(h0 if h0_cal is None else h0_cal),
                                      float(h0), float(eps), int(n_job),
                                      h.ctypes.data, paths.ctypes.data, bias.ctypes.data, var.ctypes.data,
                                      rho2.ctypes.data))
    return dict(h=h, n_paths=paths, bias=bias, var=var, rho2=rho2)


def rbf_shape(n_nodes, spacing, target_cond=1e10):
    """Shape parameter c of the inverse multiquadric at which the
    interpolation matrix of n_nodes equispaced points reaches target_cond
    (host)."""
    c = C.c_double()
    _check(lib().pdd_rbf_shape(int(n_nodes), float(spacing), float(target_cond), C.byref(c)))
    return c.value


def spectral_tables(p):
    """Accuracy of the degree-p diagonalisation of the spectral solves (host):
    (max |E V - V diag(lam)| / max |E|, max |V V^{-1} - I|)."""
    a, b = C.c_double(), C.c_double()
    _check(lib().pdd_spectral_tables(int(p), C.byref(a), C.byref(b)))
    return a.value, b.value


def _set_interp(run, w):
    """Interpolation fields of a Run from workload keys ``interp`` ("hat" or
    "rbf") and ``rbf_c``."""
    run.interp = INTERP[w.get("interp", "hat")]
    run.rbf_c = float(w.get("rbf_c", 0.0))
    return run


def knot_xy(w):
    part, kn = partition_of(w), knots_of(w)
    n, nnz = C.c_int64(), C.c_int64()
    _check(lib().pdd_pattern(C.byref(part), C.byref(kn), C.byref(n), C.byref(nnz), None, None))
    xy = np.empty(2 * n.value, dtype=np.float64)
    _check(lib().pdd_knot_xy(C.byref(part), C.byref(kn), xy.ctypes.data))
    return xy.reshape(-1, 2)


class Context:
    """A libpdd context bound to a torch device and stream."""

    def __init__(self, device=0, stream=None):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        h = C.c_void_p()
        _check(lib().pdd_create(C.byref(h), int(device), C.c_void_p(stream.cuda_stream)))
        self.h = h

    def close(self):
        if self.h:
            lib().pdd_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def check(self, status):
        _check(status, self.h)

    def sync(self):
        self.check(lib().pdd_sync(self.h))

    def set_launch(self, block=0, grid=0, paths_per_ticket=0, schedule="static"):
        sched = {"static": 0, "dynamic": 1}[schedule]
        self.check(lib().pdd_set_launch(self.h, block, grid, paths_per_ticket, sched))

    def set_refill(self, min_idle=1):
        self.check(lib().pdd_set_refill(self.h, int(min_idle)))

    def set_spare_rows(self, spare=-1):
        self.check(lib().pdd_set_spare_rows(self.h, int(spare)))

    def spare_rows(self):
        r = C.c_int32()
        self.check(lib().pdd_get_spare_rows(self.h, C.byref(r)))
        return r.value

    def set_table_read(self, read_all=False):
        """Float32 table assemblies: read only the varying fields when at most
        two vary (default), or always all seven cooperatively."""
        self.check(lib().pdd_set_table_read(self.h, 1 if read_all else 0))

    def table_fields(self):
        """(bit mask of the fields found varying, lane-per-path read used) of
        the last float32 table assembly."""
        m, r = C.c_uint32(), C.c_int32()
        self.check(lib().pdd_table_fields(self.h, C.byref(m), C.byref(r)))
        return m.value, bool(r.value)

    def refill(self):
        r = C.c_int32()
        self.check(lib().pdd_get_refill(self.h, C.byref(r)))
        return r.value

    def last_launch(self):
        g, b, t = C.c_int32(), C.c_int32(), C.c_int64()
        self.check(lib().pdd_last_launch(self.h, C.byref(g), C.byref(b), C.byref(t)))
        return g.value, b.value, t.value

    def set_timing(self, enable=True):
        self.check(lib().pdd_set_timing(self.h, 1 if enable else 0))

    def kernel_ms(self):
        """(summed assembly-kernel milliseconds, launches) since set_timing."""
        ms, n = C.c_double(), C.c_int32()
        self.check(lib().pdd_kernel_ms(self.h, C.byref(ms), C.byref(n)))
        return ms.value, n.value

    # ---- solve --------------------------------------------------------------
    def solve(self, row_ptr, col_idx, val, b, u=None, tol=1e-10, max_iter=2000, check=True, noalloc=False):
        """Solve G u = b (device tensors).  Returns (u, iterations, relative
        residual).  noalloc: pdd_solve_noalloc (the library's static scratch)."""
        n = b.numel()
        if u is None:
            u = self.torch.empty(n, dtype=self.torch.float64, device=self.device)
        it, rr = C.c_int32(), C.c_double()
        fn = lib().pdd_solve_noalloc if noalloc else lib().pdd_solve
        st = fn(self.h, n, _ptr(row_ptr), _ptr(col_idx), _ptr(val), _ptr(b), _ptr(u),
                float(tol), int(max_iter), C.byref(it), C.byref(rr))
        if check or st != ENOTCONV:
            self.check(st)
        return u, it.value, rr.value

    # ---- batches, graphs, tuning -------------------------------------------------
    def _outputs(self, w):
        n, nnz, _, _ = pattern(w)
        dev, torch = self.device, self.torch
        return dict(n=n, nnz=nnz,
                    row_ptr=torch.empty(n + 1, dtype=torch.int32, device=dev),
                    col_idx=torch.empty(max(nnz, 1), dtype=torch.int32, device=dev),
                    val=torch.empty(max(nnz, 1), dtype=torch.float64, device=dev),
                    b=torch.empty(n, dtype=torch.float64, device=dev),
                    diag=torch.empty(n * DIAG_WIDTH, dtype=torch.float64, device=dev))

    def _instance(self, w, out, precision=None, lut=None, cvp=None, npk=None, hk=None):
        run = Run(int(w["seed"]) & (2 ** 64 - 1), int(w.get("instance", 0)), PRECISION[precision or w["precision"]],
                  EXIT[w["exit_rule"]], 0, int(w["n_paths"]), None, float(w["h"]), cvp, None, None)
        _set_interp(run, w)
        if npk is not None:
            run.n_paths_per_knot = npk.ctypes.data
        if hk is not None:
            run.h_per_knot = hk.ctypes.data
        return Instance(self.coeffs_of(w, lut), partition_of(w), knots_of(w), run,
                        _ptr(out["row_ptr"]), _ptr(out["col_idx"]), _ptr(out["val"]), _ptr(out["b"]),
                        _ptr(out["diag"]))

    def batch_arrays(self, ws, outs=None, precision=None, lut=None, cv=None, n_paths_per_knot=None,
                     h_per_knot=None):
        """Instance array (and outputs) for pdd_assemble_batch / pdd_autotune;
        ``lut`` is the table of tabulated-coefficient workloads (single
        instance); ``cv`` a CVSpec shared by every instance; per-knot path
        counts and steps (host arrays) for a single instance, which
        pdd_autotune then tunes as pdd_assemble runs it."""
        outs = outs or [self._outputs(w) for w in ws]
        cvp = None
        if cv is not None:
            cvs = cv if isinstance(cv, CV) else cv.struct()
            self._keep_cv = cvs                       # the instances point at it
            cvp = C.cast(C.pointer(cvs), C.c_void_p)
        npk = None if n_paths_per_knot is None else np.ascontiguousarray(n_paths_per_knot, dtype=np.int32)
        hk = None if h_per_knot is None else np.ascontiguousarray(h_per_knot, dtype=np.float64)
        self._keep_arrays = (npk, hk)
        arr = (Instance * len(ws))(*[self._instance(w, o, precision, lut, cvp, npk, hk) for w, o in zip(ws, outs)])
        return arr, outs

    def assemble_batch(self, ws, outs=None, precision=None, arr=None, cv=None):
        """Assemble every workload of ws in one launch; returns the list of outputs."""
        if arr is None:
            arr, outs = self.batch_arrays(ws, outs, precision, cv=cv)
        self.check(lib().pdd_assemble_batch(self.h, len(arr), arr))
        self._keep_batch = arr
        return outs

    def graph_begin(self):
        self.check(lib().pdd_graph_begin(self.h))

    def graph_end(self):
        n = C.c_int32()
        self.check(lib().pdd_graph_end(self.h, C.byref(n)))
        return n.value

    def graph_launch(self):
        self.check(lib().pdd_graph_launch(self.h))

    def autotune(self, arr, reps=3):
        """Tune the launch shape for an Instance array (see batch_arrays)."""
        ms = C.c_double()
        rep = C.create_string_buffer(16384)
        self.check(lib().pdd_autotune(self.h, len(arr), arr, int(reps), C.byref(ms), rep, 16384))
        return ms.value, rep.value.decode()

    # ---- control-variate network ---------------------------------------------
    def mlp_init(self, seed=0):
        """Initial network parameters on the device (zero biases, Glorot-uniform weights)."""
        params = self.torch.empty(MLP_PARAMS, dtype=self.torch.float32, device=self.device)
        self.check(lib().pdd_mlp_init(self.h, _ptr(params), int(seed) & ((1 << 64) - 1)))
        return params

    def mlp_eval(self, params, xy):
        n = xy.shape[0]
        v = self.torch.empty(n, dtype=self.torch.float32, device=self.device)
        g = self.torch.empty(n, 2, dtype=self.torch.float32, device=self.device)
        self.check(lib().pdd_mlp_eval(self.h, _ptr(params), n, _ptr(xy), _ptr(v), _ptr(g)))
        return v, g

    def mlp_grad_bf16(self, params, xy):
        """grad v at the rows of xy through the assembly's bf16-MFMA routine."""
        n = xy.shape[0]
        g = self.torch.empty(n, 2, dtype=self.torch.float32, device=self.device)
        self.check(lib().pdd_mlp_grad_bf16(self.h, _ptr(params), n, _ptr(xy), _ptr(g)))
        return g

    def mlp_grad(self, params, xy, target):
        grad = self.torch.empty(MLP_PARAMS, dtype=self.torch.float32, device=self.device)
        loss = self.torch.empty(1, dtype=self.torch.float32, device=self.device)
        self.check(lib().pdd_mlp_grad(self.h, _ptr(params), xy.shape[0], _ptr(xy), _ptr(target), _ptr(grad), _ptr(loss)))
        return grad, loss

    def mlp_train(self, params, m, s, xy, target, order, batch, steps, step0, lr):
        losses = self.torch.empty(max(steps, 1), dtype=self.torch.float32, device=self.device)
        self.check(lib().pdd_mlp_train(self.h, _ptr(params), _ptr(m), _ptr(s), target.numel(), _ptr(xy), _ptr(target),
                                       _ptr(order), order.numel(), int(batch), int(steps), int(step0), float(lr),
                                       _ptr(losses)))
        return losses[:steps]

    def mlp_bake(self, params, w, lut_n):
        table = self.torch.empty(lut_n, lut_n, 2, dtype=self.torch.float32, device=self.device)
        part = partition_of(w)
        self.check(lib().pdd_mlp_bake_grad_lut(self.h, _ptr(params), C.byref(part), int(lut_n), _ptr(table)))
        return table

    def collect(self, w, u0, paths_per_knot, points_per_path, seed=None, exit_rule=None, lut=None):
        """Training pairs (xy [slots, 2], target [slots]); NaN targets mark unused slots."""
        n = pattern(w)[0]
        slots = n * paths_per_knot * points_per_path
        xy = self.torch.empty(slots, 2, dtype=self.torch.float32, device=self.device)
        t = self.torch.empty(slots, dtype=self.torch.float32, device=self.device)
        run = Run(int(w["seed"] if seed is None else seed), int(w.get("instance", 0)), PRECISION["fp32"],
                  EXIT[exit_rule or w["exit_rule"]], 0, int(w["n_paths"]), None, float(w["h"]), None, None, None)
        _set_interp(run, w)
        co = self.coeffs_of(w, lut)
        part, kn = partition_of(w), knots_of(w)
        self.check(lib().pdd_collect_training(self.h, C.byref(co), C.byref(part), C.byref(kn), C.byref(run),
                                              _ptr(u0), int(paths_per_knot), int(points_per_path), _ptr(xy), _ptr(t)))
        return xy, t

    def calibrate(self, w, u_knots, n_paths, h=None, seed=None, instance=0, precision=None, cv=None, lut=None):
        """Phase II sums (device float64 [n, CAL_WIDTH]) from n_paths mixed
        GM/EM paths per knot scored with the knot values u_knots."""
        n = pattern(w)[0]
        stats = self.torch.empty(n * CAL_WIDTH, dtype=self.torch.float64, device=self.device)
        cvs = None
        if cv is not None:
            cvs = cv if isinstance(cv, CV) else cv.struct()
        run = Run(int(w["seed"] if seed is None else seed) & (2 ** 64 - 1), int(instance),
                  PRECISION[precision or w["precision"]], EXIT["gm"], 0, int(n_paths), None,
                  float(w["h"] if h is None else h),
                  C.cast(C.pointer(cvs), C.c_void_p) if cvs is not None else None, None, None)
        _set_interp(run, w)
        co = self.coeffs_of(w, lut)
        part, kn = partition_of(w), knots_of(w)
        self.check(lib().pdd_calibrate(self.h, C.byref(co), C.byref(part), C.byref(kn), C.byref(run),
                                       _ptr(u_knots), _ptr(stats)))
        self._keep = (cvs,)
        return stats.view(n, CAL_WIDTH)

    def eval_subdomain(self, w, u_knots, xy, n_paths, h=None, seed=None, instance=None, precision=None,
                       exit_rule=None, lut=None):
        """u and its standard error at the points xy (device float64 [P, 2])
        inside the subdomains, from the knot values u_knots (device float64 [n])."""
        P = xy.shape[0]
        u = self.torch.empty(P, dtype=self.torch.float64, device=self.device)
        se = self.torch.empty(P, dtype=self.torch.float64, device=self.device)
        run = Run(int(w["seed"] if seed is None else seed) & (2 ** 64 - 1),
                  int(w.get("instance", 0) if instance is None else instance),
                  PRECISION[precision or w["precision"]], EXIT[exit_rule or w["exit_rule"]], 0, int(n_paths),
                  None, float(w["h"] if h is None else h), None, None, None)
        _set_interp(run, w)
        co = self.coeffs_of(w, lut)
        part, kn = partition_of(w), knots_of(w)
        self.check(lib().pdd_eval_subdomain(self.h, C.byref(co), C.byref(part), C.byref(kn), _ptr(u_knots), int(P),
                                            _ptr(xy), C.byref(run), _ptr(u), _ptr(se)))
        return u, se

    # ---- assembly ----------------------------------------------------------
    def coeffs_of(self, w, lut=None):
        par = (C.c_double * 4)(*(list(w.get("param", ())) + [0.0] * 4)[:4])
        lut_n = int(w.get("lut_n", 0)) if lut is not None else 0
        return Coeffs(KIND[w["kind"]], lut_n, par, _ptr(lut))

    # ---- pseudospectral subdomain solves ---------------------------------------
    def spectral_solve(self, w, u_knots, p, interp=None, rbf_c=None, lut=None):
        """Grid values and derivatives of every square: tensor [H^2, 3, p+1, p+1]
        (fields u, du/dx, du/dy).  interp defaults to the workload's
        ("hat" or "rbf" with w["rbf_c"])."""
        H = int(w["H"])
        grid = self.torch.empty(H * H, 3, p + 1, p + 1, dtype=self.torch.float64, device=self.device)
        mode = interp or w.get("interp", "hat")
        c = float(rbf_c if rbf_c is not None else w.get("rbf_c", 0.0)) if mode == "rbf" else 0.0
        co = self.coeffs_of(w, lut)
        part, kn = partition_of(w), knots_of(w)
        self.check(lib().pdd_spectral_solve(self.h, C.byref(co), C.byref(part), C.byref(kn), int(p), INTERP[mode], c,
                                            _ptr(u_knots), _ptr(grid)))
        return grid

    def spectral_eval(self, w, grid, p, xy):
        """u0 [n] and grad u0 [n, 2] at the rows of xy (device float64 [n, 2])."""
        n = xy.shape[0]
        u = self.torch.empty(n, dtype=self.torch.float64, device=self.device)
        g = self.torch.empty(n, 2, dtype=self.torch.float64, device=self.device)
        part = partition_of(w)
        self.check(lib().pdd_spectral_eval(self.h, C.byref(part), int(p), _ptr(grid), n, _ptr(xy), _ptr(u), _ptr(g)))
        return u, g

    def spectral_grad_lut(self, w, grid, p, lut_n):
        """grad u0 on the lut_n^2 node grid: float32 [lut_n, lut_n, 2], the
        gradient-table control variate's input."""
        table = self.torch.empty(lut_n, lut_n, 2, dtype=self.torch.float32, device=self.device)
        part = partition_of(w)
        self.check(lib().pdd_spectral_grad_lut(self.h, C.byref(part), int(p), _ptr(grid), int(lut_n), _ptr(table)))
        return table

    def assemble(self, w, out=None, lut=None, n_paths_per_knot=None, u_ref=None,
                 dump_paths=0, precision=None, exit_rule=None, seed=None, instance=None,
                 cv=None, h_per_knot=None):
        """Assemble G (CSR) and b of workload w.  Returns dict of device tensors
        row_ptr, col_idx, val, b, diag (and dump if requested).  ``out`` may hold
        preallocated tensors of the same names to write into; ``h_per_knot``
        (host array of n) gives each knot its own time step."""
        torch = self.torch
        n, nnz, _, _ = pattern(w) if out is None else (out["n"], out["nnz"], None, None)
        dev = self.device
        if out is None:
            out = dict(n=n, nnz=nnz,
                       row_ptr=torch.empty(n + 1, dtype=torch.int32, device=dev),
                       col_idx=torch.empty(max(nnz, 1), dtype=torch.int32, device=dev),
                       val=torch.empty(max(nnz, 1), dtype=torch.float64, device=dev),
                       b=torch.empty(n, dtype=torch.float64, device=dev),
                       diag=torch.empty(n * DIAG_WIDTH, dtype=torch.float64, device=dev))
        if dump_paths:
            out["dump"] = torch.full((n * dump_paths * DUMP_WIDTH,), float("nan"),
                                     dtype=torch.float64, device=dev)
        npk = None
        if n_paths_per_knot is not None:
            npk = np.ascontiguousarray(n_paths_per_knot, dtype=np.int32)
        cvs = None
        if cv is not None:
            cvs = cv if isinstance(cv, CV) else cv.struct()
        run = Run(int(w["seed"] if seed is None else seed) & (2 ** 64 - 1),
                  int(w.get("instance", 0) if instance is None else instance),
                  PRECISION[precision or w["precision"]], EXIT[exit_rule or w["exit_rule"]],
                  int(dump_paths), int(w["n_paths"]), _ptr(npk), float(w["h"]),
                  C.cast(C.pointer(cvs), C.c_void_p) if cvs is not None else None,
                  _ptr(u_ref), _ptr(out.get("dump")) if dump_paths else None)
        _set_interp(run, w)
        hk = None
        if h_per_knot is not None:
            hk = np.ascontiguousarray(h_per_knot, dtype=np.float64)
            run.h_per_knot = hk.ctypes.data
        co = self.coeffs_of(w, lut)
        part, kn = partition_of(w), knots_of(w)
        self.check(lib().pdd_assemble(self.h, C.byref(co), C.byref(part), C.byref(kn), C.byref(run),
                                      _ptr(out["row_ptr"]), _ptr(out["col_idx"]), _ptr(out["val"]),
                                      _ptr(out["b"]), _ptr(out["diag"])))
        self._keep = (npk, cvs, hk)
        return out
