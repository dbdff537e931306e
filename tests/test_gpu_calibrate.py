"""Phase II calibration on the GPU (pdd_calibrate) against the oracle: float64
same-stream sums per knot to rounding, float32 production within Monte Carlo
error, the constant-solution special case and argument checks."""
import numpy as np
import pytest

from paper_2301_05780_amd import pdd, workloads
from oracle.geometry import Geometry
from oracle.coeffs import Coefficients
from oracle import mlp as omlp
from oracle.calibrate import calibrate as oracle_calibrate, plan

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = pdd.Context(0)
    yield c
    c.close()


def _table(seed, n=65):
    rng = np.random.default_rng(seed + 100)
    th = workloads.mlp_init(seed) + rng.normal(0.0, 0.05, workloads.MLP_PARAMS)
    th = th.astype(np.float32).astype(np.float64)
    xs = np.arange(n) / (n - 1)
    X, Y = np.meshgrid(xs, xs)
    return omlp.grad_input(th, np.stack([X.ravel(), Y.ravel()], axis=1)).reshape(n, n, 2).astype(np.float32)


def _u0(g, c, rng):
    return c.exact(g.x, g.y) + rng.normal(0.0, 0.01, size=g.n)   # a slightly wrong warm-up solution


@pytest.mark.parametrize("kind,with_cv", [("varcoef", True), ("varcoef", False), ("lut", True)])
def test_fp64_same_stream_sums(ctx, kind, with_cv):
    w = dict(kind=kind, param=(), domain=(0.0, 1.0, 0.0, 1.0), H=3, m=4, ext=2, n_paths=160, h=2e-3, seed=31,
             precision="fp64", exit_rule="gm")
    tab = lut = None
    if kind == "lut":
        tab = workloads.varied_lut(65)
        w["lut_n"] = 65
        lut = torch.from_numpy(tab).cuda()
    g = Geometry(w["domain"], w["H"], w["m"], w["ext"])
    c = Coefficients(kind, (), lut=tab, lut_n=w.get("lut_n", 0), domain=w["domain"])
    u0 = _u0(g, Coefficients("poisson") if kind == "lut" else c, np.random.default_rng(3))
    spec = ocv = None
    if with_cv:
        table = _table(4)
        spec = pdd.CVSpec("grad_lut", table=torch.from_numpy(table).cuda())
        ocv = omlp.GradLutCV(table, w["domain"])
    got = ctx.calibrate(w, torch.from_numpy(u0).cuda(), w["n_paths"], instance=2, cv=spec, lut=lut).cpu().numpy()
    ctx.sync()
    ref = oracle_calibrate(g, c, u0, w["n_paths"], w["h"], w["seed"], instance=2, cv=ocv)
    for k in range(g.n):
        r = ref[k]
        scale = w["n_paths"] * (1.0 + abs(r[1]) / w["n_paths"] + abs(r[3]) / w["n_paths"]) ** 2
        assert np.all(np.abs(got[k, :6] - r[:6]) <= 1e-11 * scale), k
        assert np.array_equal(got[k, 6:], r[6:]), k
    if not with_cv:
        assert np.all(got[:, 3:6] == 0.0)


def test_fp32_production_within_monte_carlo_error(ctx):
    w = dict(workloads.poisson_small("gm"), kind="varcoef", n_paths=400, h=2e-3)
    g = Geometry(w["domain"], w["H"], w["m"], w["ext"])
    c = Coefficients("varcoef")
    u0 = _u0(g, c, np.random.default_rng(5))
    got = ctx.calibrate(w, torch.from_numpy(u0).cuda(), 400, precision="fp32").cpu().numpy()
    ctx.sync()
    ref = oracle_calibrate(g, c, u0, 400, w["h"], w["seed"], knots=[0, g.n // 2, g.n - 1])
    for k, r in ref.items():
        N = 400.0
        m, v = r[1] / N, r[2] / N - (r[1] / N) ** 2
        se = np.sqrt(max(v, 0.0) / N)
        assert abs(got[k, 1] / N - m) <= 3 * se + 1e-5, k
        assert abs(got[k, 6] / r[6] - 1.0) < 2e-3 and abs(got[k, 7] / r[7] - 1.0) < 2e-3, k


def test_constant_solution_plan(ctx):
    """u = 1 with u0 = 1: zero bias and variance, h_i = h0 and one job of paths per knot."""
    w = dict(kind="constsol", param=(), domain=(0.0, 1.0, 0.0, 1.0), H=3, m=4, ext=2, n_paths=200, h=2e-3, seed=8,
             precision="fp64", exit_rule="gm")
    n = pdd.pattern(w)[0]
    got = ctx.calibrate(w, torch.ones(n, dtype=torch.float64, device="cuda"), 200).cpu().numpy()
    ctx.sync()
    assert np.all(np.abs(got[:, 0]) < 1e-10) and np.allclose(got[:, 1], 200.0, rtol=0, atol=1e-10)
    pl = pdd.calibration_plan(got, 200, 2e-3, 0.01, 50)
    assert np.all(pl["h"] == 2e-3) and np.all(pl["n_paths"] == 50)
    ref = plan(got, 200, 2e-3, 0.01, 50)
    assert np.array_equal(pl["n_paths"], ref["n_paths"])


def test_calibrate_argument_validation(ctx):
    w = workloads.poisson_small()
    u = torch.zeros(29, dtype=torch.float64, device="cuda")
    with pytest.raises(pdd.PddError) as e:
        ctx.calibrate(w, u, 0)
    assert e.value.status == pdd.EINVAL
    params = ctx.mlp_init(0)
    with pytest.raises(pdd.PddError) as e:
        ctx.calibrate(w, u, 10, cv=pdd.CVSpec("network", params=params))
    assert e.value.status == pdd.EINVAL


@pytest.mark.parametrize("n_paths", [1, 3, 65])
def test_persistent_claims_cover_every_path(ctx, n_paths):
    """Path counts that leave the last claims partly empty (1, 3 and 65 paths
    per knot): float64 sums equal the oracle's, the step totals exactly, so
    every path ran once."""
    w = dict(kind="eq43", param=(), domain=(-100.0, 100.0, -100.0, 100.0), H=3, m=4, ext=2, n_paths=n_paths,
             h=2.0, seed=17, precision="fp64", exit_rule="gm")
    g = Geometry(w["domain"], w["H"], w["m"], w["ext"])
    c = Coefficients("eq43")
    u0 = _u0(g, c, np.random.default_rng(5))
    got = ctx.calibrate(w, torch.from_numpy(u0).cuda(), n_paths).cpu().numpy()
    ctx.sync()
    ref = oracle_calibrate(g, c, u0, n_paths, w["h"], w["seed"])
    for k in range(g.n):
        r = ref[k]
        scale = n_paths * (1.0 + abs(r[1]) / n_paths) ** 2
        assert np.all(np.abs(got[k, :6] - r[:6]) <= 1e-11 * scale), k
        assert np.array_equal(got[k, 6:], r[6:]), k


@pytest.mark.parametrize("kappa", [1e6, 1e10])
def test_rbf_scores_fp64_same_stream(ctx, kappa):
    """u0 at the exits interpolated with the RBF cardinal functions: the GPU
    applies the stencil inverse to the values once per side and sums
    alpha_i phi_i per exit, the oracle solves per exit; they agree to
    S kappa u of the scores' scale."""
    from oracle.rbf import shape_for_condition, condition
    w = dict(kind="varcoef", param=(), domain=(0.0, 1.0, 0.0, 1.0), H=3, m=4, ext=2, n_paths=120, h=2e-3, seed=33,
             precision="fp64", exit_rule="gm")
    g = Geometry(w["domain"], w["H"], w["m"], w["ext"])
    S = min(2 * w["m"] + 2 * w["ext"] + 1, g.L + 1)
    cc = shape_for_condition(S, g.dx, kappa)
    k_ = condition(np.arange(S) * g.dx, cc)
    w.update(interp="rbf", rbf_c=cc)
    c = Coefficients("varcoef")
    u0 = _u0(g, c, np.random.default_rng(6))
    got = ctx.calibrate(w, torch.from_numpy(u0).cuda(), w["n_paths"]).cpu().numpy()
    ctx.sync()
    ref = oracle_calibrate(g, c, u0, w["n_paths"], w["h"], w["seed"], interp=("rbf", cc))
    for k in range(g.n):
        r = ref[k]
        scale = w["n_paths"] * (1.0 + abs(r[1]) / w["n_paths"]) ** 2
        assert np.all(np.abs(got[k, :3] - r[:3]) <= (1e-11 + S * k_ * 2.0 ** -53) * scale), k
        assert np.array_equal(got[k, 6:], r[6:]), k
