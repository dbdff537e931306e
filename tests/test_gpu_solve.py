"""GPU solve of G u = b (mixed-precision BiCGStab with float64 refinement)
against LAPACK/SciPy on the same matrices, plus interface error versus u*."""
import numpy as np
import pytest

from paper_2301_05780_amd import pdd, workloads
from oracle.solve import solve as oracle_solve, relative_residual, rmse
from oracle.coeffs import Coefficients

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = pdd.Context(0)
    yield c
    c.close()


def _host(out, nnz):
    return (out["row_ptr"].cpu().numpy(), out["col_idx"].cpu().numpy()[:nnz],
            out["val"].cpu().numpy()[:nnz], out["b"].cpu().numpy())


@pytest.mark.parametrize("w", [workloads.poisson_small("gm"), workloads.varcoef("gm")],
                         ids=["poisson_small", "varcoef"])
def test_solve_matches_direct_solver(ctx, w):
    out = ctx.assemble(w)
    u, it, rel = ctx.solve(out["row_ptr"], out["col_idx"], out["val"][:out["nnz"]], out["b"])
    ctx.sync()
    rp, ci, val, b = _host(out, out["nnz"])
    uh = u.cpu().numpy()
    ref = oracle_solve(rp, ci, val, b)
    assert rel <= 1e-10
    assert relative_residual(rp, ci, val, b, uh) <= 1.5e-10
    assert np.allclose(uh, ref, rtol=1e-8, atol=1e-9 * np.abs(ref).max())
    # interface error against the manufactured solution (statistical + bias)
    xy = pdd.knot_xy(w)
    ue = Coefficients(w["kind"]).exact(xy[:, 0], xy[:, 1])
    assert rmse(uh, ue) < 0.05
    print(f"{w['name']}: {it} BiCGStab iterations, relres {rel:.2e}, interface RMSE {rmse(uh, ue):.4g}")


def test_zero_rhs_gives_zero(ctx):
    w = workloads.poisson_small()
    out = ctx.assemble(w)
    b0 = torch.zeros_like(out["b"])
    u, it, rel = ctx.solve(out["row_ptr"], out["col_idx"], out["val"][:out["nnz"]], b0)
    ctx.sync()
    assert it == 0 and rel == 0.0 and float(u.abs().max()) == 0.0


def test_not_converged_is_reported(ctx):
    w = workloads.varcoef()
    out = ctx.assemble(w)
    u, it, rel = ctx.solve(out["row_ptr"], out["col_idx"], out["val"][:out["nnz"]], out["b"],
                           tol=1e-14, max_iter=2, check=False)
    ctx.sync()
    assert it <= 3 and rel > 1e-14
    with pytest.raises(pdd.PddError) as e:
        ctx.solve(out["row_ptr"], out["col_idx"], out["val"][:out["nnz"]], out["b"], tol=1e-14, max_iter=2)
    assert e.value.status == pdd.ENOTCONV


def test_identity_rows(ctx):
    """A diagonal system (every patch equal to the domain would give G = I)."""
    n = 37
    rp = torch.arange(n + 1, dtype=torch.int32, device="cuda")
    ci = torch.arange(n, dtype=torch.int32, device="cuda")
    val = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.linspace(-1, 2, n, dtype=torch.float64, device="cuda")
    u, it, rel = ctx.solve(rp, ci, val, b)
    ctx.sync()
    assert rel <= 1e-10 and torch.allclose(u, b, rtol=0, atol=1e-12)
