"""pdd_solve_noalloc (the solve on the library's static device scratch, for
callers that cannot allocate) against pdd_solve through the C ABI: two calls
in a row, the second with a smaller system, each equal to the allocating
solve's result (the same kernels in the same order: identical iterates), and
sizes beyond the static array refused before any kernel runs."""
import numpy as np
import pytest

from paper_2301_05780_amd import pdd, workloads

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = pdd.Context(0)
    yield c
    c.close()


def _system(ctx, w):
    out = ctx.assemble(w)
    ctx.sync()
    return out["row_ptr"], out["col_idx"], out["val"][:out["nnz"]], out["b"]


def test_noalloc_solve_matches_the_allocating_solve(ctx):
    big = _system(ctx, dict(workloads.varcoef(), n_paths=500))
    small = _system(ctx, workloads.poisson_small())
    for sysm in (big, small):
        u_ref, it_ref, rr_ref = ctx.solve(*sysm, tol=1e-10)
        u, it, rr = ctx.solve(*sysm, tol=1e-10, noalloc=True)
        ctx.sync()
        assert it == it_ref and rr <= 1e-10
        a, b = u.cpu().numpy(), u_ref.cpu().numpy()
        assert np.all(np.isfinite(a))
        assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(b)), np.max(np.abs(a - b))


def test_noalloc_solve_refuses_sizes_beyond_its_scratch(ctx):
    # row_ptr claims 40 M nonzeros: refused from the sizes alone, before any
    # kernel reads col_idx or val
    rp = torch.tensor([0, 40_000_000], dtype=torch.int32, device="cuda")
    ci = torch.zeros(1, dtype=torch.int32, device="cuda")
    val = torch.ones(1, dtype=torch.float64, device="cuda")
    b = torch.ones(1, dtype=torch.float64, device="cuda")
    with pytest.raises(pdd.PddError) as e:
        ctx.solve(rp, ci, val, b, noalloc=True)
    assert e.value.status == pdd.EINVAL and "128 MiB" in str(e.value)
