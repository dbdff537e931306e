"""The Sec. 5 problem (eqs. 42-43) on the GPU against the oracle, on a
reduced partition of the same domain: float64 same-stream parity with the
hat and the RBF interpolation, and float32 production within 3 standard
errors.  Bars as in the hat and RBF parity tests."""
import numpy as np
import pytest

from paper_2301_05780_amd import pdd
from oracle.geometry import Geometry
from oracle.coeffs import Coefficients
from oracle.assemble import assemble as oracle_assemble, to_csr
from oracle.rbf import shape_for_condition, condition
from parity import fetch, assert_same_stream, assert_within_se

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

U = 2.0 ** -53


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = pdd.Context(0)
    yield c
    c.close()


def _w(**kw):
    w = dict(name="eq43_small", kind="eq43", param=(), domain=(-100.0, 100.0, -100.0, 100.0), H=4, m=8, ext=4,
             n_paths=100, h=1.0, seed=4, precision="fp64", exit_rule="gm")
    w.update(kw)
    return w


def _oracle(w, interp=None):
    g = Geometry(w["domain"], w["H"], w["m"], w["ext"])
    out = oracle_assemble(g, Coefficients("eq43"), w["n_paths"], w["h"], w["seed"], exit_rule=w["exit_rule"],
                          interp=interp)
    return g, to_csr(g, out["rows"])


@pytest.mark.parametrize("rule", ["gm", "naive"])
def test_hat_fp64_same_stream(ctx, rule):
    w = _w(exit_rule=rule)
    g, ref = _oracle(w)
    got = fetch(ctx.assemble(w), g)
    ctx.sync()
    assert_same_stream(got, g, ref)


def test_rbf_fp64_same_stream(ctx):
    S, dx = 17, 200.0 / 32
    c = shape_for_condition(S, dx, 1e8)
    kappa = condition(np.arange(S) * dx, c)
    w = _w(interp="rbf", rbf_c=c)
    g, ref = _oracle(w, ("rbf", c))
    got = fetch(ctx.assemble(w), g)
    ctx.sync()
    row_of = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    tol = (1e-12 + S * kappa * U) * ref["mass"]
    assert np.array_equal(got["col_idx"], g.col_idx)
    assert np.all(np.abs(got["val"] - ref["val"]) <= tol[row_of])
    assert np.all(np.abs(got["b"] - ref["b"]) <= tol)
    assert np.array_equal(got["diag"][:, :6], ref["diag"][:, :6])


def test_fp32_production_within_se(ctx):
    w = _w(precision="fp32", n_paths=300)
    g, ref = _oracle(w)
    got = fetch(ctx.assemble(w), g)
    ctx.sync()
    assert_within_se(got, g, ref, nse=3.0, floor=1e-5)
