"""Comparison helpers shared by the GPU parity tests (no test functions here).

Bars:
  * CSR pattern bit-exact;
  * float64 same-stream mode: every G and b entry within ``rel`` of the
    oracle, scaled by the row's mean absolute per-path contribution (only the
    summation order differs); step counts and exit-side counts exact;
  * float32 production mode: every entry within ``nse`` Monte Carlo standard
    errors of the oracle plus a float32 rounding floor.
"""
import numpy as np

from paper_2301_05780_amd import pdd


def fetch(out, g):
    return dict(row_ptr=out["row_ptr"].cpu().numpy(), col_idx=out["col_idx"].cpu().numpy()[:g.nnz],
                val=out["val"].cpu().numpy()[:g.nnz], b=out["b"].cpu().numpy(),
                diag=out["diag"].cpu().numpy().reshape(g.n, pdd.DIAG_WIDTH))


def assert_same_stream(got, g, ref, rel=1e-12):
    assert np.array_equal(got["row_ptr"], g.row_ptr)
    assert np.array_equal(got["col_idx"], g.col_idx)
    row_of = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    tol = rel * ref["mass"]
    dv = np.abs(got["val"] - ref["val"])
    db = np.abs(got["b"] - ref["b"])
    assert np.all(dv <= tol[row_of]), f"max G error {np.max(dv / tol[row_of]):.3g} x tol"
    assert np.all(db <= tol), f"max b error {np.max(db / tol):.3g} x tol"
    d, r = got["diag"], ref["diag"]
    assert np.array_equal(d[:, :6], r[:, :6]), "step counts / exit-side counts differ"
    assert np.allclose(d[:, 6:], r[:, 6:], rtol=1e-11, atol=1e-12 * np.max(np.abs(r[:, 6:])))


def assert_within_se(got, g, ref, nse=3.0, floor=1e-6):
    assert np.array_equal(got["row_ptr"], g.row_ptr)
    assert np.array_equal(got["col_idx"], g.col_idx)
    dv = np.abs(got["val"] - ref["val"])
    db = np.abs(got["b"] - ref["b"])
    assert np.all(dv <= nse * ref["se_val"] + floor), f"worst G {np.max(dv - nse * ref['se_val']):.3g}"
    assert np.all(db <= nse * ref["se_b"] + floor * np.maximum(1, np.abs(ref["b"]))), \
        f"worst b {np.max(db - nse * ref['se_b']):.3g}"


