"""The benchmark's workloads at full size, in the launch configuration the
benchmark times: the autotuned shape (block, grid, ticket size, schedule,
deferred refill) set by the same helpers `bench.py` uses, and for the
64-instance batch the replay of the captured HIP graph.  Sampled rows are
checked against the oracle, which computes them one knot at a time, within 3
Monte Carlo standard errors; patterns are exact and the row sums obey the
c <= 0 bound 0 <= sum_j G_kj <= 1."""
import numpy as np
import pytest

import bench
from paper_2301_05780_amd import pdd, workloads
from oracle.geometry import Geometry
from oracle.coeffs import Coefficients
from oracle.assemble import assemble as oracle_assemble

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = pdd.Context(0)
    yield c
    c.close()


def _host(out):
    nnz = out["nnz"]
    return dict(row_ptr=out["row_ptr"].cpu().numpy(), col_idx=out["col_idx"].cpu().numpy()[:nnz],
                val=out["val"].cpu().numpy()[:nnz], b=out["b"].cpu().numpy(),
                diag=out["diag"].cpu().numpy().reshape(out["n"], pdd.DIAG_WIDTH))


def _check_rows(w, got, coeffs, knots):
    g = Geometry(w["domain"], w["H"], w["m"], w["ext"])
    assert np.array_equal(got["row_ptr"], g.row_ptr) and np.array_equal(got["col_idx"], g.col_idx)
    assert np.all(np.isfinite(got["val"])) and np.all(np.isfinite(got["b"]))
    rs = np.add.reduceat(got["val"], g.row_ptr[:-1])
    assert np.all(rs > -1e-9) and np.all(rs < 1 + 1e-9)
    assert np.all(got["diag"][:, 1] == w["n_paths"])
    ref = oracle_assemble(g, coeffs, w["n_paths"], w["h"], w["seed"], instance=w.get("instance", 0),
                          exit_rule=w["exit_rule"], knots=np.asarray(knots))["rows"]
    for k in knots:
        r = ref[k]
        a, e = g.row_ptr[k], g.row_ptr[k + 1]
        assert np.all(np.abs(got["val"][a:e] - r["val"]) <= 3 * r["se_val"] + 1e-6), k
        assert abs(got["b"][k] - r["b"]) <= 3 * r["se_b"] + 1e-5, k
        # the same random stream: the step totals agree closely
        assert abs(got["diag"][k, 0] / r["diag"][0] - 1.0) < 2e-3, k


def test_varcoef_in_the_timed_configuration(ctx):
    w = workloads.varcoef()
    out, tuned = bench.tuned_single(ctx, w, tune=True)
    try:
        ctx.assemble(w, out=out)
        ctx.sync()
        assert ctx.last_launch() == tuned["shape"]
        got = _host(out)
        n = got["row_ptr"].size - 1
        rng = np.random.default_rng(3)
        knots = np.concatenate([[0, n - 1], rng.choice(n, 2, replace=False)])
        _check_rows(w, got, Coefficients("varcoef", ()), knots)
    finally:
        ctx.set_launch(0, 0, 0)
        ctx.set_refill(1)
        ctx.set_spare_rows(-1)


def test_varcoef_rbf_at_full_size(ctx):
    """The RBF view of the benchmark: full varcoef size, default launch shape,
    c at condition number 1e10 for the 33-point stencils; sampled rows
    against the oracle's per-path cardinal weights within 3 standard errors
    (plus S kappa u of the row mass for the conditioning)."""
    w = workloads.varcoef()
    c = pdd.rbf_shape(33, 1 / 128, 1e10)
    wr = dict(w, interp="rbf", rbf_c=c)
    out = ctx.assemble(wr)
    ctx.sync()
    got = _host(out)
    g = Geometry(w["domain"], w["H"], w["m"], w["ext"])
    assert np.array_equal(got["row_ptr"], g.row_ptr) and np.array_equal(got["col_idx"], g.col_idx)
    assert np.all(np.isfinite(got["val"])) and np.all(np.isfinite(got["b"]))
    n = g.n
    knots = np.concatenate([[0, n - 1], np.random.default_rng(6).choice(n, 2, replace=False)])
    ref = oracle_assemble(g, Coefficients("varcoef", ()), w["n_paths"], w["h"], w["seed"], exit_rule=w["exit_rule"],
                          knots=knots, interp=("rbf", c))["rows"]
    for k in knots:
        r = ref[k]
        a, e = g.row_ptr[k], g.row_ptr[k + 1]
        floor = 1e-6 + 33 * 1e10 * 2.0 ** -53 * r["mass"]
        assert np.all(np.abs(got["val"][a:e] - r["val"]) <= 3 * r["se_val"] + floor), k
        assert abs(got["b"][k] - r["b"]) <= 3 * r["se_b"] + floor, k
        assert abs(got["diag"][k, 0] / r["diag"][0] - 1.0) < 2e-3, k


def test_sec5_phase1_in_the_timed_configuration(ctx):
    """The Sec. 5 experiment's Phase I at full size (11,241 knots, 191-point
    RBF stencils, h0 = 0.08) in the autotuned shape the benchmark times:
    sampled rows against the oracle within 3 standard errors plus the
    conditioning floor."""
    w = workloads.sec5()
    c = pdd.rbf_shape(191, 200.0 / 630, w["rbf_condition"])
    w = dict(w, rbf_c=c)
    arr, outs = ctx.batch_arrays([w])
    try:
        ctx.autotune(arr, reps=1)
        shape = ctx.last_launch()
        out = ctx.assemble(w, out=outs[0])
        ctx.sync()
        assert ctx.last_launch() == shape
        got = _host(out)
        g = Geometry(w["domain"], w["H"], w["m"], w["ext"])
        assert np.array_equal(got["row_ptr"], g.row_ptr) and np.array_equal(got["col_idx"], g.col_idx)
        assert np.all(np.isfinite(got["val"])) and np.all(np.isfinite(got["b"]))
        knots = np.random.default_rng(8).choice(g.n, 2, replace=False)
        ref = oracle_assemble(g, Coefficients("eq43"), w["n_paths"], w["h"], w["seed"], exit_rule=w["exit_rule"],
                              knots=knots, interp=("rbf", c))["rows"]
        for k in knots:
            r = ref[k]
            a, e = g.row_ptr[k], g.row_ptr[k + 1]
            floor = 1e-6 + 191 * w["rbf_condition"] * 2.0 ** -53 * r["mass"]
            assert np.all(np.abs(got["val"][a:e] - r["val"]) <= 3 * r["se_val"] + floor), k
            assert abs(got["b"][k] - r["b"]) <= 3 * r["se_b"] + floor, k
            assert abs(got["diag"][k, 0] / r["diag"][0] - 1.0) < 5e-3, k
    finally:
        ctx.set_launch(0, 0, 0)
        ctx.set_refill(1)
        ctx.set_spare_rows(-1)


def test_sec5_calibration_at_full_size(ctx):
    """The Sec. 5 Phase II as the benchmark runs it (11,241 knots, 1000 mixed
    paths each, RBF scores with a warm-up-like u0): the sampled knots' mean
    scores within 3 standard errors of the oracle's and the step totals
    close (float32 paths against float64)."""
    from oracle.calibrate import calibrate as oracle_calibrate
    w = workloads.sec5()
    c = pdd.rbf_shape(191, 200.0 / 630, w["rbf_condition"])
    w = dict(w, rbf_c=c)
    g = Geometry(w["domain"], w["H"], w["m"], w["ext"])
    co = Coefficients("eq43")
    u0 = co.exact(g.x, g.y) + np.random.default_rng(12).normal(0.0, 0.02, g.n)
    stats = ctx.calibrate(w, torch.from_numpy(u0).cuda(), w["n_paths"], seed=3).cpu().numpy()
    ctx.sync()
    assert np.all(np.isfinite(stats))
    N = w["n_paths"]
    knots = np.random.default_rng(13).choice(g.n, 2, replace=False)
    ref = oracle_calibrate(g, co, u0, N, w["h"], 3, knots=knots, interp=("rbf", c))
    for k in knots:
        r = ref[int(k)]
        mean, var = r[1] / N, max(r[2] / N - (r[1] / N) ** 2, 0.0)
        assert abs(stats[k, 1] / N - mean) <= 3 * np.sqrt(var / N) + 1e-6, k
        assert abs(stats[k, 7] / r[7] - 1.0) < 5e-3, k


def test_large_lut_in_the_timed_configuration(ctx):
    w = workloads.large_lut()
    tab = workloads.poisson_lut(w["lut_n"])
    lut = torch.from_numpy(tab).cuda()
    out, tuned = bench.tuned_single(ctx, w, lut=lut, tune=True)
    try:
        ctx.assemble(w, out=out, lut=lut)
        ctx.sync()
        assert ctx.last_launch() == tuned["shape"]
        got = _host(out)
        n = got["row_ptr"].size - 1
        assert n == 62465
        rng = np.random.default_rng(4)
        knots = np.concatenate([[n // 2], rng.choice(n, 2, replace=False)])
        _check_rows(w, got, Coefficients("lut", lut=tab, lut_n=w["lut_n"]), knots)
    finally:
        ctx.set_launch(0, 0, 0)
        ctx.set_refill(1)
        ctx.set_spare_rows(-1)


def test_batched_graph_replay_in_the_timed_configuration():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        gctx = pdd.Context(0, stream=stream)
        ws = workloads.batched()
        arr, outs, tuned_ms = bench.tuned_batched(gctx, ws)
        assert tuned_ms > 0
        gctx.graph_begin()
        gctx.assemble_batch(ws, arr=arr)
        gctx.graph_end()
        for o in outs:
            o["b"].fill_(np.nan)
        gctx.graph_launch()
        gctx.sync()
        rng = np.random.default_rng(5)
        for i in (3, 29, 60):
            w = ws[i]
            got = _host(outs[i])
            n = got["row_ptr"].size - 1
            _check_rows(w, got, Coefficients("amplitude", w["param"]), rng.choice(n, 2, replace=False))
        for o in outs:
            assert np.all(np.isfinite(o["b"].cpu().numpy()))
        gctx.close()
