"""Batched multi-instance assembly (one persistent launch), HIP graph replay
and the autotuner."""
import numpy as np
import pytest

from paper_2301_05780_amd import pdd, workloads
from oracle.geometry import Geometry
from oracle.coeffs import Coefficients
from oracle.assemble import assemble as oracle_assemble, to_csr

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = pdd.Context(0)
    yield c
    c.close()


def _small_batch(n=5, precision="fp64"):
    ws = []
    for w in workloads.batched()[:n]:
        w = dict(w)
        w["H"] = min(w["H"], 4)
        w["m"] = min(w["m"], 6)
        w["ext"] = w["m"] // 2
        w["n_paths"] = 120 + 37 * w["instance"]
        w["h"] = 2e-3
        w["precision"] = precision
        ws.append(w)
    return ws


def _host(out):
    nnz = out["nnz"]
    return dict(row_ptr=out["row_ptr"].cpu().numpy(), col_idx=out["col_idx"].cpu().numpy()[:nnz],
                val=out["val"].cpu().numpy()[:nnz], b=out["b"].cpu().numpy(),
                diag=out["diag"].cpu().numpy().reshape(out["n"], pdd.DIAG_WIDTH))


def test_batch_equals_single_instances(ctx):
    """Instance i inside the batch = instance i assembled alone (float64
    same stream: equal up to summation order), and = the oracle."""
    ws = _small_batch()
    outs = ctx.assemble_batch(ws)
    ctx.sync()
    for i, w in enumerate(ws):
        got = _host(outs[i])
        alone = _host(ctx.assemble(w))
        ctx.sync()
        assert np.array_equal(got["row_ptr"], alone["row_ptr"]) and np.array_equal(got["col_idx"], alone["col_idx"])
        scale = np.abs(alone["b"]).max() + 1.0
        assert np.allclose(got["val"], alone["val"], rtol=0, atol=1e-13)
        assert np.allclose(got["b"], alone["b"], rtol=0, atol=1e-13 * scale)
        assert np.array_equal(got["diag"][:, :6], alone["diag"][:, :6])
    # two instances against the oracle
    for i in (0, 3):
        w = ws[i]
        g = Geometry(w["domain"], w["H"], w["m"], w["ext"])
        ref = to_csr(g, oracle_assemble(g, Coefficients("amplitude", w["param"]), w["n_paths"], w["h"], w["seed"],
                                        instance=w["instance"], exit_rule=w["exit_rule"])["rows"])
        got = _host(outs[i])
        row_of = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
        tol = 1e-12 * ref["mass"]
        assert np.all(np.abs(got["val"] - ref["val"]) <= tol[row_of])
        assert np.all(np.abs(got["b"] - ref["b"]) <= tol)


def test_graph_replay_matches_eager():
    """Capture the batch once, replay it several times with eager work and
    synchronisations in between; every replay reproduces the eager result.
    Capture needs a stream of its own (not the null stream)."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        gctx = pdd.Context(0, stream=stream)
        ws = _small_batch(4, "fp32")
        arr, outs = gctx.batch_arrays(ws)
        gctx.assemble_batch(ws, arr=arr)          # builds and caches every table
        gctx.sync()
        eager = [_host(o) for o in outs]
        for o in outs:
            o["val"].fill_(-7.0)
            o["b"].fill_(-7.0)
        gctx.graph_begin()
        gctx.assemble_batch(ws, arr=arr)
        nodes = gctx.graph_end()
        assert nodes >= 1 + len(ws)
        for rep in range(3):
            for o in outs:
                o["val"].fill_(float(rep))
                o["b"].fill_(float(rep))
            gctx.graph_launch()
            gctx.sync()
            _ = torch.ones(1000, device="cuda").sum().item()     # eager work between replays
            for i, o in enumerate(outs):
                h = _host(o)
                assert np.array_equal(h["val"], eager[i]["val"]), f"replay {rep} instance {i}"
                assert np.array_equal(h["b"], eager[i]["b"])

        # a batch the context has not seen cannot be captured
        ws2 = _small_batch(2, "fp32")
        for w in ws2:
            w["n_paths"] += 1
        arr2, _ = gctx.batch_arrays(ws2)
        gctx.graph_begin()
        with pytest.raises(pdd.PddError) as e:
            gctx.assemble_batch(ws2, arr=arr2)
        try:
            gctx.graph_end()
        except pdd.PddError:
            pass
        assert e.value.status == pdd.EINVAL
        gctx.sync()
        gctx.close()


def test_autotune_keeps_results(ctx):
    ws = _small_batch(3, "fp32")
    arr, outs = ctx.batch_arrays(ws)
    ms, report = ctx.autotune(arr, reps=2)
    assert ms > 0 and "block" in report
    # the spare-row phase (pooled tally rows: batched launches) tries both
    # block sizes, whatever the sweep before it preferred
    assert "block 256, 0 spare rows" in report and "block 128, 0 spare rows" in report, report
    ctx.assemble_batch(ws, arr=arr)
    ctx.sync()
    tuned = [_host(o) for o in outs]
    ctx.set_launch(0, 0, 0)
    ctx.set_refill(1)
    ctx.set_spare_rows(-1)
    ctx.assemble_batch(ws, arr=arr)
    ctx.sync()
    for i, o in enumerate(outs):
        h = _host(o)
        assert np.allclose(h["val"], tuned[i]["val"], rtol=0, atol=1e-12)
        assert np.allclose(h["b"], tuned[i]["b"], rtol=1e-12, atol=1e-12)


def test_batch_rejects_mixed_options(ctx):
    ws = _small_batch(2, "fp32")
    ws[1]["precision"] = "fp64"
    with pytest.raises(pdd.PddError) as e:
        ctx.assemble_batch(ws)
    assert e.value.status == pdd.EINVAL


def test_full_batched_workload(ctx):
    """The 64-instance workload at full size in one launch: patterns exact,
    row sums in [0, 1] (c = 0), sampled knots against the oracle within 3 SE."""
    ws = workloads.batched()
    outs = ctx.assemble_batch(ws)
    ctx.sync()
    rng = np.random.default_rng(0)
    for i in (0, 17, 41):
        w = ws[i]
        g = Geometry(w["domain"], w["H"], w["m"], w["ext"])
        got = _host(outs[i])
        assert np.array_equal(got["row_ptr"], g.row_ptr) and np.array_equal(got["col_idx"], g.col_idx)
        rs = np.add.reduceat(got["val"], g.row_ptr[:-1])
        assert np.all(rs > -1e-9) and np.all(rs < 1 + 1e-9)
        knots = rng.choice(g.n, 2, replace=False)
        ref = oracle_assemble(g, Coefficients("amplitude", w["param"]), w["n_paths"], w["h"], w["seed"],
                              instance=w["instance"], exit_rule="gm", knots=knots)["rows"]
        for k in knots:
            r = ref[k]
            a, e = g.row_ptr[k], g.row_ptr[k + 1]
            assert np.all(np.abs(got["val"][a:e] - r["val"]) <= 3 * r["se_val"] + 1e-6)
            assert abs(got["b"][k] - r["b"]) <= 3 * r["se_b"] + 1e-5
    for o in outs:
        assert np.all(np.isfinite(o["b"].cpu().numpy()))
