"""Edge cases of the GPU assembly against the oracle: the one-knot partition
(patch = domain, the PDD special case), a rectangular domain away from the
origin, seeds with high key bits, the dynamic schedule, graph replay of a
tabulated-coefficient assembly, and argument validation."""
import numpy as np
import pytest

from paper_2301_05780_amd import pdd, workloads
from oracle.geometry import Geometry
from oracle.coeffs import Coefficients
from oracle.assemble import assemble as oracle_assemble, to_csr
from parity import fetch, assert_same_stream

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = pdd.Context(0)
    yield c
    c.close()


def _oracle(w, lut=None):
    g = Geometry(w["domain"], w["H"], w["m"], w["ext"])
    c = Coefficients(w["kind"], w.get("param", ()), lut=lut, lut_n=w.get("lut_n", 0), domain=w["domain"])
    rows = oracle_assemble(g, c, w["n_paths"], w["h"], w["seed"], instance=w.get("instance", 0),
                           exit_rule=w["exit_rule"])["rows"]
    return g, to_csr(g, rows)


def test_single_knot_patch_is_the_domain(ctx):
    """H = 2, m = 1: one unknown, the crossing knot, whose patch is the whole
    domain, so G = [1] and b is the plain Feynman-Kac estimate of u there."""
    w = dict(kind="poisson", param=(), domain=(0.0, 1.0, 0.0, 1.0), H=2, m=1, ext=0, n_paths=2000,
             h=1e-3, seed=3, precision="fp64", exit_rule="gm")
    g, ref = _oracle(w)
    assert g.n == 1 and g.nnz == 1
    got = fetch(ctx.assemble(w), g)
    ctx.sync()
    assert_same_stream(got, g, ref)
    assert got["val"][0] == 1.0
    u = np.sin(np.pi * 0.5) ** 2 + 0.125
    assert abs(got["b"][0] - u) < 4 * ref["se_b"][0] + 5e-3


@pytest.mark.parametrize("rule", ["gm", "naive"])
def test_rectangular_domain_away_from_origin(ctx, rule):
    w = dict(kind="varcoef", param=(), domain=(-1.0, 2.0, 0.25, 1.75), H=3, m=4, ext=2, n_paths=150,
             h=2e-3, seed=17, precision="fp64", exit_rule=rule, instance=1)
    g, ref = _oracle(w)
    got = fetch(ctx.assemble(w), g)
    ctx.sync()
    assert_same_stream(got, g, ref)


def test_seed_with_high_key_bits(ctx):
    w = dict(workloads.poisson_small("gm"), n_paths=200, seed=(1 << 40) + 12345)
    g, ref = _oracle(w)
    got = fetch(ctx.assemble(w), g)
    ctx.sync()
    assert_same_stream(got, g, ref)
    # a different high word is a different stream
    w2 = dict(w, seed=(2 << 40) + 12345)
    other = fetch(ctx.assemble(w2), g)
    ctx.sync()
    assert not np.array_equal(other["b"], got["b"])


@pytest.mark.parametrize("kind", ["varcoef", "lut"])
def test_dynamic_schedule_matches_the_oracle(ctx, kind):
    """Waves claim tickets from device counters (per XCD share for the table
    family): the float64 sums may change order, nothing else."""
    w = dict(kind=kind, param=(), domain=(0.0, 1.0, 0.0, 1.0), H=4, m=8, ext=4, n_paths=200, h=2e-3,
             seed=5, precision="fp64", exit_rule="gm", instance=2)
    lut = None
    tab = None
    if kind == "lut":
        tab = workloads.varied_lut(65)
        w["lut_n"] = 65
        lut = torch.from_numpy(tab).cuda()
    g, ref = _oracle(w, tab)
    ctx.set_launch(0, 0, 64, "dynamic")
    try:
        for _ in range(2):                     # the counters are reset for the next assembly
            got = fetch(ctx.assemble(w, lut=lut), g)
            ctx.sync()
            assert_same_stream(got, g, ref)
    finally:
        ctx.set_launch(0, 0, 0)


def test_tabulated_assembly_graph_replay():
    """A single-instance float32 table assembly (bound and cell-copy kernels,
    XCD split, partial rows, finalize) captured once and replayed: every replay
    equals the eager result bit for bit."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        gctx = pdd.Context(0, stream=stream)
        tab = workloads.varied_lut(65)
        lut = torch.from_numpy(tab).cuda()
        w = dict(kind="lut", param=(), domain=(0.0, 1.0, 0.0, 1.0), H=4, m=8, ext=4, n_paths=300, h=2e-3,
                 seed=9, precision="fp32", exit_rule="gm", lut_n=65)
        out = gctx.assemble(w, lut=lut)
        gctx.sync()
        eager_val = out["val"].cpu().numpy().copy()
        eager_b = out["b"].cpu().numpy().copy()
        gctx.graph_begin()
        gctx.assemble(w, out=out, lut=lut)
        gctx.graph_end()
        for rep in range(3):
            out["val"].fill_(float(rep))
            out["b"].fill_(float(rep))
            gctx.graph_launch()
            gctx.sync()
            _ = torch.ones(1000, device="cuda").sum().item()
            assert np.array_equal(out["val"].cpu().numpy(), eager_val), rep
            assert np.array_equal(out["b"].cpu().numpy(), eager_b), rep
        gctx.close()


def test_argument_validation(ctx):
    w = workloads.poisson_small()
    xy = torch.zeros(4, 2, dtype=torch.float64, device="cuda")
    u = torch.zeros(29, dtype=torch.float64, device="cuda")
    with pytest.raises(pdd.PddError) as e:
        ctx.eval_subdomain(w, u, xy, 10, instance=1 << 31)
    assert e.value.status == pdd.EINVAL
    with pytest.raises(pdd.PddError) as e:
        ctx.eval_subdomain(w, u, xy, 0)
    assert e.value.status == pdd.EINVAL
    wl = dict(w, kind="lut", lut_n=1)
    with pytest.raises(pdd.PddError) as e:
        ctx.assemble(wl, lut=torch.zeros(8, device="cuda"))
    assert e.value.status == pdd.EINVAL
    with pytest.raises(pdd.PddError) as e:
        ctx.assemble(dict(w, exit_rule="naive", h=-1.0))
    assert e.value.status == pdd.EINVAL


@pytest.mark.parametrize("refill", [16, 64])
def test_deferred_refill_matches_the_oracle(ctx, refill):
    """A wave that refills only once `refill` lanes are idle (64: only when the
    whole wave is idle) runs the same paths: the float64 sums may change order,
    nothing else."""
    w = dict(kind="varcoef", param=(), domain=(0.0, 1.0, 0.0, 1.0), H=4, m=8, ext=4, n_paths=300, h=2e-3,
             seed=21, precision="fp64", exit_rule="gm", instance=4)
    g, ref = _oracle(w)
    ctx.set_refill(refill)
    assert ctx.refill() == refill
    try:
        got = fetch(ctx.assemble(w), g)
        ctx.sync()
        assert_same_stream(got, g, ref)
    finally:
        ctx.set_refill(1)


def test_refill_argument_validation(ctx):
    for bad in (0, 65, -3):
        with pytest.raises(pdd.PddError) as e:
            ctx.set_refill(bad)
        assert e.value.status == pdd.EINVAL


def test_empty_point_sets(ctx):
    """Zero points: the calls succeed and touch nothing."""
    w = workloads.poisson_small()
    u = torch.zeros(29, dtype=torch.float64, device="cuda")
    xy = torch.zeros(0, 2, dtype=torch.float64, device="cuda")
    val, se = ctx.eval_subdomain(w, u, xy, 10)
    ctx.sync()
    assert val.numel() == 0 and se.numel() == 0
    params = ctx.mlp_init(1)
    v, g = ctx.mlp_eval(params, torch.zeros(0, 2, dtype=torch.float32, device="cuda"))
    ctx.sync()
    assert v.numel() == 0 and g.numel() == 0


@pytest.mark.parametrize("spare", [0, 1])
def test_shared_row_pool_matches_the_oracle(ctx, spare):
    """Four waves sharing 4 (or 5) tally rows (table family), with tickets of
    16 paths so that waves often find no free row for their next ticket and
    wait: same rows as the oracle (float64 sums may change order)."""
    tab = workloads.varied_lut(65)
    w = dict(kind="lut", param=(), domain=(0.0, 1.0, 0.0, 1.0), H=4, m=8, ext=4, n_paths=150, h=2e-3,
             seed=23, precision="fp64", exit_rule="gm", instance=5, lut_n=65)
    g, ref = _oracle(w, tab)
    lut = torch.from_numpy(tab).cuda()
    ctx.set_launch(256, 0, 16, "static")
    ctx.set_spare_rows(spare)
    assert ctx.spare_rows() == spare
    try:
        for _ in range(2):
            got = fetch(ctx.assemble(w, lut=lut), g)
            ctx.sync()
            assert_same_stream(got, g, ref)
    finally:
        ctx.set_launch(0, 0, 0)
        ctx.set_spare_rows(-1)


def test_shared_row_pool_in_a_batch(ctx):
    """The batched kernel with one row per wave (no spare), dynamic schedule."""
    ws = []
    for i, w in enumerate(workloads.batched()[:3]):
        w = dict(w, H=min(w["H"], 4), m=min(w["m"], 6), n_paths=90 + 11 * i, h=2e-3, precision="fp64")
        w["ext"] = w["m"] // 2
        ws.append(w)
    ctx.set_launch(128, 0, 8, "dynamic")
    ctx.set_spare_rows(0)
    try:
        outs = ctx.assemble_batch(ws)
        ctx.sync()
        for w, o in zip(ws, outs):
            g = Geometry(w["domain"], w["H"], w["m"], w["ext"])
            c = Coefficients(w["kind"], w["param"])
            rows = oracle_assemble(g, c, w["n_paths"], w["h"], w["seed"], instance=w["instance"],
                                   exit_rule=w["exit_rule"])["rows"]
            assert_same_stream(fetch(o, g), g, to_csr(g, rows))
    finally:
        ctx.set_launch(0, 0, 0)
        ctx.set_spare_rows(-1)


def test_spare_row_argument_validation(ctx):
    with pytest.raises(pdd.PddError) as e:
        ctx.set_spare_rows(-2)
    assert e.value.status == pdd.EINVAL
