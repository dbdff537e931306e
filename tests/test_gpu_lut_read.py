"""Float32 table reads: the lane-per-path read of the varying fields against
the full cooperative read of all seven.

A field that holds one value at every node has the bilinear form
(v, 0, 0, 0) on every cell, which evaluates to v, so reading only the
varying fields changes no bit of any path: the two reads must give the same
paths (the dumped exit records), the same G and the same integer per-knot
sums exactly (static schedule, fixed launch shape).  The two kernels add
b, sum s and sum s^2 in different orders (per-lane sums flushed per ticket
against per-row sums), so those agree to float64 rounding.  The scan that
decides between them is checked on tables with zero, one, two and seven
varying fields, a constant -0 (the full read turns it into +0) and a
misaligned table pointer.
"""
import numpy as np
import pytest

from paper_2301_05780_amd import pdd, workloads

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

N = 129


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = pdd.Context(0)
    yield c
    c.set_table_read(False)
    c.close()


DUMP = 16


def _assert_same(a, b, what):
    """G, the dumped paths and the integer per-knot sums (sum K, N, the exit
    counts) bit for bit; b and the score sums to float64 rounding."""
    for k in ("val", "dump"):
        if k in a and k in b:
            x, y = a[k], b[k]
            assert torch.equal(torch.nan_to_num(x, nan=-7.0), torch.nan_to_num(y, nan=-7.0)), (what, k)
    da, db = a["diag"].view(-1, pdd.DIAG_WIDTH), b["diag"].view(-1, pdd.DIAG_WIDTH)
    assert torch.equal(da[:, :6], db[:, :6]), (what, "diag counts")
    for x, y, k in ((a["b"], b["b"], "b"), (da[:, 6:], db[:, 6:], "diag sums")):
        assert torch.allclose(x, y, rtol=1e-12, atol=1e-14), (what, k, float((x - y).abs().max()))


def _work(rule):
    return dict(kind="lut", param=(), domain=(0.0, 1.0, 0.0, 1.0), H=4, m=8, ext=4, n_paths=700,
                h=1e-3, seed=5, precision="fp32", exit_rule=rule, instance=0, lut_n=N)


def _tables():
    base = workloads.poisson_lut(N)
    xs = np.arange(N) / (N - 1)
    two = base.copy()
    two[..., 2] = np.sqrt(2.0) * (1.0 + 0.2 * np.sin(2 * np.pi * xs))[None, :]      # syy(x) and f vary
    none = base.copy()
    none[..., 6] = -1.0                                                              # every field constant
    negzero = base.copy()
    negzero[..., 3] = -0.0                                                           # dx = -0 everywhere
    return {
        "one_field": (base, 1 << 6, True),
        "two_fields": (two, (1 << 2) | (1 << 6), True),
        "no_field": (none, 0, True),
        "negative_zero": (negzero, 1 << 6, True),
        "all_fields": (workloads.varied_lut(N), 0x7F, False),
    }


@pytest.mark.parametrize("rule", ["gm", "naive"])
@pytest.mark.parametrize("name", ["one_field", "two_fields", "no_field", "negative_zero", "all_fields"])
def test_lane_read_equals_full_read(ctx, name, rule):
    tab, mask, lane = _tables()[name]
    w = _work(rule)
    lut = torch.from_numpy(np.ascontiguousarray(tab)).cuda()
    outs = []
    for read_all in (False, True):
        ctx.set_table_read(read_all)
        out = ctx.assemble(w, lut=lut, dump_paths=DUMP)
        ctx.sync()
        got_mask, got_lane = ctx.table_fields()
        assert got_mask == mask, (name, hex(got_mask))
        assert got_lane == (lane and not read_all), name
        outs.append({k: out[k][:out["nnz"]].clone() if k == "val" else out[k].clone()
                     for k in ("val", "b", "diag", "dump")})
    ctx.set_table_read(False)
    _assert_same(outs[0], outs[1], name)
    assert float(outs[0]["diag"].view(-1, pdd.DIAG_WIDTH)[:, 0].sum()) > 0


def test_misaligned_table_is_refused(ctx):
    w = _work("gm")
    flat = torch.from_numpy(workloads.poisson_lut(N)).cuda().view(-1)
    shifted = torch.empty(flat.numel() + 4, dtype=torch.float32, device="cuda")[1:]
    shifted[: flat.numel()].copy_(flat)
    with pytest.raises(pdd.PddError) as e:
        ctx.assemble(w, lut=shifted)
    assert e.value.status == pdd.EINVAL


def test_stale_lane_choice_in_a_graph_reads_the_full_layout():
    """While a graph is captured the library cannot read the layout back, so
    it launches the kernel the last eager call chose.  Captured after a
    one-field table, an assembly of a seven-field table launches the
    lane-per-path kernel on the full copy; that kernel reads the layout word
    itself and takes its full per-lane read, so every replay gives the eager
    (cooperative-read) assembly's G and integer sums bit for bit and its b
    to float64 rounding (same launch shape, static schedule), and the
    replays equal each other bit for bit."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        g = pdd.Context(0, stream=stream)
        try:
            g.set_launch(256, 64, 200, "static")
            w = _work("gm")
            full = torch.from_numpy(workloads.varied_lut(N)).cuda()
            one = torch.from_numpy(workloads.poisson_lut(N)).cuda()
            out = g.assemble(w, lut=full)
            g.sync()
            assert g.table_fields() == (0x7F, False)
            ref = {k: out[k].clone() for k in ("val", "b", "diag")}
            other = g.assemble(w, lut=one)
            g.sync()
            assert g.table_fields() == (1 << 6, True)
            g.graph_begin()
            g.assemble(w, out=out, lut=full)
            g.graph_end()
            first = None
            for rep in range(2):
                for k in ("val", "b", "diag"):
                    out[k].fill_(float("nan"))
                g.graph_launch()
                g.sync()
                assert g.table_fields() == (0x7F, False)
                got = {k: out[k].clone() for k in ("val", "b", "diag")}
                _assert_same(got, ref, ("replay", rep))
                if first is None:
                    first = got
                for k in ("val", "b", "diag"):
                    assert torch.equal(got[k], first[k]), (rep, k)
                g.assemble(w, out=other, lut=one)          # eager work between the replays
                g.sync()
        finally:
            g.close()


def test_constant_sigma_thresholds_equal_the_exact_test():
    """With sigma constant over the table, float32 GM exits use fixed exact
    thresholds instead of the candidate test plus the exact test at the
    projection.  Against a table whose sxy holds -0 at one node (a varying
    field to the scan, so the exact test runs, but every interpolated value
    and a_nn are the same), G, b and the per-knot sums agree bit for bit."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = pdd.Context(0)
    try:
        w = _work("gm")
        a = workloads.poisson_lut(N)
        b = a.copy()
        b[N // 2, N // 2, 1] = -0.0
        outs = []
        for tab, mask in ((a, 1 << 6), (b, (1 << 1) | (1 << 6))):
            out = c.assemble(w, lut=torch.from_numpy(tab).cuda())
            c.sync()
            assert c.table_fields() == (mask, True)
            outs.append(out)
        for k in ("val", "b", "diag"):
            assert torch.equal(outs[0][k], outs[1][k]), k
    finally:
        c.close()


@pytest.mark.parametrize("n", [2, 3, 6])
def test_tiny_tables(ctx, n):
    """Tables of one, four and 25 cells (every path in the first or last
    cell of a row or column, the edge clamps taken on both sides): the lane
    read gives the full read's paths, G and counts bit for bit."""
    w = dict(_work("gm"), lut_n=n)
    tab = workloads.poisson_lut(n)
    lut = torch.from_numpy(tab).cuda()
    outs = []
    for read_all in (False, True):
        ctx.set_table_read(read_all)
        out = ctx.assemble(w, lut=lut, dump_paths=DUMP)
        ctx.sync()
        assert ctx.table_fields() == (1 << 6, not read_all)
        outs.append({k: out[k].clone() for k in ("val", "b", "diag", "dump")})
    ctx.set_table_read(False)
    _assert_same(outs[0], outs[1], n)


def test_table_read_switch_rejects_other_values(ctx):
    with pytest.raises(pdd.PddError) as e:
        ctx.check(pdd.lib().pdd_set_table_read(ctx.h, 2))
    assert e.value.status == pdd.EINVAL
