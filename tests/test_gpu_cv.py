"""GPU control variate (eqs. 11, 37-38): network kernels against the float64
oracle, same-stream parity of the control-variate assembly, the training-pair
identity, and the gain of the trained network over the plain estimator."""
import numpy as np
import pytest

from paper_2301_05780_amd import pdd, workloads, cv as cvmod
from oracle import mlp as omlp
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


def _theta(seed=0, noise=0.05):
    rng = np.random.default_rng(seed + 100)
    th = workloads.mlp_init(seed) + rng.normal(0.0, noise, workloads.MLP_PARAMS)
    return th.astype(np.float32).astype(np.float64)      # exactly representable in float32


def _dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a).astype(dtype)).to("cuda")


def test_mlp_init_follows_the_counter_stream(ctx):
    """Zero biases; weight i = lim (2u - 1), u from the first Philox word at
    counter (i, 0, 0, 0): recomputed with the oracle's own generator."""
    from oracle.philox import philox4x32_10
    seed = (7 << 32) + 11
    th = ctx.mlp_init(seed).cpu().numpy().astype(np.float64)
    ctx.sync()
    w = workloads.MLP_WIDTH
    r0 = philox4x32_10(np.arange(workloads.MLP_PARAMS), 0, 0, 0, seed & 0xFFFFFFFF, seed >> 32)[0]
    u = (r0.astype(np.float64) + 0.5) * 2.0 ** -32
    fan = np.zeros(workloads.MLP_PARAMS)
    fan[0:2 * w] = w + 2                                   # W1
    fan[3 * w:3 * w + w * w] = 2 * w                       # W2
    fan[4 * w + w * w:5 * w + w * w] = w + 1               # w3
    ref = np.where(fan > 0, np.sqrt(6.0 / np.maximum(fan, 1)) * (2.0 * u - 1.0), 0.0).astype(np.float32)
    assert np.allclose(th, ref, rtol=2.0 ** -22, atol=0.0)
    assert np.all(th[fan == 0] == 0.0)
    # the uniform law of each weight block: variance lim^2 / 3
    W2 = th[3 * w:3 * w + w * w]
    lim2 = 6.0 / (2 * w)
    assert abs(W2.var() / (lim2 / 3.0) - 1.0) < 0.1
    assert np.abs(W2).max() < np.sqrt(lim2)
    other = ctx.mlp_init(seed + 1).cpu().numpy()
    assert not np.array_equal(other, th.astype(np.float32))


def test_network_eval_and_input_gradient(ctx):
    th = _theta(1)
    rng = np.random.default_rng(2)
    X = rng.uniform(-0.2, 1.2, size=(1000, 2))
    v, g = ctx.mlp_eval(_dev(th, np.float32), _dev(X, np.float32))
    ctx.sync()
    Xf = X.astype(np.float32).astype(np.float64)
    v_ref, _ = omlp.forward(th, Xf)
    g_ref = omlp.grad_input(th, Xf)
    assert np.allclose(v.cpu().numpy(), v_ref, rtol=1e-4, atol=1e-5 * np.abs(v_ref).max())
    assert np.allclose(g.cpu().numpy(), g_ref, rtol=1e-4, atol=1e-5 * np.abs(g_ref).max())


def test_loss_gradient_against_oracle(ctx):
    th = _theta(2)
    rng = np.random.default_rng(3)
    X = rng.uniform(0, 1, size=(300, 2))
    T = np.sin(3 * X[:, 0]) + X[:, 1] ** 2
    Xf, Tf = X.astype(np.float32).astype(np.float64), T.astype(np.float32).astype(np.float64)
    grad, loss = ctx.mlp_grad(_dev(th, np.float32), _dev(X, np.float32), _dev(T, np.float32))
    ctx.sync()
    l_ref, g_ref = omlp.loss_and_grad(th, Xf, Tf)
    g = grad.cpu().numpy()
    assert abs(float(loss.cpu()[0]) - l_ref) <= 1e-5 * l_ref
    assert np.linalg.norm(g - g_ref) <= 1e-4 * np.linalg.norm(g_ref)
    for lo, hi in [(0, 128), (128, 192), (192, 4288), (4288, 4352), (4352, 4416), (4416, 4417)]:
        assert np.linalg.norm(g[lo:hi] - g_ref[lo:hi]) <= 1e-4 * np.linalg.norm(g_ref[lo:hi]) + 1e-7


def test_adam_training_against_oracle(ctx):
    th0 = _theta(3, noise=0.0)
    rng = np.random.default_rng(4)
    X = rng.uniform(0, 1, size=(512, 2))
    T = np.cos(2 * X[:, 0]) * X[:, 1]
    order = workloads.minibatch_order(512, 2, seed=5)
    batch, steps = 64, 16
    Xf, Tf = X.astype(np.float32).astype(np.float64), T.astype(np.float32).astype(np.float64)
    th_ref, losses_ref = omlp.train(th0, Xf, Tf, order[:batch * steps], batch, 1e-3)
    p = _dev(th0, np.float32)
    m, s = torch.zeros_like(p), torch.zeros_like(p)
    losses = ctx.mlp_train(p, m, s, _dev(X, np.float32), _dev(T, np.float32), _dev(order, np.int32), batch, steps, 0,
                           1e-3)
    ctx.sync()
    assert np.allclose(losses.cpu().numpy(), losses_ref, rtol=1e-3)
    d_gpu = p.cpu().numpy().astype(np.float64) - th0
    d_ref = th_ref - th0
    assert np.linalg.norm(d_gpu - d_ref) <= 2e-3 * np.linalg.norm(d_ref)


def test_grad_table_bake(ctx):
    th = _theta(4)
    w = workloads.poisson_small()
    n = 33
    tab = ctx.mlp_bake(_dev(th, np.float32), w, n).cpu().numpy()
    xs = np.arange(n) / (n - 1)
    X, Y = np.meshgrid(xs, xs)
    ref = omlp.grad_input(th, np.stack([X.ravel(), Y.ravel()], axis=1)).reshape(n, n, 2)
    assert np.allclose(tab, ref, rtol=1e-4, atol=1e-5 * np.abs(ref).max())


def _fetch(out, g):
    return (out["val"].cpu().numpy()[:g.nnz], out["b"].cpu().numpy(),
            out["diag"].cpu().numpy().reshape(g.n, pdd.DIAG_WIDTH))


@pytest.mark.parametrize("mode", ["network", "grad_lut"])
def test_cv_fp64_same_stream_parity(ctx, mode):
    """float64 same-stream assembly with the control variate against the oracle
    with the same network (or the same table) to 1e-12 of the row mass."""
    w = dict(workloads.poisson_small("gm"), n_paths=200, kind="varcoef", H=3, m=6, ext=3, h=2e-3)
    g = Geometry(w["domain"], w["H"], w["m"], w["ext"])
    c = Coefficients("varcoef")
    th = _theta(5)
    if mode == "network":
        spec = pdd.CVSpec("network", params=_dev(th, np.float32))
        ocv = omlp.NetworkCV(th)
    else:
        n = 65
        xs = np.arange(n) / (n - 1)
        X, Y = np.meshgrid(xs, xs)
        table = omlp.grad_input(th, np.stack([X.ravel(), Y.ravel()], axis=1)).reshape(n, n, 2).astype(np.float32)
        spec = pdd.CVSpec("grad_lut", table=_dev(table, np.float32))
        ocv = omlp.GradLutCV(table, w["domain"])
    ref = to_csr(g, oracle_assemble(g, c, w["n_paths"], w["h"], w["seed"], exit_rule="gm", cv=ocv)["rows"])
    out = ctx.assemble(w, cv=spec)
    ctx.sync()
    val, b, diag = _fetch(out, g)
    row_of = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    tol = 1e-12 * ref["mass"]
    assert np.all(np.abs(val - ref["val"]) <= tol[row_of])
    assert np.all(np.abs(b - ref["b"]) <= tol)
    assert np.array_equal(diag[:, :6], ref["diag"][:, :6])


@pytest.mark.parametrize("mode", ["network", "grad_lut"])
def test_cv_fp32_production_within_se(ctx, mode):
    """float32 production (MFMA bf16 network or float32 table) against the
    float64 oracle with the same control variate: G unchanged, b within 3 SE."""
    w = workloads.poisson_small("gm")
    w["precision"] = "fp32"
    g = Geometry(w["domain"], w["H"], w["m"], w["ext"])
    c = Coefficients("poisson")
    th = _theta(6)
    if mode == "network":
        spec = pdd.CVSpec("network", params=_dev(th, np.float32))
        ocv = omlp.NetworkCV(th)
    else:
        n = 129
        xs = np.arange(n) / (n - 1)
        X, Y = np.meshgrid(xs, xs)
        table = omlp.grad_input(th, np.stack([X.ravel(), Y.ravel()], axis=1)).reshape(n, n, 2).astype(np.float32)
        spec = pdd.CVSpec("grad_lut", table=_dev(table, np.float32))
        ocv = omlp.GradLutCV(table, w["domain"])
    ref = to_csr(g, oracle_assemble(g, c, w["n_paths"], w["h"], w["seed"], exit_rule="gm", cv=ocv)["rows"])
    plain = ctx.assemble(w)
    ctx.sync()
    pval, pb, _ = _fetch(plain, g)
    out = ctx.assemble(w, cv=spec)
    ctx.sync()
    val, b, _ = _fetch(out, g)
    assert np.allclose(val, pval, rtol=0, atol=1e-15)              # the CV touches b only
    assert np.all(np.abs(val - ref["val"]) <= 3 * ref["se_val"] + 1e-6)
    assert np.all(np.abs(b - ref["b"]) <= 3 * ref["se_b"] + 1e-5)


def test_collected_pairs_reproduce_the_rows(ctx):
    """The first pair of every path sits at the knot and its target is the
    path's full score with u0 at the exit, so its mean over the knot's paths is
    b_k - sum_{j != k} G_kj u0_j of the assembly that used the same paths."""
    w = workloads.poisson_small("gm")
    w["precision"] = "fp32"
    out = ctx.assemble(w)
    u0, _, _ = ctx.solve(out["row_ptr"], out["col_idx"], out["val"][:out["nnz"]], out["b"])
    xy, t = ctx.collect(w, u0, w["n_paths"], 8)
    ctx.sync()
    n, nnz = out["n"], out["nnz"]
    rp = out["row_ptr"].cpu().numpy()
    ci = out["col_idx"].cpu().numpy()[:nnz]
    val = out["val"].cpu().numpy()[:nnz]
    b = out["b"].cpu().numpy()
    u = u0.cpu().numpy()
    t0 = t.cpu().numpy().reshape(n, w["n_paths"], 8)[:, :, 0]
    xy0 = xy.cpu().numpy().reshape(n, w["n_paths"], 8, 2)[:, :, 0]
    kxy = pdd.knot_xy(w)
    assert np.allclose(xy0, kxy[:, None, :].astype(np.float32))
    for k in range(n):
        a, e = rp[k], rp[k + 1]
        off = ci[a:e] != k
        expect = b[k] - np.dot(val[a:e][off], u[ci[a:e][off]])
        assert abs(t0[k].mean() - expect) <= 2e-5 * max(1.0, abs(expect))
    # later pairs: targets are finite where recorded, NaN past the exit
    tt = t.cpu().numpy()
    assert np.isfinite(tt).mean() > 0.5 and np.isnan(tt).any()


def test_trained_network_reduces_variance(ctx):
    """The network trained on the method's own pathwise estimates cuts the
    per-knot score variance (eq. 11) while b stays unbiased (eq. 38)."""
    w = workloads.poisson_small("gm")
    w["precision"] = "fp32"
    xy = pdd.knot_xy(w)
    ue = Coefficients("poisson").exact(xy[:, 0], xy[:, 1])
    u_ref = torch.from_numpy(ue).to("cuda")
    plain = ctx.assemble(w, u_ref=u_ref)
    u0, _, _ = ctx.solve(plain["row_ptr"], plain["col_idx"], plain["val"][:plain["nnz"]], plain["b"])
    params, info = cvmod.fit(ctx, w, u0, epochs=4)
    # the targets are single-path scores: the loss falls to their noise floor
    assert info["losses"][-50:].mean() < 0.9 * info["losses"][:20].mean()
    d_plain = plain["diag"].view(-1, pdd.DIAG_WIDTH).cpu().numpy().copy()
    b_plain = plain["b"].cpu().numpy().copy()
    res = {}
    for mode in ["network", "grad_lut"]:
        spec = pdd.CVSpec(mode, params=params) if mode == "network" else \
            pdd.CVSpec(mode, table=ctx.mlp_bake(params, w, 257))
        out = ctx.assemble(w, cv=spec, u_ref=u_ref)
        ctx.sync()
        d = out["diag"].view(-1, pdd.DIAG_WIDTH).cpu().numpy()
        N = d[:, 1]
        var = d[:, 7] / N - (d[:, 6] / N) ** 2
        var_p = d_plain[:, 7] / N - (d_plain[:, 6] / N) ** 2
        ratio = var_p / var
        res[mode] = ratio
        # unbiased: the control-variate b stays within a few plain standard errors
        se = np.sqrt(var_p / N)
        assert np.all(np.abs(out["b"].cpu().numpy() - b_plain) <= 4 * se + 1e-9)
    print("median variance reduction", {k: float(np.median(v)) for k, v in res.items()})
    assert np.median(res["grad_lut"]) > 5.0
    assert np.median(res["network"]) > 5.0


def test_cv_in_a_batch_fp64_same_stream(ctx):
    """Three replicas of one problem (instance words 0, 1, 2) with the gradient
    table in one batched launch: each equals the oracle's run of its instance
    to 1e-12 of the row mass."""
    w = dict(workloads.poisson_small("gm"), n_paths=120, kind="varcoef", H=3, m=6, ext=3, h=2e-3)
    g = Geometry(w["domain"], w["H"], w["m"], w["ext"])
    c = Coefficients("varcoef")
    th = _theta(6)
    n = 65
    xs = np.arange(n) / (n - 1)
    X, Y = np.meshgrid(xs, xs)
    table = omlp.grad_input(th, np.stack([X.ravel(), Y.ravel()], axis=1)).reshape(n, n, 2).astype(np.float32)
    spec = pdd.CVSpec("grad_lut", table=_dev(table, np.float32))
    ocv = omlp.GradLutCV(table, w["domain"])
    ws = [dict(w, instance=i) for i in range(3)]
    outs = ctx.assemble_batch(ws, cv=spec)
    ctx.sync()
    row_of = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    for i, out in enumerate(outs):
        ref = to_csr(g, oracle_assemble(g, c, w["n_paths"], w["h"], w["seed"], instance=i, exit_rule="gm",
                                        cv=ocv)["rows"])
        val, b, diag = _fetch(out, g)
        tol = 1e-12 * ref["mass"]
        assert np.all(np.abs(val - ref["val"]) <= tol[row_of]), i
        assert np.all(np.abs(b - ref["b"]) <= tol), i
        assert np.array_equal(diag[:, :6], ref["diag"][:, :6]), i


def test_network_cv_in_a_batch_matches_single_runs(ctx):
    """float32 network control variate: a batch of replicas gives each
    replica's single-instance result up to float64 summation order."""
    w = dict(workloads.poisson_small("gm"), n_paths=150, kind="varcoef", H=3, m=6, ext=3, h=2e-3,
             precision="fp32")
    spec = pdd.CVSpec("network", params=_dev(_theta(7), np.float32))
    ws = [dict(w, instance=i) for i in range(2)]
    outs = ctx.assemble_batch(ws, cv=spec)
    ctx.sync()
    g = Geometry(w["domain"], w["H"], w["m"], w["ext"])
    for i, out in enumerate(outs):
        single = ctx.assemble(ws[i], cv=spec)
        ctx.sync()
        a, b = _fetch(out, g), _fetch(single, g)
        assert np.allclose(a[0], b[0], rtol=0, atol=1e-9) and np.allclose(a[1], b[1], rtol=0, atol=1e-9), i
        assert np.array_equal(a[2][:, :6], b[2][:, :6]), i


def test_batch_rejects_mismatched_control_variates(ctx):
    w = dict(workloads.poisson_small("gm"), n_paths=50, kind="varcoef", precision="fp32")
    spec = pdd.CVSpec("network", params=_dev(_theta(8), np.float32))
    arr, outs = ctx.batch_arrays([w, dict(w, instance=1)], cv=spec)
    arr[1].run.cv = None
    with pytest.raises(pdd.PddError) as e:
        ctx.assemble_batch(None, arr=arr)
    assert e.value.status == pdd.EINVAL
    with pytest.raises(pdd.PddError) as e:
        ctx.assemble_batch([dict(w, precision="fp64"), dict(w, precision="fp64", instance=1)], cv=spec)
    assert e.value.status == pdd.EUNSUPPORTED


def test_network_on_a_non_unit_domain(ctx):
    """The network sees the domain's unit coordinates: the baked table on
    [-100, 100]^2 is grad v at the mapped nodes scaled by 1/200, and the
    float64 same-stream assembly with the per-step network matches the
    oracle's NetworkCV on that domain."""
    th = _theta(6)
    w = dict(kind="eq43", param=(), domain=(-100.0, 100.0, -100.0, 100.0), H=3, m=4, ext=2, n_paths=64, h=2.0,
             seed=21, precision="fp64", exit_rule="gm")
    n = 33
    tab = ctx.mlp_bake(_dev(th, np.float32), w, n).cpu().numpy()
    xs = np.arange(n) / (n - 1)
    X, Y = np.meshgrid(xs, xs)
    ref = omlp.grad_input(th, np.stack([X.ravel(), Y.ravel()], axis=1)).reshape(n, n, 2) / 200.0
    assert np.allclose(tab, ref, rtol=1e-4, atol=1e-5 * np.abs(ref).max())
    g = Geometry(w["domain"], w["H"], w["m"], w["ext"])
    spec = pdd.CVSpec("network", params=_dev(th, np.float32))
    ref = to_csr(g, oracle_assemble(g, Coefficients("eq43"), w["n_paths"], w["h"], w["seed"], exit_rule="gm",
                                    cv=omlp.NetworkCV(th, w["domain"]))["rows"])
    out = ctx.assemble(w, cv=spec)
    ctx.sync()
    val, b, diag = _fetch(out, g)
    tol = 1e-12 * ref["mass"]
    assert np.all(np.abs(b - ref["b"]) <= tol)
    assert np.array_equal(diag[:, :6], ref["diag"][:, :6])


@pytest.mark.parametrize("batch", [1536, 4096])
def test_wide_adam_steps_against_oracle(ctx, batch):
    """Batches above 1024 take the multi-workgroup step (gradient slices of
    256 points summed in workgroup order, Adam in a second kernel): the loss
    history and the parameter change follow the float64 oracle."""
    th0 = _theta(7, noise=0.0)
    rng = np.random.default_rng(11)
    n = 8192
    X = rng.uniform(0, 1, size=(n, 2))
    T = np.cos(2 * X[:, 0]) * X[:, 1] + 0.3 * np.sin(3 * X[:, 1])
    order = workloads.minibatch_order(n, 3, seed=6)
    steps = 6                      # batch * steps <= 3 n: the oracle sees the same points
    Xf, Tf = X.astype(np.float32).astype(np.float64), T.astype(np.float32).astype(np.float64)
    th_ref, losses_ref = omlp.train(th0, Xf, Tf, order[:batch * steps], batch, 1e-3)
    p = _dev(th0, np.float32)
    m, s = torch.zeros_like(p), torch.zeros_like(p)
    losses = ctx.mlp_train(p, m, s, _dev(X, np.float32), _dev(T, np.float32), _dev(order, np.int32), batch, steps, 0,
                           1e-3)
    ctx.sync()
    assert np.allclose(losses.cpu().numpy(), losses_ref, rtol=1e-3)
    d_gpu = p.cpu().numpy().astype(np.float64) - th0
    d_ref = th_ref - th0
    assert np.linalg.norm(d_gpu - d_ref) <= 2e-3 * np.linalg.norm(d_ref)
