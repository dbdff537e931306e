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


def _bf16_grad_bound(th, X):
    """First-order bound on |grad v (bf16 MFMA routine) - grad v (float64)|
    per point and component, from the rounding of the bf16 operands (unit
    roundoff u = 2^-9; float32 accumulation and the hi/lo splits of layer 1
    and of the final contraction, about 2^-16, are far below it):
      z2:  W2 and h1 rounded           |dz2_j| <= 2.01 u sum_k |W2_jk h1_k|
      g2 = 1 - tanh^2 z2:              |dg2_j| <= 2 |h2_j| g2_j |dz2_j| + u g2_j (storage)
      dh1_k = sum_j W2_jk w3_j g2_j:   W2^T w3 and g2 rounded (2 u) plus dg2
      D_k = dh1_k (1 - h1_k^2):        1 - h1^2 from the rounded h1 (2 h1^2 u), D rounded (u)
      grad v = W1^T D:                 |d grad v| <= |W1|^T |dD|."""
    W1, b1, W2, b2, w3, b3 = omlp.unpack(th)
    u = 2.0 ** -9
    h1 = np.tanh(X @ W1.T + b1)
    h2 = np.tanh(h1 @ W2.T + b2)
    g2 = 1.0 - h2 * h2
    dz2 = 2.01 * u * (np.abs(h1) @ np.abs(W2).T)
    dg2 = 2.0 * np.abs(h2) * g2 * dz2 + u * g2
    dh1 = (g2 * w3) @ W2
    ddh1 = (2.0 * u * g2 + dg2) @ np.abs(W2 * w3[:, None])
    dD = ddh1 * (1.0 - h1 * h1) + np.abs(dh1) * (2.0 * h1 * h1 + 1.0) * u
    return dD @ np.abs(W1)


def _bf16_grad_spread(th, X):
    """The same propagation with rounding errors taken as independent and
    uniform on (-u, u) (variance u^2 / 3): root-sum-square instead of absolute
    sums, the expected size of the bf16 error per point and component."""
    W1, b1, W2, b2, w3, b3 = omlp.unpack(th)
    v = (2.0 ** -9) ** 2 / 3.0
    h1 = np.tanh(X @ W1.T + b1)
    h2 = np.tanh(h1 @ W2.T + b2)
    g2 = 1.0 - h2 * h2
    dz2 = np.sqrt(2.0 * v * ((h1 * h1) @ (W2 * W2).T))
    dg2 = np.sqrt((2.0 * np.abs(h2) * g2 * dz2) ** 2 + v * g2 * g2)
    dh1 = (g2 * w3) @ W2
    ddh1 = np.sqrt((2.0 * v * g2 * g2 + dg2 * dg2) @ ((W2 * w3[:, None]) ** 2))
    dD = np.sqrt((ddh1 * (1.0 - h1 * h1)) ** 2 + dh1 * dh1 * (4.0 * h1 ** 4 + 1.0) * v)
    return np.sqrt((dD * dD) @ (W1 * W1))


@pytest.mark.parametrize("seed,n", [(1, 20011), (9, 64), (10, 1)])
def test_bf16_mfma_gradient_against_oracle(ctx, seed, n):
    """The routine the float32 network control variate runs at every step
    (bf16 MFMA, float32 accumulation) against the float64 input gradient:
    every component within twice the first-order bf16 rounding bound, the
    whole set within 2e-2 in norm (the bf16 bar), and the errors of the
    20011-point set no larger on average than the independent-rounding model
    predicts (a mis-ordered fragment or a wrong scale would add a systematic
    error far above it).  n = 20011 covers several workgroups and a ragged
    last wave, 64 exactly one wave, 1 a single lane."""
    th = _theta(seed)
    rng = np.random.default_rng(seed + 40)
    X = np.concatenate([rng.uniform(-0.2, 1.2, size=(n, 2))[:max(n - 4, 1)],
                        np.array([[0.0, 0.0], [1.0, 1.0], [0.5, 0.25], [1.2, -0.2]])])[:n]
    g = ctx.mlp_grad_bf16(_dev(th, np.float32), _dev(X, np.float32)).cpu().numpy().astype(np.float64)
    Xf = X.astype(np.float32).astype(np.float64)
    g_ref = omlp.grad_input(th, Xf)
    bound = _bf16_grad_bound(th, Xf)
    err = np.abs(g - g_ref)
    assert np.all(err <= 2.0 * bound + 1e-6), float(np.max(err / (bound + 1e-12)))
    assert np.linalg.norm(g - g_ref) <= 2e-2 * np.linalg.norm(g_ref)
    spread = _bf16_grad_spread(th, Xf)
    z = err / spread
    print(f"bf16 grad: rel. norm error {np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref):.2e}, "
          f"rms(err / spread) {np.sqrt(np.mean(z * z)):.3f}, max(err / bound) {np.max(err / bound):.3f}")
    if n >= 1000:
        assert np.sqrt(np.mean(z * z)) < 3.0


def test_network_cv_fp32_paths_against_oracle(ctx):
    """Per-path records of the float32 assembly with the per-step bf16 network
    against the float64 oracle's run with the same network on the same
    stream: step counts equal (float32 vs float64 exit flips excepted, at most
    1 %), exit points within float32 drift, and Xi of every path within the
    sum over its steps of |Y_n (sigma dW_n)| times twice the bf16 bound of
    grad v at X_n (the replayed oracle path), plus float32 summation."""
    from oracle.philox import normals_for_draw
    w = workloads.poisson_small("gm")
    w["precision"] = "fp32"
    dumps = 16
    g = Geometry(w["domain"], w["H"], w["m"], w["ext"])
    c = Coefficients("poisson")
    th = _theta(6)
    res = oracle_assemble(g, c, w["n_paths"], w["h"], w["seed"], exit_rule="gm", cv=omlp.NetworkCV(th),
                          keep_paths=True)
    out = ctx.assemble(w, cv=pdd.CVSpec("network", params=_dev(th, np.float32)), dump_paths=dumps)
    ctx.sync()
    dump = out["dump"].cpu().numpy().reshape(g.n, dumps, pdd.DUMP_WIDTH)
    sq = np.sqrt(w["h"])
    sig = np.sqrt(2.0)                                  # poisson: sigma = sqrt(2) I, Y = 1
    flips = checked = 0
    for k in range(g.n):
        p = res["paths"][k]
        K = p["K"][:dumps]
        same = dump[k, :, 0] == K
        flips += int(np.sum(~same))
        # replay the oracle's paths of this knot: X_n and the normals of every step
        ids = np.arange(dumps, dtype=np.uint64)
        x = np.tile([g.x[k], g.y[k]], (dumps, 1)).astype(np.float64)
        tol = np.zeros(dumps)
        for n in range(int(K.max())):
            first, second = normals_for_draw(n // 2, ids, k, 0, w["seed"])
            nx, ny = first if n % 2 == 0 else second
            live = n < K
            b = 2.0 * _bf16_grad_bound(th, x)
            tol += np.where(live, sig * sq * (b[:, 0] * np.abs(nx) + b[:, 1] * np.abs(ny)), 0.0)
            x = x + np.where(live[:, None], sig * sq * np.stack([nx, ny], axis=1), 0.0)
        xi_gpu, xi_ref = dump[k, same, 5], p["Xi"][:dumps][same]
        assert np.all(np.abs(xi_gpu - xi_ref) <= tol[same] + 1e-5 * (1 + K[same] * 1e-2)), k
        assert np.allclose(dump[k, same, 1], p["x"][:dumps][same], rtol=0, atol=1e-4)
        assert np.allclose(dump[k, same, 2], p["y"][:dumps][same], rtol=0, atol=1e-4)
        checked += int(same.sum())
    assert flips <= 0.01 * g.n * dumps and checked > 0


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
    b_k - sum_{j != k} G_kj u0_j of the assembly that used the same paths: the
    one with instance word PDD_COLLECT_STREAM.  The assembly with instance
    word 0 draws other paths (the pairs' own stream class)."""
    w = workloads.poisson_small("gm")
    w["precision"] = "fp32"
    out0 = ctx.assemble(w)
    u0, _, _ = ctx.solve(out0["row_ptr"], out0["col_idx"], out0["val"][:out0["nnz"]], out0["b"])
    out = ctx.assemble(dict(w, instance=pdd.COLLECT_STREAM))
    xy, t = ctx.collect(w, u0, w["n_paths"], 8)
    ctx.sync()
    b0 = out0["b"].cpu().numpy()
    assert np.mean(np.abs(b0 - out["b"].cpu().numpy()) > 1e-9) > 0.9      # other paths
    with pytest.raises(pdd.PddError) as e:
        ctx.collect(dict(w, instance=pdd.COLLECT_STREAM), u0, 4, 2)
    assert e.value.status == pdd.EINVAL
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
