"""GPU parity: the HIP library (through the C ABI) against the CPU oracle.

Tolerances: log-determinants and f within 1e-10 relative; mean within 1e-9
(max-norm relative); variances within 1e-9 per component; the adjoint
gradient within 1e-9 of the oracle's dense-inverse gradient; factor and
selected-inverse blocks within 1e-11 relative to the block norm.
"""
import math

import numpy as np
import pytest

import oracle as O
from inla_synth import THETA0, config_model, make_model

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(params=[("64", "0"), ("64", "1"), ("64", "2"), ("64", "3"), ("64", "4"),
                        ("64", "5"),
                        ("128", "0"), ("128", "3"), ("128", "4"), ("128", "5")],
                ids=["tile64", "tile64dma32", "tile64dma16", "tile64dma16s4", "tile64auto",
                     "tile64dma16w8",
                     "tile128", "tile128dma32", "tile128dma16", "tile128dma16w4"])
def tile(request, monkeypatch):
    """Run the b x b product phases on 64- or 128-wide tiles: 64 in the 64-tile
    kernel (form 0) or in the product kernel with direct-to-LDS staging (forms
    1, 2, 3: k-chunks of 32 and 16, and 16 with four LDS stages; form 4
    picks 1 or 2 by launch size; form 5: k-chunk 16 on eight waves); 128 with
    register staging (layout 0) or
    direct-to-LDS staging (layouts 3-5: 8 waves with k-chunks of 32 and 16,
    4 waves with k-chunk 16)."""
    size, variant = request.param
    monkeypatch.setenv("INLA_TILE", size)
    monkeypatch.setenv("INLA_SMALL_VARIANT" if size == "64" else "INLA_BIG_VARIANT", variant)
    return size


@pytest.fixture(scope="module")
def P():
    import paper_2204_04678_amd as P
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    P.lib()
    return P


def rel(a, b):
    return abs(a - b) / abs(b)


def rand_spd_bta(b, nt, a, seed):
    """Dense SPD matrix with the BTA pattern (strict diagonal dominance)."""
    rng = np.random.default_rng(seed)
    n = b * nt + a
    Q = np.zeros((n, n))
    for t in range(nt):
        blk = rng.uniform(-1, 1, (b, b))
        Q[t * b:(t + 1) * b, t * b:(t + 1) * b] = blk
        if t + 1 < nt:
            Q[(t + 1) * b:(t + 2) * b, t * b:(t + 1) * b] = rng.uniform(-1, 1, (b, b))
        if a:
            Q[b * nt:, t * b:(t + 1) * b] = rng.uniform(-1, 1, (a, b))
    if a:
        Q[b * nt:, b * nt:] = rng.uniform(-1, 1, (a, a))
    Q = np.tril(Q)
    Q = Q + np.tril(Q, -1).T
    Q += np.diag(np.abs(Q).sum(axis=1) + 1.0)
    return Q


def expected_factor(Q, b, nt, a):
    D, S, R, T = O.bta_factor_blocks(Q, b, nt, a)
    Di = np.stack([np.linalg.inv(D[t]) for t in range(nt)])
    Ti = np.linalg.inv(T) if a else T
    return Di, S, R, Ti


def blk_err(x, y):
    if x.size == 0:
        return 0.0
    return np.abs(x - y).max() / max(np.abs(y).max(), 1e-300)


def grad_term_magnitudes(md, theta):
    """Per component of grad f, the sum of the absolute values of the terms the
    gradient adds up: the prior term, half the two traces tr(Q^-1 dQ_k), half
    the quadratic form mu^T dQ_p_k mu and, for the noise precision, the
    residual and count terms (dense, small models only)."""
    from oracle.inla_oracle import conditional_precision, dprecision, obs_matrix, theta_params
    t = np.asarray(theta, dtype=np.float64)
    tau_y = theta_params(t)[3]
    Qp, Qc, rhs = conditional_precision(md, t)
    Sp = np.linalg.inv(Qp.toarray())
    Sc = np.linalg.inv(Qc.toarray())
    mu = np.linalg.solve(Qc.toarray(), rhs)
    dQp, dQc = dprecision(md, t)
    r = md.y - obs_matrix(md) @ mu
    pm = np.asarray(md.theta_prior_mean)
    pp = np.asarray(md.theta_prior_prec)
    out = np.empty(t.size)
    for k in range(t.size):
        out[k] = (abs(pp[k] * (t[k] - pm[k])) + 0.5 * abs(np.sum(Sp * dQp[k].toarray()))
                  + 0.5 * abs(np.sum(Sc * dQc[k].toarray())) + 0.5 * abs(mu @ (dQp[k] @ mu)))
    out[-1] += 0.5 * tau_y * float(r @ r) + 0.5 * md.m
    return out


SHAPES = [(1, 4, 2), (16, 1, 0), (64, 3, 1), (100, 3, 2), (130, 2, 3), (70, 4, 0), (200, 2, 5),
          (300, 2, 3), (257, 2, 1), (17, 3, 1), (520, 2, 2)]


@pytest.mark.parametrize("b,nt,a", SHAPES)
def test_factor_logdet_random_bta(P, tile, b, nt, a):
    print(f"factor b={b} nt={nt} a={a} tile={tile}", flush=True)
    Q = rand_spd_bta(b, nt, a, seed=b * 100 + nt * 10 + a)
    Qt = P.BtaTensors.from_blocks(*O.bta_blocks(Q, b, nt, a))
    ld, info = P.factor_logdet(Qt)
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    L = np.linalg.cholesky(Q)
    ld_ref = 2.0 * math.fsum(np.log(np.diag(L)))
    assert rel(ld.item(), ld_ref) < 1e-12
    got = Qt.to_blocks()
    exp = expected_factor(Q, b, nt, a)
    for g, e, name in zip(got, exp, "DSRT"):
        assert blk_err(g, e) < 1e-11, name


@pytest.mark.parametrize("b,nt,a", [(100, 3, 2), (64, 2, 1), (1, 5, 1), (130, 2, 0), (300, 3, 3),
                                   (257, 2, 1), (40, 1, 3), (1, 1, 0), (70, 2, 64)])
def test_solve_and_selinv_random_bta(P, tile, b, nt, a):
    print(f"solve/selinv b={b} nt={nt} a={a} tile={tile}", flush=True)
    Q = rand_spd_bta(b, nt, a, seed=7 + b + nt + a)
    n = Q.shape[0]
    Qt = P.BtaTensors.from_blocks(*O.bta_blocks(Q, b, nt, a))
    P.factor_logdet(Qt)
    rng = np.random.default_rng(3)
    r = rng.standard_normal((2, n))
    x = P.solve(Qt, torch.as_tensor(r).cuda())
    sig, diag = P.selinv(Qt, keep_sigma=True)
    torch.cuda.synchronize()
    Sinv = np.linalg.inv(Q)
    xr = np.linalg.solve(Q, r.T).T
    np.testing.assert_allclose(x.cpu().numpy(), xr, rtol=0, atol=1e-10 * np.abs(xr).max())
    np.testing.assert_allclose(diag.cpu().numpy(), np.diag(Sinv), rtol=1e-10)
    got = sig.to_blocks()
    exp = O.bta_blocks(Sinv, b, nt, a)
    for g, e, name in zip(got, exp, "DSRT"):
        assert blk_err(g, e) < 1e-10, name


@pytest.mark.parametrize("fused", ["0", "1"], ids=["batched_step", "fused_step"])
@pytest.mark.parametrize("b,nt,a", [(300, 3, 3), (257, 2, 1), (520, 2, 2), (130, 2, 0)])
def test_step_paths_factor_and_selinv(P, monkeypatch, fused, b, nt, a):
    """Both forms of the tile Cholesky step (one fused launch per step with running
    sums for the rows of inv(L_tt); or the lean launch with the next diagonal tile
    beside it and one long product per row) against the oracle."""
    print(f"step path fused={fused} b={b} nt={nt} a={a}", flush=True)
    monkeypatch.setenv("INLA_STEP_FUSED", fused)
    Q = rand_spd_bta(b, nt, a, seed=11 + b + nt + a)
    Qt = P.BtaTensors.from_blocks(*O.bta_blocks(Q, b, nt, a))
    ld, info = P.factor_logdet(Qt)
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    L = np.linalg.cholesky(Q)
    assert rel(ld.item(), 2.0 * math.fsum(np.log(np.diag(L)))) < 1e-12
    for g, e, name in zip(Qt.to_blocks(), expected_factor(Q, b, nt, a), "DSRT"):
        assert blk_err(g, e) < 1e-11, name
    sig, diag = P.selinv(Qt, keep_sigma=True)
    torch.cuda.synchronize()
    Sinv = np.linalg.inv(Q)
    np.testing.assert_allclose(diag.cpu().numpy(), np.diag(Sinv), rtol=1e-10)
    for g, e, name in zip(sig.to_blocks(), O.bta_blocks(Sinv, b, nt, a), "DSRT"):
        assert blk_err(g, e) < 1e-10, name


@pytest.mark.parametrize("width", [64, 128], ids=["tile64", "tile128"])
def test_selinv_batched_matches_stepwise(P, monkeypatch, width):
    """The selected inversion with V_t = L_{t+1,t} inv(L_tt), U_t and
    inv(L_tt)^T inv(L_tt) of every step formed up front (one launch each)
    against the step-by-step one: the same f, gradient and variances, bitwise
    with 64-wide tiles (the same products in the same order).  With 128-wide
    tiles the step-by-step launches of small models split k in two, which
    groups the terms differently: there both forms are held to the oracle."""
    print(f"selinv batched vs stepwise, tile {width}", flush=True)
    mds = [make_model(5, 3, 2, 31), make_model(8, 4, 3, 32), make_model(6, 2, 0, 33),
           make_model(4, 1, 2, 34)]
    Ms = [P.Model.from_data(m) for m in mds]
    th = np.array([[0.1, 0.8, 0.5, 2.0], [0.3, 1.1, 1.0, 3.0], [-0.2, 0.6, 0.2, 2.5],
                   [0.0, 1.0, 1.5, 4.6]])
    out = {}
    for flag in ("0", "1"):
        monkeypatch.setenv("INLA_SI_BATCH", flag)
        out[flag] = P.eval_f_grad(Ms, th, want_var=True, tile=width)
        torch.cuda.synchronize()
    for key in ("f", "grad", "var", "status"):
        if width == 64 or key == "status":
            assert torch.equal(out["0"][key], out["1"][key]), key
    voff = np.cumsum([0] + [md.n for md in mds])
    for flag in ("0", "1") if width == 128 else ("1",):
        var = out[flag]["var"].cpu().numpy()
        for i, md in enumerate(mds):
            assert rel(out[flag]["f"][i].item(), O.eval_f_dense(md, th[i])["f"]) < 1e-10
            g = out[flag]["grad"][i].cpu().numpy()
            gref = O.dense_gradient(md, th[i])
            scale = np.maximum(grad_term_magnitudes(md, th[i]), 1e-3 * np.abs(gref).max())
            assert np.max(np.abs(g - gref) / scale) < 1e-9
            vref = O.marginal_variances_dense(md, th[i])
            assert np.max(np.abs(var[voff[i]:voff[i + 1]] - vref) / vref) < 1e-9


def test_not_spd_reports_pivot(P):
    b, nt, a = 70, 3, 2
    Q = rand_spd_bta(b, nt, a, seed=5)
    bad = b * 1 + 66  # global row of the planted negative pivot
    Q[bad, bad] = -5.0
    Qt = P.BtaTensors.from_blocks(*O.bta_blocks(Q, b, nt, a))
    ld, info = P.factor_logdet(Qt)
    torch.cuda.synchronize()
    assert int(info.item()) == bad + 1
    assert math.isnan(ld.item())


def model_small(N=5, nt=3, nb=2, seed=3):
    return make_model(N, nt, nb, seed)


@pytest.mark.parametrize("shape", [(5, 3, 2), (1, 4, 2), (9, 2, 0), (10, 1, 3)])
def test_assemble(P, shape):
    md = model_small(*shape)
    M = P.Model.from_data(md)
    theta = np.array([0.2, 0.9, 0.7, 3.0])
    Qp = P.assemble(M, theta, 0)
    Qc, rhs = P.assemble(M, theta, 1)
    torch.cuda.synchronize()
    Qp_ref, Qc_ref, b_ref = O.conditional_precision(md, theta)
    for Qt, Qr in ((Qp, Qp_ref), (Qc, Qc_ref)):
        exp = O.bta_blocks(Qr, md.ns, md.nt, md.nb)
        for g, e, name in zip(Qt.to_blocks(), exp, "DSRT"):
            assert blk_err(g, e) < 1e-14, name
    np.testing.assert_allclose(rhs.cpu().numpy(), b_ref, rtol=1e-13, atol=1e-13 * np.abs(b_ref).max())


def test_eval_f_c1(P, tile):
    md = config_model("c1")
    M = P.Model.from_data(md)
    out = P.eval_f(M, THETA0, want_mu=True, want_var=True)
    torch.cuda.synchronize()
    ref = O.eval_f_dense(md, THETA0)
    assert int(out["status"].item()) == 0
    assert rel(out["f"].item(), ref["f"]) < 1e-10
    mu = out["mu"].cpu().numpy()
    assert np.abs(mu - ref["mu"]).max() / np.abs(ref["mu"]).max() < 1e-9
    var_ref = O.marginal_variances_dense(md, THETA0)
    assert np.max(np.abs(out["var"].cpu().numpy() - var_ref) / var_ref) < 1e-9


def test_logdets_c1_and_closed_form(P):
    md = config_model("c1")
    M = P.Model.from_data(md)
    Qp = P.assemble(M, THETA0, 0)
    Qc, _ = P.assemble(M, THETA0, 1)
    ldp, _ = P.factor_logdet(Qp)
    ldc, _ = P.factor_logdet(Qc)
    torch.cuda.synchronize()
    ref = O.eval_f_dense(md, THETA0)
    assert rel(ldp.item(), ref["logdet_p"]) < 1e-10
    assert rel(ldc.item(), ref["logdet_c"]) < 1e-10


def test_eval_f_grad_small(P, tile):
    md = config_model("c4small")
    M = P.Model.from_data(md)
    out = P.eval_f_grad(M, THETA0)
    torch.cuda.synchronize()
    g = out["grad"].cpu().numpy()[0]
    gref = O.dense_gradient(md, THETA0)
    assert rel(out["f"].item(), O.eval_f_dense(md, THETA0)["f"]) < 1e-10
    assert np.max(np.abs(g - gref) / np.maximum(np.abs(gref), 1e-3 * np.abs(gref).max())) < 1e-9


@pytest.mark.parametrize("N,nt,nb", [(4, 1, 2), (5, 3, 0), (1, 3, 1), (1, 1, 0), (6, 2, 64)],
                         ids=["one_step", "no_fixed", "one_node", "scalar", "max_arrow"])
def test_eval_f_grad_degenerate_models(P, N, nt, nb):
    """One time step, no fixed effects, a one-node mesh (b = 1), a 1x1 problem
    and the widest arrow the library accepts: f, grad f, mu and the variances
    against the dense oracle.  The wide-arrow mesh has more observations than
    fixed effects (144 > 64), so Q_c stays well conditioned (cond ~ 1e3); on a
    smaller mesh the fixed effects are set by their vague prior alone and
    cond(Q_c) ~ 1e7 puts the mean's rounding error itself near 1e-9."""
    print(f"degenerate model N={N} nt={nt} nb={nb}", flush=True)
    md = make_model(N, nt, nb, 5)
    M = P.Model.from_data(md)
    out = P.eval_f_grad(M, THETA0, want_mu=True, want_var=True)
    torch.cuda.synchronize()
    assert int(out["status"].item()) == 0
    ref = O.eval_f_dense(md, THETA0)
    assert rel(out["f"].item(), ref["f"]) < 1e-10
    g = out["grad"].cpu().numpy()[0]
    gref = O.dense_gradient(md, THETA0)
    # each component is a sum of trace and quadratic terms that can cancel
    # (with 64 fixed effects the two traces agree to 1e-4): rounding error is
    # bounded relative to the terms' magnitudes, not to their sum
    scale = np.maximum(grad_term_magnitudes(md, THETA0), 1e-3 * np.abs(gref).max())
    assert np.max(np.abs(g - gref) / scale) < 1e-9
    mu = out["mu"].cpu().numpy()
    assert np.abs(mu - ref["mu"]).max() / np.abs(ref["mu"]).max() < 1e-9
    var_ref = O.marginal_variances_dense(md, THETA0)
    assert np.max(np.abs(out["var"].cpu().numpy() - var_ref) / var_ref) < 1e-9


def test_new_model_is_not_served_a_destroyed_models_graph(P, monkeypatch):
    """Regression: a captured evaluation graph bakes in the device data of its
    models.  A model created after another was destroyed (possibly at the same
    host address, possibly with the same shape) must get its own results, never
    a replay of the destroyed model's graph."""
    import gc
    monkeypatch.setenv("INLA_GRAPH", "1")
    mdA = make_model(4, 3, 2, 41)
    A = P.Model.from_data(mdA)
    for _ in range(2):   # capture, then replay
        outA = P.eval_f_grad(A, THETA0, want_mu=True, want_var=True)
        torch.cuda.synchronize()
    assert rel(outA["f"].item(), O.eval_f_dense(mdA, THETA0)["f"]) < 1e-10
    del A
    gc.collect()
    # a different shape (no fixed effects), then the destroyed model's shape
    # with other data: each must match its own oracle value
    for shape, seed in (((5, 3, 0), 42), ((4, 3, 2), 43), ((5, 3, 0), 44)):
        print(f"model after destroy: shape={shape} seed={seed}", flush=True)
        md = make_model(*shape, seed)
        M = P.Model.from_data(md)
        for _ in range(2):
            out = P.eval_f_grad(M, THETA0, want_mu=True, want_var=True)
            torch.cuda.synchronize()
            ref = O.eval_f_dense(md, THETA0)
            assert int(out["status"].item()) == 0
            assert out["mu"].numel() == md.n and out["var"].numel() == md.n
            assert rel(out["f"].item(), ref["f"]) < 1e-10
            mu = out["mu"].cpu().numpy()
            assert np.abs(mu - ref["mu"]).max() / np.abs(ref["mu"]).max() < 1e-9
        del M
        gc.collect()


def test_batched_uneven_matches_single(P):
    mds = [make_model(4, 3, 2, 1), make_model(6, 2, 3, 2), make_model(9, 4, 1, 3)]
    Ms = [P.Model.from_data(m) for m in mds]
    th = np.array([[0.1, 0.8, 0.5, 2.0], [0.3, 1.1, 1.0, 3.0], [-0.2, 0.6, 0.2, 2.5]])
    out = P.eval_f_grad(Ms, th)
    torch.cuda.synchronize()
    for i, (md, M) in enumerate(zip(mds, Ms)):
        one = P.eval_f_grad(M, th[i])
        torch.cuda.synchronize()
        assert out["f"][i].item() == one["f"][0].item()
        assert torch.equal(out["grad"][i], one["grad"][0])
        assert rel(out["f"][i].item(), O.eval_f_dense(md, th[i])["f"]) < 1e-10


def test_graph_replay_matches_eager(P, monkeypatch):
    """A replayed graph (same call signature, new theta) equals the eager path bitwise."""
    md = config_model("c4small")
    M = P.Model.from_data(md)
    th1 = np.array([0.1, 0.7, 1.2, 4.0])
    th2 = np.array([-0.2, 1.1, 0.8, 4.4])
    monkeypatch.setenv("INLA_GRAPH", "1")
    P.eval_f_grad(M, th1, want_var=True)            # captures
    rep = P.eval_f_grad(M, th2, want_var=True)      # replays with the new theta
    rep2 = P.eval_f_grad(M, th2, want_var=True)     # replays again
    torch.cuda.synchronize()
    monkeypatch.setenv("INLA_GRAPH", "0")
    eag = P.eval_f_grad(M, th2, want_var=True)
    torch.cuda.synchronize()
    for key in ("f", "grad", "var"):
        assert torch.equal(rep[key], eag[key]), key
        assert torch.equal(rep2[key], eag[key]), key
    assert rel(rep["f"].item(), O.eval_f_dense(md, th2)["f"]) < 1e-10


def test_hbm_admission_waves_match_single_wave(P, monkeypatch):
    """A budget that admits one item at a time gives the same results as one wave."""
    monkeypatch.setenv("INLA_GRAPH", "0")
    mds = [make_model(5, 3, 2, 11), make_model(4, 4, 3, 12), make_model(6, 2, 1, 13)]
    Ms = [P.Model.from_data(m) for m in mds]
    th = np.array([[0.1, 0.8, 0.5, 2.0], [0.3, 1.1, 1.0, 3.0], [-0.2, 0.6, 0.2, 2.5]])
    one = P.eval_f_grad(Ms, th)
    torch.cuda.synchronize()
    waves = P.eval_f_grad(Ms, th, budget=2.0e5)
    torch.cuda.synchronize()
    assert torch.equal(one["f"], waves["f"]) and torch.equal(one["grad"], waves["grad"])
    with pytest.raises(P.InlaError):
        P.eval_f_grad(Ms, th, budget=1.0e3)


def test_shared_storage_mode_matches_two_matrix_mode(P):
    """recompute=1 (Q_prior then Q_c in one storage) gives the same results bitwise."""
    mds = [make_model(5, 3, 2, 21), make_model(8, 4, 3, 22), make_model(6, 2, 1, 23)]
    Ms = [P.Model.from_data(m) for m in mds]
    th = np.array([[0.1, 0.8, 0.5, 2.0], [0.3, 1.1, 1.0, 3.0], [-0.2, 0.6, 0.2, 2.5]])
    two = P.eval_f_grad(Ms, th, want_mu=True, want_var=True, recompute=2, tile=64)
    one = P.eval_f_grad(Ms, th, want_mu=True, want_var=True, recompute=1, tile=64)
    torch.cuda.synchronize()
    for key in ("f", "grad", "mu", "var", "status"):
        assert torch.equal(two[key], one[key]), key
    # any budget, mode and number of admission waves gives the same results
    ran = 0
    for budget in (1e5, 2e5, 4e5, 8e5, 1.6e6, 3.2e6, 6.4e6):
        for mode in (0, 1, 2):
            try:
                got = P.eval_f_grad(Ms, th, recompute=mode, tile=64, budget=budget)
            except P.InlaError:
                continue
            torch.cuda.synchronize()
            assert torch.equal(got["f"], two["f"]) and torch.equal(got["grad"], two["grad"])
            ran += 1
    assert ran >= 6
    for i, md in enumerate(mds):
        assert rel(one["f"][i].item(), O.eval_f_dense(md, th[i])["f"]) < 1e-10


def test_autotune_cache(P, tmp_path):
    """The autotuner times the tile layouts and the two Cholesky step forms
    once, stores the winner, and reuses it."""
    import json
    md = config_model("c4small")
    M = P.Model.from_data(md)
    path = tmp_path / "tune.json"
    out = P.eval_f_grad([M, M], np.stack([THETA0, THETA0 + 0.05]), autotune_cache=path)
    torch.cuda.synchronize()
    entries = json.loads(path.read_text())
    assert len(entries) == 1
    (key, val), = entries.items()
    assert key.startswith("grad:n2:") and val["tile"] in (64, 128) and val["ms"] > 0
    assert val["step"] in (-1, 0, 1)
    again = P.eval_f_grad([M, M], np.stack([THETA0, THETA0 + 0.05]), autotune_cache=path)
    torch.cuda.synchronize()
    assert len(json.loads(path.read_text())) == 1
    assert torch.equal(out["f"], again["f"])
    assert rel(out["f"][0].item(), O.eval_f_dense(md, THETA0)["f"]) < 1e-10


def test_objective_autograd(P):
    """torch.autograd through the objective gives the adjoint gradient; no-grad runs f only."""
    md = config_model("c4small")
    M = P.Model.from_data(md)
    th = torch.tensor(np.stack([THETA0, THETA0 + 0.1]), dtype=torch.float64, device="cuda",
                      requires_grad=True)
    f = P.objective(th, [M, M])
    (2.0 * f[0] + 3.0 * f[1]).backward()
    g = P.eval_f_grad([M, M], th.detach())["grad"]
    assert torch.allclose(th.grad[0], 2.0 * g[0], rtol=1e-14, atol=0)
    assert torch.allclose(th.grad[1], 3.0 * g[1], rtol=1e-14, atol=0)
    with torch.no_grad():
        f2 = P.objective(th, [M, M])
    assert torch.equal(f2, f.detach())


MULTI_TILE = [(9, 3, 0), (9, 3, 3), (12, 3, 0), (12, 3, 3)]


def check_against_dense_oracle(out, i, md, theta, voff=0):
    """f, grad f, mu and the variances of item i against the dense oracle."""
    ref = O.eval_f_dense(md, theta)
    assert int(out["status"][i].item()) == 0
    assert rel(out["f"][i].item(), ref["f"]) < 1e-10
    g = out["grad"][i].cpu().numpy()
    gref = O.dense_gradient(md, theta)
    scale = np.maximum(grad_term_magnitudes(md, theta), 1e-3 * np.abs(gref).max())
    assert np.max(np.abs(g - gref) / scale) < 1e-9, (g, gref)
    if "mu" in out:
        mu = out["mu"].cpu().numpy()[voff:voff + md.n]
        assert np.abs(mu - ref["mu"]).max() / np.abs(ref["mu"]).max() < 1e-9
    if "var" in out:
        var = out["var"].cpu().numpy()[voff:voff + md.n]
        vref = O.marginal_variances_dense(md, theta)
        assert np.max(np.abs(var - vref) / vref) < 1e-9


@pytest.mark.parametrize("N,nt,nb", MULTI_TILE)
def test_eval_f_grad_multi_tile(P, tile, N, nt, nb):
    """The adjoint where the kernels tile: b = 81 (two 64-wide tiles, one
    128-wide) and b = 144 (three 64-wide tiles, two 128-wide), with and without
    fixed effects, under every product form, against the oracle's
    dense-inverse gradient (and f, mu, variances)."""
    print(f"multi-tile adjoint N={N} nt={nt} nb={nb} tile={tile}", flush=True)
    md = make_model(N, nt, nb, 50 + N + nb)
    M = P.Model.from_data(md)
    theta = np.array([0.3, 0.9, 1.1, 3.5])
    out = P.eval_f_grad(M, theta, want_mu=True, want_var=True)
    torch.cuda.synchronize()
    check_against_dense_oracle(out, 0, md, theta)


def test_eight_wave_products_equal_four_wave_bitwise(P, monkeypatch):
    """The 64-wide products on eight waves of 32 x 16 (form 5) take every sum
    in the order the four waves of 32 x 32 (form 2) do: f, gradient, mean and
    variances agree bit for bit, on a batch of uneven multi-tile models."""
    print("eight-wave vs four-wave 64-wide products", flush=True)
    mds = [make_model(12, 3, 3, 71), make_model(9, 4, 0, 72), make_model(5, 3, 2, 73)]
    Ms = [P.Model.from_data(m) for m in mds]
    th = np.array([[0.3, 0.9, 1.1, 3.5], [-0.2, 0.6, 0.2, 2.5], [0.1, 0.8, 0.5, 2.0]])
    monkeypatch.setenv("INLA_TILE", "64")
    out = {}
    for form in ("2", "5"):
        monkeypatch.setenv("INLA_SMALL_VARIANT", form)
        out[form] = P.eval_f_grad(Ms, th, want_mu=True, want_var=True)
        torch.cuda.synchronize()
    for key in ("f", "grad", "mu", "var", "status"):
        assert torch.equal(out["2"][key], out["5"][key]), key


@pytest.mark.parametrize("fused", ["0", "1"], ids=["batched_step", "fused_step"])
@pytest.mark.parametrize("width", [64, 128], ids=["tile64", "tile128"])
def test_eval_f_grad_multi_tile_step_forms(P, monkeypatch, fused, width):
    """Both forms of the Cholesky step, with 64- and 128-wide products, on a
    multi-tile model (b = 144, nt = 3, nb = 3) against the dense oracle."""
    print(f"multi-tile step forms fused={fused} width={width}", flush=True)
    monkeypatch.setenv("INLA_STEP_FUSED", fused)
    md = make_model(12, 3, 3, 65)
    M = P.Model.from_data(md)
    theta = np.array([-0.1, 0.7, 0.6, 4.0])
    out = P.eval_f_grad(M, theta, want_mu=True, want_var=True, tile=width)
    torch.cuda.synchronize()
    check_against_dense_oracle(out, 0, md, theta)


@pytest.mark.parametrize("N,nt,nb", [(5, 3, 2), (12, 3, 3), (9, 4, 0)])
def test_eval_f_grad_rho_zero(P, N, nt, nb):
    """theta_3 = 0 (rho = 0): the time blocks decouple in the prior and the
    theta_3 derivative of Q_AR1 reduces to its off-diagonal term."""
    print(f"rho = 0: N={N} nt={nt} nb={nb}", flush=True)
    md = make_model(N, nt, nb, 70 + N)
    M = P.Model.from_data(md)
    theta = np.array([0.2, 1.0, 0.0, 3.0])
    out = P.eval_f_grad(M, theta, want_mu=True, want_var=True)
    torch.cuda.synchronize()
    check_against_dense_oracle(out, 0, md, theta)


def test_eval_status_not_positive_definite(P):
    """Items whose matrices are not numerically positive definite get status 1
    (Q_prior: tau = e^-500 makes tau^2 underflow to 0, so the space-time part of
    Q_prior is zero) or 2 (Q_c: tau_y = e^800 overflows to infinity), NaN f and
    gradient; the other items of the same batched call are unaffected."""
    md1, md2 = make_model(9, 3, 2, 81), make_model(6, 2, 0, 82)
    M1, M2 = P.Model.from_data(md1), P.Model.from_data(md2)
    th = np.array([THETA0, [-500.0, 1.0, 1.5, 4.6], [0.0, 1.0, 1.5, 800.0], THETA0])
    for fn in ("eval_f_grad", "eval_f"):
        print(f"status batch via {fn}", flush=True)
        out = getattr(P, fn)([M1, M1, M2, M2], th, want_mu=True, want_var=True)
        torch.cuda.synchronize()
        assert out["status"].cpu().tolist() == [0, 1, 2, 0]
        f = out["f"].cpu().numpy()
        assert np.isnan(f[1]) and np.isnan(f[2])
        if fn == "eval_f_grad":
            g = out["grad"].cpu().numpy()
            assert np.isnan(g[1]).all() and np.isnan(g[2]).all()
            voff = np.cumsum([0, md1.n, md1.n, md2.n])
            check_against_dense_oracle(out, 0, md1, THETA0, voff[0])
            check_against_dense_oracle(out, 3, md2, THETA0, voff[3])
            # the good items equal their single evaluations
            for i, M in ((0, M1), (3, M2)):
                one = P.eval_f_grad(M, THETA0)
                torch.cuda.synchronize()
                assert out["f"][i].item() == one["f"][0].item()
                assert torch.equal(out["grad"][i], one["grad"][0])
        else:
            assert rel(f[0], O.eval_f_dense(md1, THETA0)["f"]) < 1e-10
            assert rel(f[3], O.eval_f_dense(md2, THETA0)["f"]) < 1e-10


@pytest.mark.parametrize("si_batch", ["0", "1"], ids=["si_stepwise", "si_every_step"])
@pytest.mark.parametrize("width", [64, 128], ids=["tile64", "tile128"])
def test_keep_sigma_stores_selected_inverse(P, monkeypatch, si_batch, width):
    """keep_sigma: the selected inverse of each item's Q_c lands in caller
    storage, block by block equal to the dense inverse (Sec. "Partial
    Inversion"), and f / grad f are those of the call without it."""
    print(f"keep_sigma width={width} si_batch={si_batch}", flush=True)
    monkeypatch.setenv("INLA_SI_BATCH", si_batch)
    mds = [make_model(9, 3, 2, 91), make_model(5, 1, 3, 92), make_model(6, 4, 0, 93)]
    Ms = [P.Model.from_data(m) for m in mds]
    th = np.array([[0.1, 0.8, 0.5, 2.0], [0.3, 1.1, 1.0, 3.0], [-0.2, 0.6, 0.2, 2.5]])
    sig = [P.BtaTensors(M.b, M.nt, M.a) for M in Ms]
    out = P.eval_f_grad(Ms, th, want_var=True, tile=width, sigma=sig)
    # (keeping Sigma in caller storage eliminates every matrix from its first
    # time block on: the bitwise reference does the same)
    monkeypatch.setenv("INLA_TWIST", "0")
    ref = P.eval_f_grad(Ms, th, want_var=True, tile=width)
    torch.cuda.synchronize()
    for key in ("f", "grad", "var", "status"):
        assert torch.equal(out[key], ref[key]), key
    for i, (md, S) in enumerate(zip(mds, sig)):
        _, Qc, _ = O.conditional_precision(md, th[i])
        Sinv = np.linalg.inv(Qc.toarray())
        for g, e, name in zip(S.to_blocks(), O.bta_blocks(Sinv, md.ns, md.nt, md.nb), "DSRT"):
            assert blk_err(g, e) < 1e-10, (i, name)


@pytest.mark.parametrize("width", [64, 128], ids=["tile64", "tile128"])
def test_deferred_gradient_matches_one_pass(P, width):
    """f now and the gradient later from the kept factors (the selected
    inversions recomputed from them) equals the one-pass adjoint bit for bit;
    without room for the factors the gradient recomputes everything and still
    agrees."""
    print(f"deferred gradient width={width}", flush=True)
    mds = [make_model(9, 3, 2, 95), make_model(12, 2, 3, 96), make_model(4, 1, 0, 97)]
    Ms = [P.Model.from_data(m) for m in mds]
    th = np.array([[0.1, 0.8, 0.5, 2.0], [0.3, 1.1, 1.0, 3.0], [-0.2, 0.6, 0.2, 2.5]])
    one = P.eval_f_grad(Ms, th, want_mu=True, want_var=True, tile=width)
    st = P.EvalState(Ms, th, want_mu=True, tile=width)
    torch.cuda.synchronize()
    assert st.kept
    assert torch.equal(st.f, one["f"]) and torch.equal(st.mu, one["mu"])
    for _ in range(2):   # the kept factors serve more than one gradient
        g = st.grad(want_var=True)
        torch.cuda.synchronize()
        for key in ("f", "grad", "var", "status"):
            assert torch.equal(g[key], one[key]), key
    st.close()
    # shared storage (recompute = 1) cannot keep both factors: recomputed
    st2 = P.EvalState(Ms, th, tile=width, recompute=1)
    g2 = st2.grad()
    ref2 = P.eval_f_grad(Ms, th, tile=width, recompute=1)
    torch.cuda.synchronize()
    assert not st2.kept
    assert torch.equal(g2["grad"], ref2["grad"]) and torch.equal(g2["f"], ref2["f"])
    st2.close()
    for i, md in enumerate(mds):
        assert rel(one["f"][i].item(), O.eval_f_dense(md, th[i])["f"]) < 1e-10


def test_objective_deferred_backward(P):
    """autograd through the objective with the gradient deferred to the
    backward pass equals the forward-adjoint gradient bit for bit."""
    md = make_model(9, 3, 2, 98)
    M = P.Model.from_data(md)
    th0 = np.stack([THETA0, THETA0 + 0.1])
    a = torch.tensor(th0, dtype=torch.float64, device="cuda", requires_grad=True)
    b = torch.tensor(th0, dtype=torch.float64, device="cuda", requires_grad=True)
    fa = P.objective(a, [M, M])
    fb = P.objective(b, [M, M], defer_grad=True)
    assert torch.equal(fa.detach(), fb.detach())
    (2.0 * fa[0] + 3.0 * fa[1]).backward()
    (2.0 * fb[0] + 3.0 * fb[1]).backward()
    assert torch.equal(a.grad, b.grad)
    g = O.dense_gradient(md, THETA0)
    assert np.max(np.abs(b.grad[0].cpu().numpy() / 2.0 - g) / np.abs(g).max()) < 1e-9


@pytest.mark.parametrize("name", ["c4small", "c1"])
def test_bfgs_parallel_line_search_reaches_the_mode(P, name):
    """BFGS with the parallel line search (eight candidates per iteration in one
    batched call, a robust quadratic through them) reaches the mode the oracle
    finds with scipy's BFGS on its own dense f and gradient: the oracle's
    gradient vanishes there, f is as low, and f fell at every iteration."""
    from scipy.optimize import minimize as sp_minimize
    print(f"bfgs on {name}", flush=True)
    md = config_model(name)
    M = P.Model.from_data(md)
    res = P.minimize(M, THETA0, gtol=1e-6)
    print(f"  {res['iterations']} iterations, {res['f_evals']} f, {res['grad_evals']} f+grad, "
          f"reason {res['reason']}, theta {res['theta']}", flush=True)
    # reason 3 (no point of the interval lowered f) near the mode is the
    # rounding floor of f; the checks against the oracle below decide
    assert res["reason"] in (0, 1) or (res["reason"] == 3 and np.abs(res["grad"]).max() < 1e-5), res
    hist = res["history"]
    assert np.all(np.diff(hist[:, 0]) < 0)
    g0 = O.dense_gradient(md, THETA0)
    ref = sp_minimize(lambda th: O.eval_f_dense(md, th)["f"], THETA0,
                      jac=lambda th: O.dense_gradient(md, th), method="BFGS",
                      options=dict(gtol=1e-7, maxiter=300, hess_inv0=np.eye(4) / np.abs(g0).max()))
    g_at = O.dense_gradient(md, res["theta"])
    f_at = O.eval_f_dense(md, res["theta"])["f"]
    assert np.abs(g_at).max() <= 1e-5 * max(1.0, np.abs(g0).max() * 1e-3), g_at
    assert f_at <= ref.fun + 1e-10 * abs(ref.fun)
    assert rel(res["f"], f_at) < 1e-10
    assert np.abs(res["theta"] - ref.x).max() < 1e-3


@pytest.mark.parametrize("N,nt,nb", [(6, 4, 2), (5, 5, 0), (9, 7, 3), (12, 6, 1), (4, 9, 2)])
def test_two_sided_elimination_matches_one_sided(P, monkeypatch, N, nt, nb):
    """Eliminating the time blocks from both ends at once (a forward chain up
    to the middle block and a backward chain down to it, the default from four
    time blocks on) gives the one-sided results to rounding, and both match
    the oracle: f, grad f, mu and the variances."""
    print(f"two-sided elimination N={N} nt={nt} nb={nb}", flush=True)
    md = make_model(N, nt, nb, 100 + N + nt)
    M = P.Model.from_data(md)
    theta = np.array([0.2, 0.8, 0.9, 3.2])
    out = {}
    for flag in ("1", "0"):
        monkeypatch.setenv("INLA_TWIST", flag)
        out[flag] = P.eval_f_grad(M, theta, want_mu=True, want_var=True)
        torch.cuda.synchronize()
    for flag in ("1", "0"):
        check_against_dense_oracle(out[flag], 0, md, theta)
    a, b = out["1"], out["0"]
    assert rel(a["f"].item(), b["f"].item()) < 1e-12
    scale = np.maximum(grad_term_magnitudes(md, theta), 1e-3 * np.abs(b["grad"].cpu().numpy()).max())
    assert np.max(np.abs(a["grad"].cpu().numpy() - b["grad"].cpu().numpy()) / scale) < 1e-11
    va, vb = a["var"].cpu().numpy(), b["var"].cpu().numpy()
    assert np.max(np.abs(va - vb) / vb) < 1e-11
    ma, mb = a["mu"].cpu().numpy(), b["mu"].cpu().numpy()
    assert np.abs(ma - mb).max() / np.abs(mb).max() < 1e-11


@pytest.mark.parametrize("N,nt,nb,seed", [(4, 3, 2, 5), (9, 4, 3, 31)])
def test_integrate_matches_oracle(P, N, nt, nb, seed):
    """The integration step at the mode (Sec. "Latent Gaussian Models", eq.
    LatParam) against the oracle's: the Hessian from differences of the
    adjoint gradient, the eigen-decomposition, the axis ranges, the kept grid
    points (the same integer coordinates), their f and weights, the theta
    moments, the log evidence and the latent mixture mean and variance.  The
    second model has 64-wide tiles in two columns and four time blocks (the
    two-sided elimination).  The mode comes from scipy's BFGS on the oracle."""
    from scipy.optimize import minimize as sp_minimize
    from oracle import integrate as OI
    print(f"integrate N={N} nt={nt} nb={nb}", flush=True)
    md = make_model(N, nt, nb, seed)
    g0 = O.dense_gradient(md, THETA0)
    mode = sp_minimize(lambda th: O.eval_f_dense(md, th)["f"], THETA0,
                       jac=lambda th: O.dense_gradient(md, th), method="BFGS",
                       options=dict(gtol=1e-9, maxiter=400,
                                    hess_inv0=np.eye(4) / np.abs(g0).max())).x
    ref = OI.integrate_model(md, mode)
    # no candidate's drop is within rounding of the threshold (both sides
    # decide keep / drop in FP64 from f values that agree to ~1e-9)
    assert np.abs(ref["drops"] - 2.5).min() > 1e-4
    M = P.Model.from_data(md)
    r = P.integrate(M, mode)
    Hs = np.abs(ref["hessian"]).max()
    assert np.abs(r["hessian"] - ref["hessian"]).max() < 1e-7 * Hs
    np.testing.assert_allclose(r["eigval"], ref["eigval"], rtol=1e-6)
    np.testing.assert_allclose(r["eigvec"], ref["eigvec"], atol=1e-5)
    assert list(r["lo"]) == list(ref["lo"]) and list(r["hi"]) == list(ref["hi"])
    assert r["n_box"] == ref["n_box"] and r["n_points"] == len(ref["f"])
    pts = r["points"]
    assert np.array_equal(pts[:, :4].astype(int), ref["s"])
    np.testing.assert_allclose(pts[:, 4:8], ref["theta"], rtol=0, atol=1e-6)
    assert rel(r["f_mode"], ref["f_mode"]) < 1e-10
    assert np.abs(pts[:, 8] - ref["f"]).max() < 1e-6 * max(1.0, abs(ref["f_mode"]))
    np.testing.assert_allclose(pts[:, 9], ref["weights"], rtol=1e-5)
    np.testing.assert_allclose(r["theta_mean"], ref["theta_mean"], rtol=0, atol=1e-6)
    np.testing.assert_allclose(r["theta_cov"], ref["theta_cov"], rtol=1e-5,
                               atol=1e-7 * np.abs(ref["theta_cov"]).max())
    assert abs(r["log_evidence"] - ref["log_evidence"]) < 1e-5
    xm = r["x_mean"].cpu().numpy()
    xv = r["x_var"].cpu().numpy()
    assert np.abs(xm - ref["x_mean"]).max() < 1e-8 * np.abs(ref["x_mean"]).max()
    np.testing.assert_allclose(xv, ref["x_var"], rtol=1e-7)
    assert r["grad_evals"] == 9 and r["f_evals"] == 8 * 6 + r["n_box"] + 1 + r["n_points"]


@pytest.mark.parametrize("N,nt,nb,tile", [(12, 5, 2, "64"), (20, 4, 3, "64"), (20, 4, 3, "128"),
                                          (17, 3, 0, "128"), (9, 6, 1, "64")])
def test_band_aware_products_match_dense(P, monkeypatch, N, nt, nb, tile):
    """The products that skip the zeros outside the coupling blocks' band (the
    default) give the dense products' f, grad f, mu and variances to rounding,
    and both match the oracle; 64- and 128-wide tiles, one- and two-sided
    elimination."""
    print(f"band N={N} nt={nt} nb={nb} tile={tile}", flush=True)
    monkeypatch.setenv("INLA_TILE", tile)
    md = make_model(N, nt, nb, 300 + N + nt)
    M = P.Model.from_data(md)
    theta = np.array([0.3, 1.1, 0.7, 2.9])
    out = {}
    for flag in ("1", "0"):
        monkeypatch.setenv("INLA_BAND", flag)
        out[flag] = P.eval_f_grad(M, theta, want_mu=True, want_var=True)
    bd, dn = out["1"], out["0"]
    assert int(bd["status"].cpu()[0]) == 0
    fb, fd = float(bd["f"].cpu()[0]), float(dn["f"].cpu()[0])
    assert rel(fb, fd) < 1e-13
    gb, gd = bd["grad"].cpu().numpy()[0], dn["grad"].cpu().numpy()[0]
    assert np.abs(gb - gd).max() < 1e-11 * np.abs(gd).max()
    for key in ("mu", "var"):
        x, y = bd[key].cpu().numpy(), dn[key].cpu().numpy()
        assert np.abs(x - y).max() < 1e-12 * np.abs(y).max()
    ref = O.eval_f_dense(md, theta)
    assert rel(fb, ref["f"]) < 1e-10
    g_ref = O.dense_gradient(md, theta)
    assert np.abs(gb - g_ref).max() < 1e-9 * np.abs(g_ref).max()
    v_ref = O.marginal_variances_dense(md, theta)
    np.testing.assert_allclose(bd["var"].cpu().numpy(), v_ref, rtol=1e-9)


@pytest.mark.parametrize("N,nt,nb,seed", [(4, 3, 2, 5), (9, 4, 3, 31), (5, 3, 0, 8), (1, 1, 0, 3)])
def test_poisson_f_grad_matches_oracle(P, N, nt, nb, seed):
    """A Poisson likelihood (the inner Newton loop of a non-Gaussian
    likelihood, one factorization of Q_c(x) per iteration) against the
    oracle: f, the exact gradient with the implicit term, the mode and the
    marginal variances at the mode; a warm start at the mode converges at once
    to the same f; Gaussian responses are refused."""
    from inla_synth import poisson_counts
    from oracle import nongauss as NG
    print(f"poisson N={N} nt={nt} nb={nb}", flush=True)
    base = make_model(N, nt, nb, seed, obs_per_node=30 if N == 1 else 2)
    md = poisson_counts(base, seed=seed, level=2.0 if N == 1 else 0.5)
    M = P.Model.from_data(md)
    theta = np.array([0.1, 0.9, 0.6, 1.5])
    r = P.eval_f_grad_poisson(M, theta, want_var=True)
    assert r["status"] == 0, r
    ref = NG.eval_f(md, theta)
    g_ref = NG.gradient(md, theta)
    assert rel(r["f"], ref["f"]) < 1e-10
    assert np.abs(r["grad"] - g_ref).max() < 1e-8 * np.abs(g_ref).max()
    x = r["x"].cpu().numpy()
    assert np.abs(x - ref["x"]).max() < 1e-9 * max(1.0, np.abs(ref["x"]).max())
    _, Qc = NG.conditional_precision_at(md, theta, ref["x"])
    v_ref = np.diag(np.linalg.inv(Qc.toarray()))
    np.testing.assert_allclose(r["var"].cpu().numpy(), v_ref, rtol=1e-9)
    assert abs(r["iterations"] - ref["iterations"]) <= 1
    w = P.eval_f_grad_poisson(M, theta, x0=r["x"])
    assert w["status"] == 0 and w["iterations"] == 1
    assert rel(w["f"], r["f"]) < 1e-12
    G = P.Model.from_data(base)
    with pytest.raises(P.InlaError, match="counts"):
        P.eval_f_grad_poisson(G, theta)


def test_integrate_and_poisson_status_paths(P):
    """The drivers' failure paths: a Hessian that is not positive definite
    (a difference step so small that theta +- h e_k round to theta, so H = 0)
    is refused with INLA_ERR_NOT_SPD; Newton's method stopped after one
    iteration reports status 4 with NaN f and gradient, and the library stays
    usable (the next call with the default budget converges)."""
    from inla_synth import poisson_counts
    md = make_model(4, 3, 2, 5)
    M = P.Model.from_data(md)
    with pytest.raises(P.InlaError, match="positive definite"):
        P.integrate(M, THETA0, h=1e-300, latent=False)
    C = P.Model.from_data(poisson_counts(md, seed=5))
    theta = np.array([0.1, 0.9, 0.6, 1.5])
    r = P.eval_f_grad_poisson(C, theta, max_iter=1)
    assert r["status"] == 4 and r["iterations"] == 1
    assert math.isnan(r["f"]) and np.all(np.isnan(r["grad"]))
    ok = P.eval_f_grad_poisson(C, theta)
    assert ok["status"] == 0 and math.isfinite(ok["f"])


def test_integrate_latent_chunks_continue_one_sum(P, monkeypatch):
    """The latent mixture over the kept points is accumulated chunk by chunk
    (at most about 1 GiB of mu and variances at a time); the chunks continue
    one sequential sum, so chunks of 3 points give the one-chunk result bit for
    bit."""
    md = make_model(4, 3, 2, 5)
    M = P.Model.from_data(md)
    theta = np.array([-3.87344165, 2.44666108, 0.05611112, 4.58238323])   # near the mode
    monkeypatch.delenv("INLA_LATENT_CHUNK", raising=False)
    one = P.integrate(M, theta)
    monkeypatch.setenv("INLA_LATENT_CHUNK", "3")
    many = P.integrate(M, theta)
    assert one["n_points"] > 6
    assert torch.equal(one["x_mean"], many["x_mean"]) and torch.equal(one["x_var"], many["x_var"])
    assert np.array_equal(one["points"], many["points"])
