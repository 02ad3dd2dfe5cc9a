"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each check uses a route independent of the oracle's own computation: closed
forms from the spectrum of the grid Laplacian, the Gaussian marginal
likelihood of y, the matrix determinant lemma, kriging / Woodbury forms of the
posterior, the paper's two selected-inversion recursions, central differences
(eq. central_diff), and the arrowhead fill pattern of the paper's figure
"arrowhead_matrices".
"""
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
from inla_synth import THETA0, make_model

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def small(N=4, nt=3, nb=2, seed=11):
    return make_model(N, nt, nb, seed)


def rel(a, b):
    return abs(a - b) / abs(b)


# ---------------------------------------------------------------- spectra

def path_eigs(N):
    """Eigenvalues of the Neumann path-graph Laplacian: 4 sin^2(pi i / (2N))."""
    return 4.0 * np.sin(np.pi * np.arange(N) / (2.0 * N)) ** 2


def dct_basis(N):
    """Orthonormal DCT-II vectors: the eigenvectors of the Neumann path Laplacian."""
    x = np.arange(N)
    V = np.cos(np.pi * np.outer(x + 0.5, np.arange(N)) / N)
    V[:, 0] *= 1.0 / math.sqrt(N)
    V[:, 1:] *= math.sqrt(2.0 / N)
    return V  # V[x, i]


def closed_logdet_prior(model, theta):
    tau, kappa, rho, _ = O.theta_params(theta)
    N, h, nt, nb = model.N, model.h, model.nt, model.nb
    ns = N * N
    lam = path_eigs(N)
    k2 = kappa * kappa * h * h
    ld_s = ns * (2 * theta[0] - 2 * math.log(h)) + 2 * math.fsum(
        np.log(k2 + lam[:, None] + lam[None, :]).ravel())
    ld_ar = -(nt - 1) * math.log(1 - rho * rho) if nt > 1 else 0.0
    return ns * ld_ar + nt * ld_s + nb * math.log(model.beta_prior_prec)


@pytest.mark.parametrize("shape", [(4, 3, 2), (5, 4, 0), (3, 1, 3), (1, 5, 2), (7, 2, 1)])
@pytest.mark.parametrize("theta", [THETA0, np.array([0.3, -0.2, -0.7, 2.0]),
                                   np.array([-0.5, 0.4, 0.0, 1.0])])
def test_logdet_prior_closed_form(shape, theta):
    model = small(*shape)
    Qp = O.prior_precision(model, theta)
    L = np.linalg.cholesky(Qp.toarray())
    ld = 2.0 * math.fsum(np.log(np.diag(L)))
    ref = closed_logdet_prior(model, theta)
    assert rel(O.eval_f_dense(model, theta)["logdet_p"], ref) < 1e-12
    assert rel(ld, ref) < 1e-12


def test_prior_variance_closed_form():
    model = small(5, 4, 2)
    theta = np.array([0.3, 0.5, 0.8, 1.0])
    tau, kappa, rho, _ = O.theta_params(theta)
    N, h, nt, ns = model.N, model.h, model.nt, model.ns
    lam = path_eigs(N)
    V = dct_basis(N)
    k2 = kappa * kappa * h * h
    # (Q_s^{-1})_ss = h^2/tau^2 sum_ij phi_ij(s)^2 / (k2 + lam_i + lam_j)^2
    qinv = np.zeros(ns)
    for iy in range(N):
        for ix in range(N):
            phi2 = (V[ix, :][:, None] * V[iy, :][None, :]) ** 2  # [i (x-mode), j (y-mode)]
            qinv[iy * N + ix] = (h * h / (tau * tau)) * np.sum(
                phi2 / (k2 + lam[:, None] + lam[None, :]) ** 2)
    Sp = np.linalg.inv(O.prior_precision(model, theta).toarray())
    v = np.diag(Sp)
    np.testing.assert_allclose(v[:ns * nt], np.tile(qinv, nt), rtol=1e-11)
    np.testing.assert_allclose(v[ns * nt:], 1.0 / model.beta_prior_prec, rtol=1e-12)
    # cross-time covariance of a stationary AR1: block (t+1, t) = rho * block (t, t)
    D, S, R, T = O.bta_blocks(Sp, ns, nt, model.nb)
    for t in range(nt - 1):
        np.testing.assert_allclose(S[t], rho * D[t], rtol=1e-10, atol=1e-14 * np.abs(D[t]).max())
    assert np.abs(R).max() < 1e-14


def test_prior_traces_closed_form():
    model = small(4, 5, 2)
    theta = np.array([0.2, 0.7, 0.6, 3.0])
    tau, kappa, rho, _ = O.theta_params(theta)
    N, h, nt, ns = model.N, model.h, model.nt, model.ns
    lam = path_eigs(N)
    k2 = kappa * kappa * h * h
    Sp = np.linalg.inv(O.prior_precision(model, theta).toarray())
    dQp, _ = O.dprecision(model, theta)
    tr = [float(np.sum(Sp * d.toarray())) for d in dQp]
    assert rel(tr[0], 2 * ns * nt) < 1e-11
    assert rel(tr[1], nt * np.sum(4 * k2 / (k2 + lam[:, None] + lam[None, :]))) < 1e-11
    assert rel(tr[2], 2 * rho * ns * (nt - 1)) < 1e-11
    assert abs(tr[3]) == 0.0


def test_dprecision_matches_central_differences_of_builders():
    model = small(4, 3, 2)
    theta = np.array([0.1, 0.9, 0.5, 2.0])
    dQp, dQc = O.dprecision(model, theta)
    h = 1e-6
    for k in range(4):
        e = np.zeros(4)
        e[k] = h
        Pp, Pc, _ = O.conditional_precision(model, theta + e)
        Mp, Mc, _ = O.conditional_precision(model, theta - e)
        fdp = ((Pp - Mp) / (2 * h)).toarray()
        fdc = ((Pc - Mc) / (2 * h)).toarray()
        scale_p = max(1.0, np.abs(fdp).max())
        scale_c = max(1.0, np.abs(fdc).max())
        assert np.abs(fdp - dQp[k].toarray()).max() / scale_p < 1e-7
        assert np.abs(fdc - dQc[k].toarray()).max() / scale_c < 1e-7


# ---------------------------------------------------------------- Gaussian identities

def marginal_likelihood_f(model, theta):
    """f(theta) = -log pi(theta) - log N(y; 0, A Q_p^{-1} A^T + tau_y^{-1} I)."""
    import scipy.linalg as sla
    tau_y = O.theta_params(theta)[3]
    A = O.obs_matrix(model).toarray()
    Lp = np.linalg.cholesky(O.prior_precision(model, theta).toarray())
    W = sla.solve_triangular(Lp, A.T, lower=True)  # A Q_p^{-1} A^T = W^T W
    S = W.T @ W + np.eye(model.m) / tau_y
    sign, ld = np.linalg.slogdet(S)
    assert sign > 0
    quad = float(model.y @ np.linalg.solve(S, model.y))
    return -scipy_log_hyperprior(model, theta) + 0.5 * ld + 0.5 * quad + 0.5 * model.m * O.LOG2PI


def scipy_log_hyperprior(model, theta):
    """Independent Gaussian hyperprior N(m_k, 1/p_k) through scipy's own normal density."""
    from scipy.stats import norm
    sd = 1.0 / np.sqrt(np.asarray(model.theta_prior_prec, dtype=np.float64))
    return math.fsum(norm.logpdf(np.asarray(theta, dtype=np.float64),
                                 loc=np.asarray(model.theta_prior_mean, dtype=np.float64),
                                 scale=sd))


@pytest.mark.parametrize("mean,prec,theta", [
    (np.zeros(4), np.full(4, 0.01), THETA0),
    (np.array([0.5, -1.0, 2.0, 3.0]), np.array([1.0, 4.0, 0.25, 9.0]),
     np.array([0.3, -0.2, -0.7, 2.0])),
    (np.array([-3.0, 0.0, 0.1, 10.0]), np.array([100.0, 1e-4, 2.0, 0.5]),
     np.array([-2.5, 7.0, 0.0, -1.0])),
])
def test_log_hyperprior_is_the_gaussian_density(mean, prec, theta):
    """log pi(theta), constants included (the Gaussian hyperprior reading of
    Sec. "Latent Gaussian Models"), against scipy.stats.norm.logpdf summed over
    the four components."""
    model = small()
    model.theta_prior_mean = mean
    model.theta_prior_prec = prec
    assert rel(O.log_hyperprior(model, theta), scipy_log_hyperprior(model, theta)) < 1e-14


@pytest.mark.parametrize("shape,tol", [((4, 3, 2), 1e-10), ((3, 2, 0), 1e-10), ((2, 4, 1), 1e-10)])
def test_f_equals_marginal_likelihood(shape, tol):
    model = small(*shape)
    for theta in (THETA0, np.array([0.4, 0.2, -0.3, 1.5])):
        assert rel(O.eval_f_dense(model, theta)["f"], marginal_likelihood_f(model, theta)) < tol


@pytest.mark.slow
def test_f_equals_marginal_likelihood_c1():
    from inla_synth import config_model
    model = config_model("c1")
    # S (2000 x 2000) has condition number ~2e8 here (Var(beta) = 1e3 against a
    # noise variance of 1e-2), so the m-space route itself carries ~1e-10 relative
    # rounding error in y^T S^{-1} y; the pin is set an order of magnitude above it.
    assert rel(O.eval_f_dense(model, THETA0)["f"], marginal_likelihood_f(model, THETA0)) < 1e-9


def test_determinant_lemma_and_posterior_forms():
    model = small(4, 3, 2)
    theta = np.array([0.1, 0.8, 0.9, 3.0])
    tau_y = O.theta_params(theta)[3]
    out = O.eval_f_dense(model, theta)
    A = O.obs_matrix(model).toarray()
    Sp = np.linalg.inv(O.prior_precision(model, theta).toarray())
    M = np.eye(model.m) + tau_y * A @ Sp @ A.T
    assert rel(out["logdet_c"], out["logdet_p"] + np.linalg.slogdet(M)[1]) < 1e-11
    S = A @ Sp @ A.T + np.eye(model.m) / tau_y
    mu_krig = Sp @ A.T @ np.linalg.solve(S, model.y)
    np.testing.assert_allclose(out["mu"], mu_krig, rtol=1e-9, atol=1e-11 * np.abs(mu_krig).max())
    Sc_wood = Sp - Sp @ A.T @ np.linalg.solve(S, A @ Sp)
    np.testing.assert_allclose(O.marginal_variances_dense(model, theta), np.diag(Sc_wood),
                               rtol=1e-9)
    # 2 h(mu) = tau_y y^T y - b^T mu for h(x) = 1/2 x^T Q_p x + tau_y/2 |y - A x|^2
    _, _, b = O.conditional_precision(model, theta)
    lhs = out["quad"] + tau_y * out["rss"]
    assert rel(lhs, tau_y * float(model.y @ model.y) - float(b @ out["mu"])) < 1e-10


# ---------------------------------------------------------------- selected inversion

def test_selected_inversion_recursions_agree_with_inverse():
    model = small(3, 3, 2)
    _, Qc, _ = O.conditional_precision(model, THETA0)
    Q = Qc.toarray()
    L = np.linalg.cholesky(Q)
    Sinv = np.linalg.inv(Q)
    S1 = O.selinv_rue_martino(L)
    S2 = O.selinv_takahashi(L)
    scale = np.abs(Sinv).max()
    assert np.abs(S1 - Sinv).max() / scale < 1e-12
    assert np.abs(S2 - Sinv).max() / scale < 1e-12
    assert np.abs(S1 - S2).max() / scale < 1e-13


def test_selected_inversion_two_by_two():
    # Sigma_11 = (l21^2 + l22^2) / (l11^2 l22^2) for L = [[l11, 0], [l21, l22]]
    l11, l21, l22 = 1.7, -0.4, 0.9
    L = np.array([[l11, 0.0], [l21, l22]])
    for S in (O.selinv_rue_martino(L), O.selinv_takahashi(L)):
        assert rel(S[0, 0], (l21 ** 2 + l22 ** 2) / (l11 ** 2 * l22 ** 2)) < 1e-15
        assert rel(S[1, 1], 1.0 / l22 ** 2) < 1e-15


def test_gmrf_sample_covariance():
    """x = L^{-T} z with z ~ N(0, I) has covariance Q^{-1} (Sec. "Partial Inversion")."""
    model = small(2, 2, 1)
    _, Qc, _ = O.conditional_precision(model, np.array([0.0, 0.5, 0.3, 0.0]))
    Q = Qc.toarray()
    L = np.linalg.cholesky(Q)
    rng = np.random.default_rng(5)
    z = rng.standard_normal((Q.shape[0], 200000))
    x = np.linalg.solve(L.T, z)
    C = np.cov(x)
    Sinv = np.linalg.inv(Q)
    se = np.sqrt((Sinv ** 2 + np.outer(np.diag(Sinv), np.diag(Sinv))) / z.shape[1])
    assert np.all(np.abs(C - Sinv) < 6 * se)


# ---------------------------------------------------------------- gradient

@pytest.mark.parametrize("shape", [(4, 3, 2), (3, 1, 2), (3, 3, 0), (1, 4, 1)])
def test_gradient_matches_central_differences(shape):
    model = small(*shape)
    theta = np.array([0.2, 0.6, 0.7, 2.5])
    g = O.dense_gradient(model, theta)
    fd = O.fd_gradient(model, theta, h=1e-5)
    scale = np.abs(fd).max()
    assert np.all(np.abs(g - fd) <= 1e-7 * np.maximum(np.abs(fd), 1e-3 * scale))


# ---------------------------------------------------------------- special cases

def test_rho_zero_is_block_diagonal():
    model = small(4, 3, 0)
    theta = np.array([0.1, 0.5, 0.0, 1.0])
    Qp = O.prior_precision(model, theta).toarray()
    D, S, _, _ = O.bta_blocks(Qp, model.ns, model.nt, 0)
    assert np.abs(S).max() == 0.0
    Ls = np.linalg.cholesky(D[0])
    assert rel(O.eval_f_dense(model, theta)["logdet_p"],
               model.nt * 2 * math.fsum(np.log(np.diag(Ls)))) < 1e-13


def test_single_node_grid_is_scalar_ar1_with_arrow():
    model = small(1, 6, 2)
    theta = np.array([0.3, 0.2, 0.4, 1.0])
    tau, kappa, rho, _ = O.theta_params(theta)
    Qp = O.prior_precision(model, theta).toarray()
    qs = tau * tau * kappa ** 4 * model.h ** 2  # (tau^2/h^2) (kappa^2 h^2)^2, h = 1
    ref = qs * O.ar1_precision(6, rho).toarray()
    np.testing.assert_allclose(Qp[:6, :6], ref, rtol=1e-14)
    np.testing.assert_allclose(Qp[6:, 6:], 1e-3 * np.eye(2))


def test_fig1_arrowhead_fill_pattern():
    pats = {}
    with open(os.path.join(GOLDEN, "fig1_arrowhead.txt")) as fh:
        lines = [ln.strip() for ln in fh if ln.strip() and not ln.startswith("#")]
    for i in range(0, len(lines), 5):
        pats[lines[i]] = np.array([[c == "x" for c in row] for row in lines[i + 1:i + 5]])
    rng = np.random.default_rng(3)
    Q1 = np.where(pats["Q1"], rng.uniform(0.1, 1.0, (4, 4)), 0.0)
    Q1 = np.triu(Q1) + np.triu(Q1, 1).T + 4.0 * np.eye(4)
    L1 = O.bta_factor_blocks(Q1, 4, 1, 0)[0][0]
    assert np.array_equal(np.abs(L1) > 1e-15, pats["L1"])
    perm = [1, 2, 3, 0]  # move the dense row/column last
    Q2 = Q1[np.ix_(perm, perm)]
    assert np.array_equal(Q2 != 0, pats["Q2"])
    L2 = O.bta_factor_blocks(Q2, 4, 1, 0)[0][0]
    assert np.array_equal(np.abs(L2) > 1e-15, pats["L2"])
    # in block form with the dense row as a 1-wide arrow: no fill in the space-time part
    D, S, R, T = O.bta_factor_blocks(Q2, 1, 3, 1)
    assert np.all(S == 0.0)


# ---------------------------------------------------------------- banded route

@pytest.mark.parametrize("shape", [(5, 4, 3), (6, 2, 0), (4, 1, 2), (1, 7, 1)])
def test_banded_route_matches_dense(shape):
    model = small(*shape)
    theta = np.array([0.1, 0.9, 1.1, 3.5])
    d = O.eval_f_dense(model, theta)
    bnd = O.eval_f_banded(model, theta, return_factors=True)
    for key in ("f", "logdet_p", "logdet_c"):
        assert rel(bnd[key], d[key]) < 1e-12
    np.testing.assert_allclose(bnd["mu"], d["mu"], rtol=1e-10, atol=1e-12 * np.abs(d["mu"]).max())
    idx = np.arange(model.n)
    v = O.variance_samples_banded(bnd["factor_c"], idx)
    np.testing.assert_allclose(v, O.marginal_variances_dense(model, theta), rtol=1e-10)


# ---------------------------------------------------------------- planted mistakes

def test_pins_detect_planted_mistakes(monkeypatch):
    """Each plausible slip in the oracle must trip at least one pin above."""
    model = small(4, 3, 2)
    theta = np.array([0.2, 0.6, 0.7, 2.5])
    good_ld = closed_logdet_prior(model, theta)
    good_ml = marginal_likelihood_f(model, theta)

    # (1) wrong spatial scaling: tau instead of tau^2
    orig_sp = O.spatial_precision
    monkeypatch.setattr(O.inla_oracle, "spatial_precision",
                        lambda N, h, tau, kappa: orig_sp(N, h, math.sqrt(tau), kappa))
    assert rel(O.eval_f_dense(model, theta)["logdet_p"], good_ld) > 1e-6
    monkeypatch.undo()

    # (2) sign slip in the AR1 coupling: logdet is blind, cross-covariance is not
    orig_ar = O.ar1_precision
    monkeypatch.setattr(O.inla_oracle, "ar1_precision", lambda nt, rho: orig_ar(nt, -rho))
    Sp = np.linalg.inv(O.prior_precision(model, theta).toarray())
    D, S, _, _ = O.bta_blocks(Sp, model.ns, model.nt, model.nb)
    rho = math.tanh(theta[2])
    assert np.abs(S[0] - rho * D[0]).max() > 1e-3 * np.abs(D[0]).max()
    monkeypatch.undo()

    # (3) dropped constant in f: marginal-likelihood identity breaks
    orig_c = O.inla_oracle._combine

    def bad_combine(*a, **k):
        out = orig_c(*a, **k)
        out["f"] -= 0.5 * model.m * O.LOG2PI
        return out
    monkeypatch.setattr(O.inla_oracle, "_combine", bad_combine)
    assert rel(O.eval_f_dense(model, theta)["f"], good_ml) > 1e-6
    monkeypatch.undo()

    # (4) transposed operand in the likelihood term (A A^T-shaped slip is impossible
    #     dimensionally, so plant a missing tau_y on A^T A instead)
    orig_cp = O.conditional_precision

    def bad_cp(model_, theta_):
        Qp, Qc, b = orig_cp(model_, theta_)
        tau_y = O.theta_params(theta_)[3]
        A = O.obs_matrix(model_)
        return Qp, (Qc - (tau_y - 1.0) * (A.T @ A)).tocsr(), b
    monkeypatch.setattr(O.inla_oracle, "conditional_precision", bad_cp)
    assert rel(O.eval_f_dense(model, theta)["f"], good_ml) > 1e-6
    monkeypatch.undo()

    # (5) gradient with the wrong sign on the prior-trace term fails the FD pin
    orig_dp = O.dprecision

    def bad_dp(model_, theta_):
        dQp, dQc = orig_dp(model_, theta_)
        return [-d for d in dQp], dQc
    monkeypatch.setattr(O.inla_oracle, "dprecision", bad_dp)
    g = O.dense_gradient(model, theta)
    monkeypatch.undo()
    fd = O.fd_gradient(model, theta, h=1e-5)
    assert np.max(np.abs(g - fd) / np.maximum(np.abs(fd), 1e-3)) > 1e-4

    # (6) hyperprior without its 2 pi (log p instead of log(p / 2 pi)): both the
    #     density pin and the marginal-likelihood identity must fail
    def bad_prior(model_, theta_):
        t = np.asarray(theta_, dtype=np.float64)
        m = np.asarray(model_.theta_prior_mean, dtype=np.float64)
        p = np.asarray(model_.theta_prior_prec, dtype=np.float64)
        return float(np.sum(0.5 * np.log(p) - 0.5 * p * (t - m) ** 2))
    monkeypatch.setattr(O.inla_oracle, "log_hyperprior", bad_prior)
    monkeypatch.setattr(O, "log_hyperprior", bad_prior)
    assert rel(O.log_hyperprior(model, theta), scipy_log_hyperprior(model, theta)) > 1e-6
    assert rel(O.eval_f_dense(model, theta)["f"], good_ml) > 1e-6
    monkeypatch.undo()

    # (7) half the normalising constant dropped (1/2 log p taken as log p)
    def bad_prior2(model_, theta_):
        t = np.asarray(theta_, dtype=np.float64)
        m = np.asarray(model_.theta_prior_mean, dtype=np.float64)
        p = np.asarray(model_.theta_prior_prec, dtype=np.float64)
        return float(np.sum(np.log(p) - 0.5 * math.log(2.0 * math.pi) - 0.5 * p * (t - m) ** 2))
    monkeypatch.setattr(O.inla_oracle, "log_hyperprior", bad_prior2)
    assert rel(O.eval_f_dense(model, theta)["f"], good_ml) > 1e-6
    monkeypatch.undo()
