"""The integration step after the mode search (Sec. "Latent Gaussian Models",
Sec. "Approximating pi(x_i | y)", eq. LatParam): the oracle's FD Hessian,
standardised grid, quadrature over theta and latent mixture pinned to facts
that fix them -- closed-form Hessians, Gaussian integrals, a brute-force
lattice count, one-dimensional numerical integration of a mixture density and
the Laplace approximation as the one-point special case."""
import itertools
import math

import numpy as np
import pytest
import scipy.optimize

from inla_synth import THETA0, make_model
from oracle import inla_oracle as O
from oracle import integrate as I


# ---------------------------------------------------------------------------
# step 1: the Hessian from central differences of the gradient
# ---------------------------------------------------------------------------
def _smooth(t):
    """A non-quadratic test function with its gradient and Hessian in closed form."""
    a = np.array([0.5, 1.5, 2.0, 0.7])
    f = float(np.sum(a * np.exp(t)) + t[0] * t[1] ** 2 + math.sin(t[2] * t[3]))
    g = a * np.exp(t)
    g = g + np.array([t[1] ** 2, 2 * t[0] * t[1],
                      t[3] * math.cos(t[2] * t[3]), t[2] * math.cos(t[2] * t[3])])
    c, s = math.cos(t[2] * t[3]), math.sin(t[2] * t[3])
    H = np.diag(a * np.exp(t))
    H[0, 1] += 2 * t[1]
    H[1, 0] += 2 * t[1]
    H[1, 1] += 2 * t[0]
    H[2, 2] += -t[3] ** 2 * s
    H[3, 3] += -t[2] ** 2 * s
    H[2, 3] += c - t[2] * t[3] * s
    H[3, 2] += c - t[2] * t[3] * s
    return f, g, H


def test_fd_hessian_matches_the_closed_form():
    t = np.array([0.3, -0.4, 0.8, 1.1])
    H = I.fd_hessian(lambda x: _smooth(x)[1], t, h=1e-4)
    np.testing.assert_allclose(H, _smooth(t)[2], rtol=1e-7, atol=1e-7)
    assert np.array_equal(H, H.T)


def _quadratic(seed=3, d=4):
    rng = np.random.default_rng(seed)
    B = rng.standard_normal((d, d))
    A = B @ B.T + d * np.diag(rng.uniform(0.5, 2.0, d))
    c = rng.standard_normal(d)
    f0 = 17.25
    f = lambda t: f0 + 0.5 * float((t - c) @ A @ (t - c))
    g = lambda t: A @ (t - c)
    return A, c, f0, f, g


def test_standardised_coordinates_whiten_the_hessian():
    A, c, f0, f, g = _quadratic()
    H = I.fd_hessian(g, c)
    np.testing.assert_allclose(H, A, rtol=1e-12, atol=1e-10)
    lam, V, M = I.standardise(H)
    assert np.all(np.diff(lam) > 0)
    np.testing.assert_allclose(M.T @ A @ M, np.eye(4), atol=1e-12)
    for j in range(4):
        assert V[np.argmax(np.abs(V[:, j])), j] > 0


def test_standardise_rejects_an_indefinite_hessian():
    with pytest.raises(ValueError):
        I.standardise(np.diag([1.0, -2.0, 3.0, 4.0]))


# ---------------------------------------------------------------------------
# steps 3-4: axis ranges and the kept points
# ---------------------------------------------------------------------------
def test_kept_points_are_the_lattice_ball_of_the_gaussian():
    """For a quadratic f the drop at z = dz s is dz^2 |s|^2 / 2 exactly, so the
    kept points are the integer vectors with |s|^2 < 2 dpi / dz^2, counted here
    by brute force over a box larger than the search's."""
    A, c, f0, f, g = _quadratic()
    lam, V, M = I.standardise(I.fd_hessian(g, c))
    for dz, dpi in ((1.0, 2.4), (0.5, 1.2), (1.0, 4.6)):
        fm, lo, hi, cands = I.explore(f, c, M, dz, dpi, max_steps=8)
        r = int(math.floor(math.sqrt(2 * dpi) / dz - 1e-12))
        assert list(lo) == [r] * 4 and list(hi) == [r] * 4
        kept = {tuple(s) for s, th, fv in cands if fv - fm < dpi}
        ball = {s for s in itertools.product(range(-r - 2, r + 3), repeat=4)
                if 0.5 * dz * dz * sum(x * x for x in s) < dpi}
        assert kept == ball
    # dz = 1, dpi = 2.4: 1 + 8 + 24 + 32 + 24 points with |s|^2 = 0..4 (the
    # thresholds avoid drops equal to dpi, which rounding would decide)
    fm, lo, hi, cands = I.explore(f, c, M, 1.0, 2.4)
    assert sum(fv - fm < 2.4 for _, _, fv in cands) == 89


def test_exploration_stops_at_max_steps_and_at_failed_points():
    A, c, f0, f, g = _quadratic()
    lam, V, M = I.standardise(A)
    fm, lo, hi, _ = I.explore(f, c, M, 1.0, 1e6, max_steps=3)
    assert list(lo) == [3] * 4 and list(hi) == [3] * 4
    # a point where f cannot be evaluated (+inf) ends that direction
    fe = lambda t: math.inf if np.linalg.solve(M, t - c)[0] > 0.5 else f(t)
    fm, lo, hi, _ = I.explore(fe, c, M, 1.0, 1e6, max_steps=3)
    assert hi[0] == 0 and lo[0] == 3


# ---------------------------------------------------------------------------
# step 5: the quadrature over theta
# ---------------------------------------------------------------------------
def _gaussian_quadrature(dz, dpi, seed=3):
    A, c, f0, f, g = _quadratic(seed)
    lam, V, M = I.standardise(I.fd_hessian(g, c))
    fm, lo, hi, cands = I.explore(f, c, M, dz, dpi, max_steps=12)
    kept = [(th, fv) for s, th, fv in cands if fv - fm < dpi]
    w, mean, cov, log_ev = I.quadrature(fm, [k[1] for k in kept], [k[0] for k in kept], lam, dz)
    return A, c, f0, w, mean, cov, log_ev


@pytest.mark.parametrize("dz", [1.0, 0.75])
def test_quadrature_of_a_gaussian_gives_its_moments_and_integral(dz):
    """exp(-f) with f = f0 + (t - c)^T A (t - c) / 2 integrates to
    exp(-f0) (2 pi)^2 det(A)^{-1/2} with mean c and covariance A^{-1}; the
    lattice rule is exact to ~1e-8 for a Gaussian at these steps and the ball
    |z|^2 < 40 holds all but ~1e-7 of the mass."""
    A, c, f0, w, mean, cov, log_ev = _gaussian_quadrature(dz, 20.0)
    assert abs(w.sum() - 1.0) < 1e-14
    np.testing.assert_allclose(mean, c, rtol=0, atol=1e-12)
    np.testing.assert_allclose(cov, np.linalg.inv(A), rtol=2e-6, atol=1e-8)
    exact = -f0 + 2.0 * math.log(2 * math.pi) - 0.5 * np.linalg.slogdet(A)[1]
    assert abs(log_ev - exact) < 1e-6


def test_planted_mistakes_fail_the_gaussian_pin(monkeypatch):
    """Each slip below must break the Gaussian pin: the whitening with
    lambda^{+1/2}, M^T in place of M, and a covariance not taken about the
    mean."""
    real = I.standardise

    def wrong_power(H):
        lam, V, M = real(H)
        return lam, V, V * lam ** 0.5

    def transposed(H):
        lam, V, M = real(H)
        return lam, V, M.T.copy()

    real_quad = I.quadrature

    def uncentred(f0, kf, kt, lam, dz):
        w, mean, cov, ev = real_quad(f0, kf, kt, lam, dz)
        th = np.asarray(kt)
        return w, mean, (w[:, None] * th).T @ th, ev

    for name, fn in (("standardise", wrong_power), ("standardise", transposed),
                     ("quadrature", uncentred)):
        with monkeypatch.context() as m:
            m.setattr(I, name, fn)
            with pytest.raises(AssertionError):
                test_quadrature_of_a_gaussian_gives_its_moments_and_integral(1.0)


# ---------------------------------------------------------------------------
# step 6: the latent mixture (eq. LatParam)
# ---------------------------------------------------------------------------
def test_latent_mixture_matches_the_integrated_mixture_density():
    """Mean and variance of sum_k w_k N(mu^k, v^k) by one-dimensional
    numerical integration of the mixture density on a fine grid."""
    rng = np.random.default_rng(11)
    K, n = 3, 5
    mus = rng.normal(0.0, 2.0, (K, n)) + 40.0
    vs = rng.uniform(0.2, 1.5, (K, n))
    w = rng.uniform(0.1, 1.0, K)
    w /= w.sum()
    mean, var = I.latent_mixture(mus, vs, w)
    for i in range(n):
        x = np.linspace(mus[:, i].min() - 14, mus[:, i].max() + 14, 200001)
        p = sum(w[k] * np.exp(-0.5 * (x - mus[k, i]) ** 2 / vs[k, i]) / math.sqrt(2 * math.pi * vs[k, i])
                for k in range(K))
        m1 = np.trapezoid(x * p, x)
        m2 = np.trapezoid((x - m1) ** 2 * p, x)
        assert abs(np.trapezoid(p, x) - 1.0) < 1e-10
        assert abs(mean[i] - m1) < 1e-9 and abs(var[i] - m2) < 1e-8
    # one point: the Gaussian itself
    m, v = I.latent_mixture(mus[:1], vs[:1], [1.0])
    assert np.array_equal(m, mus[0]) and np.array_equal(v, vs[0])


# ---------------------------------------------------------------------------
# the whole step on a small model
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def small():
    md = make_model(4, 3, 2, 5)
    res = scipy.optimize.minimize(lambda t: O.eval_f_dense(md, t)["f"], THETA0,
                                  jac=lambda t: O.dense_gradient(md, t), method="BFGS",
                                  options=dict(gtol=1e-9, maxiter=400))
    return md, res.x


def test_model_hessian_agrees_with_second_differences_of_f(small):
    """Two routes to the Hessian of f at the mode: differences of the adjoint
    gradient and second differences of f alone."""
    md, t = small
    H = I.fd_hessian(lambda x: O.dense_gradient(md, x), t, h=1e-4)
    f = lambda x: O.eval_f_dense(md, x)["f"]
    h = 2e-3
    H2 = np.empty((4, 4))
    E = np.eye(4) * h
    for k in range(4):
        for j in range(4):
            H2[k, j] = (f(t + E[k] + E[j]) - f(t + E[k] - E[j]) - f(t - E[k] + E[j])
                        + f(t - E[k] - E[j])) / (4 * h * h)
    np.testing.assert_allclose(H, H2, rtol=1e-4, atol=1e-4 * np.abs(H).max())


def test_one_point_rule_is_the_laplace_approximation(small):
    """With only the mode kept and dz = sqrt(2 pi) the log evidence is the
    Laplace approximation -f* + (d/2) log 2 pi - log det(H) / 2, the theta
    moments are (theta*, 0) and the latent mixture is N(mu(theta*), v(theta*))."""
    md, t = small
    r = I.integrate_model(md, t, dz=math.sqrt(2 * math.pi), dpi=1e-9)
    assert r["theta"].shape == (1, 4) and np.array_equal(r["s"], np.zeros((1, 4)))
    lap = -r["f_mode"] + 2.0 * math.log(2 * math.pi) - 0.5 * np.linalg.slogdet(r["hessian"])[1]
    assert abs(r["log_evidence"] - lap) < 1e-10 * max(1.0, abs(lap))
    np.testing.assert_allclose(r["theta_mean"], t, rtol=0, atol=1e-15)
    assert np.abs(r["theta_cov"]).max() == 0.0
    np.testing.assert_allclose(r["x_mean"], O.eval_f_dense(md, t)["mu"], rtol=1e-14, atol=1e-14)
    np.testing.assert_allclose(r["x_var"], O.marginal_variances_dense(md, t), rtol=1e-14)


def test_model_integration_invariants(small):
    """Weights positive and summing to one, the mode kept with the largest
    weight, every kept drop below dpi, a positive definite theta covariance
    close to H^{-1} (the posterior of theta is near Gaussian here), and a
    mixture variance at least the weighted mean of the point variances."""
    md, t = small
    r = I.integrate_model(md, t)
    w = r["weights"]
    assert np.all(w > 0) and abs(w.sum() - 1.0) < 1e-14
    i0 = [k for k, s in enumerate(r["s"]) if not s.any()]
    assert len(i0) == 1 and w[i0[0]] == w.max()
    assert np.all(r["f"] - r["f_mode"] < 2.5)
    assert np.all(np.linalg.eigvalsh(r["theta_cov"]) > 0)
    Hinv = np.linalg.inv(r["hessian"])
    assert np.abs(np.diag(r["theta_cov"]) / np.diag(Hinv) - 1.0).max() < 0.5
    # law of total variance: var >= E[v]
    TH = r["theta"]
    vs = np.array([O.marginal_variances_dense(md, th) for th in TH])
    assert np.all(r["x_var"] >= w @ vs - 1e-15)
