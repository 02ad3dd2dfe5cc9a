"""The Poisson-likelihood oracle (Sec. "Latent Gaussian Models": the inner
optimisation of a non-Gaussian likelihood) pinned to facts that fix it: the
mode against a general-purpose optimiser, the gradient (with its implicit
term) against central differences of f, the one-latent-variable case against
the textbook Laplace formula, and that formula against the exact integral."""
import math

import numpy as np
import pytest
import scipy.integrate
import scipy.optimize
from scipy.special import gammaln

from inla_synth import THETA0, make_model, poisson_counts
from oracle import inla_oracle as O
from oracle import nongauss as NG


@pytest.fixture(scope="module")
def small():
    return poisson_counts(make_model(4, 3, 2, 5), seed=1)


THETA = np.array([0.1, 0.9, 0.6, 1.5])


def test_mode_is_the_maximiser(small):
    """Newton's mode is stationary and equals the maximiser a quasi-Newton
    method finds on the same objective."""
    md = small
    x, iters = NG.newton_mode(md, THETA)
    Qp = O.prior_precision(md, THETA)
    A = O.obs_matrix(md)
    grad = -(Qp @ x) + A.T @ (md.y - np.exp(A @ x))
    assert np.abs(grad).max() < 1e-9 * max(1.0, np.abs(A.T @ md.y).max())
    obj = lambda v: 0.5 * float(v @ (Qp @ v)) - NG.log_lik(md.y, A @ v)
    jac = lambda v: Qp @ v - A.T @ (md.y - np.exp(A @ v))
    ref = scipy.optimize.minimize(obj, np.zeros(md.n), jac=jac, method="L-BFGS-B",
                                  options=dict(ftol=1e-15, gtol=1e-11, maxiter=5000))
    assert np.abs(ref.x - x).max() < 1e-5 * max(1.0, np.abs(x).max())
    assert 2 <= iters < 50


def test_gradient_matches_central_differences(small):
    """The gradient with the implicit term equals central differences of f;
    without the implicit term it does not (the planted slip must fail)."""
    md = small
    g = NG.gradient(md, THETA)
    h = 1e-5
    fd = np.empty(4)
    for k in range(4):
        e = np.zeros(4)
        e[k] = h
        fd[k] = (NG.eval_f(md, THETA + e)["f"] - NG.eval_f(md, THETA - e)["f"]) / (2 * h)
    scale = np.abs(fd).max()
    assert np.abs(g - fd).max() < 1e-6 * scale, (g, fd)
    assert g[3] == pytest.approx(md.theta_prior_prec[3] * (THETA[3] - md.theta_prior_mean[3]))
    g0 = NG.gradient(md, THETA, implicit=False)
    assert np.abs(g0 - fd).max() > 1e-4 * scale


def _one_node(seed=3, per=30, level=2.0):
    md = make_model(1, 1, 0, seed, obs_per_node=per)
    return poisson_counts(md, seed=seed, level=level, spread=0.3)


def test_one_latent_variable_is_the_textbook_laplace_formula():
    """With one latent variable (a 1 x 1 grid, one time point, no fixed
    effects) f is -log pi(theta) minus the textbook Laplace approximation of
    log p(y | theta) = log int N(x; 0, 1/q) prod_i Pois(y_i; e^x) dx."""
    md = _one_node()
    for theta in (THETA0, np.array([0.4, -0.2, 0.0, 0.0])):
        r = NG.eval_f(md, theta)
        q = float(O.prior_precision(md, theta).toarray()[0, 0])
        f_lap, xs = NG.laplace_scalar(md.y, np.ones(md.m), q, O.log_hyperprior(md, theta))
        assert abs(r["x"][0] - xs) < 1e-10
        assert abs(r["f"] - f_lap) < 1e-10 * max(1.0, abs(f_lap))


def test_laplace_formula_approximates_the_exact_integral():
    """... and that approximation is within the Laplace error of the exact
    integral, computed by adaptive quadrature (total count ~ 250: the error
    is of order 1/(12 sum y))."""
    md = _one_node()
    theta = np.array([0.4, -0.2, 0.0, 0.0])
    q = float(O.prior_precision(md, theta).toarray()[0, 0])
    lp = O.log_hyperprior(md, theta)
    f_lap, xs = NG.laplace_scalar(md.y, np.ones(md.m), q, lp)
    y = md.y

    def h(v):
        return (0.5 * math.log(q / (2 * math.pi)) - 0.5 * q * v * v
                + float(np.sum(y * v - np.exp(v) - gammaln(y + 1.0))))

    h0 = h(xs)
    val, err = scipy.integrate.quad(lambda v: math.exp(h(v) - h0), xs - 3, xs + 3,
                                    epsabs=1e-14, epsrel=1e-12, limit=200)
    exact = h0 + math.log(val)
    assert y.sum() > 150
    assert abs((-lp - f_lap) - exact) < 2e-3
    # the constants matter: dropping the 1/2 log 2 pi of the Laplace formula is far off
    assert abs((-lp - f_lap - 0.5 * math.log(2 * math.pi)) - exact) > 0.5
