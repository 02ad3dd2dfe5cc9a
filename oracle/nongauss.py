"""Oracle of f(theta) and its gradient with a Poisson likelihood (test
infrastructure).

TEST INFRASTRUCTURE ONLY (see the package header): only tests/ may use it.

Paper: Sec. "Latent Gaussian Models" -- with a non-Gaussian likelihood the
Gaussian approximation pi_G(x | theta, y) of eq. (post_theta_approx) needs an
inner optimisation: its mode x* and its normalising constant are found anew in
every iteration, each iteration one more factorization of the precision of
pi_G; Sec. "Parallelization of Function Evaluations" notes that this inner
loop is what keeps automatic differentiation out of reach there.

Model (the latent Gaussian model of the Gaussian case with the likelihood
swapped; readings listed in the design notes):
  y_i ~ Poisson(exp(eta_i)), eta = A x (log link, unit exposure);
  log pi(y | x) = sum_i (y_i eta_i - exp(eta_i) - log y_i!);
  theta_4 does not enter the likelihood (only its prior);
  x* = argmax [log pi(x | theta) + log pi(y | x)], found by Newton's method:
    Q_c(x) = Q_p + A^T diag(exp(A x)) A,  Q_c(x) x_new = A^T (y + e (eta - 1)),
  from x = 0, each step halved (at most 60 times) until the objective does
  not decrease, until max |x_new - x| <= tol (1 + max |x|);
  f(theta) = -log pi(theta) - 1/2 log|Q_p| + 1/2 x*^T Q_p x* - log pi(y | x*)
             + 1/2 log|Q_c(x*)|  (the -n/2 log 2 pi of pi(x | theta) and of
             pi_G cancel).

Gradient (derived, listed in the design notes): with Sigma_c = Q_c(x*)^{-1},
dQ_k = dQ_p / dtheta_k (k = 1..3; zero for k = 4),
  df/dtheta_k = p_k (theta_k - m_k) - 1/2 tr(Q_p^{-1} dQ_k) + 1/2 x*^T dQ_k x*
                + 1/2 tr(Sigma_c dQ_k) - z^T dQ_k x*,
  z = Sigma_c A^T c,  c_i = 1/2 exp(eta*_i) (A Sigma_c A^T)_ii:
the last term is the implicit one -- x* moves with theta
(dx*/dtheta_k = -Sigma_c dQ_k x*) and log|Q_c(x*)| depends on x*
(d/dx_j 1/2 log|Q_c| = (A^T c)_j); the other terms of f are stationary in x
at the mode.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp
from scipy.special import gammaln

from . import inla_oracle as O


def log_lik(y, eta) -> float:
    """sum_i y_i eta_i - exp(eta_i) - log y_i!"""
    return float(np.sum(y * eta - np.exp(eta) - gammaln(y + 1.0)))


def newton_mode(model, theta, tol=1e-12, max_iter=200):
    """x* by Newton's method with step halving (dense solves).  Returns
    (x*, iterations)."""
    Qp = O.prior_precision(model, theta).toarray()
    A = O.obs_matrix(model)
    y = model.y
    x = np.zeros(model.n)

    def objective(v):
        return -0.5 * float(v @ (Qp @ v)) + log_lik(y, A @ v)

    gx = objective(x)
    for it in range(1, max_iter + 1):
        eta = A @ x
        e = np.exp(eta)
        Qc = Qp + (A.T @ sp.diags(e) @ A).toarray()
        xn = np.linalg.solve(Qc, A.T @ (y + e * (eta - 1.0)))
        step = 1.0
        cand = xn
        gc = objective(cand)
        halvings = 0
        while not gc >= gx and halvings < 60:
            step *= 0.5
            cand = x + step * (xn - x)
            gc = objective(cand)
            halvings += 1
        done = np.abs(cand - x).max() <= tol * (1.0 + np.abs(x).max())
        x, gx = cand, gc
        if done:
            return x, it
    raise RuntimeError("Newton's method did not converge")


def conditional_precision_at(model, theta, x):
    Qp = O.prior_precision(model, theta)
    A = O.obs_matrix(model)
    return Qp, Qp + A.T @ sp.diags(np.exp(A @ x)) @ A


def eval_f(model, theta, tol=1e-12) -> dict:
    """f(theta) at the Newton mode (dense log-determinants)."""
    t = np.asarray(theta, dtype=np.float64)
    x, iters = newton_mode(model, t, tol)
    Qp, Qc = conditional_precision_at(model, t, x)
    A = O.obs_matrix(model)
    ldp = np.linalg.slogdet(Qp.toarray())[1]
    ldc = np.linalg.slogdet(Qc.toarray())[1]
    quad = float(x @ (Qp @ x))
    ll = log_lik(model.y, A @ x)
    lp = O.log_hyperprior(model, t)
    f = -lp - 0.5 * ldp + 0.5 * quad - ll + 0.5 * ldc
    return dict(f=f, x=x, iterations=iters, logdet_p=ldp, logdet_c=ldc, quad=quad,
                log_lik=ll, log_prior=lp)


def gradient(model, theta, tol=1e-12, implicit=True) -> np.ndarray:
    """The exact gradient (explicit terms at x*, plus the implicit term)."""
    t = np.asarray(theta, dtype=np.float64)
    x, _ = newton_mode(model, t, tol)
    Qp, Qc = conditional_precision_at(model, t, x)
    A = O.obs_matrix(model)
    Sp = np.linalg.inv(Qp.toarray())
    Sc = np.linalg.inv(Qc.toarray())
    dQp, _ = O.dprecision(model, t)
    eta = A @ x
    Ad = A.toarray()
    c = 0.5 * np.exp(eta) * np.einsum("ij,jk,ik->i", Ad, Sc, Ad)
    z = Sc @ (A.T @ c)
    pm = np.asarray(model.theta_prior_mean)
    pp = np.asarray(model.theta_prior_prec)
    g = pp * (t - pm)
    for k in range(3):
        D = dQp[k]
        g[k] += (-0.5 * float(np.sum(Sp * D.toarray())) + 0.5 * float(x @ (D @ x))
                 + 0.5 * float(np.sum(Sc * D.toarray())))
        if implicit:
            g[k] -= float(z @ (D @ x))
    return g


def obs_variances(model, theta, x):
    """(A Sigma_c A^T)_ii at x (dense)."""
    _, Qc = conditional_precision_at(model, theta, x)
    Ad = O.obs_matrix(model).toarray()
    Sc = np.linalg.inv(Qc.toarray())
    return np.einsum("ij,jk,ik->i", Ad, Sc, Ad)


def laplace_scalar(y, a, q, log_prior_theta, lo=-50.0, hi=50.0):
    """Textbook Laplace approximation for ONE latent variable x ~ N(0, 1/q)
    with y_i ~ Poisson(exp(a_i x)): log p(y | theta) ~ h(x*) + 1/2 log 2 pi
    - 1/2 log(-h''(x*)), h = log N(x; 0, 1/q) + log-likelihood, x* by
    bisection on h'.  Returns -log pi(theta) - that (the f of this model)."""
    y = np.asarray(y, dtype=np.float64)
    a = np.asarray(a, dtype=np.float64)

    def dh(v):
        return -q * v + float(np.sum(a * (y - np.exp(a * v))))

    for _ in range(400):
        mid = 0.5 * (lo + hi)
        if dh(mid) > 0:
            lo = mid
        else:
            hi = mid
    xs = 0.5 * (lo + hi)
    h = (0.5 * math.log(q) - 0.5 * math.log(2 * math.pi) - 0.5 * q * xs * xs
         + float(np.sum(y * a * xs - np.exp(a * xs) - gammaln(y + 1.0))))
    h2 = q + float(np.sum(a * a * np.exp(a * xs)))
    return -log_prior_theta - (h + 0.5 * math.log(2 * math.pi) - 0.5 * math.log(h2)), xs
