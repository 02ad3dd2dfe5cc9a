"""Oracle of the integration step after the mode search (test infrastructure).

TEST INFRASTRUCTURE ONLY (see the package header): only tests/ may use it.

Paper: Sec. "Latent Gaussian Models" (the mode theta* is found, the area
around it is explored and a set of points theta^k is chosen at which
pi~(theta^k | y) is evaluated; the posterior marginals of the hyperparameters
follow by numerical integration), Sec. "Approximating pi(x_i | y)" (eq. LatParam:
the latent marginals are the integral over theta of pi(theta | y) times
pi(x_i | theta, y); with a Gaussian likelihood the latter is the Gaussian
pi_G with mean mu(theta) and variance (Q_c(theta)^{-1})_ii, which needs one
partial inversion per point), Sec. "Parallelization of Function Evaluations"
(the points and their partial inversions are independent) and the final
Hessian approximation at the mode of Sec. "Leveraging Level 1 Parallelism".

The paper gives no design of the points.  Reading taken (the grid strategy of
Rue, Martino and Chopin, 2009, listed in the design notes):

1. H = Hessian of f = -log pi~(theta | y) at theta* by central differences of
   the gradient, H[k, :] = (grad f(theta* + h e_k) - grad f(theta* - h e_k)) / 2h,
   then symmetrised.
2. H = V diag(lambda) V^T with lambda ascending and each eigenvector's
   largest-magnitude entry positive; standardised coordinates
   theta(z) = theta* + V diag(lambda^{-1/2}) z.
3. Along each of the 2d directions +-e_j in z, steps s = 1, 2, ... of length dz
   (at most max_steps) while f(theta(s dz e_j)) - f(theta*) < dpi; the range on
   that side is the number of such steps.
4. Every z = dz s, s integer, inside the box of those ranges is a candidate;
   it is kept when f(theta(z)) - f(theta*) < dpi (the mode always is).  Points
   are listed in lexicographic order of s.
5. With equal cell volumes, w_k is proportional to exp(-(f_k - f*)) and the
   weights sum to one; E[theta | y] and Cov[theta | y] are the weighted sums,
   and log pi(y) = -f* + log sum_k exp(-(f_k - f*)) + d log dz
   + log |det V diag(lambda^{-1/2})| (exp(-f) is the joint density of theta
   and y here: every normalising constant is kept in f).
6. Latent marginals as the mixture of eq. LatParam over the kept points:
   mean_i = sum_k w_k mu_i^k, var_i = sum_k w_k (v_i^k + (mu_i^k - mean_i)^2).
"""
from __future__ import annotations

import itertools
import math

import numpy as np

from . import inla_oracle as O


def fd_hessian(grad, theta, h=1e-3):
    """Central differences of the gradient along the coordinate axes,
    symmetrised: 0.5 (H + H^T)."""
    t = np.asarray(theta, dtype=np.float64)
    d = t.size
    H = np.empty((d, d))
    for k in range(d):
        e = np.zeros(d)
        e[k] = h
        H[k] = (np.asarray(grad(t + e)) - np.asarray(grad(t - e))) / (2.0 * h)
    return 0.5 * (H + H.T)


def standardise(H):
    """Eigenvalues (ascending) and eigenvectors of H with each column's
    largest-magnitude entry positive, and M = V diag(lambda^{-1/2})."""
    lam, V = np.linalg.eigh(np.asarray(H, dtype=np.float64))
    if not np.all(lam > 0.0):
        raise ValueError("Hessian at the mode is not positive definite")
    for j in range(V.shape[1]):
        if V[np.argmax(np.abs(V[:, j])), j] < 0.0:
            V[:, j] = -V[:, j]
    return lam, V, V * lam ** -0.5


def explore(f, theta_mode, M, dz=1.0, dpi=2.5, max_steps=6):
    """Steps 3-4: the axis ranges (lo, hi), and the box candidates as
    (s, theta, f) in lexicographic order of s.  f(theta) returns +inf where
    Q is not positive definite."""
    t0 = np.asarray(theta_mode, dtype=np.float64)
    d = t0.size
    f0 = f(t0)
    lo = np.zeros(d, dtype=np.int64)
    hi = np.zeros(d, dtype=np.int64)
    for j in range(d):
        for sign, rng in ((1, hi), (-1, lo)):
            for s in range(1, max_steps + 1):
                z = np.zeros(d)
                z[j] = sign * s * dz
                if not f(t0 + M @ z) - f0 < dpi:
                    break
                rng[j] = s
    cands = []
    for s in itertools.product(*[range(-int(lo[j]), int(hi[j]) + 1) for j in range(d)]):
        s = np.array(s, dtype=np.int64)
        th = t0 + M @ (dz * s)
        cands.append((s, th, f(th)))
    return f0, lo, hi, cands


def quadrature(f0, kept_f, kept_theta, lam, dz):
    """Step 5: weights, posterior mean and covariance of theta, log evidence."""
    fk = np.asarray(kept_f, dtype=np.float64)
    th = np.asarray(kept_theta, dtype=np.float64)
    u = np.exp(-(fk - f0))
    w = u / u.sum()
    mean = w @ th
    dev = th - mean
    cov = (w[:, None] * dev).T @ dev
    d = th.shape[1]
    log_ev = -f0 + math.log(u.sum()) + d * math.log(dz) - 0.5 * float(np.sum(np.log(lam)))
    return w, mean, cov, log_ev


def latent_mixture(mus, variances, w):
    """Step 6 (eq. LatParam with Gaussian conditionals): mean and variance of
    the mixture sum_k w_k N(mu^k, v^k), componentwise."""
    mus = np.asarray(mus, dtype=np.float64)
    variances = np.asarray(variances, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    mean = w @ mus
    var = w @ (variances + (mus - mean) ** 2)
    return mean, var


def _safe_f(model, theta):
    try:
        return float(O.eval_f_dense(model, theta)["f"])
    except np.linalg.LinAlgError:
        return math.inf


def integrate_model(model, theta_mode, h=1e-3, dz=1.0, dpi=2.5, max_steps=6, latent=True):
    """Steps 1-6 for one model by the dense route (small n)."""
    t0 = np.asarray(theta_mode, dtype=np.float64)
    H = fd_hessian(lambda t: O.dense_gradient(model, t), t0, h)
    lam, V, M = standardise(H)
    f = lambda t: _safe_f(model, t)
    f0, lo, hi, cands = explore(f, t0, M, dz, dpi, max_steps)
    kept = [(s, th, fv) for s, th, fv in cands if fv - f0 < dpi]
    S = np.array([c[0] for c in kept])
    TH = np.array([c[1] for c in kept])
    FK = np.array([c[2] for c in kept])
    w, mean, cov, log_ev = quadrature(f0, FK, TH, lam, dz)
    out = dict(hessian=H, eigval=lam, eigvec=V, f_mode=f0, lo=lo, hi=hi, n_box=len(cands),
               s=S, theta=TH, f=FK, weights=w, theta_mean=mean, theta_cov=cov,
               log_evidence=log_ev, drops=np.array([c[2] - f0 for c in cands]))
    if latent:
        mus, vs = [], []
        for th in TH:
            mus.append(O.eval_f_dense(model, th)["mu"])
            vs.append(O.marginal_variances_dense(model, th))
        out["x_mean"], out["x_var"] = latent_mixture(mus, vs, w)
        out["mu_mode"] = O.eval_f_dense(model, t0)["mu"]
    return out
