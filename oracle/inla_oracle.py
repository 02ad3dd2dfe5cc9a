"""Plain, slow, obviously-correct FP64 CPU oracle for the INLA objective.

TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the benchmark's
CPU-baseline leg may import this module.  It shares no code with the GPU
library: it consumes only the seeded inputs of ``inla_synth``.

What it computes (paper: "Parallelized integrated nested Laplace
approximations for fast Bayesian inference"):

* the latent Gaussian model of Sec. "Latent Gaussian Models", with the latent
  vector written without the linear predictor, x = (u, beta), Gaussian
  likelihood; the GMRF x has *precision* Q(theta);
* the objective f(theta) = -log pi~(theta | y) of Sec. "Parallel Optimization"
  built from eq. (post_theta_approx): prior of theta, prior of x, likelihood,
  and the Gaussian approximation pi_G, all at the mode x* = mu;
* log-determinants from a Cholesky factor Q = L L^T as 2 sum log L_ii, and the
  mode by forward then backward substitution (Sec. "Sparse Linear Algebra");
* marginal variances (Q_c^{-1})_ii (Sec. "Approximating pi(x_i | y)",
  Sec. "Partial Inversion"), both as the plain diagonal of the inverse and via
  the two selected-inversion recursions the paper states (eq. sel_inv_cov and
  eq. takahashi_recursion);
* the exact gradient of f (derived by differentiating the same objective; the
  paper computes it by central differences, eq. central_diff, which the tests
  use to pin it).

Readings of points the paper leaves open are listed in the design notes:
Gaussian hyperprior N(m_k, 1/p_k) with normalising constants; Neumann grid
Laplacian; stationary unit-variance AR1 in time with rho = tanh(theta_3);
fixed effects last (the arrowhead order of Sec. "Matrix Reordering").

Two evaluation routes:
* dense (numpy.linalg) for small n -- the brute force;
* bordered-banded (LAPACK dpbtrf via scipy) for the large workloads: the
  space-time part is banded with half-bandwidth ns + 2N, the fixed effects form
  a dense border handled by a Schur complement.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla
import scipy.linalg.lapack as lapack
import scipy.sparse as sp

LOG2PI = math.log(2.0 * math.pi)

__all__ = [
    "theta_params", "grid_laplacian", "spatial_precision", "ar1_precision",
    "obs_matrix", "prior_precision", "conditional_precision", "log_hyperprior",
    "dprecision", "eval_f", "eval_f_banded", "eval_f_dense", "dense_gradient",
    "fd_gradient", "marginal_variances_dense", "variance_samples_banded",
    "selinv_rue_martino", "selinv_takahashi", "bta_blocks", "bta_factor_blocks",
    "BandedFactor", "banded_factor", "LOG2PI",
]


# ---------------------------------------------------------------------------
# model: precision matrices (Sec. "Latent Gaussian Models")
# ---------------------------------------------------------------------------

def theta_params(theta):
    """theta = (log tau, log kappa, atanh rho, log tau_y) -> (tau, kappa, rho, tau_y)."""
    t = np.asarray(theta, dtype=np.float64)
    return math.exp(t[0]), math.exp(t[1]), math.tanh(t[2]), math.exp(t[3])


def grid_laplacian(N: int) -> sp.csr_matrix:
    """Graph Laplacian of the 4-neighbour N x N grid (Neumann: rows sum to 0).

    G[s,s] = number of neighbours of s, G[s,s'] = -1 for neighbours.
    Node (ix, iy) has index s = iy*N + ix.
    """
    ns = N * N
    rows, cols, vals = [], [], []
    for iy in range(N):
        for ix in range(N):
            s = iy * N + ix
            deg = 0
            for dx, dy in ((-1, 0), (1, 0), (0, -1), (0, 1)):
                jx, jy = ix + dx, iy + dy
                if 0 <= jx < N and 0 <= jy < N:
                    rows.append(s)
                    cols.append(jy * N + jx)
                    vals.append(-1.0)
                    deg += 1
            rows.append(s)
            cols.append(s)
            vals.append(float(deg))
    return sp.csr_matrix((vals, (rows, cols)), shape=(ns, ns))


def spatial_precision(N: int, h: float, tau: float, kappa: float) -> sp.csr_matrix:
    """Q_s = tau^2 (kappa^2 C + G) C^{-1} (kappa^2 C + G) with C = h^2 I."""
    ns = N * N
    G = grid_laplacian(N)
    C = (h * h) * sp.identity(ns, format="csr")
    K = kappa * kappa * C + G
    Cinv = (1.0 / (h * h)) * sp.identity(ns, format="csr")
    return (tau * tau) * (K @ Cinv @ K).tocsr()


def ar1_precision(nt: int, rho: float) -> sp.csr_matrix:
    """Stationary AR1 with unit marginal variance: precision T(rho)/(1-rho^2).

    T(rho) is tridiagonal, diagonal (1, 1+rho^2, ..., 1+rho^2, 1) and
    off-diagonal -rho.  For nt = 1 the precision is [1].
    """
    if nt == 1:
        return sp.csr_matrix(np.ones((1, 1)))
    d = np.full(nt, 1.0 + rho * rho)
    d[0] = d[-1] = 1.0
    o = np.full(nt - 1, -rho)
    T = sp.diags([o, d, o], [-1, 0, 1], format="csr")
    return T / (1.0 - rho * rho)


def obs_matrix(model) -> sp.csr_matrix:
    return sp.csr_matrix((model.A_val, model.A_col.astype(np.int64), model.A_rowptr),
                         shape=(model.m, model.n))


def _assemble_prior(model, tau, kappa, rho, Qar=None, Qsp=None):
    Qs = spatial_precision(model.N, model.h, tau, kappa) if Qsp is None else Qsp
    Qa = ar1_precision(model.nt, rho) if Qar is None else Qar
    Qst = sp.kron(Qa, Qs, format="csr")
    if model.nb == 0:
        return Qst
    return sp.block_diag([Qst, model.beta_prior_prec * sp.identity(model.nb)], format="csr")


def prior_precision(model, theta) -> sp.csr_matrix:
    """Q_p(theta) = blockdiag(Q_AR1(rho) kron Q_s(tau, kappa), beta_prec * I_nb)."""
    tau, kappa, rho, _ = theta_params(theta)
    return _assemble_prior(model, tau, kappa, rho)


def conditional_precision(model, theta):
    """Q_c = Q_p + tau_y A^T A and the right-hand side b = tau_y A^T y."""
    tau_y = theta_params(theta)[3]
    A = obs_matrix(model)
    Qp = prior_precision(model, theta)
    Qc = (Qp + tau_y * (A.T @ A)).tocsr()
    b = tau_y * (A.T @ model.y)
    return Qp, Qc, b


def log_hyperprior(model, theta) -> float:
    """log pi(theta) for independent N(m_k, 1/p_k) priors, constants included."""
    t = np.asarray(theta, dtype=np.float64)
    m = np.asarray(model.theta_prior_mean, dtype=np.float64)
    p = np.asarray(model.theta_prior_prec, dtype=np.float64)
    return float(np.sum(0.5 * np.log(p / (2.0 * math.pi)) - 0.5 * p * (t - m) ** 2))


def dprecision(model, theta):
    """Exact derivatives of (Q_p, Q_c) with respect to theta_1..theta_4.

    Returns two lists of four sparse matrices.  Derived by differentiating the
    definitions above:
      d/dtheta1: tau^2 scales the whole space-time part -> 2 Q_st;
      d/dtheta2: Q_s -> 4 tau^2 kappa^2 (kappa^2 h^2 I + G);
      d/dtheta3: Q_AR1 -> d Q_AR1 / d rho * (1 - rho^2);
      d/dtheta4: Q_p does not depend on tau_y; Q_c gains tau_y A^T A.
    """
    tau, kappa, rho, tau_y = theta_params(theta)
    N, h, nt = model.N, model.h, model.nt
    ns = N * N
    Qs = spatial_precision(N, h, tau, kappa)
    Qa = ar1_precision(nt, rho)
    G = grid_laplacian(N)
    K = kappa * kappa * h * h * sp.identity(ns, format="csr") + G
    dQs2 = (4.0 * tau * tau * kappa * kappa) * K
    if nt == 1:
        dQa3 = sp.csr_matrix((1, 1))
    else:
        r2 = 1.0 - rho * rho
        d = np.full(nt, 4.0 * rho / r2)
        d[0] = d[-1] = 2.0 * rho / r2
        o = np.full(nt - 1, -(1.0 + rho * rho) / r2)
        dQa3 = sp.diags([o, d, o], [-1, 0, 1], format="csr")

    def pad(Mst):
        if model.nb == 0:
            return Mst.tocsr()
        return sp.block_diag([Mst, sp.csr_matrix((model.nb, model.nb))], format="csr")

    dQp = [pad(2.0 * sp.kron(Qa, Qs)), pad(sp.kron(Qa, dQs2)), pad(sp.kron(dQa3, Qs)),
           sp.csr_matrix((model.n, model.n))]
    A = obs_matrix(model)
    dQc = dQp[:3] + [(tau_y * (A.T @ A)).tocsr()]
    return dQp, dQc


# ---------------------------------------------------------------------------
# dense route (brute force, small n)
# ---------------------------------------------------------------------------

def _chol_dense(Q):
    Qd = Q.toarray() if sp.issparse(Q) else np.asarray(Q)
    return np.linalg.cholesky(Qd)


def _logdet_from_chol(L) -> float:
    """log|Q| = sum_i 2 log L_ii (Sec. "Sparse Linear Algebra")."""
    return 2.0 * math.fsum(np.log(np.diag(L)))


def _solve_chol(L, b):
    """Q x = b by forward substitution L z = b then backward L^T x = z."""
    z = sla.solve_triangular(L, b, lower=True)
    return sla.solve_triangular(L.T, z, lower=False)


def eval_f_dense(model, theta) -> dict:
    """f(theta) and its parts by the dense route."""
    _, _, _, tau_y = theta_params(theta)
    Qp, Qc, b = conditional_precision(model, theta)
    Lp = _chol_dense(Qp)
    Lc = _chol_dense(Qc)
    mu = _solve_chol(Lc, b)
    return _combine(model, theta, _logdet_from_chol(Lp), _logdet_from_chol(Lc), mu, Qp, tau_y)


def _combine(model, theta, ldp, ldc, mu, Qp, tau_y) -> dict:
    """Assemble f from its parts, eq. (post_theta_approx) at x = mu, sign flipped.

    log pi(x|theta)    = -n/2 log 2pi + 1/2 log|Q_p| - 1/2 x^T Q_p x
    log pi(y|x,theta)  = -m/2 log 2pi + m/2 log tau_y - tau_y/2 |y - A x|^2
    log pi_G(x|theta,y) at its mode = -n/2 log 2pi + 1/2 log|Q_c|
    """
    A = obs_matrix(model)
    r = model.y - A @ mu
    rss = float(r @ r)
    quad = float(mu @ (Qp @ mu))
    m = model.m
    t4 = float(np.asarray(theta)[3])
    lp = log_hyperprior(model, theta)
    f = (-lp - 0.5 * ldp + 0.5 * quad - 0.5 * m * t4 + 0.5 * tau_y * rss + 0.5 * ldc
         + 0.5 * m * LOG2PI)
    return dict(f=f, logdet_p=ldp, logdet_c=ldc, mu=mu, quad=quad, rss=rss,
                log_prior=lp)


def marginal_variances_dense(model, theta) -> np.ndarray:
    """v_i = (Q_c^{-1})_ii, the plain definition."""
    _, Qc, _ = conditional_precision(model, theta)
    return np.diag(np.linalg.inv(Qc.toarray())).copy()


def dense_gradient(model, theta) -> np.ndarray:
    """Exact grad f with dense inverses (small n only).

    d f / d theta_k = p_k (theta_k - m_k) - 1/2 tr(Q_p^{-1} dQ_p_k)
                      + 1/2 tr(Q_c^{-1} dQ_c_k) + 1/2 mu^T dQ_p_k mu
                      + [k = 4] (tau_y/2 |y - A mu|^2 - m/2)
    (mu minimises the quadratic part of f, so its own theta-dependence drops
    out of the derivative.)
    """
    t = np.asarray(theta, dtype=np.float64)
    _, _, _, tau_y = theta_params(t)
    Qp, Qc, b = conditional_precision(model, t)
    Sp = np.linalg.inv(Qp.toarray())
    Sc = np.linalg.inv(Qc.toarray())
    mu = np.linalg.solve(Qc.toarray(), b)
    dQp, dQc = dprecision(model, t)
    A = obs_matrix(model)
    r = model.y - A @ mu
    g = np.empty(4)
    pm = np.asarray(model.theta_prior_mean)
    pp = np.asarray(model.theta_prior_prec)
    for k in range(4):
        trp = float(np.sum(Sp * dQp[k].toarray()))
        trc = float(np.sum(Sc * dQc[k].toarray()))
        g[k] = pp[k] * (t[k] - pm[k]) - 0.5 * trp + 0.5 * trc + 0.5 * float(mu @ (dQp[k] @ mu))
    g[3] += 0.5 * tau_y * float(r @ r) - 0.5 * model.m
    return g


def fd_gradient(model, theta, h: float = 1e-5, f=None) -> np.ndarray:
    """Central differences along the coordinate axes, eq. (central_diff)."""
    f = f or (lambda th: eval_f(model, th)["f"])
    t = np.asarray(theta, dtype=np.float64)
    g = np.empty(t.size)
    for k in range(t.size):
        e = np.zeros(t.size)
        e[k] = h
        g[k] = (f(t + e) - f(t - e)) / (2.0 * h)
    return g


# ---------------------------------------------------------------------------
# selected inversion recursions (Sec. "Partial Inversion")
# ---------------------------------------------------------------------------

def selinv_rue_martino(L):
    """Sigma on the pattern of L (plus the diagonal) by eq. (sel_inv_cov).

    Sigma_ij = delta_ij / L_ii^2 - 1/L_ii sum_{k>i, L_ki != 0} L_ki Sigma_kj,
    for i <= j, traversed from the bottom-right corner.  Entries with
    L_ji == 0 (j > i) are not needed by the recursion over the pattern of L
    because the pattern of a Cholesky factor is closed under this recursion;
    for clarity this small-n version fills the whole upper triangle.
    Returns the full symmetric matrix.
    """
    L = np.asarray(L)
    n = L.shape[0]
    S = np.zeros((n, n))
    for i in range(n - 1, -1, -1):
        nz = [k for k in range(i + 1, n) if L[k, i] != 0.0]
        for j in range(n - 1, i - 1, -1):
            acc = 0.0
            for k in nz:
                acc += L[k, i] * S[k, j]
            S[i, j] = (1.0 if i == j else 0.0) / (L[i, i] ** 2) - acc / L[i, i]
            S[j, i] = S[i, j]
    return S


def selinv_takahashi(L):
    """Sigma by eq. (takahashi_recursion) with Q = V D V^T, L = V D^{1/2}.

    Sigma_ij = delta_ij / D_ii - sum_{k>i, V_ki != 0} V_ki Sigma_kj, i <= j.
    """
    L = np.asarray(L)
    n = L.shape[0]
    dl = np.diag(L)
    V = L / dl[None, :]
    Dd = dl * dl
    S = np.zeros((n, n))
    for i in range(n - 1, -1, -1):
        nz = np.nonzero(V[i + 1:, i])[0] + i + 1
        for j in range(n - 1, i - 1, -1):
            S[i, j] = (1.0 if i == j else 0.0) / Dd[i] - float(V[nz, i] @ S[nz, j])
            S[j, i] = S[i, j]
    return S


# ---------------------------------------------------------------------------
# block views (block-tridiagonal-with-arrowhead, time-major, arrow last)
# ---------------------------------------------------------------------------

def bta_blocks(Q, b: int, nt: int, a: int):
    """Split a (dense or sparse) matrix into D[t]=(t,t), S[t]=(t+1,t), R[t]=(A,t), T=(A,A)."""
    Qd = Q.toarray() if sp.issparse(Q) else np.asarray(Q)
    nst = b * nt
    D = np.stack([Qd[t * b:(t + 1) * b, t * b:(t + 1) * b] for t in range(nt)])
    S = (np.stack([Qd[(t + 1) * b:(t + 2) * b, t * b:(t + 1) * b] for t in range(nt - 1)])
         if nt > 1 else np.zeros((0, b, b)))
    R = np.stack([Qd[nst:nst + a, t * b:(t + 1) * b] for t in range(nt)])
    T = Qd[nst:nst + a, nst:nst + a].copy()
    return D, S, R, T


def bta_factor_blocks(Q, b: int, nt: int, a: int):
    """Blocks of the dense Cholesky factor L of Q (same layout as bta_blocks)."""
    return bta_blocks(_chol_dense(Q), b, nt, a)


# ---------------------------------------------------------------------------
# bordered-banded route (large n)
# ---------------------------------------------------------------------------

class BandedFactor:
    """Cholesky of [[B, C^T], [C, T]] with B banded (lower band LB, half-bandwidth kd).

    LB: lower band of chol(B) in LAPACK format, LB[i-j, j] = L[i, j];
    W = B^{-1} C^T (nst x a);  LS = chol(T - C W).
    """

    def __init__(self, LB, W, LS, nst, a):
        self.LB, self.W, self.LS, self.nst, self.a = LB, W, LS, nst, a

    def logdet(self) -> float:
        v = 2.0 * math.fsum(np.log(self.LB[0]))
        if self.a:
            v += 2.0 * math.fsum(np.log(np.diag(self.LS)))
        return v

    def solve(self, r):
        r = np.asarray(r, dtype=np.float64)
        yB = sla.cho_solve_banded((self.LB, True), r[:self.nst])
        if not self.a:
            return yB
        xA = sla.cho_solve((self.LS, True), r[self.nst:] - self.W.T @ r[:self.nst])
        xB = yB - self.W @ xA
        return np.concatenate([xB, xA])


def _lower_band(Bsp, kd: int) -> np.ndarray:
    coo = Bsp.tocoo()
    keep = coo.row >= coo.col
    d = coo.row[keep] - coo.col[keep]
    if d.size and d.max() > kd:
        raise ValueError("matrix is wider than the requested band")
    ab = np.zeros((kd + 1, Bsp.shape[0]))
    np.add.at(ab, (d, coo.col[keep]), coo.data[keep])
    return ab


def banded_factor(Q, nst: int, kd: int) -> BandedFactor:
    Q = Q.tocsr()
    a = Q.shape[0] - nst
    B = Q[:nst, :nst]
    LB = sla.cholesky_banded(_lower_band(B, kd), lower=True, overwrite_ab=True,
                             check_finite=False)
    if a == 0:
        return BandedFactor(LB, np.zeros((nst, 0)), np.zeros((0, 0)), nst, 0)
    C = Q[nst:, :nst].toarray()
    T = Q[nst:, nst:].toarray()
    W = sla.cho_solve_banded((LB, True), C.T.copy(), check_finite=False)
    LS = np.linalg.cholesky(T - C @ W)
    return BandedFactor(LB, W, LS, nst, a)


def _bandwidth(model) -> int:
    # time-block coupling reaches one block back; Q_s has half-bandwidth 2N
    ns = model.ns
    within = min(ns - 1, 2 * model.N)
    return within if model.nt == 1 else ns + within


def eval_f_banded(model, theta, return_factors: bool = False) -> dict:
    """f(theta) by the bordered-banded route (same formula as eval_f_dense)."""
    _, _, _, tau_y = theta_params(theta)
    Qp, Qc, b = conditional_precision(model, theta)
    nst = model.ns * model.nt
    kd = _bandwidth(model)
    Fp = banded_factor(Qp, nst, kd)
    ldp = Fp.logdet()
    del Fp
    Fc = banded_factor(Qc, nst, kd)
    mu = Fc.solve(b)
    out = _combine(model, theta, ldp, Fc.logdet(), mu, Qp, tau_y)
    if return_factors:
        out["factor_c"] = Fc
    return out


def eval_f(model, theta, dense_limit: int = 3000) -> dict:
    if model.n <= dense_limit:
        return eval_f_dense(model, theta)
    return eval_f_banded(model, theta)


def variance_samples_banded(F: BandedFactor, idx) -> np.ndarray:
    """(Q^{-1})_ii for the requested indices, one unit-vector solve each.

    For i in the banded part: (Q^{-1})_ii = |L_B^{-1} e_i|^2 + (W S^{-1} W^T)_ii,
    where L_B^{-1} e_i vanishes above row i, so the triangular solve starts at i.
    For i in the border: (S^{-1})_jj.
    """
    idx = np.asarray(idx, dtype=np.int64)
    out = np.empty(idx.size)
    nst = F.nst
    Sinv = np.linalg.inv(F.LS @ F.LS.T) if F.a else np.zeros((0, 0))
    for q, i in enumerate(idx):
        if i >= nst:
            out[q] = Sinv[i - nst, i - nst]
            continue
        sub = F.LB[:, i:]
        e = np.zeros((nst - i, 1))
        e[0, 0] = 1.0
        x, info = lapack.dtbtrs(sub, e, uplo="L", trans="N", diag="N")
        if info != 0:
            raise RuntimeError("dtbtrs failed")
        v = float(x[:, 0] @ x[:, 0])
        if F.a:
            w = F.W[i]
            v += float(w @ (Sinv @ w))
        out[q] = v
    return out
