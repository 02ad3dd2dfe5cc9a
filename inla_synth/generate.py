"""Seeded synthetic workloads.

Model family (one spatio-temporal field on an N x N grid over the unit square,
nt time steps, nb fixed effects, Gaussian observations):

* grid nodes (ix, iy), ix, iy = 0..N-1, spacing h = 1/(N-1) (h = 1 when N = 1),
  node index s = iy*N + ix, latent index t*ns + s for the field at time t and
  ns*nt + c for fixed effect c (fixed effects last, the "arrow");
* m = 2*ns*nt observations, exactly 2*ns of them at each time step, in order;
  observation j sits at time t_j = j // (2*ns), at a uniform random location in
  [0,1)^2, and loads on the 4 corners of its grid cell with bilinear weights
  plus nb i.i.d. N(0,1) covariates;
* y = A x_true + 0.1 * eps with x_true, eps i.i.d. N(0,1).

Random draws, in this order, from numpy.random.default_rng(seed):
locations (m,2), covariates (m,nb), x_true (n), eps (m).

Nothing here evaluates the inference method; see the oracle and the GPU
library for that.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace

import numpy as np

# Hyperparameter point (log tau, log kappa, atanh rho, log noise precision).
THETA0 = np.array([0.0, 1.0, 1.5, 4.6])

# Seeds of the named workloads: 2204 + k for workload k.
_CONFIGS = {
    "c1": dict(N=10, nt=10, nb=2, seed=2205),
    "c2": dict(N=32, nt=50, nb=4, seed=2206),
    "c4": dict(N=40, nt=100, nb=6, seed=2208),
    "c4small": dict(N=6, nt=4, nb=6, seed=2208),
    "c5": dict(N=45, nt=200, nb=10, seed=2209),
    # the line-search workload over 6 time steps: every launch does the same
    # work as one of the 200-step run's (per-launch profiles)
    "c5short": dict(N=45, nt=6, nb=10, seed=2209),
}


@dataclass
class ModelData:
    """Host description of one model: grid, observation matrix, responses, priors."""

    N: int
    nt: int
    nb: int
    h: float
    m: int
    A_rowptr: np.ndarray  # int64, m+1
    A_col: np.ndarray  # int32, nnz
    A_val: np.ndarray  # float64, nnz
    y: np.ndarray  # float64, m
    theta_prior_mean: np.ndarray = field(default_factory=lambda: np.zeros(4))
    theta_prior_prec: np.ndarray = field(default_factory=lambda: np.full(4, 0.01))
    beta_prior_prec: float = 1e-3
    seed: int = 0

    @property
    def ns(self) -> int:
        return self.N * self.N

    @property
    def n(self) -> int:
        return self.ns * self.nt + self.nb


def make_model(N: int, nt: int, nb: int, seed: int, obs_per_node: int = 2,
               noise_sd: float = 0.1) -> ModelData:
    if N < 1 or nt < 1 or nb < 0:
        raise ValueError("need N >= 1, nt >= 1, nb >= 0")
    rng = np.random.default_rng(seed)
    ns = N * N
    nst = ns * nt
    n = nst + nb
    m = obs_per_node * ns * nt
    loc = rng.random((m, 2))
    Z = rng.standard_normal((m, nb))
    x_true = rng.standard_normal(n)
    eps = rng.standard_normal(m)

    t_of_row = np.arange(m, dtype=np.int64) // (obs_per_node * ns)
    if N == 1:
        h = 1.0
        st_cols = (t_of_row * ns)[:, None]
        st_vals = np.ones((m, 1))
    else:
        h = 1.0 / (N - 1)
        gx = loc[:, 0] / h
        gy = loc[:, 1] / h
        ix = np.minimum(np.floor(gx).astype(np.int64), N - 2)
        iy = np.minimum(np.floor(gy).astype(np.int64), N - 2)
        fx = gx - ix
        fy = gy - iy
        s00 = iy * N + ix
        base = t_of_row * ns
        # ascending column order within a row: (ix,iy), (ix+1,iy), (ix,iy+1), (ix+1,iy+1)
        st_cols = np.stack([base + s00, base + s00 + 1, base + s00 + N, base + s00 + N + 1], axis=1)
        st_vals = np.stack([(1 - fx) * (1 - fy), fx * (1 - fy), (1 - fx) * fy, fx * fy], axis=1)
    k_st = st_cols.shape[1]
    cols = np.empty((m, k_st + nb), dtype=np.int64)
    vals = np.empty((m, k_st + nb))
    cols[:, :k_st] = st_cols
    vals[:, :k_st] = st_vals
    cols[:, k_st:] = nst + np.arange(nb)[None, :]
    vals[:, k_st:] = Z
    nnz_row = k_st + nb
    rowptr = np.arange(m + 1, dtype=np.int64) * nnz_row
    col = cols.reshape(-1).astype(np.int32)
    val = vals.reshape(-1).copy()

    # y = A x_true + noise (row-wise dot products of the CSR rows)
    Ax = np.einsum("ij,ij->i", vals, x_true[cols])
    y = Ax + noise_sd * eps
    return ModelData(N=N, nt=nt, nb=nb, h=h, m=m, A_rowptr=rowptr, A_col=col, A_val=val,
                     y=y, seed=seed)


def poisson_counts(md: ModelData, seed: int = 0, level: float = 0.5, spread: float = 0.3) -> ModelData:
    """The same design with count responses for a Poisson likelihood: the log
    rate of observation i is level + spread * (standardised y_i), clipped to
    [-2, 2.5] (rates between 0.14 and 12), and the count is a seeded Poisson
    draw with that rate.  Returns a copy of md with y replaced by the counts
    (as float64)."""
    rng = np.random.default_rng(10_000 + seed)
    z = (md.y - md.y.mean()) / max(md.y.std(), 1e-300)
    log_rate = np.clip(level + spread * z, -2.0, 2.5)
    counts = rng.poisson(np.exp(log_rate)).astype(np.float64)
    return replace(md, y=counts)


def config_model(name: str) -> ModelData:
    c = _CONFIGS[name]
    return make_model(c["N"], c["nt"], c["nb"], c["seed"])


def fd_stencil(theta: np.ndarray, h: float) -> np.ndarray:
    """The 2*d+1 central-difference points: theta, then theta +/- h e_k for k = 1..d."""
    theta = np.asarray(theta, dtype=np.float64)
    d = theta.size
    pts = [theta.copy()]
    for k in range(d):
        e = np.zeros(d)
        e[k] = h
        pts.append(theta + e)
        pts.append(theta - e)
    return np.stack(pts)


def line_search_points(theta0: np.ndarray, seed: int, gamma: float = 0.5) -> np.ndarray:
    """8 points theta0 - alpha*p along a seeded unit direction p.

    Two points lie on the +p side close to theta0 and six inside the search
    interval (theta0, theta0 - gamma*p).
    """
    rng = np.random.default_rng([seed, 1])
    p = rng.standard_normal(theta0.size)
    p /= np.linalg.norm(p)
    alphas = gamma * np.array([-1 / 4, -1 / 8, 1 / 6, 2 / 6, 3 / 6, 4 / 6, 5 / 6, 1.0])
    return np.stack([theta0 - a * p for a in alphas])


def uneven_batch(count: int = 64, meta_seed: int = 2207, sides=(16, 24, 32),
                 nt_range=(20, 100), nb_range=(2, 6), theta_spread: float = 0.5,
                 build: bool = True):
    """Models of uneven (N, nt, nb), each with its own random theta.

    Returns a list of (ModelData or shape tuple, theta).  With build=False only
    the shapes (N, nt, nb, seed) are returned, which is cheap.
    """
    rng = np.random.default_rng(meta_seed)
    out = []
    for j in range(count):
        N = int(rng.choice(sides))
        nt = int(rng.integers(nt_range[0], nt_range[1] + 1))
        nb = int(rng.integers(nb_range[0], nb_range[1] + 1))
        theta = THETA0 + rng.uniform(-theta_spread, theta_spread, size=4)
        seed = meta_seed * 1000 + j
        out.append(((make_model(N, nt, nb, seed) if build else (N, nt, nb, seed)), theta))
    return out


def config_theta_batch(name: str) -> np.ndarray:
    """The theta points a named workload evaluates."""
    if name in ("c1", "c4", "c4small"):
        return THETA0[None, :].copy()
    if name == "c2":
        return fd_stencil(THETA0, 1e-3)
    if name in ("c5", "c5short"):
        return line_search_points(THETA0, _CONFIGS["c5"]["seed"])
    raise KeyError(name)
