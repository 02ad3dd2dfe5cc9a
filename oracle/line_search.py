"""Oracle of the parallel line search's robust quadratic fit.

TEST INFRASTRUCTURE ONLY (see the package header): only tests/ may use it.

Paper: Sec. "Parallel Line Search" -- a second-order polynomial q is fitted
through the evaluated line-search points by robust regression in which every
point carries a weight, the weights being the bisquare (Tukey biweight)
function of the scaled residuals; its minimiser on the search interval is the
next iterate.  The paper names the weighting but not its constants or the
scale estimate; the reading taken here (listed in the design notes): tuning
constant 4.685, residual scale = median |r| / 0.6745, iteratively reweighted
least squares from the ordinary least-squares fit until the weights change by
less than 1e-12; when the scale is zero (an exact fit through at least half
of the points) the points off the fit get weight zero.
"""
from __future__ import annotations

import numpy as np

BISQUARE_C = 4.685
MAD_TO_SD = 0.6744897501960817   # the 0.75 quantile of the standard normal


def bisquare_weights(r, scale, c=BISQUARE_C, ymax=1.0):
    """w = (1 - (r / (c s))^2)^2 inside |r| < c s, zero outside."""
    r = np.asarray(r, dtype=np.float64)
    if not scale > 1e-15 * max(ymax, 1e-300):
        return (np.abs(r) <= 1e-13 * max(ymax, 1e-300)).astype(np.float64)
    u = r / (c * scale)
    return np.where(np.abs(u) < 1.0, (1.0 - u * u) ** 2, 0.0)


def robust_quadratic_fit(x, y, c=BISQUARE_C, rounds=200, tol=1e-12):
    """Coefficients (c0, c1, c2) of q(x) = c0 + c1 x + c2 x^2 and the final
    weights, by iteratively reweighted least squares with bisquare weights."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    X = np.stack([np.ones_like(x), x, x * x], axis=1)
    ymax = float(np.abs(y).max())
    beta = np.linalg.lstsq(X, y, rcond=None)[0]
    w = np.ones_like(y)
    for _ in range(rounds):
        r = y - X @ beta
        s = float(np.median(np.abs(r))) / MAD_TO_SD
        wn = bisquare_weights(r, s, c, ymax)
        dw = float(np.abs(wn - w).max())
        w = wn
        if np.count_nonzero(w > 0) < 3:
            break
        sw = np.sqrt(w)
        beta = np.linalg.lstsq(X * sw[:, None], y * sw, rcond=None)[0]
        if dw < tol:
            break
    return beta, w


def quadratic_minimiser_on(beta, lo, hi):
    """argmin of q on [lo, hi]: the vertex when q is convex and the vertex lies
    inside, else the lower end point."""
    c0, c1, c2 = beta
    cands = [lo, hi]
    if c2 > 0:
        v = -c1 / (2 * c2)
        if lo < v < hi:
            cands.append(v)
    q = [c0 + c1 * a + c2 * a * a for a in cands]
    return cands[int(np.argmin(q))]
