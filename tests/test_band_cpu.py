"""The band of the coupling blocks (the off-diagonal time blocks c(rho) Q_s):
its half-bandwidth against the oracle's Q_s, the upper-trapezoidal shape of
L_{t+1,t} that the band-aware products rely on, and the band-aware flop
counts the benchmark reports against brute-force counts."""
import numpy as np
import pytest

import bench
from inla_synth import THETA0, make_model
from oracle import inla_oracle as O


@pytest.mark.parametrize("N", [1, 2, 3, 5, 8])
def test_halfbandwidth_is_that_of_the_spatial_precision(N):
    _, kappa = 1.3, 0.7
    Qs = O.spatial_precision(N, 1.0 / max(N - 1, 1), 1.3, kappa).tocoo()
    nz = np.abs(Qs.data) > 0
    w = int(np.abs(Qs.row[nz] - Qs.col[nz]).max()) if nz.any() else 0
    assert bench.coupling_halfbandwidth(N) == w


def test_factor_coupling_is_upper_trapezoidal():
    """L_{t+1,t} = S_t inv(L_tt)^T has exact zeros left of column r - w in
    row r when S_t has half-bandwidth w (the dense factor of the oracle)."""
    md = make_model(6, 3, 2, 4)
    b, w = md.ns, bench.coupling_halfbandwidth(6)
    _, Qc, _ = O.conditional_precision(md, THETA0)
    L = np.linalg.cholesky(Qc.toarray())
    for t in range(md.nt - 1):
        X = L[(t + 1) * b:(t + 2) * b, t * b:(t + 1) * b]
        for r in range(b):
            assert np.all(X[r, :max(0, r - w)] == 0.0)
        assert np.abs(X[w + 1:, 0]).max() == 0.0 and np.abs(X[:, -1]).max() > 0


@pytest.mark.parametrize("b,w", [(7, 0), (9, 2), (16, 5), (16, 15), (12, 20)])
def test_band_macs_match_brute_force(b, w):
    x = syrk = v = arrow = 0
    for r in range(b):
        for c in range(b):
            x += sum(1 for k in range(b) if abs(r - k) <= w and k <= c)
            if r >= c:
                syrk += sum(1 for k in range(b) if k >= r - w and k >= c - w)
            v += sum(1 for k in range(b) if k >= c and k >= r - w)
        arrow += sum(1 for k in range(b) if k >= r - w)
    got = bench.band_macs(b, w)
    assert got == (x, syrk, v, arrow)


def test_dense_counts_are_the_limit():
    b, nt, a = 30, 4, 3
    assert bench.flops_chol(b, nt, a, b - 1) == bench.flops_chol(b, nt, a)
    assert bench.flops_selinv(b, nt, a, b + 5) == bench.flops_selinv(b, nt, a)
    assert bench.flops_chol(b, nt, a, 4) < bench.flops_chol(b, nt, a)
