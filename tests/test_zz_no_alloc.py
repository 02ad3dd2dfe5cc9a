"""The allocation-free factorization (inla_factor_logdet_noalloc, through the
C ABI) against inla_factor_logdet: the same factor blocks, log-determinant and
pivot status bit for bit, on two calls in a row, the second with a smaller
matrix (so it runs on the fixed workspace the first one left dirty)."""
import math

import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    import paper_2204_04678_amd as P
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    P.lib()
    return P


def rand_spd_bta(b, nt, a, seed):
    """Dense SPD matrix with the BTA pattern (strict diagonal dominance)."""
    rng = np.random.default_rng(seed)
    n = b * nt + a
    Q = np.zeros((n, n))
    for t in range(nt):
        Q[t * b:(t + 1) * b, t * b:(t + 1) * b] = rng.uniform(-1, 1, (b, b))
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


@pytest.mark.parametrize("fused", ["0", "1"], ids=["batched_step", "fused_step"])
def test_noalloc_factor_matches_factor_logdet(P, monkeypatch, fused):
    monkeypatch.setenv("INLA_STEP_FUSED", fused)
    for (b, nt, a), seed in (((300, 3, 3), 1), ((100, 2, 2), 2)):
        print(f"noalloc factor b={b} nt={nt} a={a} fused={fused}", flush=True)
        Q = rand_spd_bta(b, nt, a, seed)
        blocks = O.bta_blocks(Q, b, nt, a)
        Qa = P.BtaTensors.from_blocks(*blocks)
        Qb = P.BtaTensors.from_blocks(*blocks)
        ld_a, info_a = P.factor_logdet(Qa)
        ld_b, info_b = P.factor_logdet_noalloc(Qb)
        torch.cuda.synchronize()
        assert int(info_b.item()) == 0 and int(info_a.item()) == 0
        assert ld_b.item() == ld_a.item()
        for X, Y in ((Qa.D, Qb.D), (Qa.S, Qb.S), (Qa.R, Qb.R), (Qa.T, Qb.T)):
            assert torch.equal(X, Y)
        ld_ref = 2.0 * math.fsum(np.log(np.diag(np.linalg.cholesky(Q))))
        assert abs(ld_b.item() - ld_ref) <= 1e-12 * abs(ld_ref)


def test_noalloc_reports_pivot_and_rejects_oversize(P):
    b, nt, a = 70, 3, 2
    Q = rand_spd_bta(b, nt, a, seed=5)
    bad = b + 66
    Q[bad, bad] = -5.0
    Qt = P.BtaTensors.from_blocks(*O.bta_blocks(Q, b, nt, a))
    ld, info = P.factor_logdet_noalloc(Qt)
    torch.cuda.synchronize()
    assert int(info.item()) == bad + 1
    assert math.isnan(ld.item())
    # a 3000 x 3000 block needs two 72 MB panels: refused before anything runs
    big = P.BtaTensors(3000, 1, 0)
    with pytest.raises(P.InlaError) as err:
        P.factor_logdet_noalloc(big)
    assert err.value.code == -3
