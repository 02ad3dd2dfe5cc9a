"""Host-only unit test of the integration step's host arithmetic
(csrc/integrate_host.h, compiled here with g++; no GPU): the Jacobi
eigen-decomposition with its sign and order convention, the box enumeration
and the quadrature, each against the oracle's (numpy) counterpart."""
import itertools
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import integrate as I

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2204_04678_amd", "csrc")


@pytest.fixture(scope="module")
def exe(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("needs g++")
    out = tmp_path_factory.mktemp("native") / "integrate_check"
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Werror", "-I" + CSRC,
                    os.path.join(HERE, "native", "integrate_check.cpp"), "-o", str(out)],
                   check=True)
    return str(out)


def run(exe, text):
    r = subprocess.run([exe], input=text, capture_output=True, text=True, check=True)
    return r.stdout.splitlines()


def _spd(seed):
    rng = np.random.default_rng(seed)
    B = rng.standard_normal((4, 4))
    return B @ B.T + np.diag(rng.uniform(0.1, 3.0, 4)) * 10 ** rng.uniform(-2, 3)


@pytest.mark.parametrize("seed", range(6))
def test_eigen_matches_the_oracle_convention(exe, seed):
    H = _spd(seed)
    if seed == 5:   # widely spread eigenvalues, as Hessians of f are
        H = np.diag([1e-2, 3.0, 5e2, 4e5]) + 1e-3 * (H + H.T)
    out = run(exe, "eig " + " ".join(repr(float(x)) for x in H.ravel()) + "\n")
    lam = np.array(out[0].split()[1:], dtype=float)
    V = np.array(out[1].split()[1:], dtype=float).reshape(4, 4)
    lam_o, V_o, _ = I.standardise(H)
    np.testing.assert_allclose(lam, lam_o, rtol=1e-12, atol=1e-12 * np.abs(lam_o).max())
    np.testing.assert_allclose(V, V_o, atol=1e-9)
    np.testing.assert_allclose(V @ np.diag(lam) @ V.T, H, rtol=0, atol=1e-12 * np.abs(H).max())


def test_box_enumeration_is_lexicographic(exe):
    lo, hi = [1, 0, 2, 1], [2, 1, 0, 3]
    out = run(exe, "box " + " ".join(map(str, lo + hi)) + "\n")
    head = out[0].split()
    expect = list(itertools.product(*[range(-l, h + 1) for l, h in zip(lo, hi)]))
    assert int(head[1]) == int(head[2]) == len(expect)
    got = [tuple(int(x) for x in line.split()) for line in out[1:]]
    assert got == expect


def test_quadrature_matches_the_oracle(exe):
    rng = np.random.default_rng(2)
    K = 17
    f0 = 1234.5
    f = f0 + rng.uniform(0.0, 2.4, K)
    th = rng.standard_normal((K, 4))
    lam = np.array([0.3, 2.0, 7.5, 40.0])
    text = f"quad 0.75 {float(f0)!r} {K} " + " ".join(repr(float(x)) for x in lam) + " "
    text += " ".join(f"{float(f[k])!r} " + " ".join(repr(float(x)) for x in th[k]) for k in range(K)) + "\n"
    vals = np.array(run(exe, text)[0].split()[1:], dtype=float)
    w, mean, cov, ev = I.quadrature(f0, f, th, lam, 0.75)
    np.testing.assert_allclose(vals[:K], w, rtol=1e-13)
    np.testing.assert_allclose(vals[K:K + 4], mean, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(vals[K + 4:K + 20].reshape(4, 4), cov, rtol=1e-11, atol=1e-14)
    assert abs(vals[-1] - ev) < 1e-12 * abs(ev)
