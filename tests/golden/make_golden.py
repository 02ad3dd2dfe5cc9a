"""Write the stored oracle values the GPU parity tests compare against.

Calls only the CPU oracle (oracle/) and the seeded input generator
(inla_synth/).  Usage (from the repository root):

    python tests/golden/make_golden.py c2 c4 c5 c3

Each workload writes tests/golden/<name>.json with f, both log-determinants,
the posterior mode at sampled indices and the marginal variances at sampled
indices (all of the fixed effects, the first and last time block's first 16
nodes, and seeded random others).

    python tests/golden/make_golden.py --grad c2

adds to an existing file the gradient of f by central differences of the
oracle's f, Richardson-extrapolated from the steps 2h and h:
g_k = (4 D_k(h) - D_k(2h)) / 3, D_k(s) = (f(theta + s e_k) - f(theta - s e_k)) / 2s,
whose truncation error is O(h^4).
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from inla_synth import THETA0, config_model, uneven_batch  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def sample_indices(md, count=96, seed=0):
    ns, nt, nb = md.ns, md.nt, md.nb
    nst = ns * nt
    idx = set(range(nst, nst + nb))
    idx.update(range(min(16, ns)))
    idx.update(range((nt - 1) * ns, (nt - 1) * ns + min(16, ns)))
    rng = np.random.default_rng(seed)
    idx.update(int(i) for i in rng.integers(0, nst, size=count))
    return np.array(sorted(idx), dtype=np.int64)


def golden_for(md, theta, variances=True):
    t0 = time.time()
    out = oracle.eval_f_banded(md, theta, return_factors=True)
    idx = sample_indices(md)
    rec = {
        "N": md.N, "nt": md.nt, "nb": md.nb, "seed": md.seed, "theta": list(map(float, theta)),
        "f": out["f"], "logdet_p": out["logdet_p"], "logdet_c": out["logdet_c"],
        "idx": idx.tolist(), "mu": out["mu"][idx].tolist(),
        "mu_absmax": float(np.abs(out["mu"]).max()),
    }
    if variances:
        rec["var"] = oracle.variance_samples_banded(out["factor_c"], idx).tolist()
    rec["oracle_seconds"] = time.time() - t0
    return rec


def fd_gradient_richardson(md, theta, h=1e-3):
    theta = np.asarray(theta, dtype=float)
    d = {}
    for s in (2 * h, h):
        g = np.zeros(theta.size)
        for k in range(theta.size):
            e = np.zeros(theta.size)
            e[k] = s
            fp = oracle.eval_f_banded(md, theta + e)["f"]
            fm = oracle.eval_f_banded(md, theta - e)["f"]
            g[k] = (fp - fm) / (2 * s)
        d[s] = g
    return (4 * d[h] - d[2 * h]) / 3, d


def add_gradient(name, h=1e-3):
    path = os.path.join(HERE, f"{name}.json")
    with open(path) as fh:
        data = json.load(fh)
    md = config_model(name)
    t0 = time.time()
    g, d = fd_gradient_richardson(md, THETA0, h)
    data["grad_fd"] = g.tolist()
    data["grad_fd_steps"] = [2 * h, h]
    data["grad_fd_central"] = {str(s): v.tolist() for s, v in d.items()}
    data["grad_fd_seconds"] = time.time() - t0
    with open(path, "w") as fh:
        json.dump(data, fh)
    print(name, "grad_fd", g.tolist(), f"{data['grad_fd_seconds']:.1f}s", flush=True)


def main(names):
    for name in names:
        if name == "c3":
            items = uneven_batch(64)
            recs = []
            for j in range(0, 64, 8):   # every eighth model of the batch
                md, th = items[j]
                r = golden_for(md, th, variances=False)
                r["item"] = j
                recs.append(r)
                print(name, j, r["f"], f"{r['oracle_seconds']:.1f}s", flush=True)
            data = {"workload": "64 uneven models (meta-seed 2207), every eighth", "items": recs}
        else:
            md = config_model(name)
            data = golden_for(md, THETA0)
            print(name, data["f"], f"{data['oracle_seconds']:.1f}s", flush=True)
        with open(os.path.join(HERE, f"{name}.json"), "w") as fh:
            json.dump(data, fh)


if __name__ == "__main__":
    if sys.argv[1:2] == ["--grad"]:
        for name in sys.argv[2:] or ["c2"]:
            add_gradient(name)
    else:
        main(sys.argv[1:] or ["c2", "c4", "c5", "c3"])
