"""Run a named synthetic workload through the library, for profilers.

    python3 -m paper_2204_04678_amd.workload c2 [steps] [--graph]
    python3 -m paper_2204_04678_amd.workload mode-integrate c2
    python3 -m paper_2204_04678_amd.workload poisson c2 [steps]

Builds the seeded model of the workload (as bench.py does), then runs `steps`
evaluations of f and its gradient (the workload's theta points, one batched
call per step) with eager kernel launches unless --graph is given, and prints
one line per step.  Nothing is timed here; the profiler does that.

mode-integrate: the steps around the hot path on one model -- the mode search
(BFGS with the parallel line search from the default theta), then the
integration step at the mode with the latent mixture marginals -- printing
the wall time of each (graph replay on) and what they did.
poisson: `steps` f + gradient evaluations with the Poisson likelihood on the
workload's design with seeded counts, the first from x = 0 and the others
warm-started at the previous mode, with their wall times.
"""
import os
import sys
import time


def mode_integrate(name):
    import numpy as np
    import torch

    import paper_2204_04678_amd as P
    from inla_synth import THETA0, config_model

    md = config_model(name)
    M = P.Model.from_data(md)
    P.eval_f_grad(M, THETA0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = P.minimize(M, THETA0)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    print(f"{name} mode: {t1 - t0:.3f} s, {res['iterations']} iterations, {res['f_evals']} f and "
          f"{res['grad_evals']} f+grad evaluations, reason {res['reason']}, f = {res['f']:.10g}, "
          f"max |grad| = {np.abs(res['grad']).max():.3g}, theta = {np.round(res['theta'], 6).tolist()}",
          flush=True)
    for latent in (False, True):
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        r = P.integrate(M, res["theta"], latent=latent)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        print(f"{name} integrate (latent marginals: {latent}): {t3 - t2:.3f} s, box {r['n_box']} "
              f"points, {r['n_points']} kept, {r['f_evals']} f and {r['grad_evals']} f+grad "
              f"evaluations, log evidence {r['log_evidence']:.10g}, "
              f"theta sd {np.round(np.sqrt(np.diag(r['theta_cov'])), 5).tolist()}", flush=True)


def poisson(name, steps):
    import numpy as np
    import torch

    import paper_2204_04678_amd as P
    from inla_synth import config_model, poisson_counts

    md = poisson_counts(config_model(name), seed=2)
    M = P.Model.from_data(md)
    theta = np.array([0.1, 0.9, 0.6, 1.5])
    x = None
    for s in range(steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = P.eval_f_grad_poisson(M, theta + 0.01 * s, x0=x)
        torch.cuda.synchronize()
        print(f"{name} poisson step {s}: {time.perf_counter() - t0:.4f} s, {r['iterations']} Newton "
              f"iterations, {r['halvings']} halvings, f = {r['f']:.12g}", flush=True)
        x = r["x"]


def main(argv):
    if argv and argv[0] == "mode-integrate":
        return mode_integrate(argv[1] if len(argv) > 1 else "c2")
    if argv and argv[0] == "poisson":
        return poisson(argv[1] if len(argv) > 1 else "c2", int(argv[2]) if len(argv) > 2 else 3)
    args = [a for a in argv if not a.startswith("--")]
    name = args[0] if args else "c2"
    steps = int(args[1]) if len(args) > 1 else 2
    if "--graph" not in argv:
        os.environ["INLA_GRAPH"] = "0"
    import numpy as np
    import torch

    import paper_2204_04678_amd as P
    from inla_synth import THETA0, config_model, config_theta_batch, uneven_batch

    if name == "c3":
        items = uneven_batch(64)
        models = [P.Model.from_data(m) for m, _ in items]
        th = np.stack([t for _, t in items])
    else:
        md = config_model(name)
        th = config_theta_batch(name) if name in ("c5", "c5short") else THETA0[None, :]
        models = [P.Model.from_data(md)] * th.shape[0]
    theta = torch.tensor(th, dtype=torch.float64, device="cuda")
    for s in range(steps):
        t0 = time.perf_counter()
        out = P.eval_f_grad(models, theta)
        torch.cuda.synchronize()
        print(f"{name} step {s}: {time.perf_counter() - t0:.4f} s, f[0] = {out['f'][0].item():.12g}",
              flush=True)


if __name__ == "__main__":
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    main(sys.argv[1:])
