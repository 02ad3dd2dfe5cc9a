"""Run a named synthetic workload through the library, for profilers.

    python3 -m paper_2204_04678_amd.workload c2 [steps] [--graph]

Builds the seeded model of the workload (as bench.py does), then runs `steps`
evaluations of f and its gradient (the workload's theta points, one batched
call per step) with eager kernel launches unless --graph is given, and prints
one line per step.  Nothing is timed here; the profiler does that.
"""
import os
import sys
import time


def main(argv):
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
