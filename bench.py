"""Benchmark: f(theta) + grad f evaluations per second on one MI355X.

Workload (default): the 32x32-grid, 50-time-step, 4-fixed-effect model
(n = 51204, block size b = 1024), FP64.  One step = one evaluation of f(theta)
and its exact gradient at theta0 through the selected-inversion adjoint:
assembly of Q_prior and Q_c, both block Cholesky factorizations and
log-determinants, the mode solve, both selected inversions with the trace
reductions, and the combination into f and grad f.  Inputs are resident in HBM
before the timed region.

Also measured in the same run (reported beside the headline, not as it):
  * the plain finite-difference baseline on the same GPU: 2*dim(theta)+1 = 9
    f-only evaluations one after another per gradient;
  * the same 9 points as one batched call;
  * the CPU oracle on the host (bounded sample), as the cpu_baseline.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6  # MI355X, dense FP64 matrix (and vector) peak, published


def flops_chol(b, nt, a):
    """Dense-block BTA Cholesky: POTRF per block, TRSM/SYRK/GEMM couplings, arrow."""
    return (nt * b ** 3 / 3 + (nt - 1) * (2 * b ** 3 + 2 * a * b * b) + nt * (a * b * b + a * a * b)
            + a ** 3 / 3)


def flops_selinv(b, nt, a):
    """Block selected inversion: per step POTRI (2/3 b^3), V (b^3), Sigma_S (2 b^3), Sigma_D (b^3)."""
    return nt * (2.0 / 3.0) * b ** 3 + (nt - 1) * 4 * b ** 3 + nt * (4 * a * b * b + 2 * a * a * b)


def kernel_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for f in ("bta_kernels.hip", "model_kernels.hip", "inla_internal.h"):
        with open(os.path.join(ROOT, "paper_2204_04678_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def hbm_traffic(config, kernel):
    """HBM bytes per dispatch of `kernel` (averaged over its instantiations,
    weighted by their dispatch counts) from the committed rocprofv3 counter
    summary of this workload (FETCH_SIZE and WRITE_SIZE, scaled by what they
    read for a plain 1 GiB copy); None when there is none or the kernel
    sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{config}_f_grad.txt")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = [json.loads(line[5:]) for line in fh if line.startswith("JSON ")]
    if not rec or rec[0]["source_sha256"] != kernel_sources_sha256():
        return None
    # every instantiation of the kernel (tile edge, layout), weighted by dispatches
    ks = [v for n, v in rec[0]["kernels"].items() if n == kernel or n.startswith(kernel + "<")]
    nd = sum(v["dispatches"] for v in ks)
    if nd == 0:
        return None
    return sum(v["hbm_bytes_per_dispatch"] * v["dispatches"] for v in ks) / nd


def cpu_baseline(md, theta, budget_s=20.0):
    """Oracle f(theta) on the host; the oracle's gradient is 2d+1 = 9 f evaluations."""
    import numpy as np

    import oracle
    try:
        from threadpoolctl import threadpool_info
        threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        threads = os.cpu_count() or 1
    t0 = time.perf_counter()
    n = 0
    while True:
        oracle.eval_f_banded(md, np.asarray(theta))
        n += 1
        if time.perf_counter() - t0 > budget_s / 2 or n >= 3:
            break
    dt = (time.perf_counter() - t0) / n
    return {"value": 1.0 / (9.0 * dt), "unit": "f+grad evals/s", "cores": int(threads),
            "kind": "oracle",
            "sample": f"{n} oracle f evaluation(s) (bordered-banded LAPACK Cholesky of Q_p and Q_c + "
                      f"solve) at the workload size, {dt:.2f} s each; f+grad by central "
                      f"differences = 9 f evaluations"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="c2", choices=["c1", "c2", "c3", "c4", "c5"],
                    help="c2 (default, the headline): 32x32x50, one theta; c3: 64 uneven models, "
                         "one batched call; c4: 40x40x100, one theta; c5: 45x45x200, the 8 "
                         "line-search points in one batched call")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-fd", action="store_true", help="skip the finite-difference baseline")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); the "
              f"batched items would shard across GPUs by theta point, which is not built.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2204_04678_amd as P
    from inla_synth import THETA0, config_model, config_theta_batch, fd_stencil, uneven_batch

    if not os.path.exists(P.binding.LIB):
        from paper_2204_04678_amd import _build
        _build.build()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)

    if args.config == "c3":
        items = uneven_batch(64)
        mds = [m for m, _ in items]
        model = [P.Model.from_data(m) for m in mds]
        theta = torch.tensor(np.stack([t for _, t in items]), dtype=torch.float64, device="cuda")
        md = mds[0]
        workload = "64 models of uneven (N in {16,24,32}, nt in [20,100], nb in [2,6]), each " \
                   "with its own theta, f+grad via adjoint, one batched call"
    else:
        md = config_model(args.config)
        mds = [md]
        model = P.Model.from_data(md)
        th = config_theta_batch(args.config) if args.config == "c5" else THETA0[None, :]
        theta = torch.tensor(th, dtype=torch.float64, device="cuda")
        mds = mds * theta.shape[0]
        workload = (f"N={md.N} (b={md.ns}), nt={md.nt}, nb={md.nb}, n={md.n}, m={md.m}, "
                    f"{theta.shape[0]} theta point(s), f+grad via adjoint")
    n_items = theta.shape[0]
    b, nt, a = md.ns, md.nt, md.nb
    F_alg = sum(2 * flops_chol(m.ns, m.nt, m.nb) + 2 * flops_selinv(m.ns, m.nt, m.nb) for m in mds)

    # Timed region: the evaluation replays its captured hipGraph (one launch of
    # the whole ~2.5k-kernel sequence per step).
    for _ in range(max(args.warmup, 1)):
        P.eval_f_grad(model, theta)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out = P.eval_f_grad(model, theta)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    step_s = (t1 - t0) / args.steps
    value = n_items / step_s

    # Kernel timing pass: the same steps launched eagerly with HIP events around
    # every kernel on its stream (events recorded inside a captured graph cannot
    # be timed), in the same process right after the timed region.
    prev_graph = os.environ.get("INLA_GRAPH")
    os.environ["INLA_GRAPH"] = "0"
    P.profile_begin()
    torch.cuda.synchronize()
    tp0 = time.perf_counter()
    for _ in range(args.steps):
        P.eval_f_grad(model, theta)
    torch.cuda.synchronize()
    tp1 = time.perf_counter()
    prof = P.profile_end()
    if prev_graph is None:
        os.environ.pop("INLA_GRAPH", None)
    else:
        os.environ["INLA_GRAPH"] = prev_graph
    eager_step_s = (tp1 - tp0) / args.steps
    f_val = out["f"].cpu().numpy().tolist()
    grad = out["grad"].cpu().numpy().tolist()
    if n_items == 1:
        f_val, grad = f_val[0], grad[0]
    elif n_items > 8:
        f_val, grad = f_val[:8], grad[:8]

    calls = max(prof["calls"], 1)
    slots, kernels = prof["slots"], prof["kernels"]
    # dominant tile kernel (by kernel symbol, as rocprof reports it) by time
    tile_kernels = {k: v for k, v in kernels.items() if k != "other" and v["launches"]}
    dom = max(tile_kernels, key=lambda k: tile_kernels[k]["ms"])
    pk = tile_kernels[dom]
    achieved = pk["flops"] / (pk["ms"] * 1e-3) / 1e12 if pk["ms"] > 0 else 0.0
    roofline = {"bound": "mfma", "kernel": dom,
                "achieved": round(achieved, 3), "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_FP64_TFLOPS, 4),
                "traffic": hbm_traffic(args.config, "inla::" + dom),
                "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE/WRITE_SIZE, copy-calibrated)",
                "launches_per_step": pk["launches"] / calls,
                "avg_launch_us": round(pk["ms"] * 1e3 / max(pk["launches"], 1), 3),
                "alg_flops_per_launch": pk["flops"] / max(pk["launches"], 1),
                "kernel_share_of_eager_step": round(pk["ms"] * 1e-3 / calls / eager_step_s, 4),
                "timing_pass": {"steps": calls, "unreadable_records": prof["bad"],
                                "eager_ms_per_step": round(eager_step_s * 1e3, 3),
                                "note": "per-kernel HIP events, eager launches of the same steps"},
                "per_kernel": {k: {"launches_per_step": v["launches"] / calls,
                                   "ms_per_step": round(v["ms"] / calls, 3),
                                   "avg_us": round(v["ms"] * 1e3 / max(v["launches"], 1), 3),
                                   "tflops": round(v["flops"] / max(v["ms"], 1e-9) / 1e9, 3)}
                               for k, v in kernels.items() if v["launches"]},
                "per_phase_ms_per_step": {k: round(v["ms"] / calls, 3)
                                          for k, v in slots.items() if v["launches"]}}

    extra = {}
    if not args.no_fd and args.config in ("c2", "c4"):
        pts = torch.tensor(fd_stencil(THETA0, 1e-3), dtype=torch.float64, device="cuda")
        reps = max(1, args.steps // 3)
        P.eval_f(model, pts[0:1])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            for i in range(pts.shape[0]):
                P.eval_f(model, pts[i:i + 1])
        torch.cuda.synchronize()
        fd_seq = (time.perf_counter() - t0) / reps
        P.eval_f(model, pts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fdb = P.eval_f(model, pts)
        torch.cuda.synchronize()
        fd_bat = (time.perf_counter() - t0) / reps
        fv = fdb["f"].cpu().numpy()
        g_fd = [(fv[1 + 2 * k] - fv[2 + 2 * k]) / 2e-3 for k in range(4)]
        extra["fd_baseline"] = {
            "grad_evals_per_s_sequential": round(1.0 / fd_seq, 4),
            "grad_evals_per_s_batched9": round(1.0 / fd_bat, 4),
            "adjoint_speedup_vs_sequential_fd": round(value * fd_seq, 3),
            "adjoint_speedup_vs_batched_fd": round(value * fd_bat, 3),
            "fd_grad_h1e-3": g_fd,
        }

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(md, theta[0].cpu().numpy())

    rec = {
        "metric": "f(theta)+grad f evaluations/s (BTA Cholesky + selected-inversion adjoint, FP64)",
        "value": round(value, 4),
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(step_s * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded grid model; no dataset)",
        "config": {"workload": workload, "b": b, "nt": nt, "a": a, "n": md.n, "items": n_items},
        "pct_fp64_peak_whole_step": round(100 * F_alg / step_s / (PEAK_FP64_TFLOPS * 1e12), 3),
        "alg_flops_per_step": F_alg,
        "f": f_val,
        "grad": grad,
        "roofline": roofline,
        "cpu_baseline": cpu,
        **extra,
    }
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
