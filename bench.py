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
  * the largest block size (45x45 grid, b = 2025, nt = 200, nb = 10): the 8
    line-search theta points in one batched call, with its own step count, as
    the "largest_block" record (evaluations/s, whole-step FP64 rate and the
    product kernel's roofline);
  * the CPU oracle on the host (bounded samples), as the cpu_baseline: all
    cores through threaded LAPACK, one thread, and the level-1 form of the
    paper's parallel scheme (the 9 central-difference points in 9 concurrent
    processes), run before anything touches the GPU.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6  # MI355X, dense FP64 matrix (and vector) peak, published


def coupling_halfbandwidth(N):
    """Half-bandwidth of the coupling blocks c(rho) Q_s of an N x N grid: Q_s
    couples nodes up to grid distance 2 (|dx| + |dy| <= 2), which in the
    row-major order is an index offset of at most 2N (N + 1 on a 2 x 2 grid)."""
    b = N * N
    if N == 1:
        return 0
    return min(2 * N, b - 1) if N >= 3 else N + 1


def band_macs(b, w):
    """Multiply-adds of the band-aware b x b products (entry by entry): X = S
    inv(L)^T with S of half-bandwidth w, the lower half of X X^T, V = X inv(L),
    and one arrow row times X^T.  With w >= b - 1 these are the dense counts."""
    r = np.arange(b, dtype=np.float64)
    lo = np.maximum(0.0, r - w)
    hi = np.minimum(b - 1.0, r + w)
    L = hi - lo + 1
    x = float(np.sum(0.5 * L * (L + 1) + (b - 1 - hi) * L))
    syrk = float(np.sum((r + 1) * (b - lo)))
    v = float(np.sum(lo * (b - lo) + 0.5 * (b - lo) * (b - lo + 1)))
    arrow = float(np.sum(b - lo))
    return x, syrk, v, arrow


def flops_chol(b, nt, a, w=None):
    """BTA Cholesky: POTRF and TRTRI per block, the coupling X = S inv(L)^T
    (TRMM), the Schur update (SYRK), the arrow couplings, the arrow block.
    w: the coupling blocks' half-bandwidth (None: dense)."""
    if w is None or w >= b - 1:
        cpl = 2 * b ** 3 + 2 * a * b * b
    else:
        x, syrk, _, arrow = band_macs(b, w)
        cpl = 2 * x + 2 * syrk + 2 * a * arrow
    return nt * b ** 3 / 3 + (nt - 1) * cpl + nt * (a * b * b + a * a * b) + a ** 3 / 3


def flops_selinv(b, nt, a, w=None):
    """Block selected inversion: per step POTRI (2/3 b^3), V = L_{t+1,t} inv(L_tt)
    (b^3 dense; band-aware with w), Sigma_S (2 b^3), Sigma_D (b^3)."""
    if w is None or w >= b - 1:
        vv = b ** 3
    else:
        vv = 2 * band_macs(b, w)[2]
    return nt * (2.0 / 3.0) * b ** 3 + (nt - 1) * (vv + 3 * b ** 3) + nt * (4 * a * b * b + 2 * a * a * b)


def product_alg_bytes(b, nt, a):
    """Compulsory HBM bytes of the b x b product phases of one f + grad
    evaluation of one item (both matrices): every operand block read once and
    every output block written once, dense blocks.  Per matrix and time step
    below the last: X = S inv(L)^T (S, inv(L) read, X written: 3 b^2), the
    Schur update (X read, the lower half of D[t+1] read and written: 2 b^2),
    V = X inv(L) (3 b^2), Sigma_S = -Sigma_D[t+1] V (3 b^2); per step
    Sigma_D (inv(L)^T inv(L) read as its stored lower half, Sigma_S and V read,
    Sigma_D written: 3.5 b^2) and inv(L)^T inv(L) itself (inv(L) read, its
    lower half written: 1.5 b^2).  The arrow rows (a << b) are left out."""
    per_matrix = (nt - 1) * 11 * b * b + nt * 5 * b * b
    return 2 * 8.0 * per_matrix


def band_of(md):
    """The half-bandwidth the library uses for this model (None with INLA_BAND=0)."""
    if os.environ.get("INLA_BAND", "1").startswith("0"):
        return None
    return coupling_halfbandwidth(md.N)


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


def host_facts():
    """Host CPU facts for the CPU baseline: logical CPUs, the CPUs this process
    may run on, the thread count the box asks for, the CPU model and the BLAS
    libraries numpy / scipy use with their thread counts."""
    facts = {"nproc": os.cpu_count(), "affinity_cpus": len(os.sched_getaffinity(0)),
             "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}
    try:
        with open("/proc/cpuinfo") as fh:
            models = [ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")]
        facts["cpu_model"] = models[0] if models else None
    except OSError:
        facts["cpu_model"] = None
    try:
        from threadpoolctl import threadpool_info
        facts["blas"] = [{"api": p.get("internal_api"), "version": p.get("version"),
                          "threads": p.get("num_threads"),
                          "library": os.path.basename(p.get("filepath", ""))}
                         for p in threadpool_info()]
    except Exception:  # pragma: no cover
        facts["blas"] = None
    return facts


_LEVEL1_CHILD = """
import json, os, sys, time
sys.path.insert(0, {root!r})
import numpy as np
import oracle
from inla_synth import config_model, fd_stencil, THETA0
md = config_model({config!r})
pt = fd_stencil(THETA0, 1e-3)[{k}]
t0 = time.time()
f = oracle.eval_f_banded(md, pt)["f"]
t1 = time.time()
print(json.dumps({{"start": t0, "end": t1, "f": f}}))
"""


def cpu_baseline(config, budget_s=30.0):
    """The oracle on the host's cores, in three modes (a baseline only, never
    the target): threaded LAPACK on all cores, one thread, and the paper's
    level-1 parallelism -- the 2d+1 = 9 central-difference points of one
    gradient as 9 concurrent processes with cores // 9 threads each.  f+grad
    by central differences costs 9 f evaluations."""
    import subprocess

    import numpy as np

    import oracle
    from inla_synth import THETA0, config_model
    facts = host_facts()
    cores = int(facts["omp_num_threads"] or facts["affinity_cpus"] or 1)
    md = config_model(config)
    theta = np.asarray(THETA0)
    modes = {}
    # (1) all cores through threaded LAPACK
    t0 = time.perf_counter()
    n = 0
    while n < 2 and time.perf_counter() - t0 < budget_s / 3:
        oracle.eval_f_banded(md, theta)
        n += 1
    dt = (time.perf_counter() - t0) / n
    modes["threaded"] = {"threads": cores, "f_evals": n, "s_per_f": round(dt, 3),
                         "f_grad_evals_per_s": 1.0 / (9.0 * dt)}
    # (2) one thread
    try:
        from threadpoolctl import threadpool_limits
        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            oracle.eval_f_banded(md, theta)
            dt1 = time.perf_counter() - t0
        modes["single_thread"] = {"threads": 1, "f_evals": 1, "s_per_f": round(dt1, 3),
                                  "f_grad_evals_per_s": 1.0 / (9.0 * dt1)}
    except ImportError:  # pragma: no cover
        pass
    # (3) level 1: the 9 stencil points in 9 concurrent processes
    per = max(1, cores // 9)
    env = dict(os.environ, OMP_NUM_THREADS=str(per), OPENBLAS_NUM_THREADS=str(per),
               MKL_NUM_THREADS=str(per))
    procs = [subprocess.Popen([sys.executable, "-c",
                               _LEVEL1_CHILD.format(root=ROOT, config=config, k=k)],
                              stdout=subprocess.PIPE, stderr=subprocess.PIPE, env=env, text=True)
             for k in range(9)]
    recs = []
    for p in procs:
        out, err = p.communicate(timeout=600)
        if p.returncode != 0:
            raise RuntimeError("level-1 oracle process failed: " + err[-2000:])
        recs.append(json.loads(out.strip().splitlines()[-1]))
    wall = max(r["end"] for r in recs) - min(r["start"] for r in recs)
    fv = [r["f"] for r in recs]
    modes["level1_9_processes"] = {
        "threads": 9 * per, "processes": 9, "threads_per_process": per,
        "fd_gradient_wall_s": round(wall, 3), "f_grad_evals_per_s": 1.0 / wall,
        "fd_grad_h1e-3": [(fv[1 + 2 * k] - fv[2 + 2 * k]) / 2e-3 for k in range(4)]}
    best = max(modes, key=lambda k: modes[k]["f_grad_evals_per_s"])
    for m in modes.values():
        m["f_grad_evals_per_s"] = round(m["f_grad_evals_per_s"], 5)
    return {"value": modes[best]["f_grad_evals_per_s"], "unit": "f+grad evals/s",
            "cores": modes[best]["threads"], "kind": "oracle",
            "sample": (f"oracle f (bordered-banded LAPACK Cholesky of Q_p and Q_c + solve) at "
                       f"{md.N}x{md.N}x{md.nt} (n={md.n}); f+grad = 9 f evaluations by central "
                       f"differences; value = fastest of the modes ({best}); threaded: {n} f "
                       f"evaluation(s), single thread: 1, level 1: one gradient"),
            "modes": modes, "host": facts}


def load_workload(P, config):
    """Models, theta batch (device) and per-item model data of a named workload."""
    import numpy as np
    import torch

    from inla_synth import THETA0, config_model, config_theta_batch, uneven_batch
    if config == "c3":
        items = uneven_batch(64)
        mds = [m for m, _ in items]
        model = [P.Model.from_data(m) for m in mds]
        theta = torch.tensor(np.stack([t for _, t in items]), dtype=torch.float64, device="cuda")
        workload = "64 models of uneven (N in {16,24,32}, nt in [20,100], nb in [2,6]), each " \
                   "with its own theta, f+grad via adjoint, one batched call"
        return model, theta, mds, workload
    md = config_model(config)
    model = P.Model.from_data(md)
    th = config_theta_batch(config) if config == "c5" else THETA0[None, :]
    theta = torch.tensor(th, dtype=torch.float64, device="cuda")
    mds = [md] * theta.shape[0]
    workload = (f"N={md.N} (b={md.ns}), nt={md.nt}, nb={md.nb}, n={md.n}, m={md.m}, "
                f"{theta.shape[0]} theta point(s), f+grad via adjoint"
                + (", one batched call" if theta.shape[0] > 1 else ""))
    return model, theta, mds, workload


def measure(P, config, model, theta, mds, steps, warmup, timing_steps):
    """Time `steps` evaluations (graph replay) after `warmup`, then an eager
    pass of `timing_steps` evaluations with HIP events around every launch;
    returns the throughput record and the roofline of the dominant tile kernel."""
    import torch
    n_items = theta.shape[0]
    F_alg = sum(2 * flops_chol(m.ns, m.nt, m.nb, band_of(m)) + 2 * flops_selinv(m.ns, m.nt, m.nb, band_of(m))
                for m in mds)
    # Timed region: the evaluation replays its captured hipGraph (one launch of
    # the whole kernel sequence per step).
    for _ in range(max(warmup, 1)):
        P.eval_f_grad(model, theta)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        out = P.eval_f_grad(model, theta)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    step_s = (t1 - t0) / steps
    value = n_items / step_s

    # Kernel timing pass: the same evaluations launched eagerly with HIP events
    # around every kernel on its stream (events recorded inside a captured
    # graph cannot be timed), in the same process right after the timed region.
    prev_graph = os.environ.get("INLA_GRAPH")
    os.environ["INLA_GRAPH"] = "0"
    P.profile_begin()
    torch.cuda.synchronize()
    tp0 = time.perf_counter()
    for _ in range(timing_steps):
        P.eval_f_grad(model, theta)
    torch.cuda.synchronize()
    tp1 = time.perf_counter()
    prof = P.profile_end()
    if prev_graph is None:
        os.environ.pop("INLA_GRAPH", None)
    else:
        os.environ["INLA_GRAPH"] = prev_graph
    eager_step_s = (tp1 - tp0) / timing_steps

    calls = max(prof["calls"], 1)
    slots, kernels = prof["slots"], prof["kernels"]
    # dominant tile kernel (by kernel symbol, as rocprof reports it) by time
    tile_kernels = {k: v for k, v in kernels.items() if k != "other" and v["launches"]}
    dom = max(tile_kernels, key=lambda k: tile_kernels[k]["ms"])
    pk = tile_kernels[dom]
    achieved = pk["flops"] / (pk["ms"] * 1e-3) / 1e12 if pk["ms"] > 0 else 0.0
    traffic = hbm_traffic(config, "inla::" + dom)
    # compulsory bytes per launch of the product kernel: the b x b product
    # phases' operand and output blocks once each, over its launches
    alg_bytes_launch = None
    if dom == "tile_product_kernel" and pk["launches"]:
        alg_bytes_launch = round(sum(product_alg_bytes(m.ns, m.nt, m.nb) for m in mds)
                                 * calls / pk["launches"], 1)
    roofline = {"bound": "mfma", "kernel": dom,
                "achieved": round(achieved, 3), "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_FP64_TFLOPS, 4),
                "traffic": traffic,
                "alg_bytes_per_launch": alg_bytes_launch,
                "traffic_over_alg_bytes": (round(traffic / alg_bytes_launch, 3)
                                           if traffic and alg_bytes_launch else None),
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
    f_val = out["f"].cpu().numpy().tolist()
    grad = out["grad"].cpu().numpy().tolist()
    return {"value": value, "step_s": step_s, "F_alg": F_alg, "f": f_val, "grad": grad,
            "roofline": roofline, "status": out["status"].cpu().numpy().tolist()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="c2", choices=["c1", "c2", "c3", "c4", "c5"],
                    help="c2 (default, the headline): 32x32x50, one theta; c3: 64 uneven models, "
                         "one batched call; c4: 40x40x100, one theta; c5: 45x45x200, the 8 "
                         "line-search points in one batched call")
    ap.add_argument("--largest-steps", type=int, default=3,
                    help="timed steps of the largest-block record (0: skip it)")
    ap.add_argument("--largest-warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-fd", action="store_true", help="skip the finite-difference baseline")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU (asked for --gpus {args.gpus}); the "
              f"batched items would shard across GPUs by theta point, which is not implemented.",
              file=sys.stderr)
        sys.exit(2)

    # the CPU baseline first: its level-1 mode starts processes, which must
    # not come from a process that has touched the GPU
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline("c2" if args.config == "c3" else args.config)

    import numpy as np
    import torch

    import paper_2204_04678_amd as P
    from inla_synth import THETA0, fd_stencil

    if not os.path.exists(P.binding.LIB):
        from paper_2204_04678_amd import _build
        _build.build()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)

    model, theta, mds, workload = load_workload(P, args.config)
    md = mds[0]
    n_items = theta.shape[0]
    r = measure(P, args.config, model, theta, mds, args.steps, args.warmup, args.steps)
    value, step_s = r["value"], r["step_s"]
    f_val, grad = r["f"], r["grad"]
    if n_items == 1:
        f_val, grad = f_val[0], grad[0]
    elif n_items > 8:
        f_val, grad = f_val[:8], grad[:8]

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

    if args.largest_steps > 0 and args.config != "c5":
        # the largest block size: free this workload's device memory first
        del model
        P.release_workspace()
        torch.cuda.empty_cache()
        t_load = time.perf_counter()
        m5, th5, mds5, wl5 = load_workload(P, "c5")
        t_load = time.perf_counter() - t_load
        r5 = measure(P, "c5", m5, th5, mds5, args.largest_steps, args.largest_warmup, 1)
        extra["largest_block"] = {
            "config": {"workload": wl5, "b": mds5[0].ns, "nt": mds5[0].nt, "a": mds5[0].nb,
                       "n": mds5[0].n, "items": th5.shape[0],
                       "coupling_halfbandwidth": band_of(mds5[0])},
            "steps": args.largest_steps, "warmup": args.largest_warmup,
            "value": round(r5["value"], 4), "unit": "evals/s",
            "ms_per_step": round(r5["step_s"] * 1e3, 3),
            "alg_flops_per_step": r5["F_alg"],
            "pct_fp64_peak_whole_step": round(100 * r5["F_alg"] / r5["step_s"]
                                              / (PEAK_FP64_TFLOPS * 1e12), 3),
            "status": r5["status"], "f": r5["f"],
            "model_setup_s": round(t_load, 2),
            "roofline": r5["roofline"]}
        del m5
        P.release_workspace()

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
        "config": {"workload": workload, "b": md.ns, "nt": md.nt, "a": md.nb, "n": md.n,
                   "items": n_items,
                   "coupling_halfbandwidth": (band_of(md) if len({m.N for m in mds}) == 1
                                              else "2N per model")},
        "build_id": P.build_id(),
        "pct_fp64_peak_whole_step": round(100 * r["F_alg"] / step_s / (PEAK_FP64_TFLOPS * 1e12), 3),
        "alg_flops_per_step": r["F_alg"],
        "f": f_val,
        "grad": grad,
        "roofline": r["roofline"],
        "cpu_baseline": cpu,
        **extra,
    }
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
