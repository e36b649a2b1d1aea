"""Frame-solve throughput of the PD+IPC solver on one MI355X.

A "step" is one frame of the quasi-static solver: a fixed number of
Algorithm-1 iterations (local step, constraint set, barrier, global step,
CCD, line search) on the face-like 50k-vertex workload.  The headline value is
the mixed-precision path's frames/s; the plain FP64 path is timed beside it.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload face50k]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# kernel families of the library's event timer
K_LOCAL, K_SIGMA_GEMV, K_FWD, K_BWD, K_BARRIER, K_TRIAL, K_RED_CHOL = 0, 1, 2, 3, 4, 5, 6

HBM_PEAK_GBS = 8000.0

# HBM bytes per local-step launch on face50k from two rocprofv3 counter passes
# (FETCH_SIZE, WRITE_SIZE), scaled by what the counters read for a plain copy
# of known size; valid only for the kernel source they were taken on
# (profiles/local_step_kernel_face50k_pmc.md).
LOCAL_STEP_TRAFFIC = {"workload": "face50k", "source_sha256_prefix": "54fa61f8b0518b46", "bytes": 103978783}


def measured_traffic(workload: str):
    import hashlib
    path = os.path.join(ROOT, "paper_2312_02999_amd", "csrc", "k_local.hip")
    with open(path, "rb") as f:
        digest = hashlib.sha256(f.read()).hexdigest()[:16]
    t = LOCAL_STEP_TRAFFIC
    ok = workload == t["workload"] and digest == t["source_sha256_prefix"]
    return t["bytes"] if ok else None


def progress(msg: str) -> None:
    """One line per finished stage on stderr (stdout carries the JSON)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def local_step_bytes(n: int, m: int) -> int:
    """Algorithmic bytes of one local-step launch (FP64 streams).

    Per tet: 4 int32 indices, 9 D_m^-1 + 1 weight + 6 actuation doubles in;
    9 rotation + 1 energy + 12 gradient-share doubles out.  Per vertex: one
    xyz triple read once.
    """
    per_tet = 4 * 4 + (9 + 1 + 6) * 8 + (9 + 1 + 12) * 8
    return m * per_tet + n * 24


def run_precision(sc, precision, steps, warmup, timer_kernel):
    import torch
    from paper_2312_02999_amd import Solver
    S = Solver(sc, iters=sc.iters, precision=precision)
    progress(f"solver ready ({'mixed' if precision else 'fp64'})")
    dev = "cuda"
    R = torch.from_numpy(np.ascontiguousarray(sc.act_R.reshape(-1, 9))).to(dev)
    seq = [torch.from_numpy(np.ascontiguousarray(sc.actuation_at((t + 1) / sc.frames))).to(dev)
           for t in range(sc.frames)]
    x = torch.from_numpy(np.ascontiguousarray(sc.X)).to(dev)
    S.set_actuation_scalar(seq[0], R)
    t = 0
    for _ in range(warmup):
        S.set_actuation_scalar(seq[min(t, len(seq) - 1)])
        x = S.solve_frame(x)
        t += 1
    progress("warm-up frames done")
    S.kernel_timer(timer_kernel)
    lat = []
    x_start, t_start = x.clone(), t
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        S.set_actuation_scalar(seq[min(t, len(seq) - 1)])
        a = time.perf_counter()
        x = S.solve_frame(x)
        lat.append(time.perf_counter() - a)
        t += 1
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    progress(f"{steps} timed frames in {wall:.2f} s")
    k_ms, k_count = S.kernel_timer(-1)
    # counters and per-stage times from an untimed replay of the same frames
    # (stage timing synchronises after the global step)
    stats = []
    xs, t = x_start, t_start
    for _ in range(steps):
        S.set_actuation_scalar(seq[min(t, len(seq) - 1)])
        xs, st = S.solve_frame(xs, stats=True)
        stats.append(st)
        t += 1
    sizes = S.sizes()
    dev_bytes = S.device_bytes()
    S.close()
    lat_ms = np.array(lat) * 1e3
    return {
        "fps": steps / wall, "ms_per_frame": 1e3 * wall / steps,
        "p50_ms": float(np.percentile(lat_ms, 50)), "p99_ms": float(np.percentile(lat_ms, 99)),
        "kernel_ms_total": k_ms, "kernel_launches": k_count, "sizes": sizes, "device_bytes": dev_bytes,
        "n_c_max": max(s["n_c"] for s in stats), "n_pt_last": stats[-1]["n_pt"], "n_ee_last": stats[-1]["n_ee"],
        "ls_failures": sum(s["ls_failures"] for s in stats),
        "refine_steps": sum(s["refine_steps"] for s in stats),
        "refine_fallbacks": sum(s["refine_fallbacks"] for s in stats),
        "cinv_rebuilds": sum(s["cinv_rebuilds"] for s in stats),
        "c_delta_max": max(s["c_delta_max"] for s in stats),
        "c_delta_sum": sum(s["c_delta_sum"] for s in stats),
        "stage_ms": {k: float(np.mean([s[k] for s in stats])) for k in ("ms_ipc", "ms_gstep", "ms_ls", "ms_misc")},
        "x_final": x.cpu().numpy(),
    }


def cpu_baseline(sc, budget_s=20.0):
    """The oracle (as it stands) on a bounded sample: whole Algorithm-1
    iterations from the rest state at full actuation until ~budget_s."""
    from oracle import fem, solver as osolver
    prob = osolver.setup_scene(sc)
    A = fem.actuation_matrices(sc.act_a, sc.act_R)
    x = sc.X.copy()
    c0 = os.times()
    t0 = time.perf_counter()
    its = 0
    while True:
        x, _, _ = osolver.iteration(prob, x, A)
        its += 1
        if time.perf_counter() - t0 > budget_s or its >= 4:
            break
    wall = time.perf_counter() - t0
    c1 = os.times()
    busy = (c1.user - c0.user) + (c1.system - c0.system)
    sec_per_it = wall / its
    # cores actually used: process CPU time over wall time (numpy/torch may
    # thread; SuperLU does not)
    return {"value": 1.0 / (sec_per_it * sc.iters), "unit": "frames/s", "cores": round(busy / wall, 2),
            "kind": "oracle", "host_cpus": os.cpu_count(),
            "sample": f"{its} oracle iteration(s) of the {sc.n}-vertex workload from rest at full actuation, "
                      f"scaled to {sc.iters} iterations/frame ({sec_per_it:.2f} s/iteration)"}


def run_adjoint(sc, n_targets=500, n_dirs=2, n_params=4, h_dir=1e-4, seed=1):
    """Adjoint of a converged frame on the face mesh against central finite
    differences of the same GPU solver (tolerance mode).  Targets are the
    converged positions of seeded proxy vertices at 0.6 x the strength field;
    the loss is taken at 0.8 x the field.  Finite differences run along seeded
    random directions in actuation space (all tets at once) and along the
    single tets with the largest gradient entries."""
    import torch
    from paper_2312_02999_amd import FP64, Solver
    dev = "cuda"
    S = Solver(sc, iters=1500, tol=1e-12, precision=FP64)
    R = torch.from_numpy(np.ascontiguousarray(sc.act_R.reshape(-1, 9))).to(dev)
    X = torch.from_numpy(np.ascontiguousarray(sc.X)).to(dev)
    rng = np.random.default_rng(seed)
    cand = np.setdiff1d(np.unique(sc.surf_tris), np.nonzero(sc.dirichlet)[0])
    tv = torch.from_numpy(rng.choice(cand, min(n_targets, cand.size), replace=False)).to(dev)

    def solve(a, x0):
        S.set_actuation_scalar(torch.from_numpy(np.ascontiguousarray(a)).to(dev), R)
        x, st = S.solve_frame(x0, stats=True)
        return x, st

    xt, st_t = solve(0.6 * sc.act_a, X)
    a = 0.8 * sc.act_a
    xs, st_s = solve(a, xt)
    loss = lambda x: float(((x[tv] - xt[tv]) ** 2).sum())
    L0 = loss(xs)
    dLdx = torch.zeros_like(xs)
    dLdx[tv] = 2.0 * (xs[tv] - xt[tv])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g = S.solve_frame_backward(dLdx)
    torch.cuda.synchronize()
    ms_bwd = 1e3 * (time.perf_counter() - t0)
    g = g.cpu().numpy()
    errs = []
    for k in range(n_dirs):
        d = rng.standard_normal(sc.m)
        fd = (loss(solve(a + h_dir * d, xs)[0]) - loss(solve(a - h_dir * d, xs)[0])) / (2 * h_dir)
        errs.append(("dir", k, float(g @ d), fd))
    top = np.argsort(-np.abs(g))[:n_params]
    for i in top:
        e = np.zeros(sc.m)
        h = 1e-3
        e[i] = h
        fd = (loss(solve(a + e, xs)[0]) - loss(solve(a - e, xs)[0])) / (2 * h)
        errs.append(("tet", int(i), float(g[i]), fd))
    S.close()
    rel = [abs(ad - fd) / max(abs(fd), 1e-300) for _, _, ad, fd in errs]
    return {"metric": "adjoint of a converged frame: backward ms and agreement with finite differences",
            "workload": f"{sc.n} vertices, {sc.m} tets, {sc.m} actuation parameters",
            "backward_ms": round(ms_bwd, 2), "loss": L0, "iters_targets": st_t["iters"],
            "iters_frame": st_s["iters"], "max_rel_err_fd": max(rel),
            "checks": [{"kind": k, "index": i, "adjoint": ad, "fd": fd} for k, i, ad, fd in errs]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="face50k")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only", choices=["fp64", "mixed"], default=None,
                    help="profile one path only (the JSON line then lacks the other)")
    ap.add_argument("--adjoint", action="store_true",
                    help="time the adjoint on the workload and check it against finite differences")
    ap.add_argument("--serving", type=int, default=0, metavar="REQUESTS",
                    help="replay a Poisson stream of this many requests through the server instead")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one 256 MiB device copy (reference for hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (the solver has no multi-GPU path); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import meshgen as mg
    from paper_2312_02999_amd import FP64, MIXED_FP32

    if args.serving:
        from paper_2312_02999_amd import serve
        for prec in (MIXED_FP32, FP64):
            progress(f"serving {args.serving} requests ({'mixed' if prec else 'fp64'})")
            rep = serve.run_serving(n_requests=args.serving, precision=prec)
            print(json.dumps({"metric": "serving: request latency and frames/s", **rep}), flush=True)
        return
    sc = mg.scene_by_name(args.workload)
    progress(f"scene {args.workload} generated (n={sc.n}, m={sc.m})")
    if args.adjoint:
        print(json.dumps(run_adjoint(sc)))
        return
    if args.only:
        r = run_precision(sc, FP64 if args.only == "fp64" else MIXED_FP32, args.steps, args.warmup, K_LOCAL)
        r.pop("x_final")
        print(json.dumps({"only": args.only, **r}))
        return
    fp64 = run_precision(sc, FP64, args.steps, args.warmup, K_LOCAL)
    mixed = run_precision(sc, MIXED_FP32, args.steps, args.warmup, K_LOCAL)
    diag = float(np.linalg.norm(sc.X.max(0) - sc.X.min(0)))
    mixed_vs_fp64 = float(np.abs(mixed["x_final"] - fp64["x_final"]).max() / diag)

    avg_ms = fp64["kernel_ms_total"] / max(fp64["kernel_launches"], 1)
    nbytes = local_step_bytes(sc.n, sc.m)
    achieved = nbytes / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    # avg_launch_us: events stamped by the dispatch itself (extended launch) on
    # the solver's stream, every local-step launch of the timed FP64 frames
    roof = {"bound": "hbm", "kernel": "local_step_kernel<double>", "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(args.workload),
            "avg_launch_us": round(avg_ms * 1e3, 2), "launches": fp64["kernel_launches"],
            "algorithmic_bytes": nbytes}
    if not args.no_cpu_baseline:
        progress("oracle baseline sample")
    cpu = None if args.no_cpu_baseline else cpu_baseline(sc)
    out = {
        "metric": "PD+IPC frames/s on 50k-vert mesh, mixed vs FP64 GPU; p50/p99 latency",
        "value": round(mixed["fps"], 3), "unit": "frames/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(mixed["ms_per_frame"], 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64 (mixed)", "data": "synthetic",
        "config": {"workload": f"{args.workload}: face-like shell n={sc.n} m={sc.m}, {sc.iters} iterations/frame, "
                               f"{sc.frames}-frame actuation ramp",
                   "n1": fp64["sizes"]["n1"], "n2": fp64["sizes"]["n2"], "factor_nnz": fp64["sizes"]["factor_nnz"]},
        "p50_ms": round(mixed["p50_ms"], 3), "p99_ms": round(mixed["p99_ms"], 3),
        "fp64": {"value": round(fp64["fps"], 3), "ms_per_step": round(fp64["ms_per_frame"], 3),
                 "p50_ms": round(fp64["p50_ms"], 3), "p99_ms": round(fp64["p99_ms"], 3),
                 "stage_ms": fp64["stage_ms"], "n_c_max": fp64["n_c_max"], "ls_failures": fp64["ls_failures"],
                 "cinv_rebuilds": fp64["cinv_rebuilds"], "c_delta_max": fp64["c_delta_max"],
                 "c_delta_sum": fp64["c_delta_sum"], "device_bytes": fp64["device_bytes"]},
        "mixed": {"stage_ms": mixed["stage_ms"], "n_c_max": mixed["n_c_max"], "ls_failures": mixed["ls_failures"],
                  "refine_steps": mixed["refine_steps"], "refine_fallbacks": mixed["refine_fallbacks"],
                  "max_rel_pos_diff_vs_fp64": mixed_vs_fp64},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))
    if args.copy_probe:
        # a plain copy of known size: its FETCH_SIZE / WRITE_SIZE per dispatch
        # scale the counters of the solver's kernels to bytes
        a = torch.ones(32 << 20, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": a.numel() * 8, "copy_probe_bytes_written": b.numel() * 8}))


if __name__ == "__main__":
    main()
