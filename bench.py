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
# dense matrix-core peaks of MI355X (TFLOP/s) by the reduced factor's type
MFMA_PEAK_TFS = {"f64": 78.6, "f32": 157.3}

# HBM bytes per timer interval of a kernel family, from two rocprofv3 counter
# passes (FETCH_SIZE, WRITE_SIZE) scaled by what the counters read for a plain
# copy of known size (--copy-probe); valid only for the workload, precision and
# kernel sources they were taken on (the summaries in profiles/ give the
# commands).  Filled in from measurements; an entry whose sources changed
# reports null.
MEASURED_TRAFFIC = {
    "reduced Cholesky (Eq. 11 system)": {
        "workload": "face50k", "precision": "mixed", "sources": ["k_dense.hip"],
        "sha256_prefix": "2bfebeeb07074475", "bytes": 1400951280},
}


def _sources_digest(files) -> str:
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2312_02999_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(family: str, workload: str, precision: str):
    t = MEASURED_TRAFFIC.get(family)
    if t is None or t["workload"] != workload or t["precision"] != precision:
        return None
    return t["bytes"] if _sources_digest(t["sources"]) == t["sha256_prefix"] else None


def progress(msg: str) -> None:
    """One line per finished stage on stderr (stdout carries the JSON)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def local_step_bytes(n: int, m: int) -> int:
    """Algorithmic bytes of one local-step (or line-search trial) launch.

    Per tet: 4 int32 indices, 9 D_m^-1 + 1 weight + 6 actuation doubles read
    once (144 B).  Per vertex: one xyz triple in and one out (48 B: x and the
    gradient, or x and the step for a trial).
    """
    return m * (4 * 4 + (9 + 1 + 6) * 8) + n * 48


# families timed in replays of the timed frames, with what one timer interval
# covers: "launch" = one kernel launch, "sweep" = one whole triangular sweep,
# "factor" = one factorisation of the reduced system
TIMED_FAMILIES = [("local_step_kernel", K_LOCAL), ("trial_energy_kernel", K_TRIAL),
                  ("forward sweep (Eq. 7, L1^-1)", K_FWD), ("backward sweep (Eq. 7, L1^-T)", K_BWD),
                  ("sigma_gemv_kernel", K_SIGMA_GEMV), ("reduced Cholesky (Eq. 11 system)", K_RED_CHOL),
                  ("barrier_kernel", K_BARRIER)]


def run_precision(sc, precision, steps, warmup, families=True, **solver_kw):
    import torch
    from paper_2312_02999_amd import Solver
    seq_np = sc.sequence()
    if warmup + steps > len(seq_np):
        print(f"warmup + steps = {warmup + steps} exceeds the {len(seq_np)}-frame actuation sequence "
              f"of this workload: every timed frame must change actuation", file=sys.stderr)
        sys.exit(2)
    S = Solver(sc, iters=sc.iters, precision=precision, **solver_kw)
    progress(f"solver ready ({'mixed' if precision else 'fp64'}{' ' + str(solver_kw) if solver_kw else ''})")
    dev = "cuda"
    R = torch.from_numpy(np.ascontiguousarray(sc.act_R.reshape(-1, 9))).to(dev)
    seq = [torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in seq_np]
    x = torch.from_numpy(np.ascontiguousarray(sc.X)).to(dev)
    S.set_actuation_scalar(seq[0], R)
    for t in range(warmup):
        S.set_actuation_scalar(seq[t])
        x = S.solve_frame(x)
    progress("warm-up frames done")
    lat = []
    x_start = x.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for t in range(warmup, warmup + steps):
        S.set_actuation_scalar(seq[t])
        a = time.perf_counter()
        x = S.solve_frame(x)
        lat.append(time.perf_counter() - a)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    progress(f"{steps} timed frames in {wall:.2f} s")

    def replay(with_stats):
        xs, out = x_start, []
        for t in range(warmup, warmup + steps):
            S.set_actuation_scalar(seq[t])
            if with_stats:
                xs, st = S.solve_frame(xs, stats=True)
                out.append((st, S.trace()))
            else:
                xs = S.solve_frame(xs)
        return xs, out

    # counters, per-iteration records and Table 1 stage times from an untimed
    # replay of the same frames (stage timing synchronises at stage ends)
    x_replay, stats = replay(True)
    same = bool(torch.equal(x_replay, x))
    # per-kernel-family durations: one more replay per family with the
    # library's HIP-event timer around that family's launches
    fam = {}
    for name, k in (TIMED_FAMILIES if families else []):
        S.kernel_timer(k)
        replay(False)
        ms, cnt = S.kernel_timer(-1)
        fam[name] = (ms, cnt)
    progress("replays done")
    sizes = S.sizes()
    dev_bytes = S.device_bytes()
    S.close()
    lat_ms = np.array(lat) * 1e3
    its = [tr for _, trs in stats for tr in trs]
    nc_frames = [st["n_c"] for st, _ in stats]
    return {
        "fps": steps / wall, "ms_per_frame": 1e3 * wall / steps,
        "p50_ms": float(np.percentile(lat_ms, 50)), "p99_ms": float(np.percentile(lat_ms, 99)),
        "families": fam, "iters_total": len(its), "sizes": sizes, "device_bytes": dev_bytes,
        "replay_bitwise_equal": same,
        "n_c_max": int(max(nc_frames)), "n_c_mean": float(np.mean([tr["n_c"] for tr in its])),
        "contact_iters": int(sum(1 for tr in its if tr["n_c"] > 0)),
        "reduced_flops": float(sum((3.0 * tr["n_c"]) ** 3 / 3.0 for tr in its if tr["n_c"] > 0)),
        "pairs_max": int(max(tr["n_pt"] + tr["n_ee"] for tr in its)),
        "ls_failures": sum(st["ls_failures"] for st, _ in stats),
        "refine_steps": sum(st["refine_steps"] for st, _ in stats),
        "refine_fallbacks": sum(st["refine_fallbacks"] for st, _ in stats),
        "cinv_rebuilds": sum(st["cinv_rebuilds"] for st, _ in stats),
        "near_ties": sum(st["near_ties"] for st, _ in stats),
        "cg_products": sum(st["pcg_iters"] for st, _ in stats),
        "stage_ms": {k: round(float(np.mean([st[k] for st, _ in stats])), 3)
                     for k in ("ms_ipc", "ms_gstep", "ms_ccd", "ms_ls", "ms_misc")},
        "x_final": x.cpu().numpy(),
    }


def rooflines(sc, r, reduced_type):
    """One roofline entry per timed kernel family: algorithmic work per timer
    interval over its mean duration."""
    n2 = r["sizes"]["n2"]
    nnz = r["sizes"]["factor_nnz"]
    out = []
    for name, (ms, cnt) in r["families"].items():
        if cnt == 0 or ms <= 0:
            continue
        avg_s = ms * 1e-3 / cnt
        e = {"kernel": name, "intervals": cnt, "total_ms": round(ms, 3), "avg_us": round(avg_s * 1e6, 2)}
        if name in ("local_step_kernel", "trial_energy_kernel"):
            work = local_step_bytes(sc.n, sc.m)
            e.update(bound="hbm", unit="GB/s", peak=HBM_PEAK_GBS, work_per_interval=work,
                     work_unit="B", per_unit="144 B/tet + 48 B/vertex")
            e["achieved"] = work / avg_s / 1e9
        elif name.startswith("forward sweep") or name.startswith("backward sweep"):
            # the forward sweep is timed in two parts per iteration
            per_it = ms * 1e-3 / max(r["iters_total"], 1)
            work = 12 * nnz
            e.update(bound="hbm", unit="GB/s", peak=HBM_PEAK_GBS, work_per_interval=work, work_unit="B",
                     per_unit="12 B per factor nonzero (value + index), 3 right-hand sides per read",
                     avg_us=round(per_it * 1e6, 2), intervals=r["iters_total"])
            e["achieved"] = work / per_it / 1e9
        elif name == "sigma_gemv_kernel":
            work = 8 * n2 * (n2 + 1) // 2
            e.update(bound="hbm", unit="GB/s", peak=HBM_PEAK_GBS, work_per_interval=work, work_unit="B",
                     per_unit="8 B per entry of the packed symmetric n2 x n2 inverse Schur complement")
            e["achieved"] = work / avg_s / 1e9
        elif name.startswith("reduced Cholesky"):
            flops_per = r["reduced_flops"] / max(cnt, 1)
            e.update(bound="mfma", unit="TFLOP/s", peak=MFMA_PEAK_TFS[reduced_type],
                     work_per_interval=flops_per, work_unit="flop", per_unit="(3 n_c)^3 / 3 per factorisation",
                     dtype=reduced_type)
            e["achieved"] = flops_per / avg_s / 1e12
        else:
            e.update(bound="alu")
        if "achieved" in e:
            e["achieved"] = round(e["achieved"], 3)
            e["frac"] = round(e["achieved"] / e["peak"], 4)
        out.append(e)
    return out


def run_dense(n: int, reps: int = 6):
    """The dense SPD factorisation and solve of the reduced system's kernels on
    a seeded n x n SPD matrix (G G^T / n + I / 2), reps times."""
    import torch
    from paper_2312_02999_amd import dense_spd
    rng = np.random.default_rng(0)
    G = rng.standard_normal((n, n))
    A = G @ G.T / n + 0.5 * np.eye(n)
    b = rng.standard_normal((n, 1))
    At = torch.tensor(A, device="cuda")
    bt = torch.tensor(b, device="cuda")
    for _ in range(reps):
        x, _ = dense_spd(At, bt)
    torch.cuda.synchronize()
    res = float(np.abs(A @ x.cpu().numpy() - b).max())
    print(json.dumps({"dense_n": n, "factorisations": reps, "max_residual": res}))


def copy_probe():
    """A plain 256 MiB device copy: its FETCH_SIZE / WRITE_SIZE per dispatch
    scale the counters of the solver's kernels to bytes."""
    import torch
    a = torch.ones(32 << 20, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": a.numel() * 8, "copy_probe_bytes_written": b.numel() * 8}))


def cpu_baseline(sc, a, budget_s=20.0):
    """The oracle (as it stands) on a bounded sample: whole Algorithm-1
    iterations from the rest state at the actuation ``a`` of the first timed
    frame, until ~budget_s (at most 4 iterations)."""
    from oracle import fem, solver as osolver
    prob = osolver.setup_scene(sc)
    A = fem.actuation_matrices(a, sc.act_R)
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
            "sample": f"{its} oracle iteration(s) of the {sc.n}-vertex workload from rest at the first timed frame's "
                      f"actuation, "
                      f"scaled to {sc.iters} iterations/frame ({sec_per_it:.2f} s/iteration)"}


def run_adjoint(sc, n_targets=500, n_dirs=2, n_params=64, h_dir=1e-4, h_param=1e-3, seed=1):
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
        e[i] = h_param
        fd = (loss(solve(a + e, xs)[0]) - loss(solve(a - e, xs)[0])) / (2 * h_param)
        errs.append(("tet", int(i), float(g[i]), fd))
        if len(errs) % 8 == 0:
            progress(f"adjoint: {len(errs)} finite-difference checks done")
    S.close()
    rel = [abs(ad - fd) / max(abs(fd), 1e-300) for _, _, ad, fd in errs]
    rel_t = sorted(r for (k, _, _, _), r in zip(errs, rel) if k == "tet")
    return {"metric": "adjoint of a converged frame: backward ms and agreement with finite differences",
            "workload": f"{sc.n} vertices, {sc.m} tets, {sc.m} actuation parameters",
            "backward_ms": round(ms_bwd, 2), "loss": L0, "iters_targets": st_t["iters"],
            "iters_frame": st_s["iters"], "max_rel_err_fd": max(rel),
            "params_checked": len(rel_t), "h_param": h_param, "h_dir": h_dir,
            "median_rel_err_params": rel_t[len(rel_t) // 2] if rel_t else None,
            "max_rel_err_params": rel_t[-1] if rel_t else None,
            "checks": [{"kind": k, "index": i, "adjoint": ad, "fd": fd} for k, i, ad, fd in errs]}


def run_table1(sc, steps, warmup, kappa0):
    """The paper's Table 1 configurations with collision on this workload, all
    FP64: the method (Schur complement and low-rank update), the Schur
    complement alone and the conjugate-gradient baseline, at kappa and at
    10 kappa (the paper states that 10x kappa nearly doubles the CG cost and
    leaves the direct step unchanged).  Per-stage times per frame (Table 1
    columns) and CG products per iteration."""
    from paper_2312_02999_amd import FP64, GSTEP_PCG, GSTEP_SCHUR, GSTEP_SCHUR_WOODBURY
    rows = []
    for kappa in (kappa0, 10.0 * kappa0):
        for name, gm in (("schur+low-rank update (the method)", GSTEP_SCHUR_WOODBURY),
                         ("schur complement only", GSTEP_SCHUR), ("PCG baseline (Eq. 5)", GSTEP_PCG)):
            r = run_precision(sc, FP64, steps, warmup, families=False, global_method=gm, kappa=kappa)
            rows.append({"config": name, "kappa": kappa, "frames_per_s": round(r["fps"], 3),
                         "ms_per_frame": round(r["ms_per_frame"], 2), "stage_ms": r["stage_ms"],
                         "n_c_mean": round(r["n_c_mean"], 1), "n_c_max": r["n_c_max"],
                         "cg_products_per_iteration": round(r["cg_products"] / max(r["iters_total"], 1), 1),
                         "ls_failures": r["ls_failures"]})
            progress(f"table 1: {name} at kappa {kappa:g} done")
    return rows


def summary(r):
    keys = ("n_c_max", "n_c_mean", "contact_iters", "iters_total", "pairs_max", "ls_failures", "refine_steps",
            "refine_fallbacks", "cinv_rebuilds", "near_ties", "stage_ms", "replay_bitwise_equal", "device_bytes")
    out = {"value": round(r["fps"], 3), "ms_per_step": round(r["ms_per_frame"], 3),
           "p50_ms": round(r["p50_ms"], 3), "p99_ms": round(r["p99_ms"], 3)}
    out.update({k: r[k] for k in keys})
    out["n_c_mean"] = round(out["n_c_mean"], 1)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="face50k")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only", choices=["fp64", "mixed"], default=None,
                    help="profile one path only (the JSON line then lacks the other)")
    ap.add_argument("--adjoint", action="store_true",
                    help="time the adjoint on the workload and check it against finite differences")
    ap.add_argument("--serving", type=int, default=0, metavar="REQUESTS",
                    help="replay a Poisson stream of this many requests through the server instead")
    ap.add_argument("--table1", action="store_true",
                    help="time the Table 1 global-step configurations at kappa and 10 kappa instead")
    ap.add_argument("--fp32-reduced-min", type=int, default=None,
                    help="mixed path: smallest reduced system solved with the refined FP32 factor")
    ap.add_argument("--adjoint-params", type=int, default=64,
                    help="with --adjoint: the actuation parameters (largest gradient entries) checked by central "
                         "differences")
    ap.add_argument("--adjoint-h", type=float, default=1e-3,
                    help="with --adjoint: the central-difference step of a single parameter")
    ap.add_argument("--dense", type=int, default=0, metavar="N",
                    help="only factor and solve a seeded N x N SPD system six times through the library's dense "
                         "kernels (for kernel traces and counters of the reduced factorisation alone)")
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
            rep = serve.run_serving(n_requests=args.serving, precision=prec,
                                    on_done=lambda k, n: progress(f"request {k}/{n} done") if k % 8 == 0 else None)
            print(json.dumps({"metric": "serving: request latency and frames/s", **rep}), flush=True)
        return
    sc = mg.scene_by_name(args.workload)
    progress(f"scene {args.workload} generated (n={sc.n}, m={sc.m})")
    if args.adjoint:
        print(json.dumps(run_adjoint(sc, n_params=args.adjoint_params, h_param=args.adjoint_h)))
        return
    if args.dense:
        run_dense(args.dense)
        return
    if args.table1:
        rows = run_table1(sc, args.steps, args.warmup, sc.kappa)
        print(json.dumps({"metric": "Table 1 global-step configurations: frames/s and stage ms per frame",
                          "workload": f"{args.workload}: n={sc.n} m={sc.m}, {sc.iters} iterations/frame, frames "
                                      f"{args.warmup}..{args.warmup + args.steps - 1} of the keyframed sequence",
                          "rows": rows}))
        return
    mixed_kw = {} if args.fp32_reduced_min is None else {"fp32_reduced_min": args.fp32_reduced_min}
    if args.only:
        prec = FP64 if args.only == "fp64" else MIXED_FP32
        r = run_precision(sc, prec, args.steps, args.warmup, **(mixed_kw if prec == MIXED_FP32 else {}))
        r.pop("x_final")
        out = {"only": args.only, **summary(r), "rooflines": rooflines(sc, r, "f64")}
        print(json.dumps(out))
        if args.copy_probe:
            copy_probe()
        return
    fp64 = run_precision(sc, FP64, args.steps, args.warmup)
    mixed = run_precision(sc, MIXED_FP32, args.steps, args.warmup, **mixed_kw)
    # the mixed path with the FP32 reduced factor (refined against FP64
    # residuals) from 2049 unknowns on, for comparison with the default
    mixed32 = run_precision(sc, MIXED_FP32, args.steps, args.warmup, families=False, fp32_reduced_min=2049)
    diag = float(np.linalg.norm(sc.X.max(0) - sc.X.min(0)))
    mixed_vs_fp64 = float(np.abs(mixed["x_final"] - fp64["x_final"]).max() / diag)
    # the mixed path factors the reduced system in FP32 from fp32_reduced_min
    # unknowns on (library default 8192)
    thr = 8192 if args.fp32_reduced_min is None else args.fp32_reduced_min
    red_type = "f32" if 3 * mixed["n_c_mean"] >= thr else "f64"
    roofs_fp64 = rooflines(sc, fp64, "f64")
    roofs_mixed = rooflines(sc, mixed, red_type)
    # the headline's roofline: the mixed path's kernel family with the most
    # time in the timed frames
    dom = max(roofs_mixed, key=lambda e: e["total_ms"])
    roof = {"bound": dom["bound"], "kernel": dom["kernel"], "achieved": dom.get("achieved"),
            "peak": dom.get("peak"), "unit": dom.get("unit"), "frac": dom.get("frac"),
            "traffic": measured_traffic(dom["kernel"], args.workload, "mixed"),
            "avg_us": dom["avg_us"], "intervals": dom["intervals"],
            "work_per_interval": dom.get("work_per_interval"), "per_unit": dom.get("per_unit")}
    if not args.no_cpu_baseline:
        progress("oracle baseline sample")
    cpu = None if args.no_cpu_baseline else cpu_baseline(sc, sc.sequence()[args.warmup])
    seq_len = len(sc.sequence())
    out = {
        "metric": "PD+IPC frames/s on 50k-vert mesh, mixed vs FP64 GPU; p50/p99 latency",
        "value": round(mixed["fps"], 3), "unit": "frames/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(mixed["ms_per_frame"], 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64 (mixed)", "data": "synthetic",
        "config": {"workload": f"{args.workload}: face-like shell n={sc.n} m={sc.m}, {sc.iters} iterations/frame, "
                               f"frames {args.warmup}..{args.warmup + args.steps - 1} of a {seq_len}-frame "
                               f"keyframed actuation sequence (every timed frame changes actuation)",
                   "n": sc.n, "m": sc.m, "n1": fp64["sizes"]["n1"], "n2": fp64["sizes"]["n2"],
                   "factor_nnz": fp64["sizes"]["factor_nnz"],
                   "contact_frac_max": round(mixed["n_c_max"] / sc.n, 4)},
        "p50_ms": round(mixed["p50_ms"], 3), "p99_ms": round(mixed["p99_ms"], 3),
        "fp64": summary(fp64),
        "mixed": {**summary(mixed), "reduced_factor_type": red_type, "max_rel_pos_diff_vs_fp64": mixed_vs_fp64},
        "mixed_fp32_reduced_from_2049": {**summary(mixed32),
                                         "max_rel_pos_diff_vs_fp64": float(np.abs(mixed32["x_final"] - fp64["x_final"]).max() / diag)},
        "roofline": roof,
        "rooflines": {"mixed": roofs_mixed, "fp64": roofs_fp64},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))
    if args.copy_probe:
        copy_probe()


if __name__ == "__main__":
    main()
