"""Continuous-batching frame-solve server on one GPU.

Requests (a mesh plus a sequence of actuation fields) arrive over time.  A
fixed set of slots, each a worker thread with its own HIP stream (default
priority), takes requests in arrival order as soon as a slot is free and the
device-memory budget admits the request's solver; frames of different
requests then run concurrently on their streams.  Solvers (with their
constant factor and inverse Schur complement) stay resident per slot and mesh
and are reused by later requests for the same mesh; idle ones are evicted
least-recently-used when memory is needed.  The library calls release the
Python interpreter lock, so slots overlap on the device.

Results do not depend on the mix: each request runs whole frames on one
solver, and every kernel is deterministic.
"""
from __future__ import annotations

import collections
import dataclasses
import threading
import time
from concurrent.futures import Future

import numpy as np
import torch

from . import FP64, MIXED_FP32, Solver


@dataclasses.dataclass
class Request:
    mesh_key: str
    scene: object
    actuations: list          # per frame: (m,) float64 strength fields
    x0: np.ndarray | None = None
    arrival: float = 0.0
    future: Future = dataclasses.field(default_factory=Future)
    start: float = 0.0
    finish: float = 0.0


def estimate_bytes(scene) -> int:
    """Rough device footprint of a solver before it exists (dominant terms)."""
    n, m = scene.n, scene.m
    n2 = int(np.sum((scene.region == 1) & (scene.dirichlet == 0)))
    per_tet = 8 * (9 + 1 + 6 + 12 + 9 + 4) + 4 * 8
    factor = 16 * 40 * n          # supernodal panels, forward copy and inverses
    n_free = int(np.sum(scene.dirichlet == 0))
    hinv = 8 * n2 * n_free        # rows x2 of H_s^-1, kept within the solver's default 4096 MiB
    if hinv > (4096 << 20):
        hinv = 0
    return int(m * per_tet + n * 200 + 8 * n2 * n2 + hinv + factor + (64 << 20))


class Server:
    """``submit(mesh_key, scene, actuations, x0)`` returns a Future of the list
    of per-frame positions (numpy, n x 3).  ``budget_bytes`` bounds the device
    memory of resident solvers; ``slots`` is the number of concurrent requests."""

    def __init__(self, budget_bytes: int, slots: int = 4, precision: int = MIXED_FP32, iters: int | None = None,
                 device: str = "cuda"):
        self.budget = int(budget_bytes)
        self.precision = precision
        self.iters = iters
        self.device = torch.device(device)
        self.queue: collections.deque[Request] = collections.deque()
        self.lock = threading.Condition()
        self.resident: dict[tuple[int, str], list] = {}     # (slot, mesh) -> [solver, bytes, last_use, busy]
        self.used = 0
        self.stop = False
        self.completed: list[Request] = []
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(slots)]
        self.workers = [threading.Thread(target=self._run, args=(k,), daemon=True) for k in range(slots)]
        for w in self.workers:
            w.start()

    # ------------------------------------------------------------------ API
    def submit(self, mesh_key, scene, actuations, x0=None, arrival=None) -> Future:
        req = Request(mesh_key, scene, list(actuations), x0, time.perf_counter() if arrival is None else arrival)
        with self.lock:
            self.queue.append(req)
            self.lock.notify_all()
        return req.future

    def close(self):
        with self.lock:
            self.stop = True
            self.lock.notify_all()
        for w in self.workers:
            w.join()
        for entry in self.resident.values():
            entry[0].close()
        self.resident.clear()

    # ------------------------------------------------------------- internals
    def _evict_for(self, need: int) -> bool:
        """Free idle resident solvers (LRU) until `need` more bytes fit."""
        while self.used + need > self.budget:
            idle = [(v[2], k) for k, v in self.resident.items() if not v[3]]
            if not idle:
                return False
            _, key = min(idle)
            solver, nbytes, _, _ = self.resident.pop(key)
            solver.close()
            self.used -= nbytes
        return True

    def _acquire(self, slot: int, req: Request):
        """Called with the lock held: a resident solver for this slot, or None."""
        key = (slot, req.mesh_key)
        if key in self.resident:
            entry = self.resident[key]
            entry[3] = True
            entry[2] = time.perf_counter()
            return entry[0]
        need = estimate_bytes(req.scene)
        if need > self.budget:
            req.future.set_exception(MemoryError(f"request needs ~{need} B, budget is {self.budget} B"))
            return False
        if not self._evict_for(need):
            return None
        self.used += need
        self.resident[key] = [None, need, time.perf_counter(), True]
        return "create"

    def _run(self, slot: int):
        stream = self.streams[slot]
        while True:
            with self.lock:
                req = None
                solver = None
                while req is None:
                    if self.stop and not self.queue:
                        return
                    if self.queue:
                        head = self.queue[0]
                        got = self._acquire(slot, head)
                        if got is False:
                            self.queue.popleft()
                            continue
                        if got is not None:
                            req = self.queue.popleft()
                            solver = got
                            break
                    self.lock.wait(timeout=0.05)
            try:
                req.start = time.perf_counter()
                if solver == "create":
                    with torch.cuda.stream(stream):
                        solver = Solver(req.scene, iters=self.iters or req.scene.iters, precision=self.precision,
                                        device=str(self.device), stream=stream)
                    real = solver.device_bytes()
                    with self.lock:
                        entry = self.resident[(slot, req.mesh_key)]
                        self.used += real - entry[1]
                        entry[0], entry[1] = solver, real
                out = self._frames(solver, req, stream)
                req.finish = time.perf_counter()
                req.future.set_result(out)
            except Exception as exc:                      # keep the slot alive
                req.finish = time.perf_counter()
                req.future.set_exception(exc)
            finally:
                with self.lock:
                    entry = self.resident.get((slot, req.mesh_key))
                    if entry is not None:
                        entry[3] = False
                        entry[2] = time.perf_counter()
                        if entry[0] is None:              # creation failed
                            self.used -= entry[1]
                            del self.resident[(slot, req.mesh_key)]
                    self.completed.append(req)
                    self.lock.notify_all()

    def _frames(self, solver, req: Request, stream):
        sc = req.scene
        with torch.cuda.stream(stream):
            R = torch.from_numpy(np.ascontiguousarray(sc.act_R.reshape(-1, 9))).to(self.device)
            x = torch.from_numpy(np.ascontiguousarray(sc.X if req.x0 is None else req.x0)).to(self.device)
            out = []
            for k, a in enumerate(req.actuations):
                at = torch.from_numpy(np.ascontiguousarray(a)).to(self.device)
                solver.set_actuation_scalar(at, R if k == 0 else None)
                x = solver.solve_frame(x)
                out.append(x.cpu().numpy())
            stream.synchronize()
        return out


def latency_report(reqs: list[Request]) -> dict:
    lat = np.array([r.finish - r.arrival for r in reqs]) * 1e3
    frames = sum(len(r.actuations) for r in reqs)
    t0 = min(r.arrival for r in reqs)
    t1 = max(r.finish for r in reqs)
    return {"requests": len(reqs), "frames": frames, "makespan_s": t1 - t0, "frames_per_s": frames / (t1 - t0),
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean())}


def poisson_workload(n_requests: int, rate: float, sizes: list[str], frames: int, seed: int = 0):
    """Arrival offsets (s) and mesh names for a Poisson stream of requests."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, n_requests)
    names = [sizes[i] for i in rng.integers(0, len(sizes), n_requests)]
    return np.cumsum(gaps) - gaps[0], names


def run_serving(n_requests=256, rate=200.0, sizes=("face5k", "face20k", "face50k", "face100k"), frames=10,
                slots=4, budget_gb=64.0, precision=MIXED_FP32, iters=None, seed=0, on_done=None):
    """Replay a Poisson arrival stream against a Server; returns the report.
    on_done(k, n), if given, is called as the k-th request (in submission
    order) has finished."""
    import meshgen as mg
    scenes = {s: mg.scene_by_name(s) for s in sorted(set(sizes))}
    offsets, names = poisson_workload(n_requests, rate, list(sizes), frames, seed)
    srv = Server(int(budget_gb * (1 << 30)), slots=slots, precision=precision, iters=iters)
    t0 = time.perf_counter()
    futs = []
    for off, nm in zip(offsets, names):
        now = time.perf_counter() - t0
        if off > now:
            time.sleep(off - now)
        sc = scenes[nm]
        seq = [sc.actuation_at((t + 1) / frames) for t in range(frames)]
        futs.append(srv.submit(nm, sc, seq, arrival=t0 + off))
    for k, f in enumerate(futs):
        f.result()
        if on_done is not None:
            on_done(k + 1, len(futs))
    rep = latency_report(srv.completed)
    srv.close()
    rep.update({"slots": slots, "rate": rate, "sizes": list(sizes), "precision": "mixed" if precision else "fp64"})
    return rep


if __name__ == "__main__":
    import argparse
    import json
    ap = argparse.ArgumentParser()
    ap.add_argument("--requests", type=int, default=256)
    ap.add_argument("--rate", type=float, default=200.0)
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--frames", type=int, default=10)
    ap.add_argument("--fp64", action="store_true")
    ap.add_argument("--sizes", default="face5k,face20k,face50k,face100k")
    args = ap.parse_args()
    rep = run_serving(args.requests, args.rate, args.sizes.split(","), args.frames, args.slots,
                      precision=FP64 if args.fp64 else MIXED_FP32)
    print(json.dumps(rep))
