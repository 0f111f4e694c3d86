"""Request server for SBD matvecs and GMRES solves on one GPU.

Each request brings its own point set (off-line part: ``sbd_plan``) and either
a right-hand side f (on-line part: one ``sbd_apply``) or a single-layer
system to solve with GMRES (``sbd_gmres``, one plan, many applies).  Requests
are admitted in arrival order while their estimated device footprint fits the
HBM budget; a pool of worker threads, each with its own HIP stream, keeps
several requests in flight so that the host-side fit of one overlaps the
kernels of another.  Fits are shared between plans (``fit_reuse``), since the
fit only depends on the kernel, eps and the annulus ratio a, and are made once at
start-up for every ratio the request sizes can need (``prefit_table``).  A GMRES solve is
planned at min(eps, rtol): the Krylov iteration converges to rtol only on an
operator that accurate (a coarser operator stalls it for many more steps);
inside the solve the library replays each Arnoldi step as a captured HIP graph.
Finished plans are released by a separate thread, so that the device-wide wait
of freeing device memory never holds a worker, into the library's large-block
cache (``sbd_set_cache_limit``), from which later plans take their memory.

Latency of a request = completion time - arrival time, including host-device
copies of its inputs and outputs.
"""
from __future__ import annotations

import math
import queue
import threading
import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Request:
    rid: int
    kind: str                      # "apply" or "gmres"
    points: np.ndarray             # [N, 2] FP64
    eps: float
    f: np.ndarray | None = None    # apply: [N] or [nrhs, N] FP64
    b: np.ndarray | None = None    # gmres: right-hand side [N]
    weights: np.ndarray | None = None
    diag: np.ndarray | None = None
    rtol: float = 1e-6
    arrival: float = 0.0           # set by the server (perf_counter seconds)


@dataclass
class Result:
    rid: int
    kind: str
    n: int
    eps: float
    precision: int
    arrival: float
    start: float
    planned: float
    finish: float
    iterations: int = 0
    relres: float = 0.0
    plan_bytes: int = 0
    out: np.ndarray | None = None
    error: str = ""

    @property
    def latency(self) -> float:
        return self.finish - self.arrival


def single_layer_diag(weights: np.ndarray) -> np.ndarray:
    """Self-panel term of the single-layer operator: the integral of
    -(1/2 pi) log|s| over a straight panel |s| <= w/2."""
    return -weights / (2 * math.pi) * (np.log(weights / 2) - 1.0)


def precision_for(req: Request) -> int:
    """FP64 far field for tight tolerances and for iterative solves, FP32 otherwise."""
    return 1 if (req.eps < 1e-4 or req.kind == "gmres") else 0


def plan_eps(req: Request) -> float:
    """Operator tolerance of a request's plan: its eps, tightened to the solve's rtol for GMRES."""
    return min(req.eps, req.rtol) if req.kind == "gmres" else req.eps


def footprint_estimate(n: int, eps: float, precision: int) -> int:
    """Conservative device bytes of one request before its plan exists (refined after planning)."""
    neigh = 40.0 * abs(math.log(eps)) ** (2 / 3) * n ** (1 / 3)
    grid = 64.0 * (abs(math.log(eps)) * n ** (2 / 3)) ** 2 * (2 if precision else 1)
    return int(n * (96 + 12 * neigh) + grid + (64 << 20))


class _Budget:
    def __init__(self, total: int):
        self.total = total
        self.used = 0
        self.cv = threading.Condition()

    def acquire(self, nbytes: int):
        nbytes = min(nbytes, self.total)
        with self.cv:
            while self.used + nbytes > self.total:
                self.cv.wait()
            self.used += nbytes
        return nbytes

    def adjust(self, held: int, actual: int) -> int:
        actual = min(actual, self.total)
        with self.cv:
            self.used += actual - held
            self.cv.notify_all()
        return actual

    def release(self, nbytes: int):
        with self.cv:
            self.used -= nbytes
            self.cv.notify_all()


class Server:
    """Worker pool serving Requests on cuda:0."""

    def __init__(self, workers: int = 4, hbm_budget: int | None = None, keep_outputs: bool = False,
                 cache_bytes: int = 48 << 30):
        import torch
        import paper_1711_07877_amd as sbd
        self.sbd = sbd
        self.torch = torch
        self.dev = torch.device("cuda:0")
        # released plan memory is kept for the next plans (sbd_set_cache_limit): freshly
        # allocated device memory costs the driver time in proportion to its volume
        sbd.sbd_set_cache_limit(cache_bytes)
        if hbm_budget is None:
            free, _ = torch.cuda.mem_get_info(self.dev)
            hbm_budget = max(int(free * 0.8) - cache_bytes, 1 << 30)
        self.budget = _Budget(hbm_budget)
        self.keep_outputs = keep_outputs
        self.q: queue.Queue = queue.Queue()
        self.results: list[Result] = []
        self.lock = threading.Lock()
        self.threads = [threading.Thread(target=self._worker, daemon=True) for _ in range(workers)]
        for t in self.threads:
            t.start()
        self.reap_q: queue.Queue = queue.Queue()
        self.reaper = threading.Thread(target=self._reap, daemon=True)
        self.reaper.start()

    # -- client side
    def submit(self, req: Request):
        req.arrival = time.perf_counter()
        self.q.put(req)

    def close(self):
        for _ in self.threads:
            self.q.put(None)
        for t in self.threads:
            t.join()
        self.reap_q.put(None)
        self.reaper.join()
        # back to plain device-synchronising frees for whoever uses the library next
        self.sbd.sbd_set_cache_limit(0)

    def _reap(self):
        """Frees finished plans (their streams are synchronised) and returns their bytes."""
        while True:
            item = self.reap_q.get()
            if item is None:
                return
            plan, held = item
            try:
                plan.free()
            finally:
                self.budget.release(held)

    def run_serial(self, requests: list[Request]) -> list[Result]:
        """One request at a time (each submitted when the previous one has finished): service times
        without queueing or overlap."""
        start = len(self.results)
        for i, r in enumerate(requests):
            self.submit(r)
            while True:
                with self.lock:
                    if len(self.results) - start > i:
                        break
                time.sleep(0.0005)
        return self.results[start:]

    def run_stream(self, requests: list[Request], gaps: list[float] | None) -> list[Result]:
        """Submit requests at cumulative inter-arrival gaps (seconds; None = all at once), wait for all."""
        start = len(self.results)
        t0 = time.perf_counter()
        due = 0.0
        for i, r in enumerate(requests):
            if gaps is not None:
                due += gaps[i]
                dt = t0 + due - time.perf_counter()
                if dt > 0:
                    time.sleep(dt)
            self.submit(r)
        while True:
            with self.lock:
                if len(self.results) - start >= len(requests):
                    return self.results[start:]
            time.sleep(0.001)

    # -- worker side
    def _worker(self):
        torch = self.torch
        stream = torch.cuda.Stream(device=self.dev)
        while True:
            req = self.q.get()
            if req is None:
                return
            try:
                res = self._serve(req, stream)
            except Exception as e:  # the request fails, the server keeps going
                now = time.perf_counter()
                res = Result(req.rid, req.kind, len(req.points), req.eps, precision_for(req), req.arrival, now, now,
                             now, error=str(e))
            with self.lock:
                self.results.append(res)

    def _serve(self, req: Request, stream) -> Result:
        torch, sbd = self.torch, self.sbd
        n = len(req.points)
        prec = precision_for(req)
        eps = plan_eps(req)
        held = self.budget.acquire(footprint_estimate(n, eps, prec))
        start = time.perf_counter()
        plan = None
        try:
            with torch.cuda.stream(stream):
                pts = torch.from_numpy(np.ascontiguousarray(req.points)).to(self.dev)
                plan = sbd.sbd_plan(pts, eps=eps, precision=prec, fit_reuse=1,
                                    max_rhs=1 if req.f is None or req.f.ndim == 1 else req.f.shape[0],
                                    stream=stream)
                planned = time.perf_counter()
                if req.kind == "apply":
                    ws_bytes = plan.workspace_bytes(plan.max_rhs)
                else:
                    ws_bytes = plan.workspace_bytes(1) + plan.gmres_workspace_bytes(30)
                held = self.budget.adjust(held, plan.plan_bytes() + ws_bytes + 64 * n)
                its, rel = 0, 0.0
                if req.kind == "apply":
                    ft = torch.from_numpy(np.ascontiguousarray(np.atleast_2d(req.f))).to(self.dev)
                    out = plan.apply(ft, stream=stream)
                else:
                    bt = torch.from_numpy(req.b).to(self.dev)
                    wt = torch.from_numpy(req.weights).to(self.dev) if req.weights is not None else None
                    dt = torch.from_numpy(req.diag).to(self.dev) if req.diag is not None else None
                    out, its, rel = plan.gmres(bt, weights=wt, diag=dt, rtol=req.rtol, stream=stream, check=False)
                host = out.to("cpu", non_blocking=False)
                stream.synchronize()
                pb = plan.plan_bytes()
        except BaseException:
            if plan is not None:
                plan.free()
            self.budget.release(held)
            raise
        finish = time.perf_counter()
        self.reap_q.put((plan, held))
        return Result(req.rid, req.kind, n, req.eps, prec, req.arrival, start, planned, finish, its, rel, pb,
                      host.numpy() if self.keep_outputs else None)


def prefit_table(eps_values, nmin: float, nmax: float, threads: int = 4) -> dict:
    """Fit once, at start-up, every annulus-ratio bucket that requests of N in [nmin, nmax]
    can need, into the library's shared fit cache (sbd_prefit).  The fit depends on the
    kernel, eps and a = delta_min / delta_max only (Section 1, off-line part), and the
    default delta_min rule gives a = |ln eps|^(2/3) / N^(2/3) whatever the curve, so a
    request never waits for a fit.  Buckets are a' = 2^(k/8); each is fitted at its
    midpoint 2^((k + 1/2) / 8), which the cache files under a'."""
    import concurrent.futures as cf
    import paper_1711_07877_amd as sbd
    jobs = []
    for eps in sorted(set(eps_values)):
        c = abs(math.log(eps)) ** (2.0 / 3.0)
        k_lo = math.floor(8.0 * math.log2(c / nmax ** (2.0 / 3.0)))
        k_hi = math.floor(8.0 * math.log2(c / nmin ** (2.0 / 3.0)))
        jobs += [(eps, 2.0 ** ((k + 0.5) / 8.0)) for k in range(k_lo, k_hi + 1) if 2.0 ** ((k + 0.5) / 8.0) < 1.0]
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        orders = list(ex.map(lambda j: sbd.sbd_prefit(j[0], j[1]), jobs))
    return {"fits": len(jobs), "seconds": round(time.perf_counter() - t0, 2), "max_P": max(orders) if orders else 0}


def make_stream(count: int, seed: int = 5, nmin: float = 1e3, nmax: float = 1e6) -> tuple[list[Request], list[float]]:
    """The serving workload: log-uniform N on random closed curves, eps in {1e-3, 1e-6},
    half applies (f ~ N(0,1)) and half GMRES(30) single-layer solves to 1e-6.
    Returns the requests and their unit-mean exponential inter-arrival gaps."""
    import synth
    reqs, gaps = [], []
    for i, s in enumerate(synth.request_stream(count, seed, nmin, nmax)):
        z = synth.serving_curve(s["n"], s["curve_seed"])
        if s["kind"] == "apply":
            f = synth.real_rhs(s["n"], s["curve_seed"] % 100000)[0]
            reqs.append(Request(i, "apply", z, s["eps"], f=f))
        else:
            w = synth.curve_weights(z)
            b = -np.log(np.hypot(z[:, 0] - 2.0, z[:, 1] - 2.0)) / (2 * math.pi)
            reqs.append(Request(i, "gmres", z, s["eps"], b=b, weights=w, diag=single_layer_diag(w)))
        gaps.append(s["gap"])
    return reqs, gaps


def percentiles(results: list[Result], service: bool = False) -> dict:
    """Latency (completion - arrival) percentiles; service=True uses completion - start."""
    lat = np.array([(r.finish - r.start) if service else r.latency for r in results if not r.error])
    if lat.size == 0:
        return {"p50_ms": None, "p99_ms": None, "mean_ms": None, "errors": len(results)}
    return {"p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 2),
            "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 2),
            "mean_ms": round(float(lat.mean()) * 1e3, 2),
            "errors": sum(1 for r in results if r.error)}


def main(argv=None):
    """Serve the synthetic request stream and print one JSON line of latency figures:
    the start-up fit table, an isolated serial pass (service times), a saturation pass
    (all requests at once), and Poisson arrivals at 0.5 / mean service time and at
    0.9 x the saturation throughput."""
    import argparse
    import json
    import sys
    ap = argparse.ArgumentParser()
    ap.add_argument("--requests", type=int, default=512)
    ap.add_argument("--workers", type=int, default=4)
    ap.add_argument("--seed", type=int, default=5)
    args = ap.parse_args(argv)
    t0 = time.perf_counter()
    reqs, gaps = make_stream(args.requests, seed=args.seed)
    print(f"generated {len(reqs)} requests in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    table = prefit_table({plan_eps(r) for r in reqs}, 1e3, 1e6)
    print(f"fit table: {table}", file=sys.stderr, flush=True)
    srv = Server(workers=args.workers)
    iso = srv.run_serial(reqs)
    tbar = float(np.mean([r.finish - r.start for r in iso]))
    print(f"isolated: mean service {tbar * 1e3:.1f} ms", file=sys.stderr, flush=True)
    t1 = time.perf_counter()
    sat = srv.run_stream(reqs, None)
    sat_rps = len(reqs) / (max(r.finish for r in sat) - t1)
    print(f"saturation: {sat_rps:.2f} req/s", file=sys.stderr, flush=True)
    out = {"requests": len(reqs), "workers": args.workers, "seed": args.seed, "fit_table": table,
           "isolated_mean_service_ms": round(tbar * 1e3, 2),
           "isolated_service": percentiles(iso, service=True),
           "saturation_req_per_s": round(sat_rps, 3),
           "errors": sum(1 for r in iso + sat if r.error)}
    for label, rate in (("poisson_half_load", 0.5 / tbar), ("poisson_0.9_saturation", 0.9 * sat_rps)):
        res = srv.run_stream(reqs, [g / rate for g in gaps])
        out[label] = dict(rate_req_per_s=round(rate, 3), **percentiles(res))
        print(f"{label}: " + json.dumps(out[label]), file=sys.stderr, flush=True)
        for msg in sorted({r.error for r in res if r.error})[:3]:
            print(f"  error: {msg}", file=sys.stderr, flush=True)
    srv.close()
    for kind in ("apply", "gmres"):
        for eps in (1e-3, 1e-6):
            sel = [r for r in iso if r.kind == kind and r.eps == eps and not r.error]
            if sel:
                out[f"isolated_{kind}_eps{eps:g}"] = {
                    "count": len(sel), "mean_n": int(np.mean([r.n for r in sel])),
                    "mean_service_ms": round(float(np.mean([r.finish - r.start for r in sel])) * 1e3, 2),
                    "mean_plan_ms": round(float(np.mean([r.planned - r.start for r in sel])) * 1e3, 2),
                    "mean_iterations": round(float(np.mean([r.iterations for r in sel])), 1)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
