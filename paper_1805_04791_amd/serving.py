"""Continuous-batching serving loop over the volume-integral-equation solver.

Requests (a medium, a frequency and 1..k incident waves) arrive as a stream.
The server

* estimates each request's device footprint with the library's own formula
  (vie_footprint_bytes) and admits it only while the admitted total fits the
  HBM budget; requests that do not fit wait, and smaller later requests may
  overtake a large one at the head of the queue;
* keeps plans (contrast + kernel tables + Krylov bases) resident in a small
  cache keyed by (kind, n, omega, medium digest): a request for a cached plan
  skips the precompute;
* runs several workers, each on its own HIP stream, so admitted requests
  overlap on the device; when queued requests share a plan key a worker
  merges their right-hand sides into one fused multi-RHS solve;
* records arrival -> completion latency per request.

The stream's inputs: by default each request's random draws are made on
the host ahead of its arrival time and its arrays (medium, incident fields)
are built on the device by the worker that serves it, on the worker's stream.
With ``--inputs host`` the arrays themselves are generated on the host by a
thread pool (and placed in pinned memory), within a host-memory budget that
also counts the inputs of requests still queued or on the device; when the
budget is spent the feeder waits, and the wait shows in the latency
(measured from the nominal arrival time).

Each right-hand side is solved with the same arithmetic whatever else runs
beside it (per-RHS convergence decisions, fixed-order reductions, tile
choices that do not change the per-pencil arithmetic), so a result is the
same alone and in the mix.

    python -m paper_1805_04791_amd.serving --requests 200 --rate 20
"""

from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import threading
import time
from collections import OrderedDict
from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np


@dataclass
class Request:
    """A solve request.  The arrays may be produced lazily by ``make`` (called
    when the request arrives), which returns (coef, mu, inc)."""
    id: int
    kind: int
    n: int
    omega: float
    nrhs: int
    coef: Optional[np.ndarray] = None       # [9][n][n][n]
    inc: Optional[np.ndarray] = None        # [nrhs][c][n][n][n]
    mu: Optional[np.ndarray] = None
    tol: float = 1e-9
    arrival: float = 0.0                    # seconds from the stream start
    key: str = ""                           # plan key; derived from the medium if empty
    make: Optional[Callable] = None
    full: bool = False
    host_bytes: int = 0                     # input bytes charged to the host budget
    recipe_fn: Optional[Callable] = None    # the request's random draws (device-side inputs)
    recipe: Optional[dict] = None

    def input_bytes(self) -> int:
        """Host bytes of the request's inputs (estimated before they exist)."""
        c = 6 if (self.full or self.mu is not None) else 3
        tensors = 9 * (2 if (self.full or self.mu is not None) else 1)
        return (tensors + self.nrhs * c) * self.n ** 3 * 16

    def release(self):
        self.coef = self.inc = self.mu = None
        self.recipe = None

    def pin(self) -> bool:
        """Move the generated inputs to pinned host memory (torch tensors), so
        that the worker's copies to the device run at full link speed.  When
        pinned memory is exhausted the inputs stay pageable (returns False)."""
        import torch
        conv = lambda a: a if a is None or isinstance(a, torch.Tensor) else torch.from_numpy(
            np.ascontiguousarray(a)).pin_memory()
        try:
            coef, mu, inc = conv(self.coef), conv(self.mu), conv(self.inc)
        except RuntimeError:
            return False
        self.coef, self.mu, self.inc = coef, mu, inc
        return True

    def materialise(self):
        if self.coef is None and self.make is not None:
            self.coef, self.mu, self.inc = self.make()
        self.full = self.mu is not None
        if not self.key:
            h = hashlib.sha1()
            h.update(np.ascontiguousarray(self.coef).view(np.uint8))
            if self.mu is not None:
                h.update(np.ascontiguousarray(self.mu).view(np.uint8))
            self.key = f"{self.kind}:{self.n}:{self.omega!r}:{h.hexdigest()[:16]}"
        return self


def device_inputs(recipe: dict, device):
    """The arrays of a serving recipe evaluated with torch on ``device``:
    coef = I + bump(x) M as [9][n][n][n] and the incident fields
    [nrhs][3][n][n][n], complex128, in the operation order of the host
    generator (the exponentials may differ from NumPy's in the last bit)."""
    import torch
    n = recipe["n"]
    f64, c128 = torch.float64, torch.complex128
    t = torch.as_tensor(recipe["axis"], dtype=f64, device=device)
    X, Y, Z = t.view(1, 1, n), t.view(1, n, 1), t.view(n, 1, 1)
    radius = 0.8
    q = (X * X + Y * Y + Z * Z) / (radius * radius)
    inside = q < 1.0
    qs = torch.where(inside, q, torch.zeros_like(q))
    b = torch.where(inside, torch.exp(1.0 - 1.0 / (1.0 - qs)), torch.zeros_like(q))
    M = torch.as_tensor(np.asarray(recipe["matrix"], dtype=np.complex128), device=device)
    coef = torch.empty((3, 3, n, n, n), dtype=c128, device=device)
    for a in range(3):
        for c in range(3):
            coef[a, c] = b * M[a, c]
            if a == c:
                coef[a, c] += 1.0
    coef = coef.reshape(9, n, n, n)
    nrhs = recipe["nrhs"]
    inc = torch.empty((nrhs, 3, n, n, n), dtype=c128, device=device)
    axis = np.asarray(recipe["axis"])
    for r in range(nrhs):
        w = recipe["waves"][r]
        if recipe["phased"]:
            d = recipe["dirs"][r]
            ex, ey, ez = (torch.as_tensor(np.exp(1j * recipe["omega"] * d[k] * axis), device=device)
                          for k in range(3))
            ph = ez.view(n, 1, 1) * ey.view(1, n, 1) * ex.view(1, 1, n)
            for a in range(3):
                torch.mul(ph, complex(w[a]), out=inc[r, a])
        else:
            for a in range(3):
                inc[r, a].fill_(complex(w[a]))
    return coef, None, inc


@dataclass
class Result:
    id: int
    density: np.ndarray
    stats: list
    arrival: float
    admitted: float
    done: float
    merged_with: List[int] = field(default_factory=list)

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class Admission:
    """Admission control by device footprint (host-only logic)."""

    def __init__(self, budget_bytes: int):
        self.budget = int(budget_bytes)
        self.used = 0
        self.peak = 0
        self.lock = threading.Condition()

    def fits(self, nbytes: int) -> bool:
        return self.used + nbytes <= self.budget or self.used == 0

    def take(self, nbytes: int):
        self.used += nbytes
        self.peak = max(self.peak, self.used)

    def give(self, nbytes: int):
        with self.lock:
            self.used -= nbytes
            self.lock.notify_all()


class PlanCache:
    """Resident plans keyed by request key; a plan is checked out by one worker at a time."""

    def __init__(self, capacity: int):
        self.capacity = capacity
        self.free: "OrderedDict[str, object]" = OrderedDict()
        self.lock = threading.Lock()
        self.hits = 0
        self.misses = 0

    def get(self, key: str):
        with self.lock:
            plan = self.free.pop(key, None)
            if plan is None:
                self.misses += 1
            else:
                self.hits += 1
            return plan

    def put(self, key: str, plan):
        with self.lock:
            if self.capacity <= 0:
                plan.close()
                return
            old = self.free.pop(key, None)
            if old is not None:
                old.close()
            self.free[key] = plan
            while len(self.free) > self.capacity:
                _, victim = self.free.popitem(last=False)
                victim.close()

    def clear(self):
        with self.lock:
            for p in self.free.values():
                p.close()
            self.free.clear()


class Server:
    def __init__(self, budget_bytes: Optional[int] = None, workers: int = 3, restart: int = 20,
                 max_batch: int = 16, plan_cache: int = 4, precision: Optional[int] = None,
                 keep_results: bool = True, gen_workers: int = 8, host_budget_bytes: int = 32 * 10 ** 9,
                 pinned_inputs: bool = False, device_inputs: bool = True, progress: int = 0):
        import torch
        from . import vie
        self.vie = vie
        self.torch = torch
        if budget_bytes is None:
            free, total = torch.cuda.mem_get_info()
            budget_bytes = int(0.7 * free)
        self.admission = Admission(budget_bytes)
        self.cache = PlanCache(plan_cache)
        self.workers = workers
        self.restart = restart
        self.max_batch = max_batch
        self.precision = vie.PREC_MIXED if precision is None else precision
        self.queue: List[Request] = []
        self.qlock = threading.Condition()
        self.results: List[Result] = []
        self.rlock = threading.Lock()
        self.t0 = time.perf_counter()
        self.closed = False
        self.inflight = 0
        self.max_inflight = 0
        self.errors: List[str] = []
        self.keep_results = keep_results
        self.pinned_inputs = pinned_inputs
        self.pin_fallbacks = 0
        # requests carrying a recipe are drawn on the host and built on the
        # device by their worker (no host copy of the arrays)
        self.device_inputs = device_inputs
        self.progress = progress  # a line on stderr every `progress` finished requests (0: none)
        self.device = torch.device("cuda")
        self.gen_workers = gen_workers
        self.host = Admission(host_budget_bytes)
        self.feeder_late = 0.0
        self.plan_s = 0.0       # summed over workers: plan creation (contrast, tables)
        self.solve_s = 0.0      # and the solves

    # ---- footprint -----------------------------------------------------------
    def footprint(self, reqs: List[Request]) -> int:
        r = reqs[0]
        nb = min(self.max_batch, sum(q.nrhs for q in reqs))
        fp = self.vie.footprint_bytes(r.kind, r.n, r.full, nb, self.restart)
        # inputs and outputs of the merged batch
        fp += 2 * sum(q.nrhs * (6 if q.full else 3) * q.n ** 3 * 16 for q in reqs)
        return int(fp)

    # ---- stream ----------------------------------------------------------------
    def now(self) -> float:
        return time.perf_counter() - self.t0

    def submit(self, req: Request):
        with self.qlock:
            self.queue.append(req)
            self.qlock.notify_all()

    def _take(self):
        """Oldest admissible request plus queued requests with the same key."""
        with self.qlock:
            while True:
                if self.closed and not self.queue:
                    return None, 0
                for i, r in enumerate(self.queue):
                    group = [r] + [q for q in self.queue[i + 1:] if q.key == r.key]
                    nb = 0
                    sel = []
                    for q in group:
                        if nb + q.nrhs > self.max_batch and sel:
                            break
                        sel.append(q)
                        nb += q.nrhs
                    fp = self.footprint(sel)
                    with self.admission.lock:
                        if self.admission.fits(fp):
                            self.admission.take(fp)
                            for q in sel:
                                self.queue.remove(q)
                            self.inflight += 1
                            self.max_inflight = max(self.max_inflight, self.inflight)
                            return sel, fp
                # nothing fits: wait for a release or an arrival
                self.qlock.wait(timeout=0.05)

    def _worker(self):
        torch = self.torch
        vie = self.vie
        stream = torch.cuda.Stream()
        while True:
            sel, fp = self._take()
            if sel is None:
                return
            admitted = self.now()
            try:
                with torch.cuda.stream(stream):
                    for q in sel:
                        if q.coef is None and q.recipe is not None:
                            q.coef, q.mu, q.inc = device_inputs(q.recipe, self.device)
                    r = sel[0]
                    plan = self.cache.get(r.key)
                    t_plan = time.perf_counter()
                    if plan is None:
                        # worker threads allocate and synchronise while others
                        # solve, which stream capture would forbid
                        plan = vie.Plan(r.kind, r.coef, omega=r.omega, mu=r.mu, precision=self.precision,
                                        max_rhs=self.max_batch, stream=stream, graphs=False)
                        stream.synchronize()
                    t_solve = time.perf_counter()
                    if len(sel) == 1:
                        inc = sel[0].inc
                    elif isinstance(sel[0].inc, torch.Tensor):
                        inc = torch.cat([q.inc for q in sel])
                    else:
                        inc = np.concatenate([q.inc for q in sel])
                    dens, _, stats, rc = plan.solve(inc, tol=min(q.tol for q in sel), restart=self.restart,
                                                    want_field=False, stream=stream)
                    dens = dens.cpu().numpy() if self.keep_results else None
                    stream.synchronize()
                    t_end = time.perf_counter()
                    self.cache.put(r.key, plan)
                    with self.rlock:
                        self.plan_s += t_solve - t_plan
                        self.solve_s += t_end - t_solve
                done = self.now()
                off = 0
                with self.rlock:
                    for q in sel:
                        k = q.nrhs
                        self.results.append(Result(q.id, dens[off:off + k] if dens is not None else None,
                                                   stats[off:off + k], q.arrival, admitted, done,
                                                   [o.id for o in sel if o.id != q.id]))
                        off += k
                        if self.progress and len(self.results) % self.progress == 0:
                            print(f"[serve] {len(self.results)} requests done at {done:.1f} s", file=sys.stderr,
                                  flush=True)
            except Exception as exc:  # keep serving; report at the end
                self.errors.append(f"request {sel[0].id}: {exc}")
            finally:
                for q in sel:
                    q.release()
                    self.host.give(q.host_bytes)
                self.admission.give(fp)
                with self.qlock:
                    self.inflight -= 1
                    self.qlock.notify_all()

    def _prepare(self, r: Request):
        if self.device_inputs and r.recipe_fn is not None:
            r.recipe = r.recipe_fn()
            return r
        r.materialise()
        if self.pinned_inputs and not r.pin():
            with self.rlock:
                self.pin_fallbacks += 1
        return r

    def run(self, stream_of: Callable[[], List[Request]], realtime: bool = True) -> List[Result]:
        """Feed the requests at their arrival times (or all at once) and serve them.

        Inputs are generated ahead by a thread pool while the host budget
        allows; request i itself waits for budget (freed as earlier requests
        finish) before it is generated."""
        from concurrent.futures import ThreadPoolExecutor
        reqs = sorted(stream_of(), key=lambda r: r.arrival)
        threads = [threading.Thread(target=self._worker, daemon=True) for _ in range(self.workers)]
        pool = ThreadPoolExecutor(max_workers=max(1, self.gen_workers))
        futures = {}
        nxt = 0

        def start(j: int, block: bool) -> bool:
            r = reqs[j]
            b = 0 if (self.device_inputs and r.recipe_fn is not None) else r.input_bytes()
            with self.host.lock:
                while not self.host.fits(b):
                    if not block:
                        return False
                    self.host.lock.wait(timeout=0.05)
                self.host.take(b)
            r.host_bytes = b
            futures[j] = pool.submit(self._prepare, r)
            return True

        self.t0 = time.perf_counter()
        for t in threads:
            t.start()
        try:
            for i, r in enumerate(reqs):
                if nxt == i:
                    start(i, True)
                    nxt += 1
                while nxt < len(reqs) and nxt - i <= 4 * max(1, self.gen_workers) and start(nxt, False):
                    nxt += 1
                futures.pop(i).result()
                if realtime:
                    delay = r.arrival - self.now()
                    if delay > 0:
                        time.sleep(delay)
                    self.feeder_late = max(self.feeder_late, -delay)
                else:
                    r.arrival = self.now()
                self.submit(r)
        finally:
            pool.shutdown(wait=True)
            with self.qlock:
                self.closed = True
                self.qlock.notify_all()
            for t in threads:
                t.join()
            self.cache.clear()
        return sorted(self.results, key=lambda x: x.id)

    def summary(self, results: List[Result]) -> dict:
        lat = np.array([r.latency for r in results]) if results else np.zeros(1)
        span = max((r.done for r in results), default=0.0) - min((r.arrival for r in results), default=0.0)
        nrhs = sum(len(r.stats) for r in results)
        conv = sum(1 for r in results for s in r.stats if s["status"] == 0)
        return {"requests": len(results), "rhs_solved": nrhs, "rhs_converged": conv,
                "solves_per_s": nrhs / span if span > 0 else None,
                "requests_per_s": len(results) / span if span > 0 else None,
                "latency_p50_ms": 1e3 * float(np.percentile(lat, 50)),
                "latency_p99_ms": 1e3 * float(np.percentile(lat, 99)),
                "latency_max_ms": 1e3 * float(lat.max()),
                "max_inflight": self.max_inflight, "peak_admitted_GB": self.admission.peak / 1e9,
                "budget_GB": self.admission.budget / 1e9, "plan_cache_hits": self.cache.hits,
                "host_peak_GB": self.host.peak / 1e9, "feeder_late_max_s": self.feeder_late,
                "worker_plan_s": self.plan_s, "worker_solve_s": self.solve_s,
                "pinned_fallbacks": self.pin_fallbacks, "device_inputs": self.device_inputs,
                "errors": self.errors[:5]}


def requests_from_generator(count: int, rate: float, grids=None, max_rhs: int = 16) -> List[Request]:
    """The seeded serving stream (Poisson arrivals; Laplace / Helmholtz / Maxwell mix).

    Media and incident fields are generated when each request arrives; every
    request has its own medium (key = its seed)."""
    from vie_inputs import generators as gen
    grids = grids or gen.SERVING_GRIDS
    out = []
    for rq in gen.serving_requests(count, rate, grids, max_rhs):
        def make(rq=rq):
            p = gen.serving_problem(rq)
            return p.coef, p.mu, p.inc
        out.append(Request(rq["id"], rq["kind"], rq["n"], rq["omega"], rq["nrhs"], arrival=rq["arrival"],
                           key=f"req{rq['item']}", make=make,
                           recipe_fn=lambda rq=rq: gen.serving_recipe(rq)))
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--requests", type=int, default=200)
    ap.add_argument("--rate", type=float, default=20.0, help="Poisson arrival rate (requests/s)")
    ap.add_argument("--grids", type=str, default="32,48,64,96,128,160")
    ap.add_argument("--max-rhs", type=int, default=16)
    ap.add_argument("--workers", type=int, default=3)
    ap.add_argument("--budget-gb", type=float, default=0.0)
    ap.add_argument("--host-budget-gb", type=float, default=24.0, help="host memory for generated inputs")
    ap.add_argument("--gen-workers", type=int, default=8, help="threads generating the stream's inputs")
    ap.add_argument("--pageable", action="store_true", help="keep the generated inputs in pageable memory")
    ap.add_argument("--inputs", choices=("device", "host"), default="device",
                    help="build each request's arrays on the device from its random draws, or on the host")
    args = ap.parse_args(argv)
    grids = tuple(int(g) for g in args.grids.split(","))
    t = time.perf_counter()
    reqs = requests_from_generator(args.requests, args.rate, grids, args.max_rhs)
    print(f"[serve] generated {len(reqs)} requests in {time.perf_counter() - t:.1f} s", file=sys.stderr, flush=True)
    srv = Server(int(args.budget_gb * 1e9) if args.budget_gb > 0 else None, workers=args.workers,
                 keep_results=False, gen_workers=args.gen_workers,
                 host_budget_bytes=int(args.host_budget_gb * 1e9), pinned_inputs=not args.pageable,
                 device_inputs=args.inputs == "device", progress=100)
    res = srv.run(lambda: reqs)
    out = srv.summary(res)
    out.update({"rate": args.rate, "grids": list(grids), "workers": args.workers})
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
