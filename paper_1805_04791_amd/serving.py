"""Continuous-batching serving loop over the volume-integral-equation solver.

Requests (a medium, a frequency and 1..k incident waves) arrive as a stream.
The server

* keeps plans (contrast, kernel tables, Krylov workspace) resident in a
  cache keyed by (kind, n, omega, medium digest); a request for a cached
  plan skips the precompute;
* serves each plan key with one worker on its own HIP stream: the worker
  opens a batch of solver slots on the plan (the library's vie_batch_*
  calls) and, at every cycle boundary of the running solve, lets queued
  requests with the same key join the free slots; finished right-hand sides
  leave at once and a request completes when all of its right-hand sides
  have; different keys are served by other workers at the same time, so
  their work overlaps on the device;
* admits by device footprint (the library's own formula, vie_footprint_bytes):
  every resident plan (serving or cached) and the input/output arrays of the
  admitted requests count against the HBM budget; idle cached plans are
  evicted (least recently used first) when a new plan needs the room, and a
  request whose plan alone exceeds the budget is refused with an error;
* records arrival -> completion latency per request, and counts the joins
  into running solves and the plan-cache hits.

The stream's inputs: by default each request's random draws are made on
the host ahead of its arrival time and its arrays (medium, incident fields)
are built on the device by the worker that serves it, on the worker's stream.
With ``--inputs host`` the arrays themselves are generated on the host by a
thread pool (and placed in pinned memory), within a host-memory budget that
also counts the inputs of requests still queued or on the device; when the
budget is spent the feeder waits, and the wait shows in the latency
(measured from the nominal arrival time).

Each right-hand side is solved with the same arithmetic whatever else runs
beside it (per-slot decisions, fixed-order reductions, tile choices that do
not change the per-pencil arithmetic), so a result is bitwise the same alone
and in the mix, whenever it joins.

    python -m paper_1805_04791_amd.serving --requests 200 --rate 20 [--media 8]
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
from collections import Counter, OrderedDict
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
    density: Optional[np.ndarray]
    stats: list
    arrival: float
    admitted: float
    done: float
    joined_running: bool = False   # joined a batch while other right-hand sides were iterating
    error: str = ""

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class Admission:
    """Admission control by device footprint (host-only logic).  A request is
    admitted only while the admitted total stays within the budget; nothing
    larger than the budget is ever admitted."""

    def __init__(self, budget_bytes: int):
        self.budget = int(budget_bytes)
        self.used = 0
        self.peak = 0
        self.lock = threading.Condition()

    def fits(self, nbytes: int) -> bool:
        return self.used + nbytes <= self.budget

    def can_ever_fit(self, nbytes: int) -> bool:
        return nbytes <= self.budget

    def take(self, nbytes: int):
        self.used += nbytes
        self.peak = max(self.peak, self.used)

    def give(self, nbytes: int):
        with self.lock:
            self.used -= nbytes
            self.lock.notify_all()


class PlanCache:
    """Idle resident plans keyed by request key, least recently used first; a
    plan is checked out by one worker at a time.  Each entry remembers the
    device bytes charged for it, released to ``on_evict`` when it is closed."""

    def __init__(self, capacity: int, on_evict: Optional[Callable[[int], None]] = None):
        self.capacity = capacity
        self.free: "OrderedDict[str, tuple]" = OrderedDict()
        self.lock = threading.Lock()
        self.hits = 0
        self.misses = 0
        self.on_evict = on_evict

    def _close(self, entries):
        # outside self.lock: on_evict takes the admission lock, which callers
        # may hold while they ask this cache for room
        for plan, nbytes in entries:
            plan.close()
            if self.on_evict:
                self.on_evict(nbytes)

    def get(self, key: str):
        """(plan, charged bytes) or None."""
        with self.lock:
            entry = self.free.pop(key, None)
            if entry is None:
                self.misses += 1
            else:
                self.hits += 1
            return entry

    def contains(self, key: str) -> bool:
        with self.lock:
            return key in self.free

    def peek(self, key: str):
        """The idle entry of `key` without checking it out (or None)."""
        with self.lock:
            return self.free.get(key)

    def put(self, key: str, plan, nbytes: int = 0):
        victims = []
        with self.lock:
            if self.capacity <= 0:
                victims.append((plan, nbytes))
            else:
                old = self.free.pop(key, None)
                if old is not None:
                    victims.append(old)
                self.free[key] = (plan, nbytes)
                while len(self.free) > self.capacity:
                    victims.append(self.free.popitem(last=False)[1])
        self._close(victims)

    def evict_one(self, keep: str = "") -> bool:
        """Closes the least recently used idle plan (not `keep`); False if none."""
        victim = None
        with self.lock:
            for k in list(self.free.keys()):
                if k != keep:
                    victim = self.free.pop(k)
                    break
        if victim is None:
            return False
        self._close([victim])
        return True

    def clear(self):
        with self.lock:
            victims = list(self.free.values())
            self.free.clear()
        self._close(victims)


class Server:
    def __init__(self, budget_bytes: Optional[int] = None, workers: int = 3, restart: int = 20,
                 max_batch: int = 16, plan_cache: int = 16, precision: Optional[int] = None,
                 keep_results: bool = True, gen_workers: int = 8, host_budget_bytes: int = 32 * 10 ** 9,
                 pinned_inputs: bool = False, device_inputs: bool = True, progress: int = 0,
                 tol: float = 1e-9, overtake_s: float = 2.0):
        import torch
        from . import vie
        self.vie = vie
        self.torch = torch
        if budget_bytes is None:
            free, total = torch.cuda.mem_get_info()
            budget_bytes = int(0.7 * free)
        self.admission = Admission(budget_bytes)
        self.cache = PlanCache(plan_cache, on_evict=self.admission.give)
        self.workers = workers
        self.restart = restart
        self.max_batch = max_batch
        self.tol = tol
        self.precision = vie.PREC_MIXED if precision is None else precision
        self.queue: List[Request] = []
        self.qlock = threading.Condition()
        self.serving = set()          # keys whose batch is open on some worker
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
        self.solve_s = 0.0      # and the batched solves
        self.plans_created = 0
        self.joins = 0          # right-hand sides added to a batch
        self.joins_running = 0  # ... while other right-hand sides of the batch were iterating
        self.batches = 0
        self.refused = 0
        # a younger request may be admitted ahead of an older one that does not
        # fit yet, until the older one has waited this long since its arrival
        self.overtake_s = overtake_s
        self.overtakes = 0
        self.seen = set()  # keys served before
        self.running = 0   # workers with an open batch
        self.repeats = set()  # keys claimed more than once
        self.closed_after_use = 0  # plans of one-off keys closed at once instead of cached
        self.returned_bytes = 0  # estimate minus resident bytes, given back after plan creation

    # ---- footprint -----------------------------------------------------------
    def plan_bytes(self, r: Request, slots: Optional[int] = None) -> int:
        """Device bytes of a new plan with a batch of `slots` (default
        max_batch) slots: an upper estimate from the grid alone."""
        nb = self.max_batch if slots is None else slots
        return int(self.vie.footprint_bytes(r.kind, r.n, r.full, nb, self.restart))

    def creation_bytes(self, r: Request) -> int:
        """Device bytes of creating a plan (the kernel-table precompute at its
        peak, or the plan with one solver slot): charged before the plan
        exists; its batch is charged once the plan knows its support."""
        return int(self.vie.footprint_bytes(r.kind, r.n, r.full, 1, 1))

    def batch_bytes(self, plan, r: Request, slots: int) -> int:
        """Device bytes that opening a batch of `slots` slots adds to a new
        plan: the Krylov vectors on the plan's support rows (basis of restart
        + 1 vectors, iterate, right-hand side, residual, work vector and best
        iterate per slot; blocks up to 1.2x larger in the library's size
        classes) and the apply workspaces for the batch."""
        info = plan.info()
        L = info["ncomp"] * info["unknown_points"]
        krylov = int(1.2 * (max(self.restart, 5) + 6) * 16 * L * slots)
        return krylov + self.resident_bytes(plan, r, slots) - int(info["device_bytes"])

    def _admit_batch(self, key: str, nbytes: int):
        """Charge a new plan's batch, waiting while it does not fit and other
        batches (which will release memory) are running; idle plans are
        evicted for room.  With nothing running it goes ahead: waiting would
        not make room."""
        with self.admission.lock:
            while not self.admission.fits(nbytes):
                if self.cache.evict_one(keep=key):
                    continue
                with self.rlock:
                    running = self.running
                if running == 0:
                    break
                self.admission.lock.wait(timeout=0.05)
            self.admission.take(nbytes)

    def resident_bytes(self, plan, r: Request, slots: int) -> int:
        """Device bytes a plan holds at most while it serves a batch of
        `slots` slots: what it holds after batch_open (contrast, tables, the
        Krylov slots on the support rows; the precompute buffers are freed)
        plus the growth of its apply workspaces, which are allocated on
        demand up to the launches' right-hand sides."""
        info = plan.info()
        c, n = (6 if r.full else 3), r.n
        p = 2 * n
        w = (p + 15) // 16 * 16  # row pitch of the y-transformed planes
        per_rhs = c * (n * n * p + n * p * w)
        grow = (max(0, slots - info["workspace_rhs_fp32"]) * per_rhs * 8 +
                max(0, slots - info["workspace_rhs_fp64"]) * per_rhs * 16)
        return int(info["device_bytes"]) + grow

    def _slots_for(self, q: Request, cached, queued: Optional[Counter] = None) -> int:
        """Batch capacity for the request's key: the full batch for a key that
        repeats (a resident plan, served before, or another queued request),
        else the request's own right-hand sides, so that a one-off medium
        does not hold Krylov vectors for joiners that never come.  queued:
        the count of each key in the queue (computed here when not given)."""
        if queued is None:
            queued = Counter(o.key for o in self.queue)
        if cached is not None or q.key in self.seen or queued[q.key] > 1:
            return self.max_batch
        return q.nrhs

    def _plan_bytes_cached(self, q: Request, slots: int) -> int:
        """plan_bytes, remembered on the request (the claim looks at every
        queued request on each pass)."""
        memo = q.__dict__.setdefault("_plan_bytes", {})
        if slots not in memo:
            memo[slots] = self.creation_bytes(q) if slots == 0 else self.plan_bytes(q, slots)
        return memo[slots]

    def _keep_plan(self, key: str) -> bool:
        """Keep an idle plan resident only for a key that has repeated or is
        queued again."""
        if key in self.repeats:
            return True
        with self.qlock:
            return any(o.key == key for o in self.queue)

    @staticmethod
    def io_bytes(r: Request) -> int:
        """The request's incident fields and densities on the device."""
        return 2 * r.nrhs * (6 if r.full else 3) * r.n ** 3 * 16

    # ---- stream ----------------------------------------------------------------
    def now(self) -> float:
        return time.perf_counter() - self.t0

    def submit(self, req: Request):
        with self.qlock:
            self.queue.append(req)
            self.qlock.notify_all()

    def _refuse(self, q: Request, why: str):
        with self.rlock:
            self.refused += 1
            self.errors.append(f"request {q.id}: {why}")
            self.results.append(Result(q.id, None, [], q.arrival, self.now(), self.now(), error=why))
        q.release()
        self.host.give(q.host_bytes)

    def _claim(self):
        """The oldest queued request whose key no worker is serving and whose
        plan and arrays fit the device budget (evicting idle cached plans for
        room): (request, its cached (plan, charged bytes) checked out or None,
        the plan bytes charged now (a new plan, or the growth of a cached one
        to more slots), the batch capacity).  A request that does not fit is
        overtaken by younger ones until it has waited overtake_s."""
        with self.qlock:
            while True:
                if self.closed and not self.queue:
                    return None, None, 0, 0
                blocked = False
                queued = Counter(o.key for o in self.queue)
                for q in list(self.queue):
                    if q.key in self.serving:
                        continue
                    if q.nrhs > self.max_batch:
                        self.queue.remove(q)
                        self._refuse(q, f"{q.nrhs} right-hand sides exceed the batch capacity {self.max_batch}")
                        continue
                    peek = self.cache.peek(q.key)
                    cached = peek is not None
                    slots = self._slots_for(q, peek, queued)
                    if cached:
                        have = peek[0].info()["krylov_slots"]
                        grow = 0 if have >= slots else (self._plan_bytes_cached(q, slots) -
                                                        self._plan_bytes_cached(q, have))
                    else:
                        # the plan's creation; its batch is charged from its own
                        # support once it exists (_admit_batch)
                        grow = self._plan_bytes_cached(q, 0)
                    need = grow + self.io_bytes(q)
                    if not self.admission.can_ever_fit(need):
                        self.queue.remove(q)
                        self._refuse(q, f"footprint {need / 1e9:.1f} GB exceeds the device budget "
                                        f"{self.admission.budget / 1e9:.1f} GB")
                        continue
                    with self.admission.lock:
                        while not self.admission.fits(need) and self.cache.evict_one(keep=q.key):
                            pass
                        if self.admission.fits(need):
                            entry = self.cache.get(q.key) if cached else None
                            if cached and entry is None:
                                continue  # evicted meanwhile: look again
                            self.admission.take(need)
                            self.queue.remove(q)
                            self.serving.add(q.key)
                            self.inflight += 1
                            self.max_inflight = max(self.max_inflight, self.inflight)
                            if q.key in self.seen:
                                self.repeats.add(q.key)
                            self.seen.add(q.key)
                            if blocked:
                                self.overtakes += 1
                            return q, entry, need - self.io_bytes(q), slots
                    if self.now() - q.arrival >= self.overtake_s:
                        break  # it has waited long enough: nothing younger goes first
                    blocked = True
                self.qlock.wait(timeout=0.05)

    def _joiners(self, key: str, free: int) -> List[Request]:
        """Queued requests of `key`, oldest first, while they fit the free slots
        and the device budget (their arrays); the first that does not fit stops
        the scan, so requests of one key keep their order."""
        out = []
        with self.qlock:
            for q in list(self.queue):
                if q.key != key:
                    continue
                if q.nrhs > free:
                    break
                with self.admission.lock:
                    if not self.admission.fits(self.io_bytes(q)):
                        break
                    self.admission.take(self.io_bytes(q))
                self.queue.remove(q)
                out.append(q)
                free -= q.nrhs
        return out

    def _inputs(self, q: Request):
        if q.coef is None and q.recipe is not None:
            q.coef, q.mu, q.inc = device_inputs(q.recipe, self.device)

    def _worker(self):
        torch = self.torch
        vie = self.vie
        stream = torch.cuda.Stream()
        while True:
            first, entry, plan_charge, cap = self._claim()
            if first is None:
                return
            key = first.key
            plan, charged = None, plan_charge
            opened = False  # this worker's batch counts in self.running
            # request id -> [request, admitted time, densities, stats, slots left, joined while running]
            open_reqs = {}
            slot_of = {}    # slot -> (request id, index within the request)
            try:
                with torch.cuda.stream(stream):
                    self._inputs(first)
                    t_plan = time.perf_counter()
                    if entry is not None:
                        plan, charged = entry[0], entry[1] + plan_charge
                    else:
                        # worker threads allocate and synchronise while others
                        # solve, which stream capture would forbid
                        plan = vie.Plan(first.kind, first.coef, omega=first.omega, mu=first.mu,
                                        precision=self.precision, max_rhs=self.max_batch, stream=stream,
                                        graphs=False)
                        stream.synchronize()
                        with self.rlock:
                            self.plans_created += 1
                    t_solve = time.perf_counter()
                    if entry is None:
                        extra = self.batch_bytes(plan, first, cap)
                        self._admit_batch(key, extra)
                        charged += extra
                    plan.batch_open(cap, tol=self.tol, restart=self.restart, stream=stream)
                    with self.rlock:
                        self.running += 1
                        opened = True
                    # the charges were estimates (a cached plan's growth from
                    # the grid alone, a new plan's batch in the largest block
                    # sizes); keep only what the plan can hold from now on
                    fit = self.resident_bytes(plan, first, cap)
                    with self.admission.lock:
                        if fit < charged:
                            self.returned_bytes += charged - fit
                        self.admission.take(fit - charged)
                        if fit < charged:
                            self.admission.lock.notify_all()
                    charged = fit
                    with self.rlock:
                        self.plan_s += t_solve - t_plan
                        self.batches += 1
                    pending = [first]
                    used = 0
                    while True:
                        for q in pending:
                            self._inputs(q)
                            got = plan.batch_add(q.inc, stream=stream)
                            open_reqs[q.id] = [q, self.now(), [None] * q.nrhs, [None] * q.nrhs, q.nrhs, used > 0]
                            for i, sl in enumerate(got):
                                slot_of[sl] = (q.id, i)
                            with self.rlock:
                                self.joins += q.nrhs
                                if used > 0:
                                    self.joins_running += q.nrhs
                            used += q.nrhs
                            q.inc = q.coef = q.mu = None   # read by batch_add (it synchronised)
                        if used == 0:
                            # nothing left: release the key atomically with the last
                            # look at the queue, so a late request starts a new batch
                            with self.qlock:
                                pending = self._joiners(key, cap)
                                if not pending:
                                    self.serving.discard(key)
                                    self.inflight -= 1
                                    self.qlock.notify_all()
                                    break
                            continue
                        plan.batch_step(stream=stream)
                        done, nfree = plan.batch_done()
                        for sl in done:
                            d, _, st, rc = plan.batch_take(sl, stream=stream)
                            rid, i = slot_of.pop(sl)
                            o = open_reqs[rid]
                            o[2][i] = d
                            o[3][i] = st
                            o[4] -= 1
                            used -= 1
                            if o[4] == 0:
                                self._finish(open_reqs.pop(rid), stream)
                        pending = self._joiners(key, cap - used)
                    plan.batch_close()
                    with self.rlock:
                        self.solve_s += time.perf_counter() - t_solve
                        self.running -= 1
                        opened = False
                if self._keep_plan(key):
                    self.cache.put(key, plan, charged)
                else:
                    # a key that has not repeated: its memory serves the next
                    # plans better in the library's block cache than held idle
                    plan.close()
                    self.admission.give(charged)
                    with self.rlock:
                        self.closed_after_use += 1
                plan = None
            except Exception as exc:  # keep serving; report at the end
                self.errors.append(f"key {key}: {exc}")
                if opened:
                    with self.rlock:
                        self.running -= 1
                for o in open_reqs.values():
                    self.admission.give(self.io_bytes(o[0]))
                    o[0].release()
                    self.host.give(o[0].host_bytes)
                if plan is not None:
                    plan.close()
                self.admission.give(charged)
                with self.qlock:
                    if key in self.serving:
                        self.serving.discard(key)
                        self.inflight -= 1
                    self.qlock.notify_all()

    def _finish(self, o, stream):
        q, admitted, dens, stats, _, joined = o
        dens_h = None
        if self.keep_results:
            dens_h = self.torch.stack(dens).cpu().numpy()
        else:
            stream.synchronize()
        done = self.now()
        self.admission.give(self.io_bytes(q))
        q.release()
        self.host.give(q.host_bytes)
        with self.rlock:
            self.results.append(Result(q.id, dens_h, stats, q.arrival, admitted, done, joined))
            if self.progress and len(self.results) % self.progress == 0:
                print(f"[serve] {len(self.results)} requests done at {done:.1f} s", file=sys.stderr, flush=True)

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
                "plans_created": self.plans_created, "batches": self.batches,
                "joins_rhs": self.joins, "joins_into_running_rhs": self.joins_running,
                "requests_joined_running": sum(1 for r in results if r.joined_running),
                "overtakes": self.overtakes, "returned_GB": self.returned_bytes / 1e9,
                "plans_closed_after_use": self.closed_after_use,
                "refused": self.refused, "errors": self.errors[:5]}


def requests_from_generator(count: int, rate: float, grids=None, max_rhs: int = 16, media: int = 0) -> List[Request]:
    """The seeded serving stream (Poisson arrivals; Laplace / Helmholtz / Maxwell mix).

    Media and incident fields are generated when each request arrives; every
    request has its own medium (key = its seed), or, with media > 0, one of a
    pool of `media` scatterers (key = the pool entry), so that plans repeat
    and requests join running batches."""
    from vie_inputs import generators as gen
    grids = grids or gen.SERVING_GRIDS
    out = []
    for rq in gen.serving_requests(count, rate, grids, max_rhs, media=media):
        def make(rq=rq):
            p = gen.serving_problem(rq)
            return p.coef, p.mu, p.inc
        key = f"pool{rq['medium_item']}" if "medium_item" in rq else f"req{rq['item']}"
        out.append(Request(rq["id"], rq["kind"], rq["n"], rq["omega"], rq["nrhs"], arrival=rq["arrival"],
                           key=key, make=make, recipe_fn=lambda rq=rq: gen.serving_recipe(rq)))
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--requests", type=int, default=200)
    ap.add_argument("--rate", type=float, default=20.0, help="Poisson arrival rate (requests/s)")
    ap.add_argument("--grids", type=str, default="32,48,64,96,128,160")
    ap.add_argument("--max-rhs", type=int, default=16)
    ap.add_argument("--workers", type=int, default=3)
    ap.add_argument("--plan-cache", type=int, default=16, help="idle plans kept resident (evicted for room)")
    ap.add_argument("--budget-gb", type=float, default=0.0)
    ap.add_argument("--host-budget-gb", type=float, default=24.0, help="host memory for generated inputs")
    ap.add_argument("--gen-workers", type=int, default=8, help="threads generating the stream's inputs")
    ap.add_argument("--pageable", action="store_true", help="keep the generated inputs in pageable memory")
    ap.add_argument("--media", type=int, default=0,
                    help="draw the scatterers from a pool of this many (0: every request its own)")
    ap.add_argument("--inputs", choices=("device", "host"), default="device",
                    help="build each request's arrays on the device from its random draws, or on the host")
    args = ap.parse_args(argv)
    grids = tuple(int(g) for g in args.grids.split(","))
    t = time.perf_counter()
    reqs = requests_from_generator(args.requests, args.rate, grids, args.max_rhs, media=args.media)
    print(f"[serve] generated {len(reqs)} requests in {time.perf_counter() - t:.1f} s", file=sys.stderr, flush=True)
    srv = Server(int(args.budget_gb * 1e9) if args.budget_gb > 0 else None, workers=args.workers,
                 keep_results=False, gen_workers=args.gen_workers,
                 host_budget_bytes=int(args.host_budget_gb * 1e9), pinned_inputs=not args.pageable,
                 device_inputs=args.inputs == "device", progress=100, plan_cache=args.plan_cache)
    res = srv.run(lambda: reqs)
    out = srv.summary(res)
    out.update({"rate": args.rate, "grids": list(grids), "workers": args.workers, "media": args.media})
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
