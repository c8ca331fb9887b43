"""Serving loop: admission by footprint (CPU) and results alone == in the mix (GPU)."""

import threading

import numpy as np
import pytest

from paper_1805_04791_amd.serving import Admission, PlanCache, Request


def test_admission_never_overcommits():
    adm = Admission(100)
    sizes = [30, 50, 40, 20, 60, 10, 90, 5]
    inflight = []
    peak = [0]
    lock = threading.Lock()

    def run(sz):
        with adm.lock:
            while not adm.fits(sz):
                adm.lock.wait()
            adm.take(sz)
        with lock:
            inflight.append(sz)
            peak[0] = max(peak[0], sum(inflight))
        with lock:
            inflight.remove(sz)
        adm.give(sz)

    ts = [threading.Thread(target=run, args=(s,)) for s in sizes]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    assert adm.used == 0
    assert adm.peak <= 100 and peak[0] <= 100


def test_admission_refuses_footprints_beyond_the_device():
    adm = Admission(100)
    assert not adm.fits(150) and not adm.can_ever_fit(150)   # not even on an empty device
    assert adm.fits(100) and adm.can_ever_fit(100)
    adm.take(60)
    assert not adm.fits(41) and adm.fits(40)


def test_plan_cache_lru_and_checkout():
    closed = []

    class P:
        def __init__(self, k):
            self.k = k

        def close(self):
            closed.append(self.k)

    freed = []
    c = PlanCache(2, on_evict=freed.append)
    for i, k in enumerate("abc"):
        c.put(k, P(k), 10 * (i + 1))
    assert closed == ["a"] and freed == [10]          # evicted plans give their bytes back
    p, nb = c.get("b")
    assert p.k == "b" and nb == 20 and c.get("b") is None     # checked out: not shared
    c.put("b", p, nb)
    assert c.hits == 1 and c.misses == 1
    assert c.evict_one(keep="c") and closed == ["a", "b"] and freed == [10, 20]
    assert not c.evict_one(keep="c")
    c.clear()
    assert closed == ["a", "b", "c"] and freed == [10, 20, 30]


def test_request_key_from_medium():
    coef = np.zeros((9, 4, 4, 4), dtype=np.complex128)
    a = Request(0, 1, 4, 2.0, 1, coef=coef, inc=np.zeros((1, 3, 4, 4, 4), complex)).materialise()
    b = Request(1, 1, 4, 2.0, 1, coef=coef.copy(), inc=np.zeros((1, 3, 4, 4, 4), complex)).materialise()
    coef2 = coef.copy()
    coef2[0, 0, 0, 0] = 1
    c = Request(2, 1, 4, 2.0, 1, coef=coef2, inc=np.zeros((1, 3, 4, 4, 4), complex)).materialise()
    assert a.key == b.key != c.key


def test_feeder_keeps_generated_inputs_within_the_host_budget():
    """The feeder generates inputs ahead of arrival but never holds more than
    the host budget (plus one request when nothing else is held); every
    request is served and its arrays are released afterwards."""
    from paper_1805_04791_amd import serving

    n, nrhs = 8, 2
    one = Request(0, 1, n, 2.0, nrhs).input_bytes()
    held = []
    lock = threading.Lock()

    class FakeServer(serving.Server):
        def plan_bytes(self, r, slots=None):
            return 0

        def creation_bytes(self, r):
            return 0

        def _worker(self):
            import time
            while True:
                q, entry, charge, slots = self._claim()
                if q is None:
                    return
                time.sleep(0.01)     # the device is slower than the stream
                with self.rlock:
                    assert q.inc is not None and q.inc.shape == (nrhs, 3, n, n, n)
                    self.results.append(serving.Result(q.id, None, [{"status": 0}] * q.nrhs, q.arrival,
                                                       self.now(), self.now()))
                with lock:
                    held.append(q)
                q.release()
                self.host.give(q.host_bytes)
                self.admission.give(charge + self.io_bytes(q))
                with self.qlock:
                    self.serving.discard(q.key)
                    self.inflight -= 1
                    self.qlock.notify_all()

    def make():
        return (np.zeros((9, n, n, n), complex), None, np.zeros((nrhs, 3, n, n, n), complex))

    reqs = [Request(i, 1, n, 2.0, nrhs, arrival=0.001 * i, key=f"k{i}", make=make) for i in range(40)]
    srv = FakeServer(budget_bytes=10 ** 12, workers=2, keep_results=False, gen_workers=4,
                     host_budget_bytes=3 * one)
    res = srv.run(lambda: reqs)
    assert [r.id for r in res] == list(range(40))
    assert srv.host.peak <= 3 * one and srv.host.used == 0
    assert all(q.coef is None and q.inc is None for q in held)


def test_batch_capacity_follows_key_repetition():
    """A one-off key opens a batch of its own right-hand sides; a key with a
    resident plan, one served before, or a second queued request opens the
    full batch so that later requests can join it."""
    from paper_1805_04791_amd import serving
    srv = serving.Server(budget_bytes=10 ** 9, workers=1, max_batch=16, keep_results=False)
    a = Request(0, 1, 8, 2.0, 3, key="a")
    b1, b2 = Request(1, 1, 8, 2.0, 5, key="b"), Request(2, 1, 8, 2.0, 2, key="b")
    srv.queue = [a, b1, b2]
    assert srv._slots_for(a, None) == 3
    assert srv._slots_for(b1, None) == 16 and srv._slots_for(b2, None) == 16
    srv.queue = [a]
    assert srv._slots_for(a, ("plan", 0)) == 16
    srv.seen.add("a")
    assert srv._slots_for(a, None) == 16


def test_batch_admission_waits_only_while_batches_run():
    """A new plan's batch is charged once the plan exists: it waits while it
    does not fit and another batch (which will release memory) is running,
    and goes ahead at once when nothing is running (waiting would not make
    room)."""
    import time
    from paper_1805_04791_amd import serving
    srv = serving.Server(budget_bytes=100, workers=1, keep_results=False)
    srv.admission.take(90)
    srv.running = 1
    done = []
    t = threading.Thread(target=lambda: (srv._admit_batch("k", 20), done.append(True)))
    t.start()
    time.sleep(0.2)
    assert not done                      # 90 + 20 > 100 while a batch runs
    srv.admission.give(50)
    t.join(timeout=5)
    assert done and srv.admission.used == 60
    srv.running = 0
    srv._admit_batch("k", 80)            # does not fit, but nothing runs
    assert srv.admission.used == 140


@pytest.mark.parametrize("overtake_s,order", [(60.0, [0, 2, 1]), (0.0, [0, 1, 2])],
                         ids=["overtake", "strict-order"])
def test_younger_requests_overtake_one_that_does_not_fit(overtake_s, order):
    """Admission order: with a device budget of 100, request 0 (30) runs while
    request 1 (80) cannot fit; request 2 (30) goes first while request 1 has
    waited less than overtake_s, and waits behind it once it has waited that
    long (overtake_s = 0: strict arrival order)."""
    import time
    from paper_1805_04791_amd import serving

    started = []
    lock = threading.Lock()

    class FakeServer(serving.Server):
        def plan_bytes(self, r, slots=None):
            return 80 if r.id == 1 else 30

        def creation_bytes(self, r):
            return self.plan_bytes(r)

        def io_bytes(self, r):
            return 0

        def _worker(self):
            while True:
                q, entry, charge, slots = self._claim()
                if q is None:
                    return
                with lock:
                    started.append(q.id)
                time.sleep(0.3 if q.id == 0 else 0.05)
                with self.rlock:
                    self.results.append(serving.Result(q.id, None, [], q.arrival, self.now(), self.now()))
                q.release()
                self.host.give(q.host_bytes)
                self.admission.give(charge + self.io_bytes(q))
                with self.qlock:
                    self.serving.discard(q.key)
                    self.inflight -= 1
                    self.qlock.notify_all()

    def make():
        return (np.zeros((9, 2, 2, 2), complex), None, np.zeros((1, 3, 2, 2, 2), complex))

    reqs = [Request(i, 1, 2, 2.0, 1, arrival=0.02 * i, key=f"k{i}", make=make) for i in range(3)]
    srv = FakeServer(budget_bytes=100, workers=2, keep_results=False, gen_workers=1, overtake_s=overtake_s)
    res = srv.run(lambda: reqs)
    assert [r.id for r in res] == [0, 1, 2] and not srv.errors
    assert started == order
    assert srv.overtakes == (1 if order[1] == 2 else 0)
    assert srv.admission.used == 0 and srv.admission.peak <= 100


@pytest.mark.gpu
@pytest.mark.parametrize("device_inputs", [True, False], ids=["device-inputs", "host-inputs"])
def test_results_alone_equal_results_in_the_mix(device_inputs):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1805_04791_amd.serving import Server, requests_from_generator
    reqs = requests_from_generator(10, rate=1e6, grids=(16, 24, 32), max_rhs=4)
    # two requests share a medium (and so a plan) to exercise merged batches
    dup = requests_from_generator(1, rate=1e6, grids=(16, 24, 32), max_rhs=4)[0]
    dup.id, dup.key, dup.make, dup.recipe_fn = 99, reqs[0].key, reqs[0].make, reqs[0].recipe_fn
    dup.kind, dup.n, dup.omega, dup.nrhs = reqs[0].kind, reqs[0].n, reqs[0].omega, reqs[0].nrhs

    def fresh(r):
        return Request(r.id, r.kind, r.n, r.omega, r.nrhs, key=r.key, make=r.make, recipe_fn=r.recipe_fn)

    alone = {}
    for r in reqs:
        srv = Server(workers=1, device_inputs=device_inputs)
        res = srv.run(lambda r=r: [fresh(r)], realtime=False)
        assert not srv.errors, srv.errors
        alone[r.id] = res[0].density
    srv = Server(workers=3, device_inputs=device_inputs)
    mix = srv.run(lambda: [fresh(r) for r in reqs + [dup]], realtime=False)
    assert not srv.errors, srv.errors
    assert len(mix) == len(reqs) + 1
    for res in mix:
        ref = alone[0 if res.id == 99 else res.id]
        assert np.array_equal(res.density, ref), res.id       # bitwise, whatever ran beside it
        assert all(s["status"] == 0 and s["rel_residual"] <= 1e-9 for s in res.stats)
    s = srv.summary(mix)
    assert s["max_inflight"] >= 1 and s["rhs_converged"] == s["rhs_solved"]


@pytest.mark.gpu
def test_joins_into_running_batches_equal_solves_alone():
    """Continuous batching: a stream over a pool of two scatterers (the seeded
    pool draws two Helmholtz media on the 64^3 grid) queued at once, served
    with batches of 4 slots, so that later requests join solves already
    running as slots free up.  Every result is bitwise the solve of that
    request alone (vie_solve on its own plan, same options), plans are
    reused, and the summary counts the joins."""
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1805_04791_amd import vie
    from paper_1805_04791_amd.serving import Server, device_inputs, requests_from_generator
    from vie_inputs import generators as gen
    reqs = requests_from_generator(14, rate=1e6, grids=(48, 64), max_rhs=3, media=2)
    assert len({r.key for r in reqs}) == 2 and {r.n for r in reqs} == {64}
    rqs = {rq["id"]: rq for rq in gen.serving_requests(14, 1e6, (48, 64), 3, media=2)}
    srv = Server(workers=2, max_batch=4, device_inputs=True)
    res = srv.run(lambda: reqs, realtime=False)
    assert not srv.errors, srv.errors
    s = srv.summary(res)
    print("[serving] joins", s["joins_rhs"], "into running", s["joins_into_running_rhs"], "plans", s["plans_created"],
          "hits", s["plan_cache_hits"], flush=True)
    assert s["joins_into_running_rhs"] > 0 and s["requests_joined_running"] > 0
    assert s["plans_created"] == 2 and s["rhs_converged"] == s["rhs_solved"]
    dev = torch.device("cuda")
    for r in res:
        coef, mu, inc = device_inputs(gen.serving_recipe(rqs[r.id]), dev)
        rq = rqs[r.id]
        plan = vie.Plan(rq["kind"], coef, omega=rq["omega"], precision=vie.PREC_MIXED, max_rhs=rq["nrhs"])
        d, _, st, rc = plan.solve(inc, tol=1e-9, restart=20, want_field=False)
        plan.close()
        assert rc == vie.OK
        assert np.array_equal(r.density, d.cpu().numpy()), r.id
        assert [x["iters"] for x in st] == [x["iters"] for x in r.stats]


def test_device_recipe_matches_host_generator():
    """The serving recipe evaluated with torch (on the CPU here) gives the host
    generator's arrays, to the rounding of the exponentials, for every kind."""
    torch = pytest.importorskip("torch")
    from paper_1805_04791_amd.serving import device_inputs
    from vie_inputs import generators as gen
    kinds = set()
    for rq in gen.serving_requests(12, 5.0, (16, 24), 3):
        p = gen.serving_problem(rq)
        coef, mu, inc = device_inputs(gen.serving_recipe(rq), torch.device("cpu"))
        assert mu is None
        assert np.abs(coef.numpy() - p.coef).max() <= 1e-14 * np.abs(p.coef).max()
        assert np.abs(inc.numpy() - p.inc).max() <= 1e-14 * np.abs(p.inc).max()
        kinds.add(rq["kind"])
    assert kinds == {0, 1, 2}
