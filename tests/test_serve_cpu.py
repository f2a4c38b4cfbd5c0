"""The serving scheduler on a simulated device (CPU only): admission by slot
count and HBM budget, first-come-first-served order, completion and latency
bookkeeping, and the Poisson arrival generator."""
import numpy as np
import pytest

from paper_2412_10249_amd import serve


class VirtualClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-6)


class SimExecutor(serve.Executor):
    """Each request advances at 1 epoch per `cost[n]` virtual seconds,
    independently of the others (one stream per slot)."""

    def __init__(self, clock, cost, foot):
        self.clock, self.cost, self.foot = clock, cost, foot
        self.state = {}
        self.peak_used = 0
        self.log = []

    def footprint(self, req):
        return self.foot[req.n]

    def start(self, req, slot):
        self.state[req.rid] = {"queued_until": self.clock(), "epochs": 0.0, "slot": slot}
        self.log.append(("start", req.rid, slot))

    def advance(self, req, epochs):
        st = self.state[req.rid]
        left = req.epochs - st["epochs"]
        if left <= 0:
            return
        e = min(epochs, left)
        st["queued_until"] = max(st["queued_until"], self.clock()) + e * self.cost[req.n]
        st["epochs"] += e
        self.clock.sleep(1e-4)  # host time per enqueue

    def finished(self, req):
        st = self.state[req.rid]
        return st["epochs"] >= req.epochs and self.clock() >= st["queued_until"]

    def release(self, req):
        self.log.append(("release", req.rid))
        del self.state[req.rid]


def _run(rate, duration, budget, slots, epochs=5.0):
    clock = VirtualClock()
    cost = {128: 1e-4, 256: 3e-4, 512: 1e-3, 1024: 5e-3}
    foot = {128: 1, 256: 4, 512: 16, 1024: 64}
    ex = SimExecutor(clock, cost, foot)
    sch = serve.Scheduler(ex, hbm_budget=budget, max_active=slots, chunk_epochs=1.0, clock=clock)
    arrivals = serve.poisson_arrivals(rate, duration, seed=7)
    used_trace = []
    orig_tick = sch.tick

    def tick():
        n = orig_tick()
        used_trace.append(sch.used)
        return n

    sch.tick = tick
    done = serve.run_load(sch, arrivals, lambda rid, n, t: serve.Request(rid, n, t, epochs), now=clock,
                          sleep=clock.sleep)
    return done, arrivals, used_trace, ex


def test_every_request_completes_and_budget_is_respected():
    done, arrivals, used, ex = _run(rate=200, duration=0.5, budget=100, slots=6)
    assert len(done) == len(arrivals) > 50
    assert max(used) <= 100
    assert all(r.latency >= r.epochs * {128: 1e-4, 256: 3e-4, 512: 1e-3, 1024: 5e-3}[r.n] - 1e-9 for r in done)
    # admission is first come first served
    starts = [rid for kind, rid, *_ in ex.log if kind == "start"]
    assert starts == sorted(starts)


def test_slots_bound_concurrency():
    done, _, _, ex = _run(rate=500, duration=0.2, budget=10 ** 6, slots=3)
    live, peak = set(), 0
    for ev in ex.log:
        if ev[0] == "start":
            live.add(ev[1])
        else:
            live.discard(ev[1])
        peak = max(peak, len(live))
    assert peak <= 3


def test_overload_grows_latency():
    light, _, _, _ = _run(rate=20, duration=1.0, budget=10 ** 6, slots=8)
    heavy, _, _, _ = _run(rate=2000, duration=0.2, budget=80, slots=2)
    assert serve.latency_summary(heavy)["p99_ms"] > serve.latency_summary(light)["p99_ms"]


def test_oversized_request_is_rejected():
    clock = VirtualClock()
    ex = SimExecutor(clock, {128: 1e-4}, {128: 10})
    sch = serve.Scheduler(ex, hbm_budget=5, max_active=2, clock=clock)
    with pytest.raises(ValueError):
        sch.submit(serve.Request(0, 128, 0.0, 1.0))


def test_poisson_arrivals_statistics():
    arr = serve.poisson_arrivals(200.0, 50.0, seed=7)
    gaps = np.diff([0.0] + [t for t, _ in arr])
    assert abs(gaps.mean() - 1 / 200) < 0.05 / 200 * 10
    sizes = np.array([n for _, n in arr])
    frac = np.mean(sizes == 128)
    assert abs(frac - 0.4) < 0.02
    assert arr == serve.poisson_arrivals(200.0, 50.0, seed=7)
