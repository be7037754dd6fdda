"""Serving on the CPU: the history store recovers every stored state exactly (Supp.
"History Recovery": recovery gives identical reconstructions), and the scheduler's
admission, grouping, retry and latency accounting, driven by a fake backend and a
simulated clock."""
import numpy as np
import pytest

import scenes
from paper_2506_21117_amd.serve import Engine, Request, StateStore, poisson_requests


def small_history(seed=5):
    return scenes.serving_history(seed=seed, n_base=3000, n_steps=4, delta_range=(200, 600))


def test_history_store_recovers_every_state_bitwise():
    states, history = small_history()
    store = StateStore.from_history(states[-1], history)
    assert store.timesteps == len(states)
    assert store.n_rows == states[-1].n + sum(h[1].n for h in history)
    for k, st in enumerate(states):
        got = store.state_arrays(k)
        for a, b in zip(got, st.param_arrays()):
            np.testing.assert_array_equal(a, b)


def test_history_static_prefix_is_shared():
    """Each state reuses the previous state's static rows: the pool grows only by the
    changed Gaussians."""
    states, history = small_history(seed=9)
    store = StateStore.from_history(states[-1], history)
    for k in range(1, len(states)):
        ind = history[k - 1][0]
        n_static = int((~ind).sum())
        np.testing.assert_array_equal(store.gathers[k][:n_static], store.gathers[k - 1][~ind])


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class FakeBackend:
    """Work takes `cost` simulated seconds per group; memory estimate is `per_view`
    bytes per view; the first launch of key (0, 64, 64) overflows once."""

    def __init__(self, clock, cost=0.01, per_view=100):
        self.clock, self.cost, self.per_view = clock, cost, per_view
        self.launches = []
        self.overflowed = set()
        self.inflight = 0
        self.max_inflight = 0

    def estimate_bytes(self, reqs):
        return self.per_view * len(reqs)

    def launch(self, reqs, slot):
        self.launches.append((tuple(r.rid for r in reqs), slot, self.clock()))
        self.inflight += 1
        self.max_inflight = max(self.max_inflight, self.inflight)
        return {"reqs": reqs, "end": self.clock() + self.cost}

    def done(self, h):
        return self.clock() >= h["end"]

    def finish(self, h):
        self.inflight -= 1
        key = h["reqs"][0].key
        if key == (0, 64, 64) and key not in self.overflowed:
            self.overflowed.add(key)
            return None
        return [f"img{r.rid}" for r in h["reqs"]]


class Cam:
    def __init__(self, w, h):
        self.width, self.height = w, h


def _advance(clock, step=0.001):
    def idle(_next):
        clock.t += step
    return idle


def test_engine_admission_grouping_and_retry():
    clock = FakeClock()
    be = FakeBackend(clock, cost=0.01, per_view=100)
    # 6 requests at t=0: three (0, 64x64), two (1, 32x32), one (0, 32x32)
    reqs = [Request(0, 0, Cam(64, 64)), Request(1, 1, Cam(32, 32)), Request(2, 0, Cam(64, 64)),
            Request(3, 0, Cam(32, 32)), Request(4, 1, Cam(32, 32)), Request(5, 0, Cam(64, 64))]
    eng = Engine(be, hbm_budget_bytes=300, max_slots=2, max_batch=2, keep_images=True)
    out, st = eng.run(reqs, clock=clock, idle=_advance(clock))
    assert sorted(c.rid for c in out) == list(range(6))
    assert {c.rid: c.image for c in out} == {i: f"img{i}" for i in range(6)}
    # grouping by (timestep, resolution), at most max_batch per group, oldest first
    groups = [g for g, _, _ in be.launches]
    first = list(dict.fromkeys(groups))
    # head request 0 grouped with 2 (same key); with 200 of 300 bytes in use nothing
    # else fits until it completes; then (1, 4) and (3,) share the budget; 5 comes last
    assert first == [(0, 2), (1, 4), (3,), (5,)]
    assert groups[1] == (0, 2)              # the overflowing group ran again first
    assert st.retries == 1
    # never more than the budget (300 bytes = 3 views) or the slots in flight
    assert st.peak_bytes <= 300 and be.max_inflight <= 2
    assert all(c.latency_ms >= 10.0 - 1e-9 for c in out)


def test_engine_rejects_requests_larger_than_the_budget():
    clock = FakeClock()
    be = FakeBackend(clock, per_view=1000)
    eng = Engine(be, hbm_budget_bytes=500, max_slots=2)
    with pytest.raises(MemoryError):
        eng.run([Request(0, 0, Cam(16, 16))], clock=clock, idle=_advance(clock))


def test_engine_admits_new_arrivals_while_others_run():
    """Continuous batching: a request arriving during another's work starts before
    that work ends when a slot is free."""
    clock = FakeClock()
    be = FakeBackend(clock, cost=0.05, per_view=1)
    reqs = [Request(0, 2, Cam(16, 16), 0.0), Request(1, 3, Cam(16, 16), 0.01)]
    eng = Engine(be, hbm_budget_bytes=10, max_slots=2)
    out, st = eng.run(reqs, clock=clock, idle=_advance(clock))
    (_, _, t0), (_, _, t1) = be.launches
    assert t0 == 0.0 and 0.01 <= t1 < 0.05
    assert st.peak_inflight == 2


def test_poisson_requests_rate():
    rng = np.random.default_rng(0)
    reqs = poisson_requests(rng, 4000, 200.0, 8, scenes.RESOLUTIONS, lambda r, w, h: Cam(w, h))
    gaps = np.diff([r.arrival for r in reqs])
    assert abs(gaps.mean() - 1 / 200.0) < 0.1 / 200.0
    assert {r.timestep for r in reqs} == set(range(8))
    assert {(r.camera.width, r.camera.height) for r in reqs} == set(scenes.RESOLUTIONS)
