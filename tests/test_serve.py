"""The serving loop's scheduler on a simulated clock: admission in arrival
order, slot and memory limits, overlap of later arrivals with running work."""
import numpy as np
import pytest

from paper_2609_30741_amd import serve


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def tick(self):
        self.t += 1e-3


class FakeExecutor:
    """Each request takes `dur[rid]` seconds of simulated time once issued;
    records what was in flight at every issue.  Like the GPU executor, a
    slot keeps the buffers of its last frame (its held bytes) after the
    frame ends, until it is trimmed or its next frame replaces them."""

    def __init__(self, clock, dur, size):
        self.clock, self.dur, self.size = clock, dur, size
        self.running = {}
        self.held = {}
        self.peak_slots = 0
        self.peak_bytes = 0.0
        self.trims = 0
        self.order = []

    def start(self):
        pass

    def need_bytes(self, r):
        return self.size[r.rid]

    def held_bytes(self, s):
        return self.held.get(s, 0.0)

    def trim(self, s):
        assert s not in self.running, "a running slot must never be trimmed"
        self.held[s] = 0.0
        self.trims += 1

    def issue(self, s, r):
        assert s not in self.running
        self.running[s] = (r, self.clock.t + self.dur[r.rid])
        self.held[s] = self.size[r.rid]
        self.order.append(r.rid)
        self.peak_slots = max(self.peak_slots, len(self.running))
        self.peak_bytes = max(self.peak_bytes, sum(self.held.values()))

    def poll(self, s, r=None):
        if s not in self.running or self.clock.t < self.running[s][1]:
            return None
        return self.running[s][1]

    def release(self, s, r):
        del self.running[s]


def run(arrivals, dur, size, slots, budget):
    clock = Clock()
    reqs = [serve.Request(i, "s", None, None, float(a)) for i, a in enumerate(arrivals)]
    ex = FakeExecutor(clock, dur, size)
    out = serve.serve(reqs, ex, slots, budget, clock=clock, idle=clock.tick)
    return out, ex


def test_every_request_completes_in_arrival_order_within_the_limits():
    rng = np.random.default_rng(0)
    n = 60
    arrivals = serve.poisson_arrivals(50.0, n, seed=1)
    dur = rng.uniform(0.02, 0.08, size=n)
    size = rng.uniform(1.0, 3.0, size=n)
    reqs, ex = run(arrivals, dur, size, slots=3, budget=6.0)
    assert ex.order == list(range(n))  # first come, first admitted
    assert ex.peak_slots <= 3 and ex.peak_bytes <= 6.0 + 1e-12
    for r in reqs:
        assert r.arrival <= r.admitted + 1e-12 <= r.done + 1e-12
        assert r.done == pytest.approx(r.admitted + dur[r.rid], abs=2e-3)
    s = serve.summary(reqs)
    assert s["requests"] == n and s["p50_ms"] <= s["p99_ms"] <= s["max_ms"]


def test_later_arrivals_join_running_work():
    # Two slots; the second request arrives while the first still runs and
    # starts at once: the work overlaps rather than waiting for a batch.
    reqs, ex = run([0.0, 0.5], [1.0, 1.0], [1.0, 1.0], slots=2, budget=10.0)
    assert reqs[1].admitted == pytest.approx(0.5, abs=2e-3)
    assert reqs[1].admitted < reqs[0].done
    # One slot: the second waits for the first.
    reqs, _ = run([0.0, 0.5], [1.0, 1.0], [1.0, 1.0], slots=1, budget=10.0)
    assert reqs[1].admitted == pytest.approx(1.0, abs=2e-3)


def test_memory_budget_holds_back_admission():
    # Free slots but not enough memory: the second request waits for the
    # first to finish although a slot is idle.
    reqs, ex = run([0.0, 0.0], [1.0, 1.0], [4.0, 4.0], slots=2, budget=6.0)
    assert reqs[1].admitted == pytest.approx(1.0, abs=2e-3)
    assert ex.peak_slots == 1


def test_a_request_larger_than_the_budget_is_refused():
    with pytest.raises(ValueError):
        run([0.0], [1.0], [7.0], slots=2, budget=6.0)


def test_poisson_arrivals_rate():
    t = serve.poisson_arrivals(90.0, 20_000, seed=3)
    assert np.all(np.diff(t) > 0)
    assert np.mean(np.diff(t)) == pytest.approx(1.0 / 90.0, rel=0.03)


def test_held_bytes_never_exceed_the_budget():
    # The budget fits two frames, there are four slots: slots keep their
    # buffers after a frame, so admission must count what idle slots hold
    # and trim them before the held total would pass the budget.
    rng = np.random.default_rng(4)
    n = 80
    arrivals = serve.poisson_arrivals(200.0, n, seed=5)
    dur = rng.uniform(0.01, 0.04, size=n)
    size = rng.choice([2.0, 3.0, 3.5], size=n)
    reqs, ex = run(arrivals, dur, size, slots=4, budget=7.0)
    assert ex.peak_bytes <= 7.0 + 1e-12
    assert ex.peak_slots >= 2
    assert ex.trims > 0
    assert ex.order == list(range(n))
    assert all(r.done >= r.admitted for r in reqs)


def test_a_slot_holding_this_size_is_reused():
    # Same-size requests one after another reuse the slot that already
    # holds their buffers: nothing is trimmed.
    reqs, ex = run([0.0, 1.5, 3.0], [1.0, 1.0, 1.0], [3.0, 3.0, 3.0], slots=3, budget=4.0)
    assert ex.trims == 0 and len({r.slot for r in reqs}) == 1
