"""Continuous-batching scheduler on the CPU: a simulated executor and clock
drive the same state machine the GPU serving loop uses."""
import pytest

import synth
from paper_2505_00690_amd.serve import Request, Scheduler, SimClock, percentile


class SimExecutor:
    """Each launch takes t0 + t_img * images seconds of simulated time; the
    workspace of a batch is ws_img bytes per image."""

    def __init__(self, clock, t0=0.002, t_img=0.001, ws_img=100):
        self.clock, self.t0, self.t_img, self.ws_img = clock, t0, t_img, ws_img
        self.running = {}
        self.launches = []

    def workspace_bytes(self, sizes):
        return self.ws_img * len(sizes)

    def launch(self, reqs, slot):
        n = sum(len(r.sizes) for r in reqs)
        done = self.clock.now() + self.t0 + self.t_img * n
        h = len(self.launches)
        self.launches.append((self.clock.now(), [r.rid for r in reqs], slot))
        self.running[h] = done
        return h

    def poll(self, h):
        return self.clock.now() >= self.running[h]

    def collect(self, h):
        self.running.pop(h)
        return [("out", h)] * len(self.launches[h][1])

    def next_event_time(self):
        return min(self.running.values()) if self.running else None


def _reqs(n, qps, seed=5004):
    return [Request(i, r.arrival_s, r.sizes)
            for i, r in enumerate(synth.draw_requests(n, qps, (224, 336), seed))]


def test_all_requests_complete_in_fifo_order():
    clock = SimClock()
    ex = SimExecutor(clock)
    reqs = _reqs(200, qps=50.0)
    st = Scheduler(ex, budget_bytes=10_000, slots=2).run(reqs, clock)
    assert sorted(r.rid for r in st.results) == list(range(200))
    for r in st.results:
        assert r.admitted >= r.arrival - 1e-12 and r.finished > r.admitted
    admitted_order = [rid for _, rids, _ in ex.launches for rid in rids]
    assert admitted_order == sorted(admitted_order)          # FIFO admission


def test_budget_is_never_exceeded_and_oversize_rejected():
    clock = SimClock()
    ex = SimExecutor(clock, ws_img=100)
    reqs = _reqs(100, qps=500.0)
    big = Request(999, 0.01, [(224, 224)] * 40)               # 4000 B > budget
    st = Scheduler(ex, budget_bytes=2_000, slots=3).run(reqs + [big], clock)
    assert st.peak_budget <= 2_000
    assert st.rejected == [999]
    assert len(st.results) == 100


def test_overlap_and_continuous_admission():
    """Under load two batches run at once, and a request that arrives while
    both slots are busy starts the moment one of them finishes."""
    clock = SimClock()
    ex = SimExecutor(clock, t0=0.01, t_img=0.0)
    reqs = [Request(0, 0.0, [(224, 224)]), Request(1, 0.001, [(224, 224)]),
            Request(2, 0.002, [(224, 224)])]
    st = Scheduler(ex, budget_bytes=10_000, slots=2).run(reqs, clock)
    assert st.max_inflight == 2
    r = {x.rid: x for x in st.results}
    assert r[0].admitted == pytest.approx(0.0)
    assert r[1].admitted == pytest.approx(0.001)
    assert r[2].admitted == pytest.approx(r[0].finished)       # slot freed at 0.010
    assert r[2].latency == pytest.approx(0.010 + 0.010 - 0.002)


def test_batch_image_limit():
    clock = SimClock()
    ex = SimExecutor(clock)
    reqs = [Request(i, 0.0, [(224, 224)] * 10) for i in range(5)]
    Scheduler(ex, budget_bytes=10**9, slots=1, max_batch_images=25).run(reqs, clock)
    assert [len(rids) for _, rids, _ in ex.launches] == [2, 2, 1]


def test_percentile_nearest_rank():
    xs = list(range(1, 101))
    assert percentile(xs, 50) == 50
    assert percentile(xs, 99) == 99
    assert percentile(xs, 100) == 100
    assert percentile([3.0], 99) == 3.0


def test_scheduler_rejects_bad_limits():
    with pytest.raises(ValueError):
        Scheduler(SimExecutor(SimClock()), budget_bytes=0)
