"""The render server's scheduling on the CPU: a scripted executor and a fake
clock stand in for the device, so admission, ordering, cancellation,
deadlines, rejection and failure paths are exercised deterministically."""
import numpy as np
import pytest

from paper_1211_5595_amd.serve import RejectedError, RenderRequest, RequestTimeout, Server


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class FakeExecutor:
    """Slots that finish a batch after 1 ms + 1 us per 1000 pixels of the clock."""

    def __init__(self, clock, slots=2, resident=1000, fail_on=None):
        self.clock, self.slots, self.resident = clock, slots, resident
        self.busy = [None] * slots
        self.launched = []     # request ids in launch order
        self.batches = []
        self.fail_on = fail_on

    def has_volume(self, vid):
        return vid in ("a", "b")

    def resident_bytes(self):
        return self.resident

    @staticmethod
    def request_bytes(req):
        return req.width * req.height * 16

    def slot_free(self):
        return None in self.busy

    def launch(self, reqs):
        if self.fail_on is not None and any(r.camera == self.fail_on for r in reqs):
            raise RuntimeError("device error")
        k = self.busy.index(None)
        dur = 1e-3 + sum(r.width * r.height for r in reqs) * 1e-9
        self.busy[k] = (self.clock() + dur, [r.camera for r in reqs])
        self.launched += [r.camera for r in reqs]
        self.batches.append([r.camera for r in reqs])
        return k

    def poll(self, k):
        return self.clock() >= self.busy[k][0]

    def finish(self, k):
        _, ids = self.busy[k]
        self.busy[k] = None
        return [f"img{i}" for i in ids], [1] * len(ids)


def req(i, side=64, vid="a", deadline=None):
    return RenderRequest(vid, i, side, side, np.zeros((4, 4), np.float32), deadline=deadline)


def run_until_idle(srv, clock, dt=1e-4, limit=100000):
    for _ in range(limit):
        srv.run_once()
        if not srv.pending():
            return
        clock.t += dt
    raise AssertionError("server did not drain")


def test_fifo_admission_and_completion():
    clock = Clock()
    ex = FakeExecutor(clock)
    srv = Server(ex, budget_bytes=10 ** 9, max_batch=4, clock=clock)
    futs = [srv.submit(req(i)) for i in range(10)]
    run_until_idle(srv, clock)
    assert ex.launched == list(range(10))
    assert [f.result() for f in futs] == [f"img{i}" for i in range(10)]
    assert all(len(b) <= 4 for b in ex.batches)


def test_budget_never_exceeded_and_big_head_not_starved():
    clock = Clock()
    ex = FakeExecutor(clock, slots=3, resident=1000)
    budget = 1000 + 3 * 256 * 256 * 16
    srv = Server(ex, budget_bytes=budget, max_batch=8, clock=clock)
    rng = np.random.default_rng(0)
    sides = [int(s) for s in rng.choice([64, 128, 256], size=60)]
    futs = []
    for i, s in enumerate(sides):
        futs.append(srv.submit(req(i, s)))
        srv.run_once()
        assert srv.peak_bytes <= budget
        clock.t += float(rng.exponential(2e-4))
    run_until_idle(srv, clock)
    assert srv.peak_bytes <= budget
    assert ex.launched == list(range(60))        # FIFO even when the head is the largest
    assert all(f.result().startswith("img") for f in futs)


def test_reject_impossible_and_unknown():
    clock = Clock()
    srv = Server(FakeExecutor(clock, resident=1000), budget_bytes=1000 + 100 * 100 * 16, clock=clock)
    with pytest.raises(RejectedError):
        srv.submit(req(0, side=101)).result(0)
    with pytest.raises(RejectedError):
        srv.submit(req(1, vid="zzz")).result(0)
    ok = srv.submit(req(2, side=100))
    run_until_idle(srv, clock)
    assert ok.result() == "img2"


def test_cancel_and_deadline():
    clock = Clock()
    ex = FakeExecutor(clock, slots=1)
    srv = Server(ex, budget_bytes=10 ** 9, max_batch=1, clock=clock)
    f0 = srv.submit(req(0, side=512))             # occupies the only slot for ~1.3 ms
    srv.run_once()
    f1 = srv.submit(req(1))
    f2 = srv.submit(req(2, deadline=clock.t + 5e-4))
    f3 = srv.submit(req(3))
    assert f1.cancel()
    run_until_idle(srv, clock)
    with pytest.raises(RuntimeError, match="cancelled"):
        f1.result(0)
    with pytest.raises(RequestTimeout):
        f2.result(0)
    assert f0.result() == "img0" and f3.result() == "img3"
    assert ex.launched == [0, 3]
    assert not f0.cancel()                         # too late once finished


def test_device_error_fails_batch_and_server_continues():
    clock = Clock()
    ex = FakeExecutor(clock, slots=1, fail_on=1)
    srv = Server(ex, budget_bytes=10 ** 9, max_batch=1, clock=clock)
    futs = [srv.submit(req(i)) for i in range(3)]
    run_until_idle(srv, clock)
    assert futs[0].result() == "img0" and futs[2].result() == "img2"
    with pytest.raises(RuntimeError, match="device error"):
        futs[1].result(0)
    assert srv.inflight_bytes == 0


def test_deterministic_replay_of_poisson_trace():
    import workloads as W

    def replay():
        clock = Clock()
        ex = FakeExecutor(clock, slots=2)
        srv = Server(ex, budget_bytes=10 ** 9, max_batch=16, clock=clock)
        trace = W.poisson_requests(300, 200, rate_hz=2000.0, n_volumes=2,
                                   volume_dims=[(64, 64, 32), (64, 64, 32)])
        futs = []
        for k, r in enumerate(trace):
            while clock.t < r["t"]:
                srv.run_once()
                clock.t = min(r["t"], clock.t + 1e-4)
            futs.append(srv.submit(req(k, side=r["side"] // 4, vid="ab"[r["volume"]])))
        run_until_idle(srv, clock)
        return ex.batches, [round(f.latency, 12) for f in futs]

    a, b = replay(), replay()
    assert a == b
    assert max(len(x) for x in a[0]) > 1          # arrivals during a batch were batched together


def test_background_thread_drains():
    import time
    ex = FakeExecutor(time.perf_counter, slots=2)
    srv = Server(ex, budget_bytes=10 ** 9, max_batch=8)
    srv.start()
    futs = [srv.submit(req(i)) for i in range(50)]
    srv.stop(drain=True)
    assert [f.result(1.0) for f in futs] == [f"img{i}" for i in range(50)]
    assert srv.latency_stats()["n"] == 50
