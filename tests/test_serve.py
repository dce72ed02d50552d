"""Serving scheduler on the CPU: a simulated executor and a virtual clock drive the
same Scheduler that runs the GPU requests (continuous batching, FIFO admission by
slots and byte budget, retry of frames that outgrew their bound)."""
import numpy as np

from paper_2503_01199_amd.serve import Request, Scheduler, request_stream


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class Handle:
    def __init__(self, req, slot, ready):
        self.req, self.slot, self.ready, self.views = req, slot, ready, 1


class Token:
    def __init__(self, done, members):
        self.done, self.members = done, members


class FakeExecutor:
    """Preparation takes `prep` s per request (overlapping across slots); a batch
    rasters after all its members are prepared and takes `raster` s per member."""

    def __init__(self, clock, prep=1e-3, raster=2e-3, overflow=None):
        self.clock = clock
        self.prep, self.raster = prep, raster
        self.overflow = dict(overflow or {})   # rid -> bytes it reports needing, once
        self.in_use = 0
        self.max_in_use = 0
        self.started, self.launched, self.finished = [], [], []

    def bytes_needed(self, req):
        return req.size

    def start(self, req, slot):
        self.in_use += 1
        self.max_in_use = max(self.max_in_use, self.in_use)
        self.started.append((self.clock.t, req.rid, slot))
        return Handle(req, slot, self.clock.t + self.prep)

    def launch(self, handles):
        t0 = max([self.clock.t] + [h.ready for h in handles])
        tok = Token(t0 + self.raster * len(handles), [h.req.rid for h in handles])
        self.launched.append((self.clock.t, tok))
        return tok

    def poll(self, token):
        return self.clock.t >= token.done

    def finish(self, h):
        self.in_use -= 1
        self.finished.append((self.clock.t, h.req.rid))
        if h.req.rid in self.overflow:
            return False, self.overflow.pop(h.req.rid)
        return True, 0


def _requests(n, gap, size=100):
    out = []
    for i in range(n):
        r = Request(i, "s", None, i * gap)
        r.size = size
        out.append(r)
    return out


def _run(reqs, ex, clock, **kw):
    def idle(t_next):
        clock.t = t_next if t_next is not None else clock.t + 1e-4
    return Scheduler(ex, **kw).run(reqs, clock=clock, idle=idle)


def test_every_request_completes_once_in_fifo_admission_order():
    clock = Clock()
    ex = FakeExecutor(clock)
    reqs = _requests(50, 0.5e-3)
    st = _run(reqs, ex, clock, budget_bytes=10_000, slots=4)
    assert len(st.latencies) == 50
    assert sorted(rid for _, rid in ex.finished) == list(range(50))
    assert [rid for _, rid, _ in ex.started] == list(range(50))  # admitted in arrival order
    assert all(r.done >= r.admitted >= r.arrival for r in reqs)
    assert ex.max_in_use <= 4


def test_budget_bounds_bytes_in_flight_and_forces_queueing():
    clock = Clock()
    ex = FakeExecutor(clock, prep=1e-3, raster=3e-3)
    reqs = _requests(20, 0.2e-3, size=100)
    st = _run(reqs, ex, clock, budget_bytes=250, slots=8)
    assert st.max_bytes_in_use <= 250
    assert ex.max_in_use == 2  # the budget, not the 8 slots, limits the flight
    assert max(st.admission_waits) > 0.0
    assert len(st.latencies) == 20


def test_arrivals_are_admitted_while_earlier_batches_run():
    """Continuous batching: a request that arrives while a batch is on the device is
    prepared and launched before that batch completes."""
    clock = Clock()
    ex = FakeExecutor(clock, prep=0.5e-3, raster=5e-3)
    reqs = _requests(10, 1e-3)
    _run(reqs, ex, clock, budget_bytes=10_000, slots=8)
    (t1, first), (t2, second) = ex.launched[0], ex.launched[1]
    assert t2 < first.done  # the second launch happened while the first batch was in flight
    assert len(ex.launched) >= 2


def test_batches_hold_everything_prepared_in_a_tick():
    clock = Clock()
    ex = FakeExecutor(clock, prep=1e-3, raster=1e-3)
    reqs = _requests(12, 0.0)  # all arrive at once
    st = _run(reqs, ex, clock, budget_bytes=10_000, slots=16, max_batch=5)
    assert st.batch_sizes[:3] == [5, 5, 2]


def test_frame_that_outgrew_its_bound_is_retried_with_the_reported_bytes():
    clock = Clock()
    ex = FakeExecutor(clock, overflow={3: 180})
    reqs = _requests(8, 1e-3, size=100)
    st = _run(reqs, ex, clock, budget_bytes=1000, slots=4)
    assert st.retries == 1 and reqs[3].retries == 1 and reqs[3].nbytes == 180
    assert len(st.latencies) == 8
    assert [rid for _, rid, _ in ex.started].count(3) == 2


def test_request_larger_than_the_budget_is_rejected_without_blocking_others():
    clock = Clock()
    ex = FakeExecutor(clock)
    reqs = _requests(6, 1e-3, size=100)
    reqs[2].size = 10_000
    st = _run(reqs, ex, clock, budget_bytes=500, slots=4)
    assert st.rejected == 1 and reqs[2].rejected
    assert len(st.latencies) == 5


def test_request_stream_is_poisson_and_mixes_resolutions():
    reqs = request_stream({"a": 6.0, "b": 3.0}, 4000, rate=200.0, seed=3)
    gaps = np.diff([0.0] + [r.arrival for r in reqs])
    assert abs(gaps.mean() - 1 / 200.0) < 0.1 / 200.0
    assert abs(gaps.std() / gaps.mean() - 1.0) < 0.1  # exponential: cv = 1
    sizes = {(r.camera.width, r.camera.height) for r in reqs}
    assert sizes == {(256, 256), (512, 512), (1280, 720), (1920, 1080)}
    assert {r.scene for r in reqs} == {"a", "b"}
