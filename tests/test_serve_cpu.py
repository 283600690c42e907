"""Scheduling logic of the continuous-batching server, on a stand-in executor
with a simulated clock (no GPU): admission by budget, arrival order, overlap
of requests that arrive while others run, and completion of every request."""
import pytest

from paper_2506_12761_amd.serve import BudgetExceeded, Executor, Request, serve

LEVELS = {"intv": 19, "cov": 7, "idm": 23}


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += dt


class FakeExecutor(Executor):
    """Programs with a level count and a memory size; one step = step_s seconds."""

    def __init__(self, clock, budget, step_s=0.1):
        self.clock, self.budget, self.step_s = clock, budget, step_s
        self.used = 0
        self.left = {}
        self.size = {}
        self.step_log = []
        self._n = 0

    def create(self, req):
        need = req.M
        if self.used + need > self.budget:
            raise BudgetExceeded("no room")
        self._n += 1
        h = self._n
        self.used += need
        self.left[h] = LEVELS[req.mode]
        self.size[h] = need
        return h

    def step(self, handles):
        self.step_log.append(sorted(handles))
        for h in handles:
            self.left[h] = max(0, self.left[h] - 1)
        self.clock.t += self.step_s

    def levels_left(self, h):
        return self.left[h]

    def destroy(self, h):
        self.used -= self.size.pop(h)
        del self.left[h]


def _reqs(spec):
    return [Request(i, client=i % 3, mode=m, M=M, l_I=16, l_S=64, d=2, arrival=t) for i, (m, M, t) in enumerate(spec)]


def test_all_complete_and_overlap():
    clk = FakeClock()
    ex = FakeExecutor(clk, budget=10_000)
    reqs = _reqs([("intv", 100, 0.0), ("cov", 100, 0.35), ("idm", 100, 0.5)])
    st = serve(reqs, ex, clock=clk, sleep=clk.sleep)
    assert st["queries"] == 3
    by = {r.rid: r for r in st["requests"]}
    # request 1 (7 levels) arrives while request 0 runs and finishes first
    assert by[1].admitted < by[0].finished and by[1].finished < by[0].finished
    assert abs(by[0].latency - 19 * 0.1) < 1e-9
    assert st["max_active"] == 3
    # steps merge the active requests
    assert any(len(s) == 3 for s in ex.step_log)


def test_budget_admission_waits_for_memory():
    clk = FakeClock()
    ex = FakeExecutor(clk, budget=250)
    reqs = _reqs([("cov", 100, 0.0), ("cov", 100, 0.0), ("cov", 100, 0.0), ("idm", 200, 0.0)])
    st = serve(reqs, ex, clock=clk, sleep=clk.sleep)
    assert st["queries"] == 4 and st["budget_rejections"] > 0
    by = {r.rid: r for r in st["requests"]}
    assert by[2].admitted >= by[0].finished  # third waits for the first two
    assert by[3].admitted >= by[2].finished  # arrival order, no overtaking
    assert ex.used == 0


def test_request_larger_than_device_is_an_error():
    clk = FakeClock()
    ex = FakeExecutor(clk, budget=50)
    with pytest.raises(RuntimeError):
        serve(_reqs([("idm", 100, 0.0)]), ex, clock=clk, sleep=clk.sleep)


def test_idle_gaps_advance_to_next_arrival():
    clk = FakeClock()
    ex = FakeExecutor(clk, budget=1000)
    st = serve(_reqs([("cov", 10, 0.0), ("cov", 10, 5.0)]), ex, clock=clk, sleep=clk.sleep)
    lat = sorted(r.latency for r in st["requests"])
    assert all(abs(x - 0.7) < 1e-9 for x in lat)


def test_cancellation_frees_memory_for_the_queue():
    """A running request cancelled by its client releases its memory at the
    next step, so a queued one is admitted before the first would have ended;
    a request cancelled while queued is never admitted."""
    clk = FakeClock()
    ex = FakeExecutor(clk, budget=100)
    reqs = _reqs([("idm", 90, 0.0), ("cov", 80, 0.05), ("intv", 10, 0.06)])
    reqs[0].cancel_at = 0.35          # running, 23 levels: cancelled after a few steps
    reqs[2].cancel_at = 0.07          # queued behind the second: cancelled before admission
    st = serve(reqs, ex, clock=clk, sleep=clk.sleep)
    assert st["cancelled"] == 2 and st["queries"] == 1
    assert reqs[0].cancelled is not None and reqs[0].finished is None
    assert reqs[2].admitted is None and reqs[2].cancelled is not None
    assert reqs[1].finished is not None and reqs[1].admitted <= 0.45  # admitted once the first was dropped
    assert ex.used == 0 and not ex.left


def test_cancel_after_finish_is_a_noop():
    clk = FakeClock()
    ex = FakeExecutor(clk, budget=100)
    reqs = _reqs([("cov", 10, 0.0)])
    reqs[0].cancel_at = 50.0
    st = serve(reqs, ex, clock=clk, sleep=clk.sleep)
    assert st["queries"] == 1 and st["cancelled"] == 0 and reqs[0].cancelled is None


class WorkExecutor(FakeExecutor):
    """Programs whose levels have a rotation count (M per level); a step costs
    its merged rotations x step_s / 1000 seconds, like the device."""

    def create(self, req):
        h = super().create(req)
        self.work = getattr(self, "work", {})
        self.work[h] = [req.M] * LEVELS[req.mode]
        return h

    def work_left(self, h):
        return sum(self.work[h][len(self.work[h]) - self.left[h]:])

    def next_work(self, h):
        return self.work[h][len(self.work[h]) - self.left[h]] if self.left[h] else 0

    def step(self, handles):
        rot = sum(self.next_work(h) for h in handles)
        self.rot_log = getattr(self, "rot_log", []) + [(len(handles), rot)]
        super().step(handles)
        self.clock.t += rot * self.step_s / 1000 - self.step_s


def test_srpt_policy_lets_small_queries_pass_a_large_one():
    """Shortest remaining work first with a rotation cap per step: a small
    query arriving while a large one runs finishes far sooner than under
    the merge-all policy, and the large one still completes; every step
    advances at least one query and respects the cap unless one level alone
    exceeds it."""
    spec = [("idm", 4000, 0.0), ("cov", 10, 0.5), ("cov", 10, 0.6)]
    res = {}
    for policy in ("all", "srpt"):
        clk = FakeClock()
        ex = WorkExecutor(clk, budget=10_000)
        st = serve(_reqs(spec), ex, clock=clk, sleep=clk.sleep, policy=policy, step_cap=100)
        assert st["queries"] == 3 and st["policy"] == policy
        res[policy] = {r.rid: r.latency for r in st["requests"]}
        assert all(len(s) >= 1 for s in ex.step_log)
        if policy == "srpt":
            assert all(n == 1 or rot <= 100 for n, rot in ex.rot_log)
            assert any(n == 1 and rot > 100 for n, rot in ex.rot_log)  # the large level runs alone
    assert res["srpt"][1] < 0.2 * res["all"][1] and res["srpt"][2] < 0.2 * res["all"][2]
    assert res["srpt"][0] <= res["all"][0] + 0.5  # the large query loses little


def test_srpt_selection_order_and_cap():
    from paper_2506_12761_amd.serve import select_step

    class Ex(FakeExecutor):
        def __init__(self):
            pass

        def work_left(self, h):
            return {1: 500, 2: 50, 3: 80, 4: 5000}[h]

        def next_work(self, h):
            return {1: 100, 2: 10, 3: 60, 4: 900}[h]

    reqs = _reqs([("idm", 1, 0.0), ("idm", 1, 0.0), ("idm", 1, 0.0), ("idm", 1, 0.0)])
    for h, r in zip((1, 2, 3, 4), reqs):
        r.handle = h
    pick = lambda cap: [r.handle for r in select_step(reqs, Ex(), "srpt", cap)]
    assert pick(None) == [2, 3, 1, 4]          # no cap: all, least remaining work first
    assert pick(100) == [2, 3]                 # 10 + 60; 100 more would pass the cap
    assert pick(200) == [2, 3, 1]
    assert pick(5) == [2]                      # always at least one
    assert [r.handle for r in select_step(reqs, Ex(), "all", 5)] == [1, 2, 3, 4]
    with pytest.raises(ValueError):
        select_step(reqs, Ex(), "fastest", None)


def test_input_bytes_of_each_mode():
    """The executor's estimate of a request's buffers: query, locations,
    payload, R and v, each 631 words of 4 bytes."""
    from paper_2506_12761_amd.serve import GpuExecutor
    ct = 631 * 4
    r = Request(0, 0, "intv", 10, 16, 64, 2, arrival=0.0)
    assert GpuExecutor._input_bytes(r) == ct * (2 * 16 + 10 * 2 * 2 * 16 + 10 * 64 + 64 + 10)
    r = Request(0, 0, "cov", 7, 20, 3, 2, arrival=0.0)
    assert GpuExecutor._input_bytes(r) == ct * (2 * 20 + 7 * 2 * 20 + 7 * 3 + 3 + 7)
    r = Request(0, 0, "idm", 5, 32, 0, 1, arrival=0.0)
    assert GpuExecutor._input_bytes(r) == ct * (32 + 5 * 32 + 0 + 0 + 5)
