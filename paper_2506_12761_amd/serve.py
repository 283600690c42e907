"""Continuous-batching server for PIR queries over the bootstrapping library.

Requests arrive over time, each a full VeLoPIR query (Algorithm 3) of one
client against that client's encrypted database, in one of the three modes.
The loop keeps every client's keys resident, admits a request when its
program (gate schedule plus intermediate ciphertexts) fits the device-memory
budget, and advances all admitted requests together: every step runs the
current circuit level of every active request in one merged batch of kernel
launches, so a request admitted while others are running joins at the next
step, and finished requests free their memory for queued ones.

Which admitted requests a step advances is the policy: "all" (every active
request, one level each) or "srpt" (shortest remaining work first: active
requests in order of blind rotations left, added while the step's rotations
stay within a cap, at least one per step), which keeps a small query from
waiting behind the huge levels of large ones.

The executor is an interface so the scheduling logic can be exercised on a
CPU with a stand-in executor; GpuExecutor drives libvlp.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field


class BudgetExceeded(Exception):
    """The executor cannot hold the request's program right now."""


@dataclass
class Request:
    rid: int
    client: int
    mode: str
    M: int
    l_I: int
    l_S: int
    d: int
    arrival: float                # seconds since the start of the run
    payload: dict = field(default_factory=dict)  # executor-specific buffers
    cancel_at: float | None = None  # the client withdraws the query at this offset, if not done by then
    admitted: float | None = None
    finished: float | None = None
    cancelled: float | None = None  # when the server dropped it after cancellation
    handle: object = None

    @property
    def latency(self) -> float | None:
        return None if self.finished is None else self.finished - self.arrival


class Executor:
    """What the server needs from a backend."""

    def create(self, req: Request):            # -> handle; raises BudgetExceeded
        raise NotImplementedError

    def step(self, handles: list) -> None:     # advance each unfinished handle by one level, wait for it
        raise NotImplementedError

    def levels_left(self, handle) -> int:
        raise NotImplementedError

    def work_left(self, handle) -> int:        # blind rotations left (for the srpt policy)
        return self.levels_left(handle)

    def next_work(self, handle) -> int:        # blind rotations of the next level
        return 1

    def destroy(self, handle) -> None:
        raise NotImplementedError

    def fetch(self, req: "Request") -> None:  # copy a finished request's result to the host
        pass


KEYSET_BYTES = 61931520 + 83886080  # transformed bootstrapping key + key-switching byte planes


class GpuExecutor(Executor):
    """libvlp programs on one device.

    keysets[client] may be loaded beforehand; otherwise key_factory(client)
    returns the client's (bk, ksk) device tensors, loaded at admission and
    dropped when the client has no request left.  input_factory(req), if
    given, returns the request's payload of device buffers (query, db_loc,
    db_pay, R, v), allocated at admission and released at destruction.  With
    `budget` (bytes), a request is admitted only while the library's memory,
    the resident keys and the held input buffers, plus what the request would
    add (its program by vlp_plan_bytes, its inputs, its keys), fit."""

    def __init__(self, ctx, keysets: dict | None = None, key_factory=None, input_factory=None,
                 budget: int | None = None):
        from . import vlp
        self.vlp = vlp
        self.ctx = ctx
        self.keysets = dict(keysets or {})
        self.key_factory = key_factory
        self.input_factory = input_factory
        self.budget = budget
        self._left = {}
        self._levels = {}
        self._req = {}
        self._users = {}
        self.input_bytes = 0

    @staticmethod
    def _input_bytes(req: Request) -> int:
        """Device bytes of a request's buffers: query, database locations and
        payload, R and v (631-word ciphertexts)."""
        d = req.d if req.mode != "idm" else 1
        loc = req.M * d * (2 if req.mode == "intv" else 1) * req.l_I
        return 631 * 4 * (d * req.l_I + loc + req.M * req.l_S + req.l_S + req.M)

    def held(self) -> int:
        """Device bytes held: the library's (programs, keysets, scratch) and the inputs."""
        return self.vlp.vlp_mem_info(self.ctx.ctx)[0] + self.input_bytes

    def create(self, req: Request):
        v = self.vlp
        shape = v.make_shape(req.mode, req.M, req.l_I, req.l_S, req.d)
        new_keys = req.client not in self.keysets
        in_bytes = self._input_bytes(req) if self.input_factory else 0
        if self.budget is not None:
            need = v.vlp_plan_bytes(shape, True) + in_bytes + (KEYSET_BYTES if new_keys else 0)
            if self.held() + need > self.budget:
                raise BudgetExceeded("request %d needs %d bytes; %d of %d held" % (req.rid, need, self.held(),
                                                                                  self.budget))
        if new_keys:
            bk, ksk = self.key_factory(req.client)
            self.keysets[req.client] = self.ctx.load_keys(bk, ksk)
            del bk, ksk
        if self.input_factory:
            req.payload = self.input_factory(req)
            self.input_bytes += in_bytes
        p = req.payload
        try:
            h = v.vlp_program_create(self.ctx.ctx, self.keysets[req.client], shape, p["query"], p["db_loc"],
                                     p.get("db_pay"), p.get("R"), p.get("v"))
        except v.VlpError as e:
            self._release(req, in_bytes, new_keys)
            if e.status == v.VLP_EBUDGET:
                raise BudgetExceeded(str(e)) from None
            raise
        n = v.vlp_program_counts(self.ctx.ctx, h)["levels"]
        self._levels[h] = [v.vlp_program_level_counts(self.ctx.ctx, h, L)["blind_rotations"] for L in range(n)]
        self._left[h] = n
        self._req[h] = (req, in_bytes)
        self._users[req.client] = self._users.get(req.client, 0) + 1
        return h

    def _release(self, req: Request, in_bytes: int, drop_keys: bool) -> None:
        if self.input_factory:
            kept = {"R_host": req.payload["R_host"]} if "R_host" in req.payload else {}
            req.payload = kept
            self.input_bytes -= in_bytes
        if drop_keys and self.key_factory and req.client in self.keysets:
            self.ctx.drop_keys(self.keysets.pop(req.client))
        if self.input_factory or self.key_factory:
            # Freed tensors go back to the device, not to torch's cache, so the
            # library's own allocations can use the memory.
            self.ctx.torch.cuda.empty_cache()

    def step(self, handles):
        if not handles:
            return
        self.vlp.vlp_step(self.ctx.ctx, handles)
        self.vlp.vlp_sync(self.ctx.ctx)
        for h in handles:
            if self._left[h] > 0:
                self._left[h] -= 1

    def levels_left(self, handle) -> int:
        return self._left[handle]

    def work_left(self, handle) -> int:
        lv = self._levels[handle]
        return sum(lv[len(lv) - self._left[handle]:])

    def next_work(self, handle) -> int:
        lv = self._levels[handle]
        return lv[len(lv) - self._left[handle]] if self._left[handle] else 0

    def destroy(self, handle):
        self._left.pop(handle, None)
        self._levels.pop(handle, None)
        self.vlp.vlp_program_destroy(self.ctx.ctx, handle)
        req, in_bytes = self._req.pop(handle)
        self._users[req.client] -= 1
        self._release(req, in_bytes, self._users[req.client] == 0)

    def fetch(self, req):
        R = req.payload.get("R")
        req.payload["R_host"] = self.ctx.to_host(R).copy() if R is not None else None


def select_step(active: list, executor: Executor, policy: str, step_cap: int | None) -> list:
    """The active requests a step advances (see the module docstring)."""
    if policy == "all":
        return list(active)
    if policy != "srpt":
        raise ValueError("unknown policy %r" % policy)
    order = sorted(active, key=lambda r: (executor.work_left(r.handle), r.arrival, r.rid))
    chosen, total = [], 0
    for r in order:
        w = executor.next_work(r.handle)
        if chosen and step_cap is not None and total + w > step_cap:
            continue
        chosen.append(r)
        total += w
    return chosen


def serve(requests: list[Request], executor: Executor, max_active: int | None = None,
          clock=time.perf_counter, sleep=time.sleep, log=None, policy: str = "all",
          step_cap: int | None = None) -> dict:
    """Run the request stream to completion; returns latency statistics.

    Arrival times are offsets from the start.  A request is admitted at the
    first step boundary after its arrival at which the executor accepts it
    (arrival order, no overtaking); each step advances the admitted requests
    the policy selects by one circuit level each.  A request's latency runs
    from its arrival to its result copied to the host.  A request whose
    cancel_at has passed is dropped at the next step boundary: never admitted
    if still queued, otherwise its program is destroyed and its memory freed
    for the queue."""
    pending = sorted(requests, key=lambda r: (r.arrival, r.rid))
    waiting: list[Request] = []
    active: list[Request] = []
    done: list[Request] = []
    dropped: list[Request] = []
    t0 = clock()
    steps = 0
    max_active_seen = 0
    rejected_attempts = 0
    while pending or waiting or active:
        now = clock() - t0
        while pending and pending[0].arrival <= now:
            waiting.append(pending.pop(0))
        # Cancellations: queued requests leave the queue, running ones free their memory.
        gone = [r for r in waiting + active if r.cancel_at is not None and r.cancel_at <= now]
        for r in gone:
            if r.handle is not None:
                executor.destroy(r.handle)
                r.handle = None
            r.cancelled = now
            dropped.append(r)
        if gone:
            waiting = [r for r in waiting if r.cancelled is None]
            active = [r for r in active if r.cancelled is None]
            if not (pending or waiting or active):
                break
        # Admission in arrival order while memory allows.
        while waiting and (max_active is None or len(active) < max_active):
            r = waiting[0]
            try:
                r.handle = executor.create(r)
            except BudgetExceeded:
                rejected_attempts += 1
                break
            r.admitted = clock() - t0
            active.append(waiting.pop(0))
        if not active:
            if not waiting and pending:  # idle until the next arrival
                sleep(max(0.0, pending[0].arrival - (clock() - t0)))
                continue
            if waiting:
                raise RuntimeError("request %d cannot be admitted even on an idle device" % waiting[0].rid)
            continue
        executor.step([r.handle for r in select_step(active, executor, policy, step_cap)])
        steps += 1
        max_active_seen = max(max_active_seen, len(active))
        still = []
        for r in active:
            if executor.levels_left(r.handle) == 0:
                executor.fetch(r)  # the result on the host ends the request's latency
                r.finished = clock() - t0
                executor.destroy(r.handle)
                r.handle = None
                done.append(r)
            else:
                still.append(r)
        active = still
        if log and steps % 10 == 0:
            log("step %d: %d active, %d waiting, %d done" % (steps, len(active), len(waiting), len(done)))
    wall = clock() - t0
    lat = sorted(r.latency for r in done)
    return {
        "policy": policy,
        "step_cap": step_cap,
        "queries": len(done),
        "wall_s": wall,
        "queries_per_s": len(done) / wall if wall > 0 else None,
        "p50_ms": 1e3 * percentile(lat, 50),
        "p99_ms": 1e3 * percentile(lat, 99),
        "mean_ms": 1e3 * sum(lat) / len(lat) if lat else None,
        "steps": steps,
        "max_active": max_active_seen,
        "budget_rejections": rejected_attempts,
        "cancelled": len(dropped),
        "requests": done,
    }


def percentile(xs, p):
    if not xs:
        return float("nan")
    xs = sorted(xs)
    k = (len(xs) - 1) * p / 100.0
    f = int(k)
    c = min(f + 1, len(xs) - 1)
    return xs[f] + (xs[c] - xs[f]) * (k - f)


def poisson_arrivals(rate: float, count: int, rng) -> list[float]:
    """Arrival offsets of a Poisson process of the given rate (per second)."""
    t, out = 0.0, []
    for _ in range(count):
        t += float(rng.exponential(1.0 / rate))
        out.append(t)
    return out

