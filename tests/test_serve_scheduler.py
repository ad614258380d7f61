"""The serving scheduler on the CPU with a fake executor and a virtual clock
(no GPU): admission in arrival order under the slot, byte and ray limits, the
backlog, reuse of freed slots, cancellation before and after admission, and
failures injected at admission and in a step."""
import dataclasses

import pytest

from paper_2005_11976_amd.serve import Scheduler


@dataclasses.dataclass
class Req:
    rid: int
    cls: int
    arrival: float


class Handle:
    def __init__(self, q, total):
        self.q, self.total, self.cursor, self.rec = q, total, 0, None


class FakeExecutor:
    """Steps take `dt` seconds of virtual time; admissions and steps can be
    made to fail; every call is logged."""

    def __init__(self, steps_of, dt=1.0, fail_admit=(), fail_step_at=None):
        self.t, self.dt, self.steps_of = 0.0, dt, steps_of
        self.fail_admit, self.fail_step_at = set(fail_admit), fail_step_at
        self.log, self.live, self.released = [], set(), []
        self.step_sizes = []

    def now(self):
        return self.t

    def wait_until(self, t):
        self.t = max(self.t, t)

    def admit(self, q, now):
        if q.rid in self.fail_admit:
            raise RuntimeError("admission of %d failed" % q.rid)
        self.log.append(("admit", q.rid, now))
        self.live.add(q.rid)
        return Handle(q, self.steps_of[q.cls])

    def step(self, hs):
        self.step_sizes.append(len(hs))
        if self.fail_step_at is not None and len(self.step_sizes) == self.fail_step_at:
            raise RuntimeError("step failed")
        self.t += self.dt

    def finish(self, h, rec):
        rec.finished = self.t
        rec.latency = self.t - rec.arrival
        return ("result", h.q.rid)

    def release(self, h):
        self.released.append(h.q.rid)
        self.live.discard(h.q.rid)

    def drain(self, records):
        pass


def sched(max_active=4, budget=100, fill=10):
    # class 0: 10 bytes, 2 rays; class 1: 40 bytes, 6 rays
    return Scheduler(lambda c: (10, 40)[c], lambda c: (2, 6)[c], max_active, budget, 0, fill)


def test_all_served_in_arrival_order_with_slot_reuse():
    reqs = [Req(i, 0, 0.5 * i) for i in range(10)]
    ex = FakeExecutor(steps_of=(3, 3))
    recs, res = sched(max_active=3).run(reqs, ex)
    assert [r.status for r in recs] == ["done"] * 10
    assert set(res) == set(range(10))
    admits = [e[1] for e in ex.log if e[0] == "admit"]
    assert admits == list(range(10))                 # arrival order
    assert max(ex.step_sizes) == 3                   # never more than the slots
    assert len(ex.step_sizes) < 10 * 3               # scans shared steps
    assert not ex.live and sorted(ex.released) == list(range(10))   # every slot freed


def test_budget_and_ray_cap_limit_admission():
    # two class-1 scans would need 80 bytes (fits 100) but 12 rays (cap 10):
    # they run one after the other (admission in order blocks the class-0
    # scans behind the second), then the second packs with both class-0 ones
    reqs = [Req(0, 1, 0.0), Req(1, 1, 0.0), Req(2, 0, 0.0), Req(3, 0, 0.0)]
    ex = FakeExecutor(steps_of=(2, 2))
    s = sched(max_active=4, budget=100, fill=10)
    recs, _ = s.run(reqs, ex)
    assert all(r.status == "done" for r in recs)
    adm = {r.rid: r.admitted for r in recs}
    assert adm[0] == 0.0 and adm[1] == 2.0 and adm[2] == 2.0 and adm[3] == 2.0
    assert ex.step_sizes == [1, 1, 3, 3] and s.peak_active == 3
    ex2 = FakeExecutor(steps_of=(2, 2))
    s2 = sched(max_active=4, budget=45, fill=100)   # bytes: one class-1 scan at a time
    recs2, _ = s2.run([Req(0, 1, 0.0), Req(1, 1, 0.0), Req(2, 0, 0.0)], ex2)
    assert all(r.status == "done" for r in recs2) and s2.peak_active == 1
    ex3 = FakeExecutor(steps_of=(2, 2))
    s3 = sched(max_active=4, budget=100, fill=100)
    s3.run([Req(0, 0, 0.0), Req(1, 0, 0.0), Req(2, 1, 0.0)], ex3)
    assert s3.peak_active == 3                       # everything fits: one batch


def test_backlog_latency_grows_when_arrivals_outpace_service():
    reqs = [Req(i, 0, 0.1 * i) for i in range(12)]
    ex = FakeExecutor(steps_of=(4, 4))
    recs, _ = sched(max_active=2).run(reqs, ex)
    lat = [r.latency for r in recs]
    assert lat[-1] > 3 * lat[0]                      # later requests wait in the backlog
    assert all(r.admitted >= r.arrival for r in recs)


def test_cancellation_before_and_after_admission():
    reqs = [Req(i, 0, 0.0) for i in range(4)] + [Req(4, 0, 10.0)]
    ex = FakeExecutor(steps_of=(5, 5))
    # 1 is cancelled while running (t = 2), 3 waits in the queue and is cancelled at t = 1,
    # 4 is cancelled before it arrives
    recs, res = sched(max_active=2).run(reqs, ex, cancel={1: 2.0, 3: 1.0, 4: 5.0})
    st = {r.rid: r.status for r in recs}
    assert st == {0: "done", 1: "cancelled", 2: "done", 3: "cancelled", 4: "cancelled"}
    assert set(res) == {0, 2}
    assert 3 not in [e[1] for e in ex.log] and 4 not in [e[1] for e in ex.log]
    assert not ex.live                               # the cancelled scan's slot was freed


def test_injected_failures():
    reqs = [Req(i, 0, 0.0) for i in range(6)]
    ex = FakeExecutor(steps_of=(3, 3), fail_admit={2}, fail_step_at=2)
    recs, res = sched(max_active=2).run(reqs, ex)
    st = {r.rid: r.status for r in recs}
    assert st[2] == "failed" and "admission" in [r for r in recs if r.rid == 2][0].error
    # the second step failed: the two scans in it (0 and 1) fail, the rest are served
    assert st[0] == "failed" and st[1] == "failed"
    assert st[3] == st[4] == st[5] == "done" and set(res) == {3, 4, 5}
    assert not ex.live


def test_oversized_request_fails_and_queue_goes_on():
    reqs = [Req(0, 1, 0.0), Req(1, 0, 0.0)]
    ex = FakeExecutor(steps_of=(1, 1))
    recs, res = sched(budget=30).run(reqs, ex)
    assert recs[0].status == "failed" and "budget" in recs[0].error
    assert recs[1].status == "done" and set(res) == {1}


def test_bounded_bypass_of_a_head_waiting_for_rays():
    # a class-1 scan runs (6 of 10 rays); the next class-1 scan waits for rays,
    # and up to `bypass` class-0 scans behind it (2 rays each) run meanwhile
    reqs = [Req(0, 1, 0.0), Req(1, 1, 0.0)] + [Req(2 + i, 0, 0.0) for i in range(5)]
    ex = FakeExecutor(steps_of=(1, 4))
    s = Scheduler(lambda c: (10, 40)[c], lambda c: (2, 6)[c], 8, 1000, 0, 10, bypass=2)
    recs, _ = s.run(reqs, ex)
    assert all(r.status == "done" for r in recs)
    admits = [e[1] for e in ex.log if e[0] == "admit"]
    assert admits[:3] == [0, 2, 3]        # two class-0 scans pass the waiting class-1 scan
    assert admits[3] == 1                 # then the head is waited for
    assert s.bypassed == 2
    ex0 = FakeExecutor(steps_of=(1, 4))
    s0 = Scheduler(lambda c: (10, 40)[c], lambda c: (2, 6)[c], 8, 1000, 0, 10, bypass=0)
    s0.run(reqs, ex0)
    assert [e[1] for e in ex0.log if e[0] == "admit"][:2] == [0, 1]   # strict arrival order
