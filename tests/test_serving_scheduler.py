"""CPU tests of the serving loop's admission and grouping logic (no GPU)."""

import dataclasses

import pytest

from paper_0807_4494_amd.serving import (BATCH_MAX, SEG_MAX, Scheduler, Server, footprint_bytes, pair_order,
                                         percentile)


@dataclasses.dataclass
class Req:
    rid: int
    L: int
    spin: int
    batch: int
    arrival_s: float = 0.0
    seed: int = 0
    timeout_s: float = None


def ws(L, spin, batch):
    # same shape as the library's: two regions of max(panel, grid) FP32 reals
    N = 2 * L - 1
    r = max(L * 4 * batch * L * 4, batch * L * N * 2 * 4)
    return 2 * ((r + 255) // 256 * 256)


def test_footprint_counts_buffers_and_workspace():
    L, B = 64, 3
    N = 2 * L - 1
    assert footprint_bytes(L, B, 1000) == B * (2 * L * L + L * N) * 8 + 1000
    assert footprint_bytes(L, B, 0, cbytes=16) == B * (2 * L * L + L * N) * 16


def test_groups_same_L_and_spin_in_arrival_order():
    s = Scheduler(1 << 40, ws, by_spin=True)
    reqs = [Req(0, 64, 0, 2), Req(1, 128, 0, 1), Req(2, 64, 0, 5), Req(3, 64, 1, 1), Req(4, 64, 0, 1)]
    for r in reqs:
        s.arrive(r)
    g = s.next_group()
    assert [r.rid for r in g.requests] == [0, 2, 4] and g.batch == 8 and (g.L, g.spin) == (64, 0)
    assert g.nbytes == footprint_bytes(64, 8, ws(64, 0, 8))
    g2 = s.next_group()
    assert [r.rid for r in g2.requests] == [1]
    g3 = s.next_group()
    assert [r.rid for r in g3.requests] == [3]
    assert s.next_group() is None
    assert s.used == g.nbytes + g2.nbytes + g3.nbytes
    for grp in (g, g2, g3):
        s.release(grp)
    assert s.used == 0


def test_group_respects_batch_limit():
    s = Scheduler(1 << 40, ws)
    for i in range(5):
        s.arrive(Req(i, 64, 2, 30))
    g = s.next_group()
    assert g.batch <= BATCH_MAX and [r.rid for r in g.requests] == [0, 1]
    g = s.next_group()
    assert [r.rid for r in g.requests] == [2, 3]


def test_admission_by_memory_keeps_head_of_line_order():
    one = footprint_bytes(256, 4, ws(256, 0, 4))
    s = Scheduler(int(1.5 * one), ws)
    s.arrive(Req(0, 256, 0, 4))
    s.arrive(Req(1, 256, 0, 4))     # would not fit beside request 0 in one group
    s.arrive(Req(2, 64, 0, 1))      # small, but behind request 1
    g0 = s.next_group()
    assert [r.rid for r in g0.requests] == [0]
    # request 1 does not fit while 0 is in flight, and 2 may not overtake it
    assert s.next_group() is None
    s.release(g0)
    g1 = s.next_group()
    assert [r.rid for r in g1.requests] == [1]
    g2 = s.next_group()
    assert [r.rid for r in g2.requests] == [2]


def test_requests_that_can_never_fit_are_rejected():
    s = Scheduler(1000, ws)
    with pytest.raises(ValueError):
        s.arrive(Req(0, 64, 0, 1))
    s2 = Scheduler(1 << 40, ws)
    with pytest.raises(ValueError):
        s2.arrive(Req(0, 64, 0, BATCH_MAX + 1))


def test_percentile_nearest_rank():
    xs = list(range(1, 101))
    assert percentile(xs, 50) == 50
    assert percentile(xs, 99) == 99
    assert percentile(xs, 100) == 100
    assert percentile([3.0], 99) == 3.0


def test_groups_same_L_across_spins_in_segments():
    s = Scheduler(1 << 40, ws)
    reqs = [Req(0, 64, 0, 2), Req(1, 128, 0, 1), Req(2, 64, 2, 5), Req(3, 64, 0, 1), Req(4, 64, -2, 3)]
    for r in reqs:
        s.arrive(r)
    g = s.next_group()
    # one call at L = 64: segments in order of first appearance, requests grouped by segment
    assert g.L == 64 and g.segments == [(0, 3), (2, 5), (-2, 3)] and g.batch == 11
    assert [r.rid for r in g.requests] == [0, 3, 2, 4]
    assert g.spin is None
    g2 = s.next_group()
    assert [r.rid for r in g2.requests] == [1] and g2.spin == 0


def test_opposite_spins_are_adjacent_segments():
    # -s right after s, so that the library shares one contraction between them
    assert pair_order([1, 2, 0, -1, -2, 3]) == [1, -1, 2, -2, 0, 3]
    assert pair_order([0, -2, 1, 2]) == [0, -2, 2, 1]
    assert pair_order([0]) == [0]
    s = Scheduler(1 << 40, ws)
    for r in [Req(0, 64, 1, 2), Req(1, 64, 2, 1), Req(2, 64, -1, 3), Req(3, 64, 1, 1)]:
        s.arrive(r)
    g = s.next_group()
    assert g.segments == [(1, 3), (-1, 3), (2, 1)]
    assert [r.rid for r in g.requests] == [0, 3, 2, 1]


def test_group_respects_segment_limit():
    s = Scheduler(1 << 40, ws)
    for i in range(SEG_MAX + 2):
        s.arrive(Req(i, 64, i, 1))
    g = s.next_group()
    assert len(g.segments) == SEG_MAX and [r.rid for r in g.requests] == list(range(SEG_MAX))
    assert [r.rid for r in s.next_group().requests] == [SEG_MAX, SEG_MAX + 1]


# ---- the loop over a simulated executor: timing, timeouts, cancels, faults ----

class FakeExecutor:
    """Virtual clock; a group takes service(group) seconds after its launch;
    launches numbered in ``fail_launch`` raise, completions in
    ``fail_complete`` report failure."""
    cbytes = 8

    def __init__(self, service=lambda g: 1e-3 * g.batch, fail_launch=(), fail_complete=(), tick=1e-4):
        self.service, self.fail_launch, self.fail_complete, self.tick = service, set(fail_launch), \
            set(fail_complete), tick
        self.launched = []

    def workspace(self, L, spin, batch):
        return ws(L, spin, batch)

    def begin(self):
        self.t = 0.0

    def now(self):
        return self.t

    def idle(self):
        self.t += self.tick

    def end(self):
        pass

    def launch(self, group, slot, keep):
        k = len(self.launched)
        self.launched.append(group)
        if k in self.fail_launch:
            raise RuntimeError("injected launch failure")
        kept = {r.rid: ("outputs of", r.rid) for r in group.requests if r.rid in keep}
        return {"k": k, "done": self.t + self.service(group)}, kept

    def poll(self, h):
        if self.t < h["done"]:
            return None
        if h["k"] in self.fail_complete:
            return ("failed", "injected completion failure")
        return ("ok", h["done"])


def _status(results):
    return {r.rid: r.status for r in results}


def test_loop_serves_every_request_in_same_L_groups():
    ex = FakeExecutor()
    srv = Server(ex, streams=1, budget_bytes=1 << 40)
    reqs = [Req(0, 64, 0, 1), Req(1, 96, 1, 2), Req(2, 64, -1, 3), Req(3, 96, 1, 1), Req(4, 64, 2, 1)]
    res, kept, st = srv.run(reqs, keep=[2], closed_loop=True)
    assert _status(res) == {i: "ok" for i in range(5)}
    assert [g.L for g in ex.launched] == [64, 96]
    assert ex.launched[0].segments == [(0, 1), (-1, 3), (2, 1)]
    assert kept == {2: ("outputs of", 2)}
    assert st["requests"] == 5 and st["mean_group_size"] == (3 * 3 + 2 * 2) / 5
    assert st["failed"] == st["timeouts"] == st["cancelled"] == 0


def test_waiting_requests_time_out():
    # one slot, busy 10 ms with request 0; requests 1 and 2 (other L, so not
    # grouped with it) wait; 1 has a 5 ms deadline, 2 none
    ex = FakeExecutor(service=lambda g: 10e-3)
    srv = Server(ex, streams=1, budget_bytes=1 << 40)
    reqs = [Req(0, 64, 0, 1), Req(1, 96, 0, 1, arrival_s=1e-3, timeout_s=5e-3), Req(2, 128, 0, 1, arrival_s=1e-3)]
    res, _, st = srv.run(reqs)
    assert _status(res) == {0: "ok", 1: "timeout", 2: "ok"}
    t1 = [r for r in res if r.rid == 1][0]
    assert 6e-3 <= t1.done_s <= 7e-3            # dropped just after its deadline
    assert st["timeouts"] == 1 and st["requests"] == 2


def test_cancel_waiting_and_in_flight_requests():
    ex = FakeExecutor(service=lambda g: 10e-3)
    srv = Server(ex, streams=1, budget_bytes=1 << 40)
    reqs = [Req(0, 64, 0, 1), Req(1, 96, 0, 1), Req(2, 128, 0, 1), Req(3, 160, 0, 1, arrival_s=50e-3)]
    asked = set()

    def tick(now):
        if now >= 2e-3 and not asked:
            asked.add(1)
            srv.cancel(0)     # in flight: runs to completion, reported cancelled
            srv.cancel(1)     # waiting: removed before launch
            srv.cancel(3)     # not arrived yet: cancelled on arrival
    res, _, st = srv.run(reqs, on_tick=tick)
    assert _status(res) == {0: "cancelled", 1: "cancelled", 2: "ok", 3: "cancelled"}
    assert [g.L for g in ex.launched] == [64, 128]     # request 1 never launched, nor 3
    assert st["cancelled"] == 3 and st["requests"] == 1


def test_failed_launch_and_completion_fail_only_their_groups():
    # launch 0 raises, launch 1 completes with an error; the loop keeps
    # serving, releases their memory and slots, and reports them failed
    ex = FakeExecutor(fail_launch={0}, fail_complete={1})
    one = footprint_bytes(64, 1, ws(64, 0, 1))
    # room for two one-map groups at a time; by_spin keeps the six requests
    # (one L, six spins) in six groups
    srv = Server(ex, streams=2, budget_bytes=2 * one + 1, by_spin=True)
    reqs = [Req(i, 64, i, 1) for i in range(6)]
    res, _, st = srv.run(reqs, closed_loop=True)
    assert _status(res) == {0: "failed", 1: "failed", 2: "ok", 3: "ok", 4: "ok", 5: "ok"}
    assert st["failed"] == 2 and st["requests"] == 4
    assert st["peak_admitted_bytes"] <= st["budget_bytes"]
