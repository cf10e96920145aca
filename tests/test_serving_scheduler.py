"""CPU tests of the serving loop's admission and grouping logic (no GPU)."""

import dataclasses

import pytest

from paper_0807_4494_amd.serving import BATCH_MAX, Scheduler, footprint_bytes, percentile


@dataclasses.dataclass
class Req:
    rid: int
    L: int
    spin: int
    batch: int
    arrival_s: float = 0.0
    seed: int = 0


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
    s = Scheduler(1 << 40, ws)
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
