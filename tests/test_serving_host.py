"""Host-side checks of the serving admission policy (no GPU)."""
from __future__ import annotations

from paper_2505_10168_amd.serving import Admission


class R:
    def __init__(self, rid, size):
        self.rid, self.size = rid, size


def test_fcfs_when_the_head_fits():
    a = Admission(budget=100)
    q = [R(0, 30), R(1, 10)]
    assert a.pick(q, free=100, footprint=lambda r: r.size) == 0


def test_backfill_small_requests_past_a_large_head():
    a = Admission(budget=100, max_bypass=2)
    q = [R(0, 90), R(1, 10), R(2, 10), R(3, 10)]
    fp = lambda r: r.size  # noqa: E731
    assert a.pick(q, free=50, footprint=fp) == 1
    q.pop(1)
    assert a.pick(q, free=40, footprint=fp) == 1
    q.pop(1)
    # the head has been passed over max_bypass times: wait for memory
    assert a.pick(q, free=30, footprint=fp) is None
    # once the head fits it goes first and the bypass count resets
    assert a.pick(q, free=95, footprint=fp) == 0
    assert a.bypassed == 0


def test_nothing_fits():
    a = Admission(budget=100)
    assert a.pick([R(0, 60), R(1, 70)], free=50, footprint=lambda r: r.size) is None
    assert a.pick([], free=50, footprint=lambda r: r.size) is None
