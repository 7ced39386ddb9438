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


def _server_stub(budget, footprints):
    """A Server with its bookkeeping only (no GPU, no worker threads), to drive the real
    _admit / _release logic."""
    import collections
    import threading

    from paper_2505_10168_amd.serving import Server, ServerStats

    srv = Server.__new__(Server)
    srv.admission = Admission(budget)
    srv.stats = ServerStats()
    srv._cv = threading.Condition()
    srv._waiting = []
    srv._in_use = 0
    srv._in_flight = 0
    srv._idle = collections.OrderedDict()
    srv._idle_bytes = 0
    srv.keep_resident = True
    srv._footprint = lambda req, options=None: footprints[req.key()]
    return srv


class Req:
    def __init__(self, key, with_adjoint=False):
        self._key, self.with_adjoint = key, with_adjoint
        self.dofs, self.n_el = 10, 1

    def key(self):
        return self._key


class FakeSolver:
    closed = False

    def close(self):
        self.closed = True


def test_reused_hierarchy_is_not_counted_twice():
    """An idle hierarchy that a request can reuse is part of the budget already in use:
    a request whose whole footprint does not fit beside the requests in flight waits,
    even if an idle hierarchy of its key exists."""
    from paper_2505_10168_amd.serving import Server
    fp = {"a": 80, "b": 50}
    srv = _server_stub(100, fp)
    out = Server._outputs(Req("a"))
    # an idle hierarchy of key "a" (its bytes without outputs) and a request "b" in flight
    srv._idle[1] = ("a", FakeSolver(), fp["a"] - out)
    srv._idle_bytes = fp["a"] - out
    srv._in_use = 50
    srv._in_flight = 1
    srv._waiting.append(Req("a"))
    with srv._cv:
        assert srv._admit() is None          # 80 > 100 - 50: must wait, reuse or not
    srv._in_use = 0
    srv._in_flight = 0
    with srv._cv:
        req, solver, total = srv._admit()    # now it fits; the idle hierarchy is reused
    assert solver is not None and total == 80 and srv._in_use == 80 and srv._idle_bytes == 0
    assert srv._in_use + srv._idle_bytes <= srv.admission.budget
