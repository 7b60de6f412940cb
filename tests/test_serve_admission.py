"""Host logic of the serving front end: HBM admission of setups and the context cache (no GPU).

Fake solvers stand in for set-up contexts: they report device bytes and a peak, and record close().
"""
import pytest

from paper_2406_06283_amd import serve


class FakeSolver:
    def __init__(self, nbytes, peak=None):
        self.nbytes = nbytes
        self.peak = nbytes if peak is None else peak
        self.closed = False

    def stats(self):
        return {"device_bytes": self.nbytes, "peak_device_bytes": self.peak}

    def close(self):
        self.closed = True


def test_reservations_count_against_the_budget():
    c = serve.ContextCache(100)
    assert c.reserve("a", 60)
    assert c.bytes == 60
    assert not c.reserve("b", 50)           # a's setup is in flight: its reservation holds the room
    c.insert("a", FakeSolver(30, peak=55))
    assert c.bytes == 30 and c.overshoots == 0
    assert c.reserve("b", 50) and c.bytes == 80


def test_eviction_is_lru_over_idle_contexts_only():
    c = serve.ContextCache(100)
    sa, sb, sc = FakeSolver(40), FakeSolver(40), FakeSolver(40)
    for k, s in (("a", sa), ("b", sb)):
        assert c.reserve(k, 40)
        c.insert(k, s)
    c.acquire("a")                           # a busy, b idle (and a most recently used)
    assert c.reserve("c", 40)
    assert sb.closed and not sa.closed and "b" not in c and c.evictions == 1
    c.insert("c", sc)
    assert c.reserve("d", 40)               # c is the only idle context: it goes, a stays
    assert sc.closed and not sa.closed and c.bytes == 80


def test_eviction_frees_enough_when_possible():
    c = serve.ContextCache(100)
    sa, sb = FakeSolver(50), FakeSolver(40)
    c.reserve("a", 50)
    c.insert("a", sa)
    c.reserve("b", 40)
    c.insert("b", sb)
    c.acquire("b")
    assert c.reserve("c", 60)               # a (idle) goes, b (busy) stays
    assert sa.closed and not sb.closed and c.bytes == 100
    assert not c.reserve("d", 1)            # b busy, c pending: nothing can go


def test_insert_overshoot_and_over_budget_are_counted():
    c = serve.ContextCache(100)
    c.reserve("a", 50)
    c.insert("a", FakeSolver(50))
    c.acquire("a")
    c.reserve("b", 40)
    c.insert("b", FakeSolver(70, peak=90))   # estimate too low: peak 90 > 40, and 50 + 70 > 100
    assert c.overshoots == 1
    assert c.over_budget == 1 and "b" in c   # the new context is never the one evicted
    c.release("a")
    c.reserve("x", 0)                       # any later make_room evicts the idle a first
    assert "a" not in c and c.bytes == 70


def test_admission_dispatches_in_order_without_overtaking():
    c = serve.ContextCache(100)
    est = {"big": 80, "s1": 30, "s2": 10, "huge": 101}
    sent = []
    adm = serve.SetupAdmission(c, est.__getitem__, sent.append)
    adm.request("s1")
    adm.request("big")
    adm.request("s2")
    adm.request("s1")                       # already queued: once
    assert adm.pump() == 1 and sent == ["s1"]   # big (80) does not fit beside s1's 30; s2 waits behind it
    adm.finished("s1", FakeSolver(20))
    assert adm.pump() == 2 and sent == ["s1", "big", "s2"]   # s1 (idle) evicted for big
    assert "s1" not in c and c.evictions == 1
    adm.request("big")                      # in setup: not queued again
    assert list(adm.blocked) == []
    adm.failed("big")
    assert c.bytes == 10 and "big" not in adm.in_setup
    adm.request("huge")
    with pytest.raises(ValueError):
        adm.pump()


def test_cached_key_is_not_set_up_again():
    c = serve.ContextCache(100)
    sent = []
    adm = serve.SetupAdmission(c, lambda k: 10, sent.append)
    adm.request("a")
    adm.pump()
    adm.finished("a", FakeSolver(10))
    adm.request("a")
    assert adm.pump() == 0 and sent == ["a"]


def test_admission_keeps_at_most_max_in_flight_setups():
    c = serve.ContextCache(1000)
    sent = []
    adm = serve.SetupAdmission(c, lambda k: 10, sent.append, max_in_flight=2)
    for k in "abcd":
        adm.request(k)
    assert adm.pump() == 2 and sent == ["a", "b"] and c.bytes == 20
    adm.finished("a", FakeSolver(5))
    assert adm.pump() == 1 and sent == ["a", "b", "c"]
