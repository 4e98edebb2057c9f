"""Host logic of the serving loop: admission by device-memory footprint,
no overtaking, and merging of waiting contraction requests into one launch
(no device needed)."""
import pytest

from paper_2106_13062_amd import _lib as C
from paper_2106_13062_amd.serve import AdmissionError, PlanCache, Request, Scheduler


def req(rid, kind, key="S", fp=10, t=0.0):
    r = Request(rid, kind, t, key)
    r.footprint = fp
    return r


def test_contractions_merge_by_sketch_and_keep_order():
    s = Scheduler(cap_bytes=1e9, max_group=3, max_inflight=8)
    for k, (kind, key) in enumerate([("contract", "A"), ("cp", "x"), ("contract", "A"), ("contract", "B"),
                                     ("contract", "A"), ("contract", "A")]):
        s.submit(req(k, kind, key))
    groups = s.next_groups()
    ids = [[r.rid for r in g] for g, _ in groups]
    # head group: up to 3 A-contractions; then the CP build; then the B one;
    # the 4th A waits for the next A group
    assert ids[0] == [0, 2, 4]
    assert ids[1] == [1]
    assert ids[2] == [3]
    assert ids[3] == [5]
    assert not s.waiting
    assert s.inflight_groups == 4 and s.inflight_bytes == 60


def test_admission_by_footprint_without_overtaking():
    s = Scheduler(cap_bytes=100, max_group=8, max_inflight=8)
    s.resident_bytes = 20
    s.submit(req(0, "cp", fp=50))
    s.submit(req(1, "coo", fp=40))      # would not fit next to request 0
    s.submit(req(2, "cp", fp=5))        # would fit, but must not overtake 1
    g = s.next_groups()
    assert [[r.rid for r in m] for m, _ in g] == [[0]]
    assert [r.rid for r in s.waiting] == [1, 2]
    s.release(50)
    g = s.next_groups()
    assert [[r.rid for r in m] for m, _ in g] == [[1], [2]]
    assert s.inflight_bytes == 45


def test_group_footprint_bounded_by_cap():
    s = Scheduler(cap_bytes=35, max_group=100, max_inflight=8)
    for k in range(10):
        s.submit(req(k, "contract", "A", fp=10))
    g = s.next_groups()
    assert len(g) == 1 and len(g[0][0]) == 3 and g[0][1] == 30
    assert len(s.waiting) == 7
    assert [r.rid for r in s.waiting] == [3, 4, 5, 6, 7, 8, 9]


def test_inflight_limit_and_oversize_request():
    s = Scheduler(cap_bytes=1e6, max_group=4, max_inflight=2)
    for k in range(5):
        s.submit(req(k, "cp", fp=1))
    assert len(s.next_groups()) == 2
    assert len(s.next_groups()) == 0
    s.release(1)
    assert len(s.next_groups()) == 1
    with pytest.raises(AdmissionError) as e:
        s.submit(req(9, "cp", fp=2e6))
    assert e.value.status == C.FCS_EADMIT


class _FakePlan:
    def __init__(self, key, nbytes):
        self.key, self.nbytes, self.closed = key, nbytes, False


def test_plan_cache_evicts_least_recently_used_unpinned_plans():
    """Hash tables of plans that nothing uses leave the cache (and the
    admission total) once the cache holds more than its limit; plans of
    resident sketches or staged inputs stay."""
    s = Scheduler(cap_bytes=1e9)
    cache = PlanCache(s, limit_bytes=300, make=lambda k: _FakePlan(k, 100), nbytes=lambda p: p.nbytes,
                      close=lambda p: setattr(p, "closed", True))
    a, b, c = cache.get("a"), cache.get("b"), cache.get("c")
    assert s.resident_bytes == 300 and cache.bytes == 300
    cache.pin("a")                      # a resident sketch uses plan a
    cache.get("b")                      # b is now the most recently used
    d = cache.get("d")                  # over the limit: c goes (a is pinned, b recent)
    assert c.closed and not a.closed and not b.closed and not d.closed
    assert set(cache.plans) == {"a", "b", "d"}
    assert s.resident_bytes == 300
    e = cache.get("e")                  # b is now the oldest unpinned plan
    assert b.closed and set(cache.plans) == {"a", "d", "e"}
    cache.unpin("a")
    cache.get("f")                      # a is unpinned and oldest
    assert a.closed and set(cache.plans) == {"d", "e", "f"} and s.resident_bytes == 300
    assert cache.get("f") is not None and not e.closed
    # a long stream of distinct keys never grows the resident total past the limit
    for k in range(100):
        cache.get(("k", k))
        assert s.resident_bytes <= 300


def test_plan_cache_keeps_pinned_plans_over_the_limit():
    s = Scheduler(cap_bytes=1e9)
    cache = PlanCache(s, limit_bytes=150, make=lambda k: _FakePlan(k, 100), nbytes=lambda p: p.nbytes)
    cache.get("a")
    cache.pin("a")
    cache.get("b")
    cache.pin("b")
    assert set(cache.plans) == {"a", "b"} and s.resident_bytes == 200
    cache.unpin("b")                    # b is unpinned: the cache shrinks to its limit
    assert set(cache.plans) == {"a"} and s.resident_bytes == 100
