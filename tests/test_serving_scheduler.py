"""Admission and residency policy of the serving loop (host logic only)."""
from paper_1809_03745_amd.serving import Request, Scheduler


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


def _req(rid, key, cells, arrival=0.0):
    return Request(rid, key, cells, make_problem=None, make_rho=None, arrival=arrival)


def _admit(s):
    p = s.next_admissible()
    assert p is not None
    req, entry, evict = p
    return req, entry, evict


def test_rejects_what_cannot_fit_an_empty_device():
    s = Scheduler(budget_bytes=10_000, slots=2, bytes_per_cell=10)
    r = _req(0, "a", 1000)
    assert not s.offer(r) and r.rejected
    assert s.stats["rejected"] == 1


def test_reuses_idle_hierarchy_and_counts_hits():
    s = Scheduler(budget_bytes=1 << 20, slots=2, bytes_per_cell=10)
    s.offer(_req(0, "a", 100))
    req, e, _ = _admit(s)
    s.set_up(e, 3000)
    s.finish(req, e)
    s.offer(_req(1, "a", 100))
    req2, e2, _ = _admit(s)
    assert e2 is e and req2.hit
    assert s.stats["hits"] == 1 and s.stats["misses"] == 1


def test_slots_bound_concurrency():
    s = Scheduler(budget_bytes=1 << 30, slots=2, bytes_per_cell=10)
    for i in range(3):
        s.offer(_req(i, ("k", i), 100))
    _admit(s)
    _admit(s)
    assert s.next_admissible() is None
    assert s.running == 2


def test_lru_eviction_and_high_water_within_budget():
    vec = _req(0, "x", 100).vec_bytes()
    budget = 2 * 1000 + vec + 500      # two hierarchies and one request, not three
    s = Scheduler(budget_bytes=budget, slots=1, bytes_per_cell=10)
    clock = Clock()
    s.clock = clock
    for i, key in enumerate(["a", "b", "c", "a"]):
        s.offer(_req(i, key, 100))
        req, e, evict = _admit(s)
        for v in evict:                 # the executor frees evicted hierarchies before a setup
            s.released(v)
        if e.handle is None and not e.ready:
            s.set_up(e, 1000)
        clock.t += 1.0
        s.finish(req, e)
        assert s.reserved() <= budget
        if key == "c":
            assert [v.key for v in evict] == ["a"]   # least recently used goes first
    assert s.high_water <= budget
    assert s.stats["evicted"] >= 1


def test_first_fit_then_no_bypass_for_a_starved_head():
    vec = _req(0, "x", 100).vec_bytes()
    s = Scheduler(budget_bytes=3000 + 2 * vec, slots=4, bytes_per_cell=10, max_bypass_s=0.5)
    clock = Clock()
    s.clock = clock
    s.offer(_req(0, "big0", 200))          # estimate 2000 + vec
    r0, e0, _ = _admit(s)
    s.set_up(e0, 2000)
    s.offer(_req(1, "big1", 200, arrival=0.0))  # does not fit beside big0
    s.offer(_req(2, "small", 10, arrival=0.0))  # fits: may pass the head
    r, e, _ = _admit(s)
    assert r.rid == 2
    s.offer(_req(3, "small2", 10, arrival=0.0))
    clock.t = 1.0                           # the head has now waited too long
    assert s.next_admissible() is None


def test_same_key_waits_for_its_busy_hierarchy():
    s = Scheduler(budget_bytes=1 << 30, slots=4, bytes_per_cell=10)
    s.clock = Clock()
    s.offer(_req(0, "a", 100))
    r0, e0, _ = _admit(s)
    s.set_up(e0, 1000)
    s.offer(_req(1, "a", 100))
    s.offer(_req(2, "b", 100))
    r, e, _ = _admit(s)            # "b" passes the waiting "a"
    assert r.rid == 2
    assert s.next_admissible() is None
    s.finish(r0, e0)
    r1, e1, _ = _admit(s)
    assert r1.rid == 1 and e1 is e0 and r1.hit
    assert sum(1 for x in s.entries if x.key == "a") == 1


def test_evicted_bytes_stay_reserved_until_released():
    """An evicted hierarchy is freed by the executor after admission; until
    it reports the release, its bytes still count against the budget, so a
    concurrent admission cannot overcommit the device."""
    vec = _req(0, "x", 100).vec_bytes()
    budget = 1000 + vec + 500           # one hierarchy and one request's vectors
    s = Scheduler(budget_bytes=budget, slots=2, bytes_per_cell=10)
    s.offer(_req(0, "a", 100))
    r, e, _ = _admit(s)
    s.set_up(e, 1000)
    s.finish(r, e)
    s.offer(_req(1, "b", 100))          # needs "a" evicted
    r1, e1, ev = _admit(s)
    assert ev == [e]
    assert s.reserved() >= 1000 + 1000 + vec   # a's bytes held while it is being freed
    s.offer(_req(2, "c", 100))
    assert s.next_admissible() is None  # would exceed the budget before a is freed
    assert s.reserved() <= budget + 1000
    s.released(e)
    assert s.releasing == 0
    assert s.reserved() == 1000 + vec


def _greq(rid, key, cells, arrival=0.0):
    return Request(rid, key, cells, make_problem=None, make_rho=None, arrival=arrival, group_key=key)


def test_coalesces_queued_requests_of_one_group():
    """An admitted small request takes queued requests of its group along (in
    queue order, up to the batch size); others stay queued; finishing the
    group frees every member's vectors."""
    s = Scheduler(budget_bytes=1 << 24, slots=2, bytes_per_cell=10, coalesce=3)
    g = [_greq(i, "g", 100) for i in range(4)]
    other = _req(9, "h", 100)
    s.offer(g[0])
    s.offer(other)
    for r in g[1:]:
        s.offer(r)
    req, e, _ = _admit(s)
    assert req is g[0] and req.members == [g[0], g[1], g[2]]
    assert s.vec_reserved == sum(m.vec_bytes() for m in req.members)
    assert list(s.queue) == [other, g[3]]
    assert s.stats["coalesced_groups"] == 1 and s.stats["coalesced_requests"] == 3
    # the group's batch is busy: the fourth waits, the other key runs
    req2, e2, _ = _admit(s)
    assert req2 is other and req2.members == [other]
    assert s.next_admissible() is None
    s.set_up(e, 5000)
    s.finish(req, e)
    assert s.vec_reserved == other.vec_bytes()
    assert s.stats["completed"] == 3
    req3, e3, _ = _admit(s)
    assert req3 is g[3] and e3 is e and req3.members == [g[3]]


def test_coalesced_vectors_must_fit_the_budget():
    s = Scheduler(budget_bytes=200_000, slots=1, bytes_per_cell=10, coalesce=8)
    g = [_greq(i, "g", 2000) for i in range(8)]
    for r in g:
        s.offer(r)
    req, e, _ = _admit(s)
    # hierarchy estimate 10 B x 2000 cells x 8 boxes, then 16.5 KB per member
    assert len(req.members) >= 1
    assert s.reserved() <= s.budget
    assert len(req.members) + len(s.queue) == 8
    assert len(s.queue) > 0


def test_group_estimate_counts_every_box():
    s = Scheduler(budget_bytes=1 << 30, slots=1, bytes_per_cell=10, coalesce=4)
    assert s.hier_estimate(_greq(0, "g", 100)) == 4 * 10 * 100
    assert s.hier_estimate(_req(1, "h", 100)) == 10 * 100
