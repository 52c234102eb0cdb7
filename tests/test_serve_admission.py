"""Host-side admission policy of the serving loop (no GPU)."""
import numpy as np
import pytest

from paper_2510_10256_amd.serve import Admission, Request


def _req(k, sid):
    return Request(rid=k, sid=sid, x=np.zeros((1, 3)))


def test_budget_slots_and_one_request_per_scene():
    rng = np.random.default_rng(3)
    sizes = rng.integers(10, 60, size=40)
    adm = Admission(budget_bytes=200, slots=3, footprint=lambda s: int(sizes[s]))
    running = []
    started = 0
    for k in range(2000):
        adm.arrive(_req(k, int(rng.integers(40))))
        for req, create, evict in adm.plan():
            assert req.sid not in [r.sid for r in running]
            for s2 in evict:
                assert all(r.sid != s2 for r in running), "evicted a busy scene"
            running.append(req)
            started += 1
        assert adm.used <= adm.budget
        assert len(running) <= 3
        assert sum(adm.resident.values()) == adm.used
        if running and rng.random() < 0.7:  # complete a random running request
            r = running.pop(int(rng.integers(len(running))))
            adm.done(r)
    assert started > 1000


def test_lru_eviction_of_idle_scenes():
    adm = Admission(budget_bytes=100, slots=4, footprint=lambda s: 40)
    for k, sid in enumerate([0, 1]):
        adm.arrive(_req(k, sid))
    started = adm.plan()
    assert [r.sid for r, _, _ in started] == [0, 1] and all(c for _, c, _ in started)
    for r, _, _ in started:
        adm.done(r)
    adm.arrive(_req(2, 0))          # touch scene 0 again: scene 1 is now least recent
    (r0, create, evict), = adm.plan()
    assert not create and evict == []
    adm.arrive(_req(3, 2))          # needs room: evicts idle scene 1, not busy scene 0
    (r2, create, evict), = adm.plan()
    assert create and evict == [1]
    assert list(adm.resident) == [0, 2]


def test_busy_scene_waits_and_is_bypassed_without_starving():
    adm = Admission(budget_bytes=1000, slots=2, footprint=lambda s: 10, max_bypass=3)
    adm.arrive(_req(0, 5))
    (first, _, _), = adm.plan()
    adm.arrive(_req(1, 5))          # same scene: must wait
    adm.arrive(_req(2, 6))
    got = adm.plan()
    assert [r.sid for r, _, _ in got] == [6]
    assert [r.rid for r in adm.queue] == [1]


def test_large_scene_is_not_starved():
    # scene 9 needs the whole budget; small requests keep arriving
    sizes = {9: 100}
    adm = Admission(budget_bytes=100, slots=4, footprint=lambda s: sizes.get(s, 30), max_bypass=2)
    adm.arrive(_req(0, 1))
    (small, _, _), = adm.plan()
    adm.arrive(_req(1, 9))          # cannot fit while scene 1 is busy
    k = 2
    started_9 = False
    for step in range(20):
        adm.arrive(_req(k, 2 + step % 3))
        k += 1
        for r, _, _ in adm.plan():
            if r.sid == 9:
                started_9 = True
        if small is not None and step == 4:
            adm.done(small)
            small = None
        for sid in list(adm.busy):
            if sid != 9 and (small is None or sid != small.sid):
                adm.done(_req(-1, sid))
        if started_9:
            break
    assert started_9


def test_scene_above_budget_is_refused():
    adm = Admission(budget_bytes=50, slots=1, footprint=lambda s: 51)
    with pytest.raises(ValueError):
        adm.arrive(_req(0, 0))
