"""Host-side tests of the serving policy (no GPU)."""
import pytest

from paper_2201_02309_amd.serve import Arena, plan_key


def test_arena_first_fit_and_coalescing():
    a = Arena(100 * 256)
    x = a.alloc(60 * 256)
    assert x == 0
    assert a.alloc(50 * 256) is None            # would exceed: waits
    y = a.alloc(40 * 256)
    assert y == 60 * 256 and a.used == 100 * 256
    a.release(x, 60 * 256)
    z = a.alloc(50 * 256)                       # first fit in the freed range
    assert z == 0 and a.used == 90 * 256
    a.release(y, 40 * 256)
    a.release(z, 50 * 256)
    assert a.free == [(0, 100 * 256)] and a.used == 0   # fully coalesced


def test_arena_rounds_to_256_bytes_and_fragments():
    a = Arena(4 * 256)
    p = [a.alloc(1) for _ in range(4)]          # 1 byte takes one 256-byte unit
    assert p == [0, 256, 512, 768] and a.alloc(1) is None
    a.release(p[1], 1)
    a.release(p[3], 1)
    assert a.alloc(512) is None                 # two free units, not contiguous
    a.release(p[2], 1)
    assert a.alloc(512) == 256


def test_arena_rejects_request_larger_than_budget():
    a = Arena(10 * 256)
    with pytest.raises(ValueError):
        a.alloc(11 * 256)


def test_plan_key_distinguishes_geometries():
    g = {"R": 570.0, "D": 1040.0, "feed_per_turn": 50.0, "n_views": 100}
    gr = {"nx": 8, "dx": 1.0}
    assert plan_key(g, gr) == plan_key(dict(g), dict(gr))
    assert plan_key(g, gr) != plan_key(dict(g, feed_per_turn=50.0000001), gr)
    assert plan_key(g, gr) != plan_key(g, dict(gr, nx=9))
    assert plan_key(g, gr, bp_slices=8) != plan_key(g, gr)


def test_failed_plan_build_is_reported_per_request():
    """A geometry whose plan cannot be built fails that key only: poll raises PlanFailed on
    every later call, and other keys keep working (the server rejects the request with an
    error instead of stopping its loop)."""
    import time

    from paper_2201_02309_amd.serve import PlanCache, PlanFailed

    cache = PlanCache(device=None, workers=1)

    def build(geom, grid):
        if geom["feed_per_turn"] < 0:
            raise ValueError("feed must be positive")
        return type("P", (), {"info": {"table_bytes": 256}})(), 0.0
    cache._build = build
    g = {"R": 570.0, "D": 1040.0, "feed_per_turn": 50.0, "n_views": 100}
    gr = {"nx": 8, "dx": 1.0}
    bad, _ = cache.request(dict(g, feed_per_turn=-1.0), gr)
    good, _ = cache.request(g, gr)
    deadline = time.time() + 10
    while cache.poll(good) is None and time.time() < deadline:
        time.sleep(0.01)
    assert cache.poll(good) is not None
    for _ in range(2):
        with pytest.raises(PlanFailed, match="feed must be positive"):
            cache.poll(bad)
    cache.close()


def test_plan_cache_evicts_least_recently_used_unheld_plans():
    """Beyond the table budget the least recently used plans are dropped, never one that a
    request in flight holds (acquire / release); a held plan goes once released."""
    import time

    from paper_2201_02309_amd.serve import PlanCache

    cache = PlanCache(device=None, workers=1, table_budget=3 * 1000)
    cache._build = lambda geom, grid: (type("P", (), {"info": {"table_bytes": 1000}})(), 0.0)
    gr = {"nx": 8, "dx": 1.0}

    def get(feed):
        key, _ = cache.request({"feed_per_turn": feed}, gr)
        deadline = time.time() + 10
        while cache.poll(key) is None and time.time() < deadline:
            time.sleep(0.005)
        return key

    keys = [get(40.0 + i) for i in range(3)]
    cache.acquire(keys[0])                       # in flight
    k3 = get(50.0)                               # 4 plans > budget: keys[1] (LRU, unheld) goes
    assert keys[0] in cache.plans and keys[1] not in cache.plans and cache.evicted == 1
    assert cache.table_bytes == 3000
    get(51.0)                                    # next unheld: keys[2]
    assert keys[0] in cache.plans and keys[2] not in cache.plans and k3 in cache.plans
    cache.release(keys[0])                       # released while over no budget: kept
    assert keys[0] in cache.plans and cache.table_bytes == 3000
    get(52.0)                                    # now keys[0] is the least recently used
    assert keys[0] not in cache.plans and cache.evicted == 3
    cache.close()
