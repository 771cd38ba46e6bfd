"""Host-side tests of the serving policy (no GPU)."""
import pytest

from paper_2201_02309_amd.serve import Admission, plan_key


def test_admission_fcfs_under_budget():
    a = Admission(100)
    assert a.try_admit(60)
    assert not a.try_admit(50)          # would exceed: waits
    assert a.try_admit(40)
    a.release(60)
    assert a.try_admit(50)
    assert a.used == 90


def test_admission_rejects_request_larger_than_budget():
    a = Admission(10)
    with pytest.raises(ValueError):
        a.try_admit(11)


def test_plan_key_distinguishes_geometries():
    g = {"R": 570.0, "D": 1040.0, "feed_per_turn": 50.0, "n_views": 100}
    gr = {"nx": 8, "dx": 1.0}
    assert plan_key(g, gr) == plan_key(dict(g), dict(gr))
    assert plan_key(g, gr) != plan_key(dict(g, feed_per_turn=50.0000001), gr)
    assert plan_key(g, gr) != plan_key(g, dict(gr, nx=9))
    assert plan_key(g, gr, bp_slices=8) != plan_key(g, gr)
