"""Admission control of the serving loop (pure host logic, no GPU)."""
from paper_2405_15573_amd.serving import Admission, solve_footprint


def test_footprint_grows_with_size_and_rhs():
    assert solve_footprint(1000, 2, 50) == 2 * solve_footprint(1000, 1, 50)
    # the Krylov basis and work vectors grow with n; the least-squares state does not
    assert solve_footprint(2000, 1, 50) - solve_footprint(1000, 1, 50) == 16 * 1000 * (50 + 13)
    assert solve_footprint(1000, 1, 50) > solve_footprint(1000, 1, 10)


def test_admit_queue_release_in_order():
    a = Admission(budget_bytes=100)
    for rid, nb in ((0, 60), (1, 30), (2, 50), (3, 10)):
        assert a.offer(rid, nb)
    got = [r for r, _ in a.admit()]
    assert got == [0, 1]                 # 2 does not fit; 3 may not overtake it
    assert a.used == 90 and a.active == 2
    a.release(60)                        # request 0 finishes
    got = [r for r, _ in a.admit()]
    assert got == [2, 3]
    assert a.used == 90
    a.release(30)
    a.release(50)
    a.release(10)
    assert a.used == 0 and a.active == 0 and not a.queue


def test_reject_larger_than_budget_and_cap_active():
    a = Admission(budget_bytes=100, max_active=2)
    assert not a.offer("huge", 101)
    assert a.rejected == ["huge"]
    for rid in range(4):
        a.offer(rid, 10)
    assert [r for r, _ in a.admit()] == [0, 1]
    a.release(10)
    assert [r for r, _ in a.admit()] == [2]


def test_release_below_zero_is_an_error():
    a = Admission(budget_bytes=10)
    try:
        a.release(5)
    except RuntimeError:
        return
    raise AssertionError("expected an accounting error")
