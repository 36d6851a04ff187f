"""Host-side admission policy of the serving loop (no GPU)."""
import random

import pytest


def load_admission():
    import paper_1107_1525_amd.serve as serve

    return serve.Admission


class Req:
    def __init__(self, footprint, arrival):
        self.footprint = footprint
        self.arrival = arrival
        self.admitted = None


def test_fifo_budget_and_no_starvation():
    Admission = load_admission()
    rng = random.Random(5)
    budget = 1000
    adm = Admission(budget)
    reqs = [Req(rng.randint(1, 400), t * 0.5) for t in range(300)]
    for r in reqs:
        adm.submit(r)
    now, live, order = 0.0, [], []
    while adm.waiting or live:
        for r in adm.admit(now):
            live.append((r, now + rng.uniform(0.1, 3.0)))
            order.append(r)
        assert adm.in_use <= budget
        assert adm.in_use == sum(r.footprint for r, _ in live)
        now += 0.25
        for r, end in list(live):
            if end <= now:
                adm.release(r)
                live.remove((r, end))
    assert order == reqs  # admitted in arrival order: none overtaken, none starved
    assert all(r.admitted >= r.arrival for r in reqs)
    assert adm.in_use == 0


def test_admits_many_at_once_when_they_fit():
    Admission = load_admission()
    adm = Admission(100)
    for k in range(10):
        adm.submit(Req(10, 0.0))
    assert len(adm.admit(0.0)) == 10 and adm.in_use == 100
    adm2 = Admission(100, max_batch=3)
    for k in range(10):
        adm2.submit(Req(10, 0.0))
    assert len(adm2.admit(0.0)) == 3


def test_rejects_oversized_and_waits_for_arrival():
    Admission = load_admission()
    adm = Admission(100)
    with pytest.raises(ValueError):
        adm.submit(Req(101, 0.0))
    adm.submit(Req(10, 5.0))
    assert adm.admit(1.0) == [] and len(adm.admit(5.0)) == 1


def test_adjust_and_hold():
    Admission = load_admission()
    adm = Admission(100)
    for k in range(4):
        adm.submit(Req(20, 0.0), worst=60)  # admitted on its estimate, could never need more than 60
    with pytest.raises(ValueError):
        adm.submit(Req(20, 0.0), worst=101)  # could never run
    got = adm.admit(0.0)
    assert len(got) == 4 and adm.in_use == 80
    assert not adm.adjust(got[1], 30) and adm.in_use == 80 and got[1].footprint == 20  # the growth does not fit yet
    assert adm.adjust(got[2], -5) and adm.in_use == 75 and got[2].footprint == 15  # a shorter code gives bytes back
    adm.release(got[0])
    assert adm.adjust(got[1], 30) and adm.in_use == 85 and got[1].footprint == 50
    adm.submit(Req(5, 0.0))
    assert adm.admit(0.0, hold=True) == []  # a batch waiting for its growth holds new admissions
    assert len(adm.admit(0.0)) == 1
    for r in got[1:]:
        adm.release(r)
    assert adm.in_use == 5
