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
