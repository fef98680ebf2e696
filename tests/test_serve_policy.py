"""Host-side scheduling of the continuous-batching server, without a GPU.

The device work is replaced by a fake that counts the steps each resident
problem receives; the policy must admit in arrival order under the slot and
byte budgets, never step a problem past its own count, retire each problem
exactly at its last step and free its budget for the next arrivals.
"""
import dataclasses

import pytest

from paper_2511_21031_amd.serve import Server


@dataclasses.dataclass
class Req:
    rid: int
    arrival: float
    steps: int
    size: int


class _Ev:
    def query(self):
        return True

    def synchronize(self):
        pass


class FakeServer(Server):
    def _setup(self):
        self.slots = {}
        self.free = list(range(self.max_slots))
        self.log = []           # ("admit", rid, used_after) / ("step", k, rids)
        self.steps_done = {}

    def _admit(self, rec, case):
        slot = self.free.pop(0)
        self.slots[slot] = rec.rid
        self.steps_done[rec.rid] = 0
        self.log.append(("admit", rec.rid, self.used + rec.footprint))
        return slot

    def _step(self, k, nactive):
        rids = sorted(self.slots.values())
        for r in rids:
            self.steps_done[r] += k
        self.log.append(("step", k, rids))

    def _remove(self, slot):
        del self.slots[slot]
        self.free.append(slot)

    def _finish(self, done):
        return _Ev(), None

    def _collect(self, copies, i):
        return 0, -1, -1, None

    def _drain(self):
        pass


def _run(reqs, budget, slots, chunk):
    srv = FakeServer(budget, max_slots=slots, chunk=chunk, footprint=lambda req: req.size)
    recs = srv.run(reqs, make_case=lambda r: r, time_scale=0.0)
    return srv, recs


@pytest.mark.parametrize("budget,slots,chunk", [(100, 3, 4), (35, 8, 7), (1000, 2, 1), (60, 64, 100)])
def test_every_problem_gets_exactly_its_steps(budget, slots, chunk):
    import random
    rng = random.Random(budget * 7 + slots)
    reqs = [Req(i, 0.0, rng.randint(1, 30), rng.randint(5, 35)) for i in range(40)]
    srv, recs = _run(reqs, budget, slots, chunk)
    assert [r.rid for r in recs] == list(range(40))
    for r in reqs:
        assert srv.steps_done[r.rid] == r.steps
    assert all(rec.finished >= 0 and rec.error == 0 for rec in recs)
    assert srv.used == 0
    # budget and slots hold at every admission; chunks never exceed the chunk size
    for entry in srv.log:
        if entry[0] == "admit":
            assert entry[2] <= budget
        else:
            assert 1 <= entry[1] <= chunk and len(entry[2]) <= slots
    assert srv.peak_used <= budget and srv.peak_active <= slots


def test_admission_is_in_arrival_order_and_waits_for_budget():
    reqs = [Req(0, 0.0, 10, 60), Req(1, 0.0, 3, 30), Req(2, 0.0, 2, 50), Req(3, 0.0, 1, 10)]
    srv, recs = _run(reqs, budget=100, slots=8, chunk=100)
    admits = [e[1] for e in srv.log if e[0] == "admit"]
    assert admits == [0, 1, 2, 3]
    # request 2 (50 B) does not fit beside 0 and 1 (90 B): it waits although 3 (10 B) would fit,
    # and is admitted only after request 1 retires
    first_steps = [e for e in srv.log if e[0] == "step"][0]
    assert first_steps[2] == [0, 1] and first_steps[1] == 3
    i2 = next(i for i, e in enumerate(srv.log) if e[:2] == ("admit", 2))
    i1_done = max(i for i, e in enumerate(srv.log) if e[0] == "step" and 1 in e[2])
    assert i2 > i1_done


def test_oversized_request_is_rejected():
    with pytest.raises(ValueError):
        _run([Req(0, 0.0, 1, 200)], budget=100, slots=4, chunk=4)


def test_new_arrivals_join_a_running_batch():
    """Continuous batching: a problem admitted later shares step calls with earlier ones."""
    reqs = [Req(0, 0.0, 50, 10), Req(1, 0.0, 5, 10), Req(2, 0.0, 5, 10)]
    srv, _ = _run(reqs, budget=20, slots=8, chunk=5)
    steps = [e for e in srv.log if e[0] == "step"]
    assert steps[0][2] == [0, 1]
    assert [0, 2] in [s[2] for s in steps]
