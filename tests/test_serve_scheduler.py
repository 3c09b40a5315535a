"""CPU checks of the serving scheduler (continuous batching) with stand-in
cases: the library's batched step is replaced by a recorder, so only the
admission, tick and retirement logic runs.  Every request must get exactly
its steps, start no earlier than its arrival, never exceed the memory budget
or the slot count, and a tick must never carry a case past its last step."""
import itertools

import pytest

import paper_2303_10783_amd.serve as S


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-4)


def _run(monkeypatch, reqs, multi_step, step_s=0.002, **kw):
    clock = FakeClock()
    log = []
    live = {}

    class Case:
        ids = itertools.count()

        def __init__(self, case, device=None):
            self.id = next(Case.ids)
            self.case = case
            self.steps = 0
            live[self.id] = self

        def set_graph(self, on):
            pass

        def read_fields(self):
            return {"steps": self.steps}

        def close(self):
            del live[self.id]

    class Batch:
        def __init__(self, cases):
            self.cases = list(cases)

        def step(self, nsteps):
            assert len(nsteps) == len(self.cases)
            for c, k in zip(self.cases, nsteps):
                assert k >= 1
                c.steps += k
            log.append((clock.t, [c.case["rid"] for c in self.cases], list(nsteps)))
            clock.t += step_s * max(nsteps)
            return [{} for _ in self.cases]

        def close(self):
            pass

    monkeypatch.setattr(S, "Case", Case)
    monkeypatch.setattr(S, "Batch", Batch)
    monkeypatch.setattr(S, "sol_footprint_bytes", lambda case: case["fp"])
    srv = S.Server(multi_step=multi_step, **kw)
    out = srv.run(reqs, clock=clock, sleep=clock.sleep)
    assert not live                                      # every case closed
    return srv, out, log


def _requests(n=12, seed=3):
    import numpy as np
    rng = np.random.default_rng(seed)
    t, out = 0.0, []
    for i in range(n):
        t += rng.exponential(0.01)
        case = {"grid": {"dim": 2, "nx": 10, "ny": 10}, "rid": i, "fp": int(rng.integers(1, 5)) * 100}
        out.append(S.Request(case=case, steps=int(rng.integers(3, 40)), arrival=t, rid=i))
    return out


@pytest.mark.parametrize("multi_step", [False, True])
def test_every_request_gets_exactly_its_steps(monkeypatch, multi_step):
    reqs = _requests()
    srv, out, log = _run(monkeypatch, reqs, multi_step, hbm_budget_bytes=700, max_active=4)
    assert out["requests"] == len(reqs)
    for r in out["done"]:
        assert r.result["steps"] == r.steps
        assert r.admitted >= r.arrival
        assert r.finished >= r.admitted
    # slots and budget were respected at every tick
    fp = {r.rid: r.case["fp"] for r in reqs}
    for _, members, _ in log:
        assert len(members) <= 4
        assert sum(fp[m] for m in members) <= 700


def test_multi_step_ticks_take_fewer_synchronisations(monkeypatch):
    r1, r2 = _requests(), _requests()
    _, _, log1 = _run(monkeypatch, r1, False, hbm_budget_bytes=700, max_active=4)
    _, _, log2 = _run(monkeypatch, r2, True, hbm_budget_bytes=700, max_active=4)
    assert len(log2) < len(log1)
    assert sum(sum(k) for _, _, k in log1) == sum(sum(k) for _, _, k in log2)


def test_free_slot_arrival_is_not_held_back(monkeypatch):
    # one long request running, a second arrives later with a free slot: the
    # long request's tick must end by the arrival (one step of slack)
    a = S.Request(case={"grid": {"dim": 2, "nx": 4, "ny": 4}, "rid": 0, "fp": 1}, steps=1000, arrival=0.0, rid=0)
    b = S.Request(case={"grid": {"dim": 2, "nx": 4, "ny": 4}, "rid": 1, "fp": 1}, steps=5, arrival=0.05, rid=1)
    srv, out, log = _run(monkeypatch, [a, b], True, step_s=0.002, max_active=4)
    rb = [r for r in out["done"] if r.rid == 1][0]
    assert rb.admitted - rb.arrival <= 2 * 0.002 + 1e-9


def test_over_budget_request_is_refused_alone(monkeypatch):
    """A request larger than the whole memory budget is refused with a reason;
    every other request of the stream is still served."""
    reqs = _requests(8)
    reqs[3].case["fp"] = 10_000
    srv, out, _ = _run(monkeypatch, reqs, True, hbm_budget_bytes=700, max_active=4)
    assert out["requests"] == 7
    assert [r.rid for r in out["rejected"]] == [3]
    assert "over the budget" in out["rejected"][0].error
    assert ("reject" in [ev for _, ev, _ in srv.log])


def test_backfill_lets_small_request_pass_a_waiting_large_one(monkeypatch):
    """While a large request waits for memory, a later small one that fits is
    admitted ahead of it; without backfill it waits behind the large one."""
    def reqs():
        mk = lambda rid, fp, steps, t: S.Request(case={"grid": {"dim": 2, "nx": 4, "ny": 4}, "rid": rid, "fp": fp},
                                                   steps=steps, arrival=t, rid=rid)
        return [mk(0, 600, 200, 0.0), mk(1, 600, 5, 0.001), mk(2, 100, 5, 0.002)]
    _, out, _ = _run(monkeypatch, reqs(), True, hbm_budget_bytes=800, max_active=4)
    adm = {r.rid: r.admitted for r in out["done"]}
    assert adm[2] < adm[1]
    _, out, _ = _run(monkeypatch, reqs(), True, hbm_budget_bytes=800, max_active=4, backfill=False)
    adm = {r.rid: r.admitted for r in out["done"]}
    assert adm[2] >= adm[1]


def test_backfill_stops_once_the_head_waited_too_long(monkeypatch):
    """A stream of small requests cannot hold a large one back forever: once
    it has waited max_wait_s no later request goes ahead of it."""
    mk = lambda rid, fp, steps, t: S.Request(case={"grid": {"dim": 2, "nx": 4, "ny": 4}, "rid": rid, "fp": fp},
                                               steps=steps, arrival=t, rid=rid)
    reqs = [mk(0, 500, 30, 0.0), mk(1, 600, 5, 0.001)] + [mk(2 + i, 100, 30, 0.002 + 0.01 * i) for i in range(40)]
    _, out, _ = _run(monkeypatch, reqs, True, hbm_budget_bytes=800, max_active=8, max_wait_s=0.05)
    r1 = [r for r in out["done"] if r.rid == 1][0]
    late = [r for r in out["done"] if r.rid >= 2 and r.arrival > r1.arrival + 0.05]
    assert late and all(r.admitted >= r1.admitted for r in late)
