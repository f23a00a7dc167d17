"""The serving loop's host logic on the CPU, against a mock executor that
scripts each request's behaviour: first-come-first-served admission under an
HBM budget and a slot limit, rejection of oversize requests, slot reuse, the
per-request walk through Algorithm 1's (outer, mode) loops, retirement on a
sweep without updates or at k_max, and the latency summary."""
import types

import numpy as np

from paper_2307_03276_amd import serve


class MockExecutor:
    def __init__(self, sizes, converge_at, nmodes):
        self.sizes, self.converge_at, self.nmodes = sizes, converge_at, nmodes
        self.slots = {}            # slot -> (request id, mode)
        self.admitted, self.events = [], []
        self.max_used_slots = 0
        self.rounds = []           # ids that ran, per round

    def footprint(self, req):
        return self.sizes[req.id]

    def admit(self, req):
        self.admitted.append(req.id)
        return {"id": req.id, "k": 0}

    def mode_begin(self, h, n, k):
        h["k"] = k
        self.events.append((h["id"], "begin", k, n))

    def set_slot(self, slot, h, n):
        self.slots[slot] = (h, n)
        self.max_used_slots = max(self.max_used_slots, len(self.slots))

    def clear_slot(self, slot):
        del self.slots[slot]

    def commit(self):
        pass

    def hold(self, flags):
        self.held = list(flags)

    def run_round(self, lmax):
        n_slots = max(self.slots) + 1 if self.slots else 1
        viol = np.zeros(n_slots)
        upd = np.zeros(n_slots, dtype=np.int32)
        done = np.zeros(n_slots, dtype=np.int32)
        held = getattr(self, "held", [])
        self.rounds.append(sorted(h["id"] for s, (h, n) in self.slots.items() if not (s < len(held) and held[s])))
        for slot, (h, n) in self.slots.items():
            if slot < len(held) and held[slot]:
                done[slot] = 1  # a held slot does no work
                continue
            c = self.converge_at[h["id"]]
            conv = c is not None and h["k"] >= c
            upd[slot] = 0 if conv else lmax
            viol[slot] = 1e-6 if conv else 0.5
            done[slot] = int(conv)
        return viol, upd, done

    def mode_end(self, h, n):
        self.events.append((h["id"], "end", h["k"], n))

    def advance(self, items):
        for h, end, begin, k in items:
            self.mode_end(h, end)
            if begin is not None:
                self.mode_begin(h, begin, k)

    def retire(self, h):
        return np.ones(2), [np.zeros((3, 2))] * self.nmodes, -1.0


def _reqs(count, nmodes=3, nnz=None):
    return [serve.Request(id=i, X=types.SimpleNamespace(dims=(5,) * nmodes, nnz=(nnz[i] if nnz else 10)), M=None,
                          arrival=0.0) for i in range(count)]


def test_fifo_admission_budget_and_rejection():
    sizes = {0: 6, 1: 5, 2: 20, 3: 3, 4: 4}
    ex = MockExecutor(sizes, {i: 1 for i in sizes}, 3)
    srv = serve.Server(budget_bytes=10, max_slots=4, kmax=5, lmax=2, tol=1e-4, executor=ex)
    for r in _reqs(5):
        srv.submit(r)
    used_max = 0.0
    while srv.tick():
        used_max = max(used_max, srv.used)
    assert used_max <= 10 and srv.peak_used <= 10
    # request 3 (size 3) fits next to request 0 but waits behind request 1: first come, first served
    assert ex.admitted == [0, 1, 3, 4]
    rejected = [r for r in srv.done if "rejected" in r.stats]
    assert [r.id for r in rejected] == [2]
    assert len(srv.done) == 5 and srv.used == 0


def test_slot_limit_and_reuse():
    sizes = {i: 1 for i in range(7)}
    ex = MockExecutor(sizes, {i: 1 + i % 3 for i in range(7)}, 2)
    srv = serve.Server(budget_bytes=1e9, max_slots=2, kmax=10, lmax=3, tol=1e-4, executor=ex)
    done = srv.run_trace(_reqs(7, nmodes=2))
    assert len(done) == 7 and ex.max_used_slots <= 2 and srv.peak_active <= 2
    assert sorted(ex.admitted) == list(range(7))


def test_loop_walk_and_retirement():
    """Request 0 stops updating from sweep 2 (converged after it), request 1
    never does (retires at k_max); each walks begin/end over every mode of
    every sweep in order."""
    ex = MockExecutor({0: 1, 1: 1}, {0: 2, 1: None}, 3)
    srv = serve.Server(budget_bytes=10, max_slots=2, kmax=4, lmax=5, tol=1e-4, executor=ex)
    done = {r.id: r for r in srv.run_trace(_reqs(2))}
    assert done[0].stats["outer_iters"] == 2 and done[0].stats["converged"]
    assert done[0].stats["inner_updates"] == 1 * 3 * 5  # sweep 1 updates every mode, sweep 2 none
    assert done[1].stats["outer_iters"] == 4 and not done[1].stats["converged"]
    assert done[1].stats["inner_updates"] == 4 * 3 * 5
    walk = [(k, n, e) for (i, e, k, n) in ex.events if i == 1]
    expect = []
    for k in range(1, 5):
        for n in range(3):
            expect += [(k, n, "begin"), (k, n, "end")]
    assert walk == expect


def test_tol_zero_runs_every_sweep():
    ex = MockExecutor({0: 1}, {0: 1}, 3)
    srv = serve.Server(budget_bytes=10, max_slots=1, kmax=3, lmax=2, tol=0.0, executor=ex)
    r = srv.run_trace(_reqs(1))[0]
    assert r.stats["outer_iters"] == 3 and not r.stats["converged"]


def test_latency_summary():
    ex = MockExecutor({i: 1 for i in range(4)}, {i: 1 for i in range(4)}, 3)
    srv = serve.Server(budget_bytes=10, max_slots=2, kmax=3, lmax=2, tol=1e-4, executor=ex)
    reqs = _reqs(4)
    for i, r in enumerate(reqs):
        r.arrival = 0.002 * i
    done = srv.run_trace(reqs)
    s = serve.latency_summary(done)
    assert s["completed"] == 4 and s["rejected"] == 0
    assert s["p99_from_arrival_s"] >= s["p50_from_arrival_s"] >= 0
    assert all(r.t_done >= r.t_admit >= r.arrival for r in done)


def test_srpt_runs_least_remaining_work_first():
    """Shortest remaining work first under a per-round cap of nonzeros: each
    round runs the requests with the least work left (nonzeros x mode rounds
    left) until the cap, at least one; held requests do not advance. Queued
    requests are ranked with the active ones and admitted only when a round
    takes them. Short requests finish first; every request still finishes its
    k_max sweeps."""
    nnz = {0: 100, 1: 10, 2: 1000, 3: 40}
    ex = MockExecutor({i: 1 for i in nnz}, {i: None for i in nnz}, 3)
    srv = serve.Server(budget_bytes=10, max_slots=4, kmax=2, lmax=2, tol=1e-4, executor=ex, policy="srpt",
                       round_cap=60)
    done = srv.run_trace(_reqs(4, nnz=[nnz[i] for i in range(4)]))
    assert [r.id for r in done] == [1, 3, 0, 2]
    assert all(r.stats["outer_iters"] == 2 for r in done)
    for ran in ex.rounds:
        assert len(ran) == 1 or sum(nnz[i] for i in ran) <= 60
    assert ex.rounds[0] == [1, 3]  # 10 + 40 <= 60; 100 and 1000 wait
    # submitted in id order, admitted by remaining work, each only when its round comes
    assert ex.admitted == [1, 3, 0, 2]
    by_id = {r.id: r for r in done}
    assert by_id[0].t_admit >= by_id[3].t_done and by_id[2].t_admit >= by_id[0].t_done
    walk = [(k, n, e) for (i, e, k, n) in ex.events if i == 2]
    assert walk == [(k, n, e) for k in (1, 2) for n in range(3) for e in ("begin", "end")]
    assert "rejected" not in done[0].stats


def test_policy_all_runs_everyone():
    ex = MockExecutor({i: 1 for i in range(3)}, {i: None for i in range(3)}, 2)
    srv = serve.Server(budget_bytes=10, max_slots=3, kmax=2, lmax=2, tol=1e-4, executor=ex)
    srv.run_trace(_reqs(3, nmodes=2))
    assert all(r == [0, 1, 2] for r in ex.rounds)


def test_srpt_round_cap_follows_the_pending_work():
    """The shortest-first round cap is an eighth of the active and queued
    requests' nonzeros, clamped to [round_cap_min, round_cap]; a floor above
    the ceiling is lowered to it."""
    ex = MockExecutor({}, {}, 3)
    srv = serve.Server(budget_bytes=1e12, max_slots=4, kmax=2, lmax=2, tol=1e-4, executor=ex, policy="srpt",
                       round_cap=800, round_cap_min=100)
    assert srv.cap() == 100  # nothing pending: the floor
    for r in _reqs(3, nnz=[400, 2000, 3000]):
        srv.submit(r)
    assert srv.cap() == 675  # 5400 / 8
    srv.submit(_reqs(1, nnz=[8000])[0])
    assert srv.cap() == 800  # 13400 / 8 above the ceiling
    assert serve.Server(executor=ex, policy="srpt", round_cap=60).cap() == 60


def test_srpt_small_rounds_under_a_light_load():
    """Under a light load the cap stays near its floor (an eighth of 980
    pending nonzeros here, far below the ceiling), so the short requests run
    together and never share a round with the long one."""
    nnz = {0: 50, 1: 10, 2: 900, 3: 20}
    ex = MockExecutor({i: 1 for i in nnz}, {i: None for i in nnz}, 3)
    srv = serve.Server(budget_bytes=10, max_slots=4, kmax=2, lmax=2, tol=1e-4, executor=ex, policy="srpt",
                       round_cap=2000, round_cap_min=100)
    done = srv.run_trace(_reqs(4, nnz=[nnz[i] for i in range(4)]))
    assert [r.id for r in done] == [1, 3, 0, 2]
    assert all(2 not in ran or len(ran) == 1 for ran in ex.rounds)
    assert ex.rounds[0] == [0, 1, 3]  # 10 + 20 + 50 <= 980 / 8 < 10 + 20 + 50 + 900
