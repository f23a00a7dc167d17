"""Continuous-batching service: results in the mix equal results alone and the
plain cpapr_solve path, FP64 results match the oracle's Algorithm 1, the HBM
budget bounds admission, and oversize requests are rejected.

FP64 factor matrices are held normwise and column-wise (lambda elementwise):
after many MU steps the order of the tile-boundary atomic additions leaves
~1e-16 differences that tiny, decaying factor entries amplify in relative
terms (see assert_iterate_parity)."""
import numpy as np
import pytest

import oracle
from paper_2307_03276_amd import cpapr, serve, synth
from tests.gpu_util import assert_iterate_parity, assert_parity, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _setup():
    import torch
    assert torch.cuda.is_available()
    oracle.build(force=False)
    cpapr.load()


def _requests(count, seed=0, nnz=(2_000, 30_000)):
    rng = np.random.default_rng(seed)
    reqs = []
    for q in range(count):
        nm = int(rng.integers(3, 5))
        dims = tuple(int(d) for d in rng.integers(30, 300, size=nm))
        n = int(np.exp(rng.uniform(np.log(nnz[0]), np.log(nnz[1]))))
        R = int(rng.choice([10, 16, 32]))
        X = synth.random_tensor(5000 + q, dims, n, zipf=(1.1,) * nm)
        M = synth.random_model(5000 + q, dims, R)
        reqs.append(serve.Request(id=q, X=X, M=M, arrival=0.0))
    return reqs


def _clone(r):
    return serve.Request(id=r.id, X=r.X, M=r.M.copy(), arrival=r.arrival)


def test_mix_equals_alone_and_oracle_fp64():
    kw = dict(kmax=6, lmax=5, tol=1e-4, precision=cpapr.CPAPR_FP64)
    reqs = _requests(8)
    mix = serve.results_to_host(serve.Server(max_slots=8, **kw).run_trace([_clone(r) for r in reqs]))
    mix = {r.id: r for r in mix}
    for r in reqs:
        alone = serve.results_to_host(serve.Server(max_slots=1, **kw).run_trace([_clone(r)]))[0]
        m = mix[r.id]
        assert m.stats["outer_iters"] == alone.stats["outer_iters"]
        assert m.stats["inner_updates"] == alone.stats["inner_updates"]
        assert_parity(m.result_lam, alone.result_lam, 1e-12, "lambda mix vs alone")
        for a, b in zip(m.result_factors, alone.result_factors):
            assert_iterate_parity(a, b, 1e-12, "factor mix vs alone")
        out, st = oracle.solve(r.X, r.M, kmax=6, lmax=5, tau=1e-4)
        assert m.stats["outer_iters"] == st["outer_iters"]
        assert m.stats["inner_updates"] == st["inner_updates"]
        assert_parity(m.result_lam, out.lam, 1e-12, "lambda vs oracle")
        for a, b in zip(m.result_factors, out.factors):
            assert_iterate_parity(a, b, 1e-12, "factor vs oracle")
        assert abs(m.stats["loglik"] - oracle.loglik(r.X, out)) <= 1e-12 * abs(m.stats["loglik"])


def test_mix_mixed_precision_matches_plain_path():
    kw = dict(kmax=5, lmax=5, tol=1e-4)
    reqs = _requests(6, seed=1)
    done = {r.id: r for r in serve.results_to_host(serve.Server(max_slots=6, precision=cpapr.CPAPR_MIXED, **kw).run_trace(
        [_clone(r) for r in reqs]))}
    for r in reqs:
        lam, facs, st = serve.solve_one(_clone(r), precision=cpapr.CPAPR_MIXED, **kw)
        lam, facs = host(lam), [host(a) for a in facs]
        m = done[r.id]
        assert m.stats["outer_iters"] == st["outer_iters"] and m.stats["inner_updates"] == st["inner_iters"]
        assert_parity(m.result_lam, lam, 1e-10, "lambda")
        for a, b in zip(m.result_factors, facs):
            assert_parity(a, b, 1e-10, "factor", elementwise=False)


def test_budget_bounds_admission_and_rejects_oversize():
    reqs = _requests(5, seed=2)
    probe = serve.Server(max_slots=4, kmax=2, lmax=2, tol=0.0)
    biggest = max(probe.footprint(r) for r in reqs)
    srv = serve.Server(budget_bytes=biggest * 1.5, max_slots=4, kmax=2, lmax=2, tol=0.0)
    done = srv.run_trace([_clone(r) for r in reqs])
    assert len(done) == 5 and all("rejected" not in r.stats for r in done)
    assert srv.peak_used <= biggest * 1.5
    # the budget binds (all five do not fit at once), and no more requests were
    # ever active together than the smallest footprints the budget holds
    sizes = sorted(probe.footprint(r) for r in reqs)
    assert sum(sizes) > biggest * 1.5
    most = max(k for k in range(1, 6) if sum(sizes[:k]) <= biggest * 1.5)
    assert srv.peak_active <= most
    tiny = serve.Server(budget_bytes=1000, max_slots=4, kmax=2, lmax=2, tol=0.0)
    out = tiny.run_trace([_clone(reqs[0])])
    assert out[0].stats.get("rejected")


def test_arrivals_over_time_and_latency_summary():
    reqs = _requests(6, seed=3)
    for i, r in enumerate(reqs):
        r.arrival = 0.01 * i
    srv = serve.Server(max_slots=3, kmax=3, lmax=3, tol=1e-4)
    done = srv.run_trace(reqs)
    s = serve.latency_summary(done)
    assert s["completed"] == 6 and s["p99_from_arrival_s"] >= s["p50_from_arrival_s"] > 0
    assert all(r.t_done >= r.t_admit >= r.arrival for r in done)


def test_srpt_rounds_give_the_same_results():
    """Shortest-remaining-work rounds hold some requests each round (their
    slots do no work); every request still computes exactly what it computes
    when all run every round."""
    kw = dict(kmax=4, lmax=4, tol=1e-4, precision=cpapr.CPAPR_FP64)
    reqs = _requests(6, seed=3)
    allr = {r.id: r for r in serve.results_to_host(serve.Server(max_slots=6, **kw).run_trace([_clone(r) for r in reqs]))}
    cap = sorted(r.X.nnz for r in reqs)[2]  # about two requests per round
    srv = serve.Server(max_slots=6, policy="srpt", round_cap=cap, **kw)
    srpt = {r.id: r for r in serve.results_to_host(srv.run_trace([_clone(r) for r in reqs]))}
    assert srv.ticks > max(r.stats["outer_iters"] for r in srpt.values()) * 4  # rounds were split
    for r in reqs:
        a, s = allr[r.id], srpt[r.id]
        assert s.stats["outer_iters"] == a.stats["outer_iters"]
        assert s.stats["inner_updates"] == a.stats["inner_updates"]
        assert_parity(s.result_lam, a.result_lam, 1e-12, "lambda")
        for x, y in zip(s.result_factors, a.result_factors):
            assert_iterate_parity(x, y, 1e-12, "factor")


def test_held_slot_does_no_work():
    import torch
    from tests.gpu_util import dev, host
    reqs = _requests(2, seed=4)
    b = cpapr.Batch(2, 1 << 16)
    items = []
    for sl, r in enumerate(reqs):
        P = cpapr.Plan.from_tensor(r.X, r.M.rank, lmax=3, tol=0.0)
        A = [dev(a) for a in r.M.factors]
        B = dev(r.M.factors[0] * r.M.lam)
        Phi = torch.full((r.X.dims[0], r.M.rank), 5.0, dtype=torch.float64, device="cuda")
        b.set(sl, P, 0, B, A, Phi)
        items.append((P, A, B, Phi))
    b.commit()
    B1, Phi1 = host(items[1][2]).copy(), host(items[1][3]).copy()
    b.hold([0, 1])
    b.inner(3)
    viol, upd, done = b.status()
    assert done[1] == 1 and upd[1] == 0 and upd[0] == 3
    assert np.array_equal(host(items[1][2]), B1) and np.array_equal(host(items[1][3]), Phi1)
    Bo, _, _, _ = oracle.mu_inner(reqs[0].X, 0, reqs[0].M.factors[0] * reqs[0].M.lam, reqs[0].M.factors, lmax=3)
    assert_parity(host(items[0][2]), Bo, 1e-12, "slot 0")
    b.hold([0, 0])
    b.inner(3)
    assert b.status()[1][1] == 3  # released: runs again
    b.close()
    for P, *_ in items:
        P.close()
