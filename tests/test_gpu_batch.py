"""Batched Phi (persistent launches over many plans, optionally replayed as a
hipGraph): every slot against the FP64 oracle, alone-vs-in-the-mix against the
single-plan path, graph replays checked one by one with eager work in between,
and slot changes picked up by an existing graph."""
import numpy as np
import pytest

import oracle
from paper_2307_03276_amd import cpapr, synth
from tests.gpu_util import assert_parity, dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _setup():
    import torch
    assert torch.cuda.is_available()
    oracle.build(force=False)
    cpapr.load()


def _case(i, rng):
    nm = int(rng.integers(2, 5))
    dims = tuple(int(d) for d in rng.integers(20, 400, size=nm))
    nnz = int(np.exp(rng.uniform(np.log(50), np.log(40_000))))
    R = int(rng.choice([8, 10, 16, 32]))
    zipf = tuple(1.1 if rng.random() < 0.5 else None for _ in range(nm))
    X = synth.random_tensor(1000 + i, dims, nnz, zipf=zipf)
    M = synth.random_model(1000 + i, dims, R)
    return X, M


def _build(cases, precision=cpapr.CPAPR_FP64, seed=0, persistent=False):
    import torch
    rng = np.random.default_rng(seed)
    items = []
    for X, M in cases:
        P = cpapr.Plan.from_tensor(X, M.rank, precision=precision)
        n = int(rng.integers(0, X.nmodes))
        A = [dev(a) for a in M.factors]
        Bh = M.factors[n] * M.lam
        Phi = torch.full((X.dims[n], M.rank), np.nan, dtype=torch.float64, device="cuda")
        items.append(dict(X=X, M=M, P=P, n=n, A=A, Bh=Bh, B=dev(Bh), Phi=Phi))
    tiles = sum(it["P"].tiles() for it in items)
    batch = cpapr.Batch(len(items) + 3, tiles + 16, persistent=persistent)
    for s, it in enumerate(items):
        batch.set(s, it["P"], it["n"], it["B"], it["A"], it["Phi"])
    return items, batch


@pytest.mark.parametrize("persistent", [False, True])
def test_batch_matches_oracle_and_single_plan(persistent):
    import torch
    rng = np.random.default_rng(1)
    cases = [_case(i, rng) for i in range(40)]
    items, batch = _build(cases, persistent=persistent)
    batch.commit()
    batch.run(use_graph=False)
    torch.cuda.synchronize()
    for it in items:
        got = host(it["Phi"])
        ref = oracle.phi(it["X"], it["n"], it["Bh"], it["M"].factors)
        assert_parity(got, ref, 1e-12, f"slot dims={it['X'].dims} R={it['M'].rank}")
        alone = host(it["P"].phi(it["n"], it["B"], it["A"]))
        assert_parity(got, alone, 1e-13, "alone vs in the mix")
    batch.close()


@pytest.mark.parametrize("persistent", [False, True])
def test_batch_graph_replays_and_slot_changes(persistent):
    import torch
    rng = np.random.default_rng(2)
    cases = [_case(100 + i, rng) for i in range(24)]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        items, batch = _build(cases, seed=3, persistent=persistent)
        batch.commit()
        batch.run(use_graph=False)
        torch.cuda.synchronize()
        eager = [host(it["Phi"]).copy() for it in items]
        for rep in range(3):
            for it in items:
                it["Phi"].fill_(np.nan)
            _ = torch.ones(1000, device="cuda").sum().item()  # unrelated eager work between replays
            batch.run(use_graph=True)
            torch.cuda.synchronize()
            for it, e in zip(items, eager):
                assert_parity(host(it["Phi"]), e, 1e-13, f"replay {rep}")
        # change operands of some slots (new B), recommit, replay the same graph
        for s in range(0, len(items), 3):
            it = items[s]
            it["Bh"] = it["Bh"] * 1.5
            it["B"].copy_(dev(it["Bh"]))
        batch.commit()
        batch.run(use_graph=True)
        torch.cuda.synchronize()
        for it in items:
            ref = oracle.phi(it["X"], it["n"], it["Bh"], it["M"].factors)
            assert_parity(host(it["Phi"]), ref, 1e-12, "after slot change")
        # drop half the slots: the graph keeps working on the rest
        for s in range(0, len(items), 2):
            batch.clear(s)
        batch.commit()
        for it in items:
            it["Phi"].fill_(np.nan)
        batch.run(use_graph=True)
        torch.cuda.synchronize()
        for s, it in enumerate(items):
            if s % 2 == 0:
                assert np.isnan(host(it["Phi"])).all()  # not touched
            else:
                ref = oracle.phi(it["X"], it["n"], it["Bh"], it["M"].factors)
                assert_parity(host(it["Phi"]), ref, 1e-12, "subset")
        batch.close()


def test_batch_mixed_precision():
    import torch
    rng = np.random.default_rng(4)
    cases = [_case(200 + i, rng) for i in range(16)]
    items, batch = _build(cases, precision=cpapr.CPAPR_MIXED, seed=5)
    batch.commit()
    batch.run()
    torch.cuda.synchronize()
    for it in items:
        ref = oracle.phi(it["X"], it["n"], it["Bh"], it["M"].factors)
        assert_parity(host(it["Phi"]), ref, 1e-5, "mixed slot")
    batch.close()


def test_batch_errors():
    import torch
    X, M, _ = synth.config_small()
    P32 = cpapr.Plan.from_tensor(X, 10, group=32)  # no batched kernel for 32-lane groups
    b = cpapr.Batch(2, 100)
    A = [dev(a) for a in M.factors]
    B = dev(M.factors[0] * M.lam)
    Phi = torch.empty((100, 10), dtype=torch.float64, device="cuda")
    with pytest.raises(cpapr.CpaprError) as ei:
        b.set(0, P32, 0, B, A, Phi)
    assert ei.value.code == -6
    with pytest.raises(cpapr.CpaprError):
        b.set(5, cpapr.Plan.from_tensor(X, 10), 0, B, A, Phi)  # slot out of range
    P = cpapr.Plan.from_tensor(X, 10)
    b.set(0, P, 0, B, A, Phi)
    with pytest.raises(cpapr.CpaprError) as ei:
        b.run()  # not committed
    assert ei.value.code == -1
    small = cpapr.Batch(2, 1)
    small.set(0, P, 0, B, A, Phi)
    with pytest.raises(cpapr.CpaprError) as ei:
        small.commit()
    assert ei.value.code == -4


def test_batch_inner_loop_equals_mu_inner_per_slot():
    """The batched inner loop with per-slot KKT stops gives, slot by slot, what
    cpapr_mu_inner gives for that plan alone (B, last Phi, updates)."""
    import torch
    rng = np.random.default_rng(9)
    cases = [_case(300 + i, rng) for i in range(12)]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        items = []
        for X, M in cases:
            n = int(rng.integers(0, X.nmodes))
            Bh = M.factors[n] * M.lam
            _, _, hist, _ = oracle.mu_inner(X, n, Bh, M.factors, lmax=12)
            tol = float(hist[int(rng.integers(2, 10))]) * 1.0001  # each slot stops at its own iteration
            P = cpapr.Plan.from_tensor(X, M.rank, lmax=12, tol=tol)
            A = [dev(a) for a in M.factors]
            Phi = torch.zeros((X.dims[n], M.rank), dtype=torch.float64, device="cuda")
            items.append(dict(X=X, M=M, P=P, n=n, A=A, Bh=Bh, B=dev(Bh), Phi=Phi, tol=tol))
        b = cpapr.Batch(len(items), sum(it["P"].tiles() for it in items) + 1)
        for s, it in enumerate(items):
            b.set(s, it["P"], it["n"], it["B"], it["A"], it["Phi"])
        b.commit()
        for use_graph in (False, True, True):
            for it in items:
                it["B"].copy_(dev(it["Bh"]))
            b.inner(12, use_graph=use_graph)
            viol, upd, done = b.status()
            for s, it in enumerate(items):
                Bo, Po, hist, nup = oracle.mu_inner(it["X"], it["n"], it["Bh"], it["M"].factors, lmax=12,
                                                    tau=it["tol"])
                assert upd[s] == nup and done[s] == (1 if nup < 12 else 0)
                assert_parity(host(it["B"]), Bo, 1e-12, f"B slot {s}")
                assert_parity(host(it["Phi"]), Po, 1e-12, f"Phi slot {s}")
        b.close()
