"""Whole-solve parity (Algorithm 1) at the benchmark sizes, every factor entry
and lambda against the oracle's own solve of the same tensor:

* 3-way 200k x 150k x 20k, 20M Zipf(1.1) nonzeros, R = 16: two outer
  iterations of ten inner MU steps per mode, so the S shift of the second outer
  iteration runs on the factors the first one left; FP64 at 1e-12 (lambda
  elementwise, factors normwise and column-wise), FP32-stored factors at 1e-5
  normwise;
* 4-way 1M x 200k x 10k x 500, 100M nonzeros, R = 32: one outer iteration of
  two inner steps per mode in FP64 at 1e-12.

The oracle's solves run single-threaded for about two minutes each; they are
started in background threads when this module begins (the oracle's C calls
release the interpreter lock), so they overlap each other and the GPU work."""
import concurrent.futures as cf
import time

import numpy as np
import pytest

import oracle
from paper_2307_03276_amd import cpapr, synth
from tests.gpu_util import assert_iterate_parity, assert_parity, bucket_errors, colmax_errors, dev, host

pytestmark = pytest.mark.gpu

C2_SCHED = dict(kmax=2, lmax=10)
C3_SCHED = dict(kmax=1, lmax=2)


def _gen_and_solve(cfg, sched, gen_box):
    X, M, s = cfg()
    gen_box.set_result((X, M, s))
    t0 = time.perf_counter()
    out, ost = oracle.solve(X, M, tau=0.0, eps=s["eps"], **sched)
    return out, ost, time.perf_counter() - t0


@pytest.fixture(scope="module")
def jobs():
    import torch
    assert torch.cuda.is_available()
    oracle.build(force=False)
    pool = cf.ThreadPoolExecutor(max_workers=2)
    gens = {"zipf3": cf.Future(), "zipf4": cf.Future()}
    futs = {"zipf3": pool.submit(_gen_and_solve, synth.config_zipf3, C2_SCHED, gens["zipf3"]),
            "zipf4": pool.submit(_gen_and_solve, synth.config_zipf4, C3_SCHED, gens["zipf4"])}
    print("oracle solves started in the background", flush=True)
    yield gens, futs
    pool.shutdown(wait=True)


def _gpu_solve(X, M, sched, precision):
    P = cpapr.Plan.from_tensor(X, M.rank, precision=precision, tol=0.0, eps=1e-10, **sched)
    lam = dev(M.lam)
    A = [dev(a) for a in M.factors]
    st = P.solve(lam, A)
    P.close()
    return host(lam), [host(a) for a in A], st


def _oracle(jobs, name):
    gens, futs = jobs
    out, ost, secs = futs[name].result(timeout=900)
    print(f"{name}: oracle solve took {secs:.1f} s", flush=True)
    return out, ost


@pytest.mark.timeout(900)
@pytest.mark.parametrize("precision,tol", [(cpapr.CPAPR_FP64, 1e-12), (cpapr.CPAPR_MIXED, 1e-5)])
def test_solve_zipf3_fullsize(jobs, precision, tol):
    X, M, s = jobs[0]["zipf3"].result(timeout=300)
    lam, A, st = _gpu_solve(X, M, C2_SCHED, precision)
    out, ost = _oracle(jobs, "zipf3")
    assert st["outer_iters"] == ost["outer_iters"] == C2_SCHED["kmax"]
    assert st["inner_iters"] == ost["inner_updates"] == C2_SCHED["kmax"] * C2_SCHED["lmax"] * X.nmodes
    fp64 = precision == cpapr.CPAPR_FP64
    assert_parity(lam, out.lam, tol, "lambda")
    for n in range(X.nmodes):
        print(f"zipf3 {'fp64' if fp64 else 'mixed'} A{n}: elementwise by size {bucket_errors(A[n], out.factors[n])}, "
              f"column-wise {colmax_errors(A[n], out.factors[n]):.2e}", flush=True)
        if fp64:
            assert_iterate_parity(A[n], out.factors[n], tol, f"A{n}")
        else:
            assert_parity(A[n], out.factors[n], tol, f"A{n}", elementwise=False)
    # the columns sum to one and lambda carries the mass (Algorithm 1's normalisation)
    for n in range(X.nmodes):
        np.testing.assert_allclose(A[n].sum(axis=0), 1.0, rtol=1e-12 if fp64 else 1e-6)


@pytest.mark.timeout(900)
def test_solve_zipf4_fullsize(jobs):
    X, M, s = jobs[0]["zipf4"].result(timeout=600)
    lam, A, st = _gpu_solve(X, M, C3_SCHED, cpapr.CPAPR_FP64)
    out, ost = _oracle(jobs, "zipf4")
    assert st["outer_iters"] == ost["outer_iters"] == 1
    assert st["inner_iters"] == ost["inner_updates"] == C3_SCHED["lmax"] * X.nmodes
    assert_parity(lam, out.lam, 1e-12, "lambda")
    for n in range(X.nmodes):
        print(f"zipf4 fp64 A{n}: elementwise by size {bucket_errors(A[n], out.factors[n])}, "
              f"column-wise {colmax_errors(A[n], out.factors[n]):.2e}", flush=True)
        assert_iterate_parity(A[n], out.factors[n], 1e-12, f"A{n}")
