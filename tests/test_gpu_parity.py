"""GPU parity: the HIP path through the C ABI against the FP64 oracle, element by
element on the same seeded inputs.

Gate (FP64): normwise and elementwise relative error <= 1e-12, and exact zeros
where the oracle has exact zeros (rows without nonzeros); factor matrices of
whole solves are held column-wise (every entry against its column's largest,
see assert_iterate_parity). Mixed precision (FP32-stored factors widened to
FP64 as they are gathered): <= 1e-5. Sizes span many tiles
and a ragged tail; the edge cases cover empty and single-entry tensors, empty
rows, clamped divisors, duplicates, one row spanning the whole tensor, every
supported lane-group / rank-block shape, and N from 2 to 8."""
import numpy as np
import pytest

import oracle
from paper_2307_03276_amd import cpapr, synth
from tests.gpu_util import assert_iterate_parity, assert_parity, dev, host

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOLMIX = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _setup():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    oracle.build(force=False)
    cpapr.load()


def _phi_case(X, M, R=None, modes=None, tol=TOL64, eps=1e-10, B_scale=1.0, **kw):
    R = M.rank if R is None else R
    P = cpapr.Plan.from_tensor(X, R, **kw)
    A = [dev(a) for a in M.factors]
    out = []
    for n in (range(X.nmodes) if modes is None else modes):
        Bh = M.factors[n] * M.lam * B_scale
        got = host(P.phi(n, dev(Bh), A, eps=eps))
        ref = oracle.phi(X, n, Bh, M.factors, eps=eps)
        out.append(assert_parity(got, ref, tol, f"mode {n}"))
    P.close()
    return out


def test_phi_small_config_every_mode():
    X, M, sched = synth.config_small()
    _phi_case(X, M)


@pytest.mark.parametrize("R", [1, 2, 5, 8, 10, 16, 17, 32, 33, 64, 100, 128, 256])
def test_phi_ranks(R):
    X = synth.random_tensor(R, (300, 200, 50), 20_000 + 37 * R, zipf=(1.1, None, 1.2))
    M = synth.random_model(R, X.dims, R)
    _phi_case(X, M)


@pytest.mark.parametrize("dims", [(50, 60), (20, 30, 40, 10), (9, 8, 7, 6, 5), (4, 5, 3, 6, 2, 3, 4, 5)])
def test_phi_modes(dims):
    X = synth.random_tensor(7, dims, 15_000, zipf=(1.1,) * len(dims))
    M = synth.random_model(7, dims, 12)
    _phi_case(X, M)


@pytest.mark.parametrize("group,R", [(4, 4), (4, 16), (8, 8), (8, 16), (16, 16), (16, 32), (16, 64),
                                     (32, 32), (32, 100), (64, 10), (64, 256)])
@pytest.mark.parametrize("chunk", [1, 3, 17, 0])
def test_phi_launch_shapes(group, R, chunk):
    X = synth.random_tensor(group * R + chunk, (500, 90, 40), 9_001, zipf=(1.3, 1.1, None))
    M = synth.random_model(3, X.dims, R)
    _phi_case(X, M, group=group, chunk=chunk)


@pytest.mark.parametrize("sort", [0, 1])
@pytest.mark.parametrize("dims", [(300, 2000, 50), (40, 30, 20, 10)])
def test_phi_sort_modes(sort, dims):
    X = synth.random_tensor(17, dims, 60_000, zipf=(1.1,) * len(dims))
    M = synth.random_model(17, dims, 16)
    _phi_case(X, M, sort=sort)


def _key_width(dim):
    b = 0
    while b < 31 and (1 << b) < dim:
        b += 1
    return b


def _expected_order(X, n, sort):
    """Stable order by i_n, or (ROW_COL) by i_n then the largest other mode's
    coordinate, both in one 32-bit key: the coordinate keeps its high bits."""
    key = X.idx[n].astype(np.uint64)
    if sort == cpapr.CPAPR_SORT_ROW_COL:
        sec = max((m for m in range(X.nmodes) if m != n), key=lambda m: X.dims[m])
        bits, sbits = _key_width(X.dims[n]), _key_width(X.dims[sec])
        keep = min(sbits, 32 - bits)
        key = (key << np.uint64(keep)) | (X.idx[sec].astype(np.uint64) >> np.uint64(sbits - keep))
    return np.argsort(key, kind="stable")


@pytest.mark.parametrize("sort", [0, 1])
@pytest.mark.parametrize("dims", [(3000, 2000, 100), ((1 << 17) + 1, (1 << 16) + 1, 300),
                                  (40, 1 << 20, 30, 1 << 14)])
def test_plan_order_is_the_stable_key_order(sort, dims):
    """A plan orders each mode's nonzeros exactly as the stable sort by its key:
    a plan of the tensor given already in that order (which a stable sort leaves
    as it is) has the same tiles and summation order, so deterministic Phi
    agrees bit for bit; any other order of a row's nonzeros changes its sums'
    rounding. Two of the shapes need more than 32 key bits in ROW_COL, so the
    secondary coordinate loses low bits there."""
    X = synth.random_tensor(21, dims, 200_000, zipf=(1.1,) * len(dims))
    M = synth.random_model(21, dims, 16)
    A = [dev(a) for a in M.factors]
    P = cpapr.Plan.from_tensor(X, 16, deterministic=1, sort=sort)
    for n in range(X.nmodes):
        o = _expected_order(X, n, sort)
        Xs = synth.SparseTensor(X.dims, np.ascontiguousarray(X.idx[:, o]), X.vals[o].copy())
        Q = cpapr.Plan.from_tensor(Xs, 16, deterministic=1, sort=sort)
        assert P.shape() == Q.shape() and P.segments(n) == Q.segments(n)
        B = dev(M.factors[n] * M.lam)
        a, b = host(P.phi(n, B, A)), host(Q.phi(n, B, A))
        assert np.array_equal(a, b), f"mode {n}: the plan's order is not the stable key order"
        Q.close()
    P.close()


def test_phi_one_row_spans_everything():
    """Every nonzero in one row of mode 0: the row crosses every tile boundary."""
    rng = np.random.default_rng(5)
    nnz = 300_001
    idx = np.stack([np.full(nnz, 3), rng.integers(0, 70, nnz), rng.integers(0, 30, nnz)]).astype(np.int32)
    X = synth.SparseTensor((10, 70, 30), idx, 1.0 + rng.poisson(2.0, nnz).astype(np.float64))
    M = synth.random_model(5, X.dims, 16)
    _phi_case(X, M)
    _phi_case(X, M, chunk=5)


def test_phi_empty_rows_duplicates_and_clamp():
    X = synth.random_tensor(9, (1000, 40, 30), 5000, zipf=(1.5, 1.1, 1.1))  # many empty rows, many duplicates
    M = synth.random_model(9, X.dims, 8)
    # scale B down so that part of the nonzeros hit the eps floor
    Bh = M.factors[0] * M.lam * 1e-3
    P = cpapr.Plan.from_tensor(X, 8)
    A = [dev(a) for a in M.factors]
    Pi_dot = None
    eps = 1e-4
    got = host(P.phi(0, dev(Bh), A, eps=eps))
    ref = oracle.phi(X, 0, Bh, M.factors, eps=eps)
    assert_parity(got, ref, TOL64, "clamped")
    assert np.sum(np.all(ref == 0, axis=1)) > 100  # empty rows really present
    P.close()


def test_phi_degenerate_sizes():
    # nnz = 0: Phi is all zero
    import torch
    X0 = synth.SparseTensor((5, 4, 3), np.zeros((3, 0), dtype=np.int32), np.zeros(0))
    M = synth.random_model(1, X0.dims, 4)
    P = cpapr.Plan.from_tensor(X0, 4)
    out = P.phi(1, dev(M.factors[1] * M.lam), [dev(a) for a in M.factors])
    assert torch.count_nonzero(out).item() == 0
    P.close()
    # a single nonzero; a mode of size 1
    X1 = synth.SparseTensor((1, 4, 3), np.array([[0], [2], [1]], dtype=np.int32), np.array([5.0]))
    _phi_case(X1, synth.random_model(2, X1.dims, 3))
    # ragged tail: nnz just past a tile multiple
    X2 = synth.random_tensor(3, (700, 600, 500), 4 * 1024 + 1, zipf=(1.1, 1.1, 1.1))
    _phi_case(X2, synth.random_model(3, X2.dims, 16))


def test_phi_quotient_within_a_few_ulps():
    """The per-nonzero quotient x / max(b.pi, eps), formed from the reciprocal
    estimate and one Newton step, against the oracle's correctly rounded
    division: a 2-way tensor with R = 1 and one nonzero per row of mode 0, so
    Phi[i] = (x / (b_i a_j)) a_j and every other operation is exact or rounded
    identically on both sides. The Newton step squares the estimate's relative
    error e: |error| <= e^2 + 3 * 2^-53 or so; an estimate good to 2^-23.5
    keeps it within 32 * 2^-52 (measured: 10.2 * 2^-52). Without the Newton
    step, or with a wrong one, the error is of the order of e itself (~1e-7)."""
    rng = np.random.default_rng(21)
    I, J = 1_000_000, 5000
    idx = np.stack([np.arange(I), rng.integers(0, J, I)]).astype(np.int32)
    X = synth.SparseTensor((I, J), idx, rng.integers(1, 1000, I).astype(np.float64))
    A = [rng.uniform(0.5, 2.0, (I, 1)), rng.uniform(0.5, 2.0, (J, 1))]
    P = cpapr.Plan.from_tensor(X, 1)
    got = host(P.phi(0, dev(A[0]), [dev(a) for a in A]))
    ref = oracle.phi(X, 0, A[0], A)
    rel = np.abs(got - ref) / np.abs(ref)
    print(f"quotient: largest relative difference {rel.max():.3e} ({rel.max() / 2.0 ** -52:.2f} x 2^-52), "
          f"{np.count_nonzero(rel)} of {I} rows differ", flush=True)
    assert rel.max() <= 32 * 2.0 ** -52
    P.close()


@pytest.mark.parametrize("dims", [(300, 200, 50), (400, 90), (60, 50, 40, 30)])
def test_phi_values_not_exact_in_fp32(dims):
    """Plans of up to three modes stage each nonzero from a packed 16-byte
    record with the value in FP32, when every value is exact there (counts);
    a value that is not (here counts + 0.1) keeps the separate arrays with the
    FP64 value; four-mode plans always read the arrays. All against the
    oracle."""
    X = synth.random_tensor(23, dims, 30_000, zipf=(1.2,) + (None,) * (len(dims) - 1))
    M = synth.random_model(23, dims, 16)
    Xf = synth.SparseTensor(X.dims, X.idx, X.vals + 0.1)
    _phi_case(Xf, M)
    _phi_case(X, M)


@pytest.mark.parametrize("group,R", [(4, 8), (8, 16), (16, 32), (32, 64), (64, 100)])
@pytest.mark.parametrize("precision", [cpapr.CPAPR_FP64, cpapr.CPAPR_MIXED])
def test_phi_four_way_packed_shapes(group, R, precision):
    """Four-way plans at lane-group shapes from 4 to 64 lanes, both
    precisions, non-integer values, several tiles and a ragged tail."""
    X = synth.random_tensor(31 + R, (700, 300, 90, 20), 50_003, zipf=(1.2, 1.1, None, None))
    X = synth.SparseTensor(X.dims, X.idx, X.vals * 0.75 + 0.01)
    M = synth.random_model(31, X.dims, R)
    _phi_case(X, M, tol=TOL64 if precision == cpapr.CPAPR_FP64 else TOLMIX, precision=precision,
              group=group, chunk=0)


def test_phi_atomic_variant_matches():
    X, M, _ = synth.config_small()
    _phi_case(X, M, variant=cpapr.CPAPR_VARIANT_ATOMIC)
    X = synth.random_tensor(2, (400, 300, 200), 60_000, zipf=(1.1, 1.1, 1.1))
    _phi_case(X, synth.random_model(2, X.dims, 16), variant=cpapr.CPAPR_VARIANT_ATOMIC)


@pytest.mark.parametrize("R", [8, 10, 16, 32])
def test_phi_mixed_precision(R):
    X = synth.random_tensor(11, (2000, 1500, 300), 200_000, zipf=(1.1, 1.1, 1.1), mu=3.0)
    M = synth.random_model(11, X.dims, R)
    _phi_case(X, M, tol=TOLMIX, precision=cpapr.CPAPR_MIXED)


def test_phi_deterministic_repeat():
    X = synth.random_tensor(13, (3000, 2000, 100), 300_000, zipf=(1.1, 1.1, 1.1))
    M = synth.random_model(13, X.dims, 16)
    P = cpapr.Plan.from_tensor(X, 16)
    A = [dev(a) for a in M.factors]
    B = dev(M.factors[0] * M.lam)
    a = host(P.phi(0, B, A))
    b = host(P.phi(0, B, A))
    # rows that cross tile boundaries use atomics; results agree to the gate either way
    assert_parity(a, b, 1e-14, "repeat")
    P.close()


def test_prof_sampled_records_every_kth_launch():
    """Kernel timing sampled every 3rd Phi launch: of 10 launches alternating
    modes 0 and 1, launches 0, 3, 6 and 9 are recorded, with their modes and
    positive durations."""
    X, M, _ = synth.config_small()
    P = cpapr.Plan.from_tensor(X, M.rank)
    A = [dev(a) for a in M.factors]
    Bs = [dev(M.factors[n] * M.lam) for n in range(2)]
    cpapr.cpapr_prof_enable_sampled(16, 3)
    try:
        for i in range(10):
            P.phi(i % 2, Bs[i % 2], A)
        recs = cpapr.cpapr_prof_read(16)
    finally:
        cpapr.cpapr_prof_disable()
    assert [m for m, _ in recs] == [0, 1, 0, 1]
    assert all(ms > 0 for _, ms in recs)
    P.close()


def test_deterministic_mode_repeats_bit_for_bit():
    """Deterministic plans: Phi, MTTKRP, a solve and PQNR row solves repeat bit
    for bit, and still match the oracle; heavy Zipf rows span many tiles."""
    import numpy as np
    X = synth.random_tensor(13, (3000, 2000, 100), 300_000, zipf=(1.2, 1.1, 1.1))
    M = synth.random_model(13, X.dims, 16)
    P = cpapr.Plan.from_tensor(X, 16, deterministic=1, kmax=2, lmax=3, tol=0.0)
    A = [dev(a) for a in M.factors]
    for n in range(3):
        Bh = M.factors[n] * M.lam
        B = dev(Bh)
        a, b = host(P.phi(n, B, A)), host(P.phi(n, B, A))
        assert np.array_equal(a, b), f"Phi mode {n} differs between runs"
        assert_parity(a, oracle.phi(X, n, Bh, M.factors), TOL64, f"deterministic Phi mode {n}")
        m1, m2 = host(P.mttkrp(n, A)), host(P.mttkrp(n, A))
        assert np.array_equal(m1, m2)
        assert_parity(m1, oracle.mttkrp(X, n, M.factors), TOL64, f"deterministic MTTKRP mode {n}")
    outs = []
    for _ in range(2):
        lam = dev(M.lam)
        Af = [dev(a) for a in M.factors]
        P.solve(lam, Af)
        outs.append([host(lam)] + [host(x) for x in Af])
    for x, y in zip(*outs):
        assert np.array_equal(x, y), "solve differs between runs"
    with pytest.raises(cpapr.CpaprError) as ei:
        P.set_shape(8, 8)  # 256-nonzero tiles are fine; 64 are not
        P.set_shape(8, 2)
    assert ei.value.code == -6
    P.close()
    Pq = cpapr.Plan.from_tensor(X, 16, deterministic=1, lmax=4, tol=0.0, method=cpapr.CPAPR_METHOD_PQNR)
    res = []
    for _ in range(2):
        B = dev(M.factors[0] * M.lam)
        Pq.pqnr_inner(0, B, A)
        res.append(host(B))
    assert np.array_equal(res[0], res[1]), "PQNR differs between runs"
    Pq.close()


def test_plan_segments_counts():
    X, M, _ = synth.config_small()
    P = cpapr.Plan.from_tensor(X, 10)
    for n in range(3):
        assert P.segments(n) == np.unique(X.idx[n]).size
    P.close()


def test_invalid_inputs_are_rejected():
    import torch
    X, M, _ = synth.config_small()
    idx = X.idx.copy()
    idx[1, 17] = 80  # out of range for mode 1 (size 80)
    with pytest.raises(cpapr.CpaprError) as ei:
        cpapr.Plan(X.dims, dev(idx), dev(X.vals), 10)
    assert ei.value.code == -2
    vals = X.vals.copy()
    vals[5] = 0.0
    with pytest.raises(cpapr.CpaprError) as ei:
        cpapr.Plan(X.dims, dev(X.idx), dev(vals), 10)
    assert ei.value.code == -3
    vals[5] = np.nan
    with pytest.raises(cpapr.CpaprError) as ei:
        cpapr.Plan(X.dims, dev(X.idx), dev(vals), 10)
    assert ei.value.code == -3


# ---------------------------------------------------------------- MU inner loop, solve, loglik

def test_launch_policy_model_shapes():
    """Default launch shape from the launch-policy model of the tensor. A large
    tensor gets 512-nonzero tiles with lanes by rank, except 17 <= R <= 32
    (16 x 2 on 256-nonzero tiles in FP64, 8 x 4 on 1024 with FP32-stored
    factors) and 5 <= R <= 16 with packed nonzero records (values exact in
    FP32, up to three modes: 1024-nonzero tiles); a smaller one tiles of the
    largest power of two <= nnz/900 (at least 32), on 16 lanes up to 128
    nonzeros, lanes by rank at 256 and 512 (16 at 256 for 9 <= R <= 16 with
    FP32-stored factors); deterministic plans keep tiles of at least 128. Explicit shapes are kept, and the model returns when
    the shape is reset. In a batch a plan on the model's shape takes the large
    tensor's shape."""
    X, M, _ = synth.config_small()  # 10,000 nonzeros, R = 10
    P = cpapr.Plan.from_tensor(X, 10)
    assert P.shape() == (16, 2)
    assert P.batch_shape() == (8, 32) and P.tiles() == 10
    P.set_shape(8, 40)
    assert P.shape() == (8, 40) and P.batch_shape() == (8, 40)
    assert P.tiles() == -(-10_000 // (32 * 40))
    P.set_shape(0, 0)
    assert P.shape() == (16, 2) and P.batch_shape() == (8, 32)
    P.set_shape(8, 0)
    assert P.shape() == (8, 1) and P.batch_shape() == (8, 1)
    P.close()
    Pd = cpapr.Plan.from_tensor(X, 10, deterministic=1)
    assert Pd.shape() == (16, 8)
    Pd.close()
    cases = {300_000: [(16, cpapr.CPAPR_FP64, (8, 8)), (8, cpapr.CPAPR_MIXED, (8, 8)),
                       (16, cpapr.CPAPR_MIXED, (16, 16)), (32, cpapr.CPAPR_FP64, (16, 16))],
             600_000: [(16, cpapr.CPAPR_FP64, (8, 16)), (16, cpapr.CPAPR_MIXED, (8, 16)),
                       (32, cpapr.CPAPR_FP64, (16, 16)), (32, cpapr.CPAPR_MIXED, (8, 16)),
                       (8, cpapr.CPAPR_FP64, (8, 16)), (64, cpapr.CPAPR_FP64, (16, 32))],
             1_100_000: [(32, cpapr.CPAPR_MIXED, (8, 32)), (32, cpapr.CPAPR_FP64, (16, 16)),
                         (16, cpapr.CPAPR_FP64, (8, 32))]}
    big = {(16, cpapr.CPAPR_FP64): (8, 32), (8, cpapr.CPAPR_MIXED): (8, 32), (16, cpapr.CPAPR_MIXED): (8, 32),
           (32, cpapr.CPAPR_FP64): (16, 16), (32, cpapr.CPAPR_MIXED): (8, 32), (8, cpapr.CPAPR_FP64): (8, 32),
           (64, cpapr.CPAPR_FP64): (16, 32)}
    for nnz, want in cases.items():
        Xn = synth.random_tensor(nnz % 97, (400, 300, 200), nnz)
        for R, prec, shape in want:
            Pn = cpapr.Plan.from_tensor(Xn, R, precision=prec)
            assert Pn.shape() == shape, (nnz, R, prec, Pn.shape())
            assert Pn.batch_shape() == big[(R, prec)], (nnz, R, prec, Pn.batch_shape())
            Pn.close()
    # values not exact in FP32: no packed records, so 512-nonzero tiles
    Xn = synth.random_tensor(7, (400, 300, 200), 1_100_000)
    Xf = synth.SparseTensor(Xn.dims, Xn.idx, Xn.vals + 0.1)
    Pf = cpapr.Plan.from_tensor(Xf, 16)
    assert Pf.shape() == (8, 16) and Pf.batch_shape() == (8, 16)
    Pf.close()


def test_mu_inner_fixed_schedule():
    X, M, _ = synth.config_small()
    P = cpapr.Plan.from_tensor(X, 10, lmax=10, tol=0.0)
    A = [dev(a) for a in M.factors]
    for n in range(3):
        Bh = M.factors[n] * M.lam
        B = dev(Bh)
        phi_last, st = P.mu_inner(n, B, A)
        Bo, Po, hist, nup = oracle.mu_inner(X, n, Bh, M.factors, lmax=10)
        assert st["inner_iters"] == nup == 10 and st["phi_evals"] == 10
        assert_parity(host(B), Bo, TOL64, f"B mode {n}")
        assert_parity(host(phi_last), Po, TOL64, f"Phi mode {n}")
        assert abs(st["kkt_violation"] - hist[-1]) <= 1e-12 * max(1.0, hist[-1])
    P.close()


def test_mu_inner_kkt_stop():
    X, M, _ = synth.config_small()
    n = 1
    Bh = M.factors[n] * M.lam
    _, _, hist, _ = oracle.mu_inner(X, n, Bh, M.factors, lmax=30)
    tau = float(hist[6]) * 1.001  # lands between two iterations' violations
    Bo, Po, hist_o, nup_o = oracle.mu_inner(X, n, Bh, M.factors, lmax=30, tau=tau)
    assert 0 < nup_o < 30
    P = cpapr.Plan.from_tensor(X, 10, lmax=30, tol=tau)
    B = dev(Bh)
    phi_last, st = P.mu_inner(n, B, [dev(a) for a in M.factors])
    assert st["inner_iters"] == nup_o
    assert st["phi_evals"] == nup_o + 1  # the Phi that triggered the stop is computed too
    assert_parity(host(B), Bo, TOL64, "B")
    assert_parity(host(phi_last), Po, TOL64, "Phi_last")
    P.close()


def _solve_case(X, M, kmax, lmax, tau, tol, elementwise=True, **kw):
    import torch
    P = cpapr.Plan.from_tensor(X, M.rank, kmax=kmax, lmax=lmax, tol=tau, **kw)
    lam = dev(M.lam)
    A = [dev(a) for a in M.factors]
    st = P.solve(lam, A)
    torch.cuda.synchronize()
    out, ost = oracle.solve(X, M, kmax=kmax, lmax=lmax, tau=tau)
    assert st["outer_iters"] == ost["outer_iters"]
    assert st["inner_iters"] == ost["inner_updates"]
    # one Phi per update, plus one per inner loop that stopped on the KKT test
    assert st["inner_iters"] <= st["phi_evals"] <= st["inner_iters"] + st["outer_iters"] * X.nmodes
    assert bool(st["converged"]) == ost["converged"]
    assert_parity(host(lam), out.lam, tol, "lambda")
    for n in range(X.nmodes):
        if elementwise:
            assert_iterate_parity(host(A[n]), out.factors[n], tol, f"A{n}")
        else:
            assert_parity(host(A[n]), out.factors[n], tol, f"A{n}", elementwise=False)
    ll = oracle.loglik(X, out)
    assert abs(st["loglik"] - ll) <= max(tol, 1e-12) * abs(ll)
    P.close()
    return st, ost


def test_solve_small_config_fixed_schedule():
    X, M, s = synth.config_small()
    _solve_case(X, M, s["kmax"], s["lmax"], 0.0, TOL64)


def test_solve_to_kkt_tolerance_with_shift():
    X = synth.random_tensor(21, (60, 50, 40, 8), 12_000, zipf=(1.2, 1.2, None, None))
    M = synth.random_model(21, X.dims, 6)
    M.factors[0][3, 2] = 0.0  # an inadmissible zero for the S shift to lift
    st, ost = _solve_case(X, M, 30, 10, 1e-4, TOL64)


@pytest.mark.parametrize("dims,R,nnz,seed", [
    ((6, 5, 4, 3, 5, 4, 3, 2), 3, 400, 31),     # eight modes
    ((30, 20, 10), 256, 3000, 32),              # the largest rank
    ((1, 40, 1), 4, 60, 33),                    # single-row modes
    ((50, 40, 30), 5, 1, 34),                   # one nonzero
])
def test_solve_unusual_shapes(dims, R, nnz, seed):
    """Full fixed-schedule solves at the edges of the supported shapes."""
    X = synth.random_tensor(seed, dims, nnz)
    M = synth.random_model(seed, dims, R)
    _solve_case(X, M, 3, 4, 0.0, TOL64)


def test_solve_all_duplicates():
    """Every nonzero at the same cell: one row per mode holds all of them."""
    import numpy as np
    dims = (7, 6, 5)
    idx = np.tile(np.array([[3], [2], [4]], dtype=np.int32), (1, 500))
    X = synth.SparseTensor(dims, idx, np.full(500, 2.0))
    M = synth.random_model(35, dims, 4)
    _solve_case(X, M, 3, 5, 0.0, TOL64)


def test_solve_mixed_precision_fixed_schedule():
    """Mixed precision against the FP64 oracle over 10 x 10 MU steps: lambda and
    every factor within 1e-5 normwise; the log-likelihood within 1e-5."""
    X, M, s = synth.config_small()
    _solve_case(X, M, s["kmax"], s["lmax"], 0.0, TOLMIX, elementwise=False, precision=cpapr.CPAPR_MIXED)


def test_loglik_matches_oracle():
    X = synth.random_tensor(31, (500, 400, 300), 100_000, zipf=(1.1, 1.1, None))
    M = synth.random_model(31, X.dims, 16)
    P = cpapr.Plan.from_tensor(X, 16)
    got = P.loglik(dev(M.lam), [dev(a) for a in M.factors])
    ref = oracle.loglik(X, M)
    assert abs(got - ref) <= TOL64 * abs(ref)
    P.close()


@pytest.mark.parametrize("dims,R", [((300, 200, 100), 16), ((40, 30, 20, 10), 10)])
def test_mttkrp_matches_oracle(dims, R):
    X = synth.random_tensor(41, dims, 40_000, zipf=(1.1,) * len(dims))
    M = synth.random_model(41, dims, R)
    P = cpapr.Plan.from_tensor(X, R)
    A = [dev(a) for a in M.factors]
    for n in range(len(dims)):
        assert_parity(host(P.mttkrp(n, A)), oracle.mttkrp(X, n, M.factors), TOL64, f"mode {n}")
    P.close()


def test_phi_and_inner_loop_random_sweep():
    """Thirty seeded random cases (2-6 modes, dims 1-300, R 1-48, uniform or
    Zipf coordinates, FP64 and mixed): Phi of every mode and a 3-step inner
    loop of one mode against the oracle."""
    import numpy as np
    rng = np.random.default_rng(77)
    for case in range(30):
        N = int(rng.integers(2, 7))
        dims = tuple(int(d) for d in rng.integers(1, 300, size=N))
        nnz = int(rng.integers(1, 5000))
        R = int(rng.integers(1, 49))
        zipf = tuple(1.1 if rng.random() < 0.5 else None for _ in range(N))
        mixed = bool(rng.random() < 0.3)
        X = synth.random_tensor(500 + case, dims, nnz, zipf=zipf)
        M = synth.random_model(500 + case, dims, R)
        prec = cpapr.CPAPR_MIXED if mixed else cpapr.CPAPR_FP64
        tol = TOLMIX if mixed else TOL64
        P = cpapr.Plan.from_tensor(X, R, precision=prec, lmax=3, tol=0.0)
        A = [dev(a) for a in M.factors]
        for n in range(N):
            Bh = M.factors[n] * M.lam
            got = host(P.phi(n, dev(Bh), A))
            assert_parity(got, oracle.phi(X, n, Bh, M.factors), tol, f"case {case} dims={dims} R={R} mode {n}")
        n = int(rng.integers(0, N))
        Bh = M.factors[n] * M.lam
        B = dev(Bh)
        P.mu_inner(n, B, A)
        Bo, _, _, _ = oracle.mu_inner(X, n, Bh, M.factors, lmax=3)
        assert_parity(host(B), Bo, tol, f"case {case} inner loop", elementwise=not mixed)
        P.close()


@pytest.mark.parametrize("dims,R,nnz,zipf", [
    ((100, 80, 60), 10, 10_000, None),
    ((300, 200, 50), 16, 30_001, (1.1, None, 1.2)),
    ((50, 60), 5, 4_000, (1.1, 1.1)),
    ((9, 8, 7, 6, 5), 33, 6_000, None),
    ((40, 30, 20), 8, 0, None),
])
def test_phi_coo_transient_matches_oracle(dims, R, nnz, zipf):
    """Phi of a COO tensor without a plan (the one mode sorted into a caller
    workspace): every mode against the oracle; an empty tensor gives Phi = 0."""
    import torch
    X = synth.random_tensor(61, dims, nnz, zipf=zipf or ())
    M = synth.random_model(61, dims, R)
    idx, vals = dev(X.idx), dev(X.vals)
    A = [dev(a) for a in M.factors]
    for n in range(len(dims)):
        Bh = M.factors[n] * M.lam
        out = torch.full((dims[n], R), 7.0, dtype=torch.float64, device="cuda")  # overwritten
        cpapr.phi_coo(X.dims, idx, vals, n, R, dev(Bh), A, out=out)
        assert_parity(host(out), oracle.phi(X, n, Bh, M.factors), TOL64, f"mode {n}")


def test_phi_coo_rejects_bad_input_and_workspace():
    import torch
    X = synth.random_tensor(62, (30, 20, 10), 500)
    M = synth.random_model(62, X.dims, 4)
    idx, vals = dev(X.idx), dev(X.vals)
    A = [dev(a) for a in M.factors]
    B = dev(M.factors[0] * M.lam)
    out = torch.empty((30, 4), dtype=torch.float64, device="cuda")
    coo = cpapr.make_coo(X.dims, idx, vals)
    need = cpapr.cpapr_phi_coo_workspace_size(coo, 0, 4)
    small = torch.empty(need - 256, dtype=torch.uint8, device="cuda")
    with pytest.raises(cpapr.CpaprError) as ei:
        cpapr.cpapr_phi_coo(coo, 0, 4, B, A, 1e-10, out, small)
    assert ei.value.code == cpapr.CPAPR_EWORKSPACE
    bad = X.idx.copy()
    bad[1, 17] = 20  # outside mode 1
    with pytest.raises(cpapr.CpaprError) as ei:
        cpapr.phi_coo(X.dims, dev(bad), vals, 0, 4, B, A, out=out)
    assert ei.value.code == cpapr.CPAPR_EINDEX
    with pytest.raises(cpapr.CpaprError) as ei:
        cpapr.phi_coo(X.dims, idx, vals, 3, 4, B, A, out=out)
    assert ei.value.code == cpapr.CPAPR_EINVAL


@pytest.mark.parametrize("dims,R", [((300, 200, 50), 8), ((300, 200, 50), 16), ((300, 200, 50), 30),
                                    ((60, 50), 16), ((40, 30, 20, 10), 10)])
def test_phi_xr_variant_matches_oracle(dims, R):
    """The reduce-scatter tile (CPAPR_VARIANT_XR) on the shapes it is built
    for (8 lanes x 1, 2 or 4 columns; N = 2..4), in both precisions."""
    X = synth.random_tensor(81, dims, 25_000, zipf=(1.1,) * len(dims))
    M = synth.random_model(81, dims, R)
    _phi_case(X, M, variant=cpapr.CPAPR_VARIANT_XR)
    _phi_case(X, M, variant=cpapr.CPAPR_VARIANT_XR, precision=cpapr.CPAPR_MIXED, tol=TOLMIX)
