"""CPU-side checks of the C ABI: the library loads, exports every function that
include/cpapr.h declares, and rejects bad arguments on the host before any
device work (no compute calls are made here)."""
import ctypes as C
import os
import re

import pytest

from paper_2307_03276_amd import cpapr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "cpapr.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cpapr_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(cpapr.LIB_PATH):
        from paper_2307_03276_amd import build
        build.build()
    return cpapr.load()


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert "cpapr_phi" in names and "cpapr_mu_inner" in names and "cpapr_solve" in names
    for n in names:
        assert hasattr(lib, n), f"{n} declared in cpapr.h but not exported"
    assert set(names) == set(cpapr.EXPORTED)


def test_params_default(lib):
    p = cpapr.cpapr_params_default()
    assert (p.kmax, p.lmax, p.tol, p.eps, p.kappa, p.kappa_tol) == (10, 10, 1e-4, 1e-10, 0.01, 1e-10)
    assert p.precision == cpapr.CPAPR_FP64 and p.variant == 0 and p.group == 0 and p.chunk == 0
    assert p.sort == cpapr.CPAPR_SORT_ROW_COL and p.method == cpapr.CPAPR_METHOD_MU and p.deterministic == 0


def _coo(dims, nnz):
    d = (C.c_int64 * len(dims))(*dims)
    c = cpapr.cpapr_coo(len(dims), C.cast(d, C.POINTER(C.c_int64)), nnz, None, None)
    c._keep = d
    return c


def _size(coo, R, p):
    n = C.c_size_t(0)
    return cpapr.load().cpapr_plan_workspace_size(C.byref(coo), R, C.byref(p), C.byref(n)), n.value


def test_workspace_size_grows_with_problem(lib):
    p = cpapr.cpapr_params_default()
    rc, a = _size(_coo([100, 80, 60], 10_000), 10, p)
    assert rc == 0 and a > 0
    rc, b = _size(_coo([100, 80, 60], 20_000), 10, p)
    assert rc == 0 and b > a
    # three sorted copies of (3 x int32 + fp64) per nonzero at least
    assert b >= 3 * 20_000 * (3 * 4 + 8)
    pm = cpapr.cpapr_params_default(precision=cpapr.CPAPR_MIXED)
    rc, c = _size(_coo([100, 80, 60], 20_000), 10, pm)
    assert rc == 0 and c > b  # FP32 factor copies


@pytest.mark.parametrize("dims,nnz,R,field,val,code", [
    ([100], 10, 4, None, None, -1),                       # one mode
    ([5] * 9, 10, 4, None, None, -1),                     # nine modes
    ([0, 4, 5], 10, 4, None, None, -6),                   # empty mode
    ([4, 5, 6], -1, 4, None, None, -1),                   # negative nnz
    ([4, 5, 6], 2 ** 31, 4, None, None, -6),              # nnz too large
    ([4, 5, 6], 10, 0, None, None, -6),                   # rank 0
    ([4, 5, 6], 10, 257, None, None, -6),                 # rank too large
    ([4, 5, 6], 10, 4, "lmax", 0, -1),
    ([4, 5, 6], 10, 4, "lmax", 5000, -1),
    ([4, 5, 6], 10, 4, "kmax", 0, -1),
    ([4, 5, 6], 10, 4, "eps", 0.0, -1),
    ([4, 5, 6], 10, 4, "precision", 7, -1),
    ([4, 5, 6], 10, 4, "group", 12, -1),
    ([4, 5, 6], 10, 40, "group", 8, -6),                  # R > 4 * group
    ([4, 5, 6], 10, 4, "variant", 9, -1),
    ([4, 5, 6], 10, 4, "sort", 5, -1),
    ([4, 5, 6], 10, 4, "method", 7, -1),
    ([4, 5, 6], 10, 4, "deterministic", 2, -1),
    ([2 ** 27, 5, 6], 10, 64, None, None, -6),          # I x R reaches 2^32 (32-bit row offsets)
    ([2 ** 26, 5, 6], 10, 63, None, None, 0),           # just below
    ([4, 5, 6, 7, 8], 10, 32, "group", 16, 0),           # N = 5: 16 lanes x 2 ranks is built
    ([4, 5, 6, 7, 8], 10, 64, "group", 16, -6),          # N = 5: 16 lanes x 4 ranks is not
])
def test_workspace_size_rejects(lib, dims, nnz, R, field, val, code):
    p = cpapr.cpapr_params_default()
    if field:
        setattr(p, field, val)
    rc, _ = _size(_coo(dims, nnz), R, p)
    assert rc == code
    if code:
        assert cpapr.cpapr_last_error()


def test_deterministic_params(lib):
    coo = _coo([100, 80, 60], 10_000)
    p = cpapr.cpapr_params_default(deterministic=1)
    rc, a = _size(coo, 16, p)
    rc0, b = _size(coo, 16, cpapr.cpapr_params_default())
    assert rc == 0 and rc0 == 0 and a >= b
    rc, _ = _size(coo, 16, cpapr.cpapr_params_default(deterministic=1, variant=2))
    assert rc == -6  # the atomic variant cannot be deterministic


def test_pqnr_params(lib):
    """PQNR needs FP64; its plans carry the row-solve state in the workspace."""
    coo = _coo([100, 80, 60], 10_000)
    mu = cpapr.cpapr_params_default()
    pq = cpapr.cpapr_params_default(method=cpapr.CPAPR_METHOD_PQNR)
    rc, a = _size(coo, 16, mu)
    rc2, b = _size(coo, 16, pq)
    assert rc == 0 and rc2 == 0 and b >= a
    pm = cpapr.cpapr_params_default(method=cpapr.CPAPR_METHOD_PQNR, precision=cpapr.CPAPR_MIXED)
    rc, _ = _size(coo, 16, pm)
    assert rc == -6


def test_pdnr_params(lib):
    """PDNR needs FP64, R <= 64 and atomics; its workspace holds an R x R
    Hessian and the Phi row per row of the largest mode (exactly that growth
    over PQNR's single-matrix buffers, up to alignment)."""
    dims = [5000, 80, 60]
    coo = _coo(dims, 10_000)
    mu = cpapr.cpapr_params_default()
    pd = cpapr.cpapr_params_default(method=cpapr.CPAPR_METHOD_PDNR)
    for R in (1, 16, 33, 64):
        rc, a = _size(coo, R, mu)
        rc2, b = _size(coo, R, pd)
        assert rc == 0 and rc2 == 0 and b >= a
        hess = max(dims) * (R * R + R) * 8
        if R >= 16:  # below that the plan's sort scratch, shared with this region, dominates
            assert hess <= b - a <= hess + max(dims) * (4 * R * 8 + 7 * 8) + 16 * 256
    for bad in (dict(precision=cpapr.CPAPR_MIXED), dict(deterministic=1)):
        rc, _ = _size(coo, 16, cpapr.cpapr_params_default(method=cpapr.CPAPR_METHOD_PDNR, **bad))
        assert rc == -6
    rc, _ = _size(coo, 65, pd)
    assert rc == -6
    rc, _ = _size(coo, 16, cpapr.cpapr_params_default(method=3))
    assert rc == -1


def test_plan_create_host_checks(lib):
    p = cpapr.cpapr_params_default()
    coo = _coo([4, 5, 6], 10)
    h = C.c_void_p()
    # idx / vals NULL with nnz > 0
    assert lib.cpapr_plan_create(C.byref(coo), 4, C.byref(p), None, 0, None, C.byref(h)) == -1
    coo0 = _coo([4, 5, 6], 0)
    assert lib.cpapr_plan_create(C.byref(coo0), 4, C.byref(p), None, 0, None, C.byref(h)) == -4
    assert lib.cpapr_plan_create(C.byref(coo0), 4, C.byref(p), 0x1001, 1 << 20, None, C.byref(h)) == -4
    assert lib.cpapr_plan_create(C.byref(coo0), 4, C.byref(p), 0x1000, 16, None, C.byref(h)) == -4
    assert "small" in cpapr.cpapr_last_error()


def test_calls_reject_null_plan(lib):
    arr = (C.c_void_p * 3)()
    assert lib.cpapr_phi(None, 0, None, arr, 1e-10, None, None) == -1
    assert lib.cpapr_mu_inner(None, 0, None, arr, None, None, None) == -1
    assert lib.cpapr_pqnr_inner(None, 0, None, arr, None, None) == -1
    assert lib.cpapr_solve(None, None, arr, None, None) == -1
    assert lib.cpapr_loglik(None, None, arr, 1e-10, None, None) == -1
    assert lib.cpapr_mttkrp(None, 0, arr, None, None) == -1
    assert lib.cpapr_plan_segments(None, 0) == -1
    g = C.c_int32(0)
    assert lib.cpapr_plan_shape(None, C.byref(g), C.byref(g)) == -1
    assert lib.cpapr_plan_batch_shape(None, C.byref(g), C.byref(g)) == -1
    # batched mode steps: no items is a no-op; a NULL plan or array is refused before any launch
    assert lib.cpapr_modes_advance(0, None, None, None, None, None, None, None, None, None) == 0
    assert lib.cpapr_modes_advance(-1, None, None, None, None, None, None, None, None, None) == -1
    one = (C.c_void_p * 1)()
    i1 = (C.c_int32 * 1)(0)
    assert lib.cpapr_modes_advance(1, one, i1, i1, i1, one, one, one, None, None) == -1
    assert lib.cpapr_modes_advance(1, None, i1, i1, i1, one, one, one, None, None) == -1


def test_prof_rejects_bad_arguments(lib):
    """Kernel-timing switches: capacity outside [1, 2^20] and a sampling
    stride below 1 are refused before any event is made."""
    assert lib.cpapr_prof_enable(0) == -1
    assert lib.cpapr_prof_enable_sampled(0, 1) == -1
    assert lib.cpapr_prof_enable_sampled(16, 0) == -1
    assert lib.cpapr_prof_enable_sampled(16, -3) == -1
    assert lib.cpapr_prof_disable() == 0


def test_phi_coo_workspace_size(lib):
    """Transient Phi's workspace: one mode's sorted copy plus its sort's
    scratch; grows with nnz; rejects a bad mode or rank (host checks only)."""
    import ctypes as C
    def size(dims, nnz, mode, R):
        d = (C.c_int64 * len(dims))(*dims)
        coo = cpapr.cpapr_coo(len(dims), C.cast(d, C.POINTER(C.c_int64)), nnz, None, None)
        n = C.c_size_t(0)
        rc = lib.cpapr_phi_coo_workspace_size(C.byref(coo), mode, R, C.byref(n))
        return rc, n.value
    rc1, a = size([40, 30, 20], 1000, 0, 8)
    rc2, b = size([40, 30, 20], 100_000, 0, 8)
    assert rc1 == rc2 == 0 and 0 < a < b
    assert b >= 100_000 * (4 + 8 + 8)  # at least the sorted copy of one mode
    assert size([40, 30, 20], 1000, 3, 8)[0] == cpapr.CPAPR_EINVAL
    assert size([40, 30, 20], 1000, -1, 8)[0] == cpapr.CPAPR_EINVAL
    assert size([40, 30, 20], 1000, 0, 0)[0] == cpapr.CPAPR_EUNSUPPORTED
