"""The no-allocation transient Phi (cpapr_phi_coo_noalloc) through the C ABI
against the workspace entry point it varies (cpapr_phi_coo, the same sort and
Phi kernels): every mode of two tensors in a row, the second smaller, so the
second call reuses the static scratch the first one filled; its size limit is
refused before any device work."""
import ctypes as C

import numpy as np
import pytest

from paper_2307_03276_amd import cpapr, synth
from tests.gpu_util import assert_parity, dev, host

pytestmark = pytest.mark.gpu


def _noalloc(X, n, R, B, A):
    import torch
    idx, vals = dev(X.idx), dev(X.vals)
    coo = cpapr.make_coo(X.dims, idx, vals)
    out = torch.full((X.dims[n], R), np.nan, dtype=torch.float64, device="cuda")
    cpapr.cpapr_phi_coo_noalloc(coo, n, R, B, A, 1e-10, out)
    return host(out)


def test_noalloc_matches_workspace_entry_point():
    import torch
    assert torch.cuda.is_available()
    cases = [((400, 300, 200), 200_000, 16, (1.1, 1.1, None)), ((90, 80, 70), 30_000, 10, (None, 1.2, None))]
    for seed, (dims, nnz, R, zipf) in enumerate(cases):
        X = synth.random_tensor(70 + seed, dims, nnz, zipf=zipf)
        M = synth.random_model(70 + seed, dims, R)
        A = [dev(a) for a in M.factors]
        idx, vals = dev(X.idx), dev(X.vals)
        for n in range(len(dims)):
            B = dev(M.factors[n] * M.lam)
            ref = host(cpapr.phi_coo(X.dims, idx, vals, n, R, B, A))
            got = _noalloc(X, n, R, B, A)
            assert_parity(got, ref, 1e-12, f"tensor {seed} mode {n}")


def test_noalloc_refuses_oversize_tensor():
    d = (C.c_int64 * 3)(4000, 3000, 2000)
    coo = cpapr.cpapr_coo(3, C.cast(d, C.POINTER(C.c_int64)), 20_000_000, 1, 1)  # never dereferenced
    n = C.c_size_t(0)
    assert cpapr.load().cpapr_phi_coo_workspace_size(C.byref(coo), 0, 8, C.byref(n)) == 0
    assert n.value > cpapr.NOALLOC_SCRATCH_BYTES
    rc = cpapr.load().cpapr_phi_coo_noalloc(C.byref(coo), 0, 8, 1, None, 1e-10, 1, None)
    assert rc == cpapr.CPAPR_EUNSUPPORTED
    assert b"scratch" in cpapr.load().cpapr_last_error()
