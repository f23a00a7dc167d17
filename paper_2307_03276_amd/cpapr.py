"""Python binding of libcpapr (include/cpapr.h): ctypes marshalling only.

Functions carry the C names (``cpapr_phi``, ``cpapr_mu_inner``, ``cpapr_solve``,
...). Device buffers are ``torch.Tensor`` on the GPU (their ``data_ptr`` is
passed); PyTorch supplies device memory and the current stream, every step of
the computation runs in the library's HIP kernels. There is no CPU fallback:
if the library is not built, or no GPU is present, calls raise.

:class:`Plan` owns a plan and its workspace tensor and offers the same calls
as methods.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from typing import Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcpapr.so")

CPAPR_FP64 = 0
CPAPR_MIXED = 1
CPAPR_VARIANT_AUTO = 0
CPAPR_VARIANT_SEGMENTED = 1
CPAPR_VARIANT_ATOMIC = 2
CPAPR_VARIANT_XR = 3
CPAPR_SORT_ROW = 0
CPAPR_SORT_ROW_COL = 1
CPAPR_METHOD_MU = 0
CPAPR_METHOD_PQNR = 1
CPAPR_METHOD_PDNR = 2
MAX_MODES = 8
CPAPR_OK = 0
CPAPR_EINVAL = -1
CPAPR_EINDEX = -2
CPAPR_EVALUE = -3
CPAPR_EWORKSPACE = -4
CPAPR_EHIP = -5
CPAPR_EUNSUPPORTED = -6


class CpaprError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"cpapr error {code}: {msg}")
        self.code = code


class cpapr_coo(C.Structure):
    _fields_ = [("nmodes", C.c_int32), ("dims", C.POINTER(C.c_int64)), ("nnz", C.c_int64),
                ("idx", C.c_void_p), ("vals", C.c_void_p)]


class cpapr_params(C.Structure):
    _fields_ = [("kmax", C.c_int32), ("lmax", C.c_int32), ("tol", C.c_double), ("eps", C.c_double),
                ("kappa", C.c_double), ("kappa_tol", C.c_double), ("precision", C.c_int32),
                ("variant", C.c_int32), ("group", C.c_int32), ("chunk", C.c_int32), ("sort", C.c_int32),
                ("method", C.c_int32), ("deterministic", C.c_int32)]


class cpapr_stats(C.Structure):
    _fields_ = [("outer_iters", C.c_int32), ("converged", C.c_int32), ("inner_iters", C.c_int64),
                ("kkt_violation", C.c_double), ("loglik", C.c_double), ("phi_evals", C.c_int64),
                ("row_steps", C.c_int64), ("trial_evals", C.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None


def load():
    """Load libcpapr.so; raises if it is missing (no fallback path exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_2307_03276_amd.build`")
    lib = C.CDLL(LIB_PATH)
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    P = C.POINTER
    sig = {
        "cpapr_params_default": (None, [P(cpapr_params)]),
        "cpapr_plan_workspace_size": (C.c_int, [P(cpapr_coo), i32, P(cpapr_params), P(C.c_size_t)]),
        "cpapr_plan_create": (C.c_int, [P(cpapr_coo), i32, P(cpapr_params), vp, C.c_size_t, vp, P(vp)]),
        "cpapr_plan_destroy": (C.c_int, [vp]),
        "cpapr_plan_segments": (i64, [vp, i32]),
        "cpapr_plan_set_shape": (C.c_int, [vp, i32, i32]),
        "cpapr_plan_shape": (C.c_int, [vp, P(i32), P(i32)]),
        "cpapr_plan_batch_shape": (C.c_int, [vp, P(i32), P(i32)]),
        "cpapr_phi": (C.c_int, [vp, i32, vp, P(vp), dbl, vp, vp]),
        "cpapr_phi_coo_workspace_size": (C.c_int, [P(cpapr_coo), i32, i32, P(C.c_size_t)]),
        "cpapr_phi_coo": (C.c_int, [P(cpapr_coo), i32, i32, vp, P(vp), dbl, vp, vp, C.c_size_t, vp]),
        "cpapr_phi_coo_noalloc": (C.c_int, [P(cpapr_coo), i32, i32, vp, P(vp), dbl, vp, vp]),
        "cpapr_mu_inner": (C.c_int, [vp, i32, vp, P(vp), vp, P(cpapr_stats), vp]),
        "cpapr_pqnr_inner": (C.c_int, [vp, i32, vp, P(vp), P(cpapr_stats), vp]),
        "cpapr_pdnr_inner": (C.c_int, [vp, i32, vp, P(vp), P(cpapr_stats), vp]),
        "cpapr_row_stats": (C.c_int, [vp, i32, vp, vp, vp]),
        "cpapr_solve": (C.c_int, [vp, vp, P(vp), P(cpapr_stats), vp]),
        "cpapr_loglik": (C.c_int, [vp, vp, P(vp), dbl, P(dbl), vp]),
        "cpapr_mttkrp": (C.c_int, [vp, i32, P(vp), vp, vp]),
        "cpapr_batch_workspace_size": (C.c_int, [i32, i64, P(C.c_size_t)]),
        "cpapr_batch_tiles": (i64, [vp]),
        "cpapr_batch_create": (C.c_int, [i32, i64, vp, C.c_size_t, P(vp)]),
        "cpapr_batch_create2": (C.c_int, [i32, i64, i32, vp, C.c_size_t, P(vp)]),
        "cpapr_batch_destroy": (C.c_int, [vp]),
        "cpapr_batch_set": (C.c_int, [vp, i32, vp, i32, vp, P(vp), vp, i32]),
        "cpapr_batch_mu": (C.c_int, [vp, vp]),
        "cpapr_batch_status": (C.c_int, [vp, P(dbl), P(i32), P(i32), vp]),
        "cpapr_batch_inner": (C.c_int, [vp, i32, i32, vp]),
        "cpapr_batch_hold": (C.c_int, [vp, P(i32), vp]),
        "cpapr_mode_begin": (C.c_int, [vp, i32, i32, vp, vp, vp, vp, vp]),
        "cpapr_mode_end": (C.c_int, [vp, i32, vp, vp, vp, vp]),
        "cpapr_modes_advance": (C.c_int, [i32, P(vp), P(i32), P(i32), P(i32), P(vp), P(vp), P(vp), P(vp), vp]),
        "cpapr_plan_sync_f32": (C.c_int, [vp, P(vp), vp]),
        "cpapr_batch_clear": (C.c_int, [vp, i32]),
        "cpapr_batch_commit": (C.c_int, [vp, vp]),
        "cpapr_batch_run": (C.c_int, [vp, i32, vp]),
        "cpapr_prof_enable": (C.c_int, [i32]),
        "cpapr_prof_enable_sampled": (C.c_int, [i32, i32]),
        "cpapr_prof_disable": (C.c_int, []),
        "cpapr_prof_read": (C.c_int, [P(i32), P(C.c_float), i32]),
        "cpapr_last_error": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


EXPORTED = ("cpapr_params_default", "cpapr_plan_workspace_size", "cpapr_plan_create", "cpapr_plan_destroy",
            "cpapr_plan_segments", "cpapr_plan_set_shape", "cpapr_plan_shape",
            "cpapr_plan_batch_shape", "cpapr_phi", "cpapr_phi_coo_workspace_size",
            "cpapr_phi_coo", "cpapr_phi_coo_noalloc", "cpapr_mu_inner", "cpapr_pqnr_inner",
            "cpapr_pdnr_inner", "cpapr_row_stats", "cpapr_solve", "cpapr_loglik",
            "cpapr_mttkrp", "cpapr_batch_workspace_size", "cpapr_batch_tiles", "cpapr_batch_create", "cpapr_batch_create2",
            "cpapr_batch_destroy", "cpapr_batch_set", "cpapr_batch_clear", "cpapr_batch_commit", "cpapr_batch_run",
            "cpapr_batch_mu", "cpapr_batch_inner", "cpapr_batch_hold", "cpapr_batch_status", "cpapr_mode_begin", "cpapr_mode_end", "cpapr_modes_advance", "cpapr_plan_sync_f32",
            "cpapr_prof_enable", "cpapr_prof_enable_sampled", "cpapr_prof_disable", "cpapr_prof_read",
            "cpapr_last_error")


def _check(rc: int):
    if rc < 0:
        raise CpaprError(rc, load().cpapr_last_error().decode())
    return rc


def _stream(stream=None) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _ptr_array(tensors: Sequence) -> C.Array:
    arr = (C.c_void_p * len(tensors))()
    for i, t in enumerate(tensors):
        arr[i] = None if t is None else t.data_ptr()
    return arr


def _need_cuda(t, name, dtype=None):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA/HIP tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must have dtype {dtype}")


def cpapr_params_default(**overrides) -> cpapr_params:
    p = cpapr_params()
    load().cpapr_params_default(C.byref(p))
    for k, v in overrides.items():
        setattr(p, k, v)
    return p


def make_coo(dims: Sequence[int], idx, vals):
    """COO descriptor for device tensors idx (int32 [N, nnz]) and vals (float64 [nnz])."""
    import torch
    _need_cuda(idx, "idx", torch.int32)
    _need_cuda(vals, "vals", torch.float64)
    d = (C.c_int64 * len(dims))(*[int(x) for x in dims])
    coo = cpapr_coo(len(dims), C.cast(d, C.POINTER(C.c_int64)), int(vals.shape[0]), idx.data_ptr(),
                    vals.data_ptr())
    coo._keep = (d, idx, vals)
    return coo


def cpapr_plan_workspace_size(coo: cpapr_coo, R: int, params: cpapr_params) -> int:
    n = C.c_size_t(0)
    _check(load().cpapr_plan_workspace_size(C.byref(coo), R, C.byref(params), C.byref(n)))
    return n.value


def cpapr_plan_create(coo, R, params, ws, stream=None):
    h = C.c_void_p()
    _check(load().cpapr_plan_create(C.byref(coo), R, C.byref(params), ws.data_ptr(), ws.numel() * ws.element_size(),
                                    _stream(stream), C.byref(h)))
    return h


def cpapr_plan_destroy(h):
    return _check(load().cpapr_plan_destroy(h))


def cpapr_plan_set_shape(h, group: int, chunk: int):
    return _check(load().cpapr_plan_set_shape(h, group, chunk))


def cpapr_plan_shape(h):
    g, c = C.c_int32(0), C.c_int32(0)
    _check(load().cpapr_plan_shape(h, C.byref(g), C.byref(c)))
    return g.value, c.value


def cpapr_plan_batch_shape(h):
    g, c = C.c_int32(0), C.c_int32(0)
    _check(load().cpapr_plan_batch_shape(h, C.byref(g), C.byref(c)))
    return g.value, c.value


def cpapr_plan_segments(h, mode: int) -> int:
    return int(load().cpapr_plan_segments(h, mode))


def cpapr_phi(h, mode, B, A, eps, Phi, stream=None):
    return _check(load().cpapr_phi(h, mode, B.data_ptr(), _ptr_array(A), eps, Phi.data_ptr(), _stream(stream)))


def cpapr_phi_coo_workspace_size(coo: cpapr_coo, mode: int, R: int) -> int:
    n = C.c_size_t(0)
    _check(load().cpapr_phi_coo_workspace_size(C.byref(coo), mode, R, C.byref(n)))
    return int(n.value)


def cpapr_phi_coo(coo, mode, R, B, A, eps, Phi, ws, stream=None):
    """Transient Phi of a COO tensor (no plan); ws: a device uint8 tensor of at least the queried size."""
    import torch
    _need_cuda(B, "B", torch.float64)
    _need_cuda(Phi, "Phi", torch.float64)
    _need_cuda(ws, "ws")
    _check(load().cpapr_phi_coo(C.byref(coo), mode, R, B.data_ptr(), _ptr_array(A), eps, Phi.data_ptr(),
                                ws.data_ptr(), ws.numel() * ws.element_size(), _stream(stream)))


NOALLOC_SCRATCH_BYTES = 128 << 20


def cpapr_phi_coo_noalloc(coo, mode, R, B, A, eps, Phi, stream=None):
    """Transient Phi with the library's static device scratch (no workspace, no allocation)."""
    import torch
    _need_cuda(B, "B", torch.float64)
    _need_cuda(Phi, "Phi", torch.float64)
    _check(load().cpapr_phi_coo_noalloc(C.byref(coo), mode, R, B.data_ptr(), _ptr_array(A), eps, Phi.data_ptr(),
                                        _stream(stream)))


def phi_coo(dims, idx, vals, mode, R, B, A, eps=1e-10, out=None, stream=None):
    """Transient Phi(mode) of device COO arrays (idx int32 [N, nnz], vals float64 [nnz])."""
    import torch
    coo = make_coo(dims, idx, vals)
    nbytes = cpapr_phi_coo_workspace_size(coo, mode, R)
    ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=B.device)
    if out is None:
        out = torch.empty((int(dims[mode]), R), dtype=torch.float64, device=B.device)
    cpapr_phi_coo(coo, mode, R, B, A, eps, out, ws, stream)
    return out


def cpapr_mu_inner(h, mode, B, A, Phi_last, stream=None) -> dict:
    st = cpapr_stats()
    _check(load().cpapr_mu_inner(h, mode, B.data_ptr(), _ptr_array(A), Phi_last.data_ptr(), C.byref(st),
                                 _stream(stream)))
    return st.as_dict()


def cpapr_pqnr_inner(h, mode, B, A, stream=None) -> dict:
    st = cpapr_stats()
    _check(load().cpapr_pqnr_inner(h, mode, B.data_ptr(), _ptr_array(A), C.byref(st), _stream(stream)))
    return st.as_dict()


def cpapr_pdnr_inner(h, mode, B, A, stream=None) -> dict:
    st = cpapr_stats()
    _check(load().cpapr_pdnr_inner(h, mode, B.data_ptr(), _ptr_array(A), C.byref(st), _stream(stream)))
    return st.as_dict()


def cpapr_row_stats(h, mode, steps, viol, stream=None):
    """Per-row steps (int32) and last KKT violation (float64) of the last row-solve call, into device tensors."""
    if steps is not None:
        _need_cuda(steps, "steps")
    if viol is not None:
        _need_cuda(viol, "viol")
    _check(load().cpapr_row_stats(h, mode, steps.data_ptr() if steps is not None else None,
                                  viol.data_ptr() if viol is not None else None, _stream(stream)))


def cpapr_solve(h, lam, A, stream=None) -> dict:
    st = cpapr_stats()
    _check(load().cpapr_solve(h, lam.data_ptr(), _ptr_array(A), C.byref(st), _stream(stream)))
    return st.as_dict()


def cpapr_loglik(h, lam, A, eps, stream=None) -> float:
    out = C.c_double(0)
    _check(load().cpapr_loglik(h, lam.data_ptr(), _ptr_array(A), eps, C.byref(out), _stream(stream)))
    return out.value


def cpapr_mttkrp(h, mode, A, M, stream=None):
    return _check(load().cpapr_mttkrp(h, mode, _ptr_array(A), M.data_ptr(), _stream(stream)))


def cpapr_batch_workspace_size(max_slots: int, max_tiles: int) -> int:
    n = C.c_size_t(0)
    _check(load().cpapr_batch_workspace_size(max_slots, max_tiles, C.byref(n)))
    return n.value


def cpapr_batch_tiles(plan_handle) -> int:
    return int(load().cpapr_batch_tiles(plan_handle))


CPAPR_BATCH_PERSISTENT = 1
CPAPR_BATCH_SKIP_HELD = 2


def cpapr_batch_create(max_slots, max_tiles, ws, flags=0):
    h = C.c_void_p()
    _check(load().cpapr_batch_create2(max_slots, max_tiles, flags, ws.data_ptr(), ws.numel() * ws.element_size(),
                                      C.byref(h)))
    return h


def cpapr_batch_destroy(h):
    return _check(load().cpapr_batch_destroy(h))


CPAPR_BATCH_F32_CURRENT = 1


def cpapr_batch_set(h, slot, plan_handle, mode, B, A, Phi, flags=0):
    return _check(load().cpapr_batch_set(h, slot, plan_handle, mode, B.data_ptr(), _ptr_array(A), Phi.data_ptr(),
                                         flags))


def cpapr_batch_mu(h, stream=None):
    return _check(load().cpapr_batch_mu(h, _stream(stream)))


def cpapr_batch_inner(h, lmax, use_graph=False, stream=None):
    return _check(load().cpapr_batch_inner(h, lmax, 1 if use_graph else 0, _stream(stream)))


def cpapr_batch_hold(h, hold, stream=None):
    """Hold flags (sequence of max_slots ints, nonzero = hold) for the following runs."""
    arr = (C.c_int32 * len(hold))(*[int(bool(x)) for x in hold])
    _check(load().cpapr_batch_hold(h, arr, _stream(stream)))


def cpapr_batch_status(h, max_slots, stream=None):
    viol = (C.c_double * max_slots)()
    upd = (C.c_int32 * max_slots)()
    done = (C.c_int32 * max_slots)()
    _check(load().cpapr_batch_status(h, viol, upd, done, _stream(stream)))
    return list(viol), list(upd), list(done)


def cpapr_mode_begin(h, mode, outer_iter, lam, A_mode, phi_prev, B, stream=None):
    return _check(load().cpapr_mode_begin(h, mode, outer_iter, lam.data_ptr(), A_mode.data_ptr(),
                                          None if phi_prev is None else phi_prev.data_ptr(), B.data_ptr(),
                                          _stream(stream)))


def cpapr_mode_end(h, mode, B, lam, A_mode, stream=None):
    return _check(load().cpapr_mode_end(h, mode, B.data_ptr(), lam.data_ptr(), A_mode.data_ptr(), _stream(stream)))


def cpapr_modes_advance(items, stream=None):
    """Mode steps of many solves in one call. items: sequence of (plan handle,
    end mode or -1, begin mode or -1, outer iteration, lambda device pointer,
    ctypes array of the plan's factor device pointers, B device pointer,
    previous-Phi device pointer or None), all plain integers / ctypes arrays
    (pointers are taken once per solve, not per call)."""
    n = len(items)
    if n == 0:
        return 0
    plans = (C.c_void_p * n)(*[it[0] for it in items])
    ends = (C.c_int32 * n)(*[it[1] for it in items])
    begins = (C.c_int32 * n)(*[it[2] for it in items])
    outer = (C.c_int32 * n)(*[it[3] for it in items])
    lam = (C.c_void_p * n)(*[it[4] for it in items])
    fac = (C.c_void_p * n)(*[C.cast(it[5], C.c_void_p) for it in items])
    B = (C.c_void_p * n)(*[it[6] for it in items])
    prev = (C.c_void_p * n)(*[it[7] for it in items])
    return _check(load().cpapr_modes_advance(n, plans, ends, begins, outer, lam, fac, B, prev, _stream(stream)))


def cpapr_plan_sync_f32(h, A, stream=None):
    return _check(load().cpapr_plan_sync_f32(h, _ptr_array(A), _stream(stream)))


def cpapr_batch_clear(h, slot):
    return _check(load().cpapr_batch_clear(h, slot))


def cpapr_batch_commit(h, stream=None):
    return _check(load().cpapr_batch_commit(h, _stream(stream)))


def cpapr_batch_run(h, use_graph=False, stream=None):
    return _check(load().cpapr_batch_run(h, 1 if use_graph else 0, _stream(stream)))


class Batch:
    """Slots of Phi work items run in persistent launches (optionally as a hipGraph)."""

    def __init__(self, max_slots: int, max_tiles: int, device="cuda", persistent: bool = False,
                 skip_held: bool = False):
        import torch
        self.max_slots, self.max_tiles = int(max_slots), int(max_tiles)
        nbytes = cpapr_batch_workspace_size(self.max_slots, self.max_tiles)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.handle = cpapr_batch_create(self.max_slots, self.max_tiles, self.ws,
                                         (CPAPR_BATCH_PERSISTENT if persistent else 0) |
                                         (CPAPR_BATCH_SKIP_HELD if skip_held else 0))
        self._keep = {}

    def set(self, slot, plan, mode, B, A, Phi, flags=0):
        cpapr_batch_set(self.handle, slot, plan.handle, mode, B, A, Phi, flags)
        self._keep[slot] = (plan, B, list(A), Phi)

    def clear(self, slot):
        cpapr_batch_clear(self.handle, slot)
        self._keep.pop(slot, None)

    def commit(self, stream=None):
        cpapr_batch_commit(self.handle, stream)

    def run(self, use_graph=False, stream=None):
        cpapr_batch_run(self.handle, use_graph, stream)

    def mu(self, stream=None):
        cpapr_batch_mu(self.handle, stream)

    def inner(self, lmax, use_graph=False, stream=None):
        cpapr_batch_inner(self.handle, lmax, use_graph, stream)

    def hold(self, flags, stream=None):
        cpapr_batch_hold(self.handle, list(flags), stream)

    def status(self, stream=None):
        return cpapr_batch_status(self.handle, self.max_slots, stream)

    def close(self):
        if getattr(self, "handle", None) is not None:
            cpapr_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def cpapr_prof_enable(capacity: int):
    return _check(load().cpapr_prof_enable(capacity))


def cpapr_prof_enable_sampled(capacity: int, every: int):
    return _check(load().cpapr_prof_enable_sampled(capacity, every))


def cpapr_prof_disable():
    return _check(load().cpapr_prof_disable())


def cpapr_prof_read(cap: int = 1 << 16):
    modes = (C.c_int32 * cap)()
    ms = (C.c_float * cap)()
    n = _check(load().cpapr_prof_read(modes, ms, cap))
    return [(modes[i], ms[i]) for i in range(n)]


def cpapr_last_error() -> str:
    return load().cpapr_last_error().decode()


class Plan:
    """A plan for one tensor (device COO) at rank R, owning its workspace tensor."""

    def __init__(self, dims, idx, vals, R: int, params: Optional[cpapr_params] = None, stream=None, **kw):
        import torch
        self.dims = tuple(int(d) for d in dims)
        self.R = int(R)
        self.params = params if params is not None else cpapr_params_default(**kw)
        coo = make_coo(self.dims, idx, vals)
        self.nnz = int(vals.shape[0])
        nbytes = cpapr_plan_workspace_size(coo, self.R, self.params)
        self.ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=idx.device)
        self.handle = cpapr_plan_create(coo, self.R, self.params, self.ws, stream)

    @classmethod
    def from_tensor(cls, X, R, device="cuda", **kw):
        import torch
        idx = torch.from_numpy(X.idx).to(device)
        vals = torch.from_numpy(X.vals).to(device)
        return cls(X.dims, idx, vals, R, **kw)

    def set_shape(self, group, chunk):
        cpapr_plan_set_shape(self.handle, group, chunk)
        self.params.group, self.params.chunk = group, chunk

    def shape(self):
        """(lanes per nonzero, nonzeros per lane group per tile) of the Phi launch."""
        return cpapr_plan_shape(self.handle)

    def batch_shape(self):
        """(lanes per nonzero, nonzeros per lane group per tile) of this plan's slots in a batch."""
        return cpapr_plan_batch_shape(self.handle)

    def tiles(self):
        """Tiles one slot of this plan takes in a batch."""
        return cpapr_batch_tiles(self.handle)

    def segments(self, mode):
        return cpapr_plan_segments(self.handle, mode)

    def phi(self, mode, B, A, eps=None, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty((self.dims[mode], self.R), dtype=torch.float64, device=B.device)
        cpapr_phi(self.handle, mode, B, A, self.params.eps if eps is None else eps, out, stream)
        return out

    def mu_inner(self, mode, B, A, phi_last=None, stream=None):
        import torch
        if phi_last is None:
            phi_last = torch.empty((self.dims[mode], self.R), dtype=torch.float64, device=B.device)
        st = cpapr_mu_inner(self.handle, mode, B, A, phi_last, stream)
        return phi_last, st

    def pqnr_inner(self, mode, B, A, stream=None):
        """PQNR row solves of one mode (plan created with method=CPAPR_METHOD_PQNR); B in/out."""
        return cpapr_pqnr_inner(self.handle, mode, B, A, stream)

    def pdnr_inner(self, mode, B, A, stream=None):
        """PDNR row solves of one mode (plan created with method=CPAPR_METHOD_PDNR); B in/out."""
        return cpapr_pdnr_inner(self.handle, mode, B, A, stream)

    def row_stats(self, mode, stream=None):
        """(steps, viol) per row of `mode` after its last row-solve call, as host arrays."""
        import torch
        steps = torch.empty(self.dims[mode], dtype=torch.int32, device="cuda")
        viol = torch.empty(self.dims[mode], dtype=torch.float64, device="cuda")
        cpapr_row_stats(self.handle, mode, steps, viol, stream)
        torch.cuda.current_stream().synchronize() if stream is None else stream.synchronize()
        return steps.cpu().numpy(), viol.cpu().numpy()

    def solve(self, lam, A, stream=None):
        return cpapr_solve(self.handle, lam, A, stream)

    def loglik(self, lam, A, eps=None, stream=None):
        return cpapr_loglik(self.handle, lam, A, self.params.eps if eps is None else eps, stream)

    def mttkrp(self, mode, A, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty((self.dims[mode], self.R), dtype=torch.float64, device=A[0].device)
        cpapr_mttkrp(self.handle, mode, A, out, stream)
        return out

    def close(self):
        if getattr(self, "handle", None) is not None:
            cpapr_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
