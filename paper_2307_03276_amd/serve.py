"""Continuous-batching CP-APR MU solver service on one GPU.

Requests (a sparse count tensor, an initial model, a rank) arrive over time.
A request is admitted when a batch slot is free and its device footprint fits
the HBM budget (first come, first served); on admission its tensor is uploaded,
its plan built (per-mode device sort) and its model placed on the device. Every
tick runs the MU inner loop (Algorithm 1) of the current mode for *all* active requests
together: the whole inner loop of each request's current mode runs as one
device sequence (cpapr_batch_inner: l_max x {batched Phi, batched KKT + MU
update}, a request whose KKT test stops it doing no further work; optionally a
replayed hipGraph), followed by one status read-back. The host then advances
each request's (outer k, mode n) state exactly as Algorithm 1's loops do;
mode transitions run the per-mode prologue / epilogue kernels
(cpapr_mode_begin / cpapr_mode_end). A request retires when an outer sweep
makes no update (tol > 0) or after k_max sweeps; its memory returns to the
budget and queued requests are admitted.

Round policy: "all" admits first come, first served, whatever fits, and runs
every active request in every round. "srpt" (shortest remaining work first)
ranks the active and the queued requests together by remaining work (nonzeros
x mode rounds left) and runs the shortest until the round holds its cap of
nonzeros (at least one request). The cap follows the load: an eighth of the
nonzeros of all active and queued requests, clamped to [round_cap_min,
round_cap]. Under a light load small rounds let short requests finish without
sharing rounds with long ones; under a deep queue large rounds spread each
round's fixed costs (launches, the status read-back, the host's bookkeeping)
over more work. Queued requests are admitted (uploaded and
sorted) only when the ranking puts them in a round, and active ones outside it
are held (their slots do no work and their state stays as it is). Short
requests then finish without waiting for the long ones, or for the uploads of
requests that will not run soon, while the GPU still gets a full round of work.
A steady stream of short requests can hold a long one back indefinitely.

Each request's arithmetic is independent of the others in the batch (same
kernels, same per-plan tiling), so its result is the same alone and in the mix
up to the order of the few atomic additions at tile boundaries.
"""
from __future__ import annotations

import dataclasses
import time
from collections import deque
from typing import List, Optional

import numpy as np

from . import cpapr


@dataclasses.dataclass
class Request:
    id: int
    X: object  # synth.SparseTensor (host)
    M: object  # synth.Model (host), initial guess
    arrival: float = 0.0  # seconds from the start of the trace
    # filled by the server
    t_admit: Optional[float] = None
    t_done: Optional[float] = None
    # the final model, left in device memory (torch tensors) when the request
    # completes; results_to_host() turns them into host arrays
    result_lam: Optional[object] = None
    result_factors: Optional[List[object]] = None
    stats: dict = dataclasses.field(default_factory=dict)


class _Active:
    """Loop counters of an admitted request; `h` is the executor's handle."""

    def __init__(self, req: Request, slot: int, h, nbytes: int):
        self.req, self.slot, self.h = req, slot, h
        self.nbytes = nbytes
        self.N = len(req.X.dims)
        self.k, self.n = 1, 0
        self.any_update = False
        self.updates = 0
        self.last_viol = [0.0] * self.N
        self.dirty = True  # slot operands changed since the last commit


class GpuExecutor:
    """Device side of the service: plans, factors and one batch whose slots
    hold the active requests' current modes (the C ABI's batch calls)."""

    def __init__(self, params: dict, max_slots: int, max_tiles: int, use_graph: bool, stream, compute_loglik: bool,
                 skip_held: bool = False):
        import torch
        self.params = params
        # skip_held: held slots are left out of the launches, so the held set
        # changes the launch shapes; rounds then run as direct launches (a
        # captured graph would be re-captured whenever the set changes)
        self.commit_on_hold = skip_held
        self.use_graph = use_graph and not skip_held
        self.compute_loglik = compute_loglik
        self.stream = stream if stream is not None else torch.cuda.Stream()
        self.batch = cpapr.Batch(max_slots, max_tiles, skip_held=skip_held)
        self.flags = cpapr.CPAPR_BATCH_F32_CURRENT if params["precision"] == cpapr.CPAPR_MIXED else 0

    def footprint(self, req: Request) -> int:
        """Device bytes a request holds while active: plan workspace, factors,
        B, the last Phi of every mode and lambda (its upload buffers are freed
        once the plan is built)."""
        X, R = req.X, req.M.rank
        d = (cpapr.C.c_int64 * len(X.dims))(*X.dims)
        coo = cpapr.cpapr_coo(len(X.dims), cpapr.C.cast(d, cpapr.C.POINTER(cpapr.C.c_int64)), X.nnz, None, None)
        ws = cpapr.cpapr_plan_workspace_size(coo, R, cpapr.cpapr_params_default(**self.params))
        mats = sum(X.dims) * R * 8
        return int(ws + 2 * mats + max(X.dims) * R * 8 + R * 8)

    def admit(self, req: Request):
        """Upload the tensor, build its plan (device sort) and place the model."""
        import torch
        with torch.cuda.stream(self.stream):
            idx = torch.from_numpy(req.X.idx).to("cuda", non_blocking=False)
            vals = torch.from_numpy(req.X.vals).to("cuda", non_blocking=False)
            plan = cpapr.Plan(req.X.dims, idx, vals, req.M.rank, stream=self.stream, **self.params)
            del idx, vals
            h = dict(plan=plan, lam=torch.from_numpy(req.M.lam).to("cuda"),
                     A=[torch.from_numpy(a).to("cuda") for a in req.M.factors],
                     B=torch.empty((max(req.X.dims), req.M.rank), dtype=torch.float64, device="cuda"),
                     phi=[torch.zeros((d, req.M.rank), dtype=torch.float64, device="cuda") for d in req.X.dims])
            cpapr.cpapr_plan_sync_f32(plan.handle, h["A"], self.stream)
        # device pointers taken once per request, for the batched mode steps
        h["ptrs"] = dict(plan=plan.handle.value, lam=h["lam"].data_ptr(), A=cpapr._ptr_array(h["A"]),
                         B=h["B"].data_ptr(), phi=[p.data_ptr() for p in h["phi"]])
        return h

    def mode_begin(self, h, n: int, k: int):
        cpapr.cpapr_mode_begin(h["plan"].handle, n, k, h["lam"], h["A"][n], h["phi"][n] if k > 1 else None, h["B"],
                               self.stream)

    def set_slot(self, slot: int, h, n: int):
        self.batch.set(slot, h["plan"], n, h["B"], h["A"], h["phi"][n], self.flags)

    def clear_slot(self, slot: int):
        self.batch.clear(slot)

    def commit(self):
        self.batch.commit(self.stream)

    def hold(self, flags):
        """Per-slot hold flags for the following rounds (held slots do no work)."""
        self.batch.hold(flags, self.stream)

    def run_round(self, lmax: int):
        """The whole inner loop of every slot's mode; per-slot (viol, updates, done)."""
        self.batch.inner(lmax, use_graph=self.use_graph, stream=self.stream)
        return self.batch.status(self.stream)

    def mode_end(self, h, n: int):
        cpapr.cpapr_mode_end(h["plan"].handle, n, h["B"], h["lam"], h["A"][n], self.stream)

    def advance(self, items):
        """Mode steps of many requests in one call: items of (h, mode to end,
        mode to begin or None, outer iteration of the begun mode)."""
        rows = []
        for h, end, begin, k in items:
            p = h["ptrs"]
            rows.append((p["plan"], end, -1 if begin is None else begin, k, p["lam"], p["A"], p["B"],
                         p["phi"][begin] if begin is not None and k > 1 else None))
        cpapr.cpapr_modes_advance(rows, self.stream)

    def retire(self, h):
        """The final model (lambda and the factors, left in device memory for
        the caller) and its log-likelihood; frees the rest of the request's
        device memory (plan, B, the last Phi of every mode)."""
        ll = h["plan"].loglik(h["lam"], h["A"], stream=self.stream) if self.compute_loglik else None
        self.stream.synchronize()
        lam, facs = h["lam"], list(h["A"])
        h["plan"].close()
        h.clear()
        return lam, facs, ll


class Server:
    """Admission, slots and the per-request loop state of Algorithm 1 over an
    executor (the GPU executor by default)."""

    def __init__(self, budget_bytes: float = 200e9, max_slots: int = 64, max_tiles: int = 1 << 22,
                 kmax: int = 20, lmax: int = 10, tol: float = 1e-4, eps: float = 1e-10,
                 precision: int = cpapr.CPAPR_MIXED, use_graph: bool = True, stream=None,
                 compute_loglik: bool = True, executor=None, policy: str = "all", round_cap: float = 32e6,
                 round_cap_min: float = 4e6):
        self.budget = float(budget_bytes)
        self.used = 0.0
        self.max_slots = max_slots
        self.params = dict(kmax=kmax, lmax=lmax, tol=tol, eps=eps, precision=precision)
        self.ex = executor if executor is not None else GpuExecutor(self.params, max_slots, max_tiles, use_graph,
                                                                   stream, compute_loglik,
                                                                   skip_held=policy == "srpt")
        self.queue: deque = deque()
        self.active: List[_Active] = []
        self.free_slots = list(range(max_slots - 1, -1, -1))
        self.done: List[Request] = []
        self.ticks = 0
        self.t0 = time.perf_counter()
        self.peak_active = 0
        self.peak_used = 0.0
        self._need_commit = True
        if policy not in ("all", "srpt"):
            raise ValueError("policy must be 'all' or 'srpt'")
        self.policy = policy
        self.round_cap = float(round_cap)
        self.round_cap_min = min(float(round_cap_min), self.round_cap)
        self._held = None  # hold flags last sent to the executor
        # host seconds per phase of tick(): admission (upload + plan build),
        # batch commit, hold flags, the round (device time + status read-back),
        # advancing the loop state (mode epilogue / prologue), retirement
        # (log-likelihood and the result's copy to the host)
        self.phase_s = dict(admit=0.0, commit=0.0, hold=0.0, round=0.0, advance=0.0, retire=0.0)

    # ------------------------------------------------------------------ admission
    def footprint(self, req: Request) -> int:
        return self.ex.footprint(req)

    def submit(self, req: Request):
        req.stats["t_submit"] = time.perf_counter() - self.t0
        self.queue.append(req)

    def _admit(self):
        while self.queue and self.free_slots:
            req = self.queue[0]
            if not self._admit_one(req):
                break  # first come, first served: wait for memory

    def _admit_one(self, req: Request) -> bool:
        """Admit a queued request if a slot is free and it fits the budget
        (rejecting it for good when it exceeds the whole budget). Returns
        whether it left the queue."""
        need = self.footprint(req)
        if need > self.budget:
            self.queue.remove(req)
            req.stats["rejected"] = "larger than the HBM budget"
            req.t_done = time.perf_counter() - self.t0
            self.done.append(req)
            return True
        if not self.free_slots or self.used + need > self.budget:
            return False
        self.queue.remove(req)
        slot = self.free_slots.pop()
        act = _Active(req, slot, self.ex.admit(req), need)
        self.used += need
        self.peak_used = max(self.peak_used, self.used)
        req.t_admit = time.perf_counter() - self.t0
        self._mode_begin(act)
        self.active.append(act)
        self.peak_active = max(self.peak_active, len(self.active))
        return True

    def _admit_srpt(self):
        """Admit the queued requests that the shortest-remaining-work ranking
        puts in the next round."""
        for item in self._ranked_round(with_queue=True):
            if isinstance(item, Request):
                self._admit_one(item)

    # ------------------------------------------------------------------ per request
    def _mode_begin(self, a: _Active):
        self.ex.mode_begin(a.h, a.n, a.k)
        a.dirty = True

    def _retire(self, a: _Active):
        req = a.req
        lam, facs, ll = self.ex.retire(a.h)
        if ll is not None:
            req.stats["loglik"] = ll
        req.result_lam, req.result_factors = lam, facs
        req.stats.update(outer_iters=a.k, inner_updates=a.updates,
                         converged=bool(self.params["tol"] > 0 and not a.any_update),
                         kkt=max(a.last_viol))
        req.t_done = time.perf_counter() - self.t0
        self.ex.clear_slot(a.slot)
        self._need_commit = True
        self.free_slots.append(a.slot)
        self.used -= a.nbytes
        self.done.append(req)

    # ------------------------------------------------------------------ tick
    def tick(self) -> bool:
        """Admit what fits, then run the inner loop of every active request's
        current mode together (one device sequence, stops decided on the
        device) and advance each request to its next mode. Returns False when
        nothing is active or queued."""
        clock = time.perf_counter
        t = clock()
        if self.policy == "all":
            self._admit()
        else:
            self._admit_srpt()
        t, dt = clock(), clock() - t
        self.phase_s["admit"] += dt
        if not self.active:
            return bool(self.queue)
        lmax, kmax, tol = self.params["lmax"], self.params["kmax"], self.params["tol"]
        run = self._select()
        held = [0] * self.max_slots
        for a in self.active:
            if a not in run:
                held[a.slot] = 1
        hold_changed = held != self._held and (self._held is not None or any(held))
        if hold_changed:
            self.ex.hold(held)
            self._held = held
        t, dt = clock(), clock() - t
        self.phase_s["hold"] += dt
        changed = False
        for a in self.active:
            if a.dirty:
                self.ex.set_slot(a.slot, a.h, a.n)
                a.dirty = False
                changed = True
        if changed or self._need_commit or (hold_changed and getattr(self.ex, "commit_on_hold", False)):
            self.ex.commit()
            self._need_commit = False
        t, dt = clock(), clock() - t
        self.phase_s["commit"] += dt
        # the whole inner loop of every running request's current mode, stops on the device
        viol, updates, done = self.ex.run_round(lmax)
        self.ticks += 1
        t, dt = clock(), clock() - t
        self.phase_s["round"] += dt
        keep, steps, retiring = [], [], []
        for a in self.active:
            if a not in run:
                keep.append(a)  # held this round: nothing ran
                continue
            a.last_viol[a.n] = viol[a.slot]
            a.updates += updates[a.slot]
            if updates[a.slot] > 0:
                a.any_update = True
            # mode finished: lambda and normalisation, then the next mode
            end = a.n
            a.n += 1
            if a.n == a.N:
                a.n = 0
                if (tol > 0 and not a.any_update) or a.k >= kmax:
                    steps.append((a.h, end, None, a.k))
                    retiring.append(a)
                    continue
                a.k += 1
                a.any_update = False
            steps.append((a.h, end, a.n, a.k))
            a.dirty = True
            keep.append(a)
        self.ex.advance(steps)
        t, dt = clock(), clock() - t
        self.phase_s["advance"] += dt
        for a in retiring:
            self._retire(a)
        self.active = keep
        self.phase_s["retire"] += clock() - t
        return bool(self.active or self.queue)

    def _remaining(self, a) -> float:
        """Work left for a request (active, or queued with all of it left): its
        nonzeros times the mode rounds left."""
        if isinstance(a, Request):
            return float(a.X.nnz) * self.params["kmax"] * len(a.X.dims)
        rounds = (self.params["kmax"] - a.k) * a.N + (a.N - a.n)
        return float(a.req.X.nnz) * rounds

    def _ranked_round(self, with_queue: bool) -> list:
        """Shortest remaining work first: the active (and, with_queue, queued)
        requests of the next round, until it holds the round's cap of nonzeros."""
        items = list(self.active) + (list(self.queue) if with_queue else [])
        nnz = lambda q: float(q.X.nnz if isinstance(q, Request) else q.req.X.nnz)  # noqa: E731
        rid = lambda q: q.id if isinstance(q, Request) else q.req.id  # noqa: E731
        cap = self.cap()
        out, work = [], 0.0
        for q in sorted(items, key=lambda q: (self._remaining(q), rid(q))):
            if out and work + nnz(q) > cap:
                break
            out.append(q)
            work += nnz(q)
        return out

    def cap(self) -> float:
        """Nonzeros a shortest-first round may hold: an eighth of the active and
        queued requests' nonzeros, within [round_cap_min, round_cap]."""
        pending = sum(float(a.req.X.nnz) for a in self.active) + sum(float(r.X.nnz) for r in self.queue)
        return min(self.round_cap, max(self.round_cap_min, pending / 8.0))

    def _select(self) -> set:
        """The active requests that run this round."""
        if self.policy == "all":
            return set(self.active)
        return set(self._ranked_round(with_queue=False))

    # ------------------------------------------------------------------ driving a trace
    def run_trace(self, requests: List[Request], time_limit: float = 600.0) -> List[Request]:
        """Replay arrivals in wall-clock time (request.arrival seconds after
        start) and serve until every request is done."""
        pending = deque(sorted(requests, key=lambda r: r.arrival))
        self.t0 = time.perf_counter()
        while pending or self.active or self.queue:
            now = time.perf_counter() - self.t0
            while pending and pending[0].arrival <= now:
                self.submit(pending.popleft())
            if not self.tick() and pending:
                time.sleep(max(0.0, min(0.001, pending[0].arrival - (time.perf_counter() - self.t0))))
            if time.perf_counter() - self.t0 > time_limit:
                raise TimeoutError("serving trace did not finish in time")
        return self.done


def results_to_host(reqs: List[Request]) -> List[Request]:
    """Copy completed requests' models from device memory into host arrays."""
    for r in reqs:
        if r.result_lam is not None and not isinstance(r.result_lam, np.ndarray):
            r.result_lam = r.result_lam.cpu().numpy()
            r.result_factors = [a.cpu().numpy() for a in r.result_factors]
    return reqs


def solve_one(req: Request, precision=cpapr.CPAPR_MIXED, kmax=20, lmax=10, tol=1e-4, eps=1e-10, stream=None):
    """The plain path: one request on its own with cpapr_solve. Returns the
    final model in device memory (lambda, factors) and the solve's stats."""
    import torch
    stream = stream if stream is not None else torch.cuda.current_stream()
    with torch.cuda.stream(stream):
        idx = torch.from_numpy(req.X.idx).to("cuda")
        vals = torch.from_numpy(req.X.vals).to("cuda")
        plan = cpapr.Plan(req.X.dims, idx, vals, req.M.rank, stream=stream, kmax=kmax, lmax=lmax, tol=tol, eps=eps,
                          precision=precision)
        del idx, vals
        lam = torch.from_numpy(req.M.lam).to("cuda")
        A = [torch.from_numpy(a).to("cuda") for a in req.M.factors]
        st = plan.solve(lam, A, stream=stream)
        plan.close()
        return lam, A, st


def latency_summary(done: List[Request]) -> dict:
    ok = [r for r in done if "rejected" not in r.stats]
    if not ok:
        return {}
    ttc = np.array([r.t_done - r.arrival for r in ok])
    tadm = np.array([r.t_done - r.t_admit for r in ok])
    span = max(r.t_done for r in ok) - min(r.arrival for r in ok)
    return {"completed": len(ok), "rejected": len(done) - len(ok),
            "p50_from_arrival_s": float(np.percentile(ttc, 50)), "p99_from_arrival_s": float(np.percentile(ttc, 99)),
            "p50_from_admission_s": float(np.percentile(tadm, 50)),
            "p99_from_admission_s": float(np.percentile(tadm, 99)),
            "solves_per_s": len(ok) / span if span > 0 else float("inf")}
