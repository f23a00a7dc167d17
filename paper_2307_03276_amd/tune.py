"""Autotuner for the Phi launch shape, measured on the device.

The segmented Phi kernel has three free choices that change its speed but not
its result (up to summation order): the lanes per nonzero G (with R <= G*RPL
rank columns spread over them, "rank blocking"), the nonzeros each lane group
walks per tile ("chunk"), and the order of the nonzeros inside a row of the
sorted copy (input order, or by the largest other mode's coordinate). The
paper finds that such launch-policy choices swing Phi's speed widely and that
the best one differs by tensor and by mode (Section 4); here they are chosen by
timing candidates on the real work.

Classes are (number of modes, rank, precision). For a batch, every class is
tuned on the batched launch of its own slots; the result is cached in a JSON
file keyed by the class and the log2 of its mean nonzero count.
"""
from __future__ import annotations

import json
import math
import os
import time
from typing import Dict, Iterable, List, Optional, Sequence, Tuple

from . import cpapr

GROUPS = (4, 8, 16)
CHUNKS = (2, 4, 8, 16, 32, 64)


def rank_block(R: int, G: int) -> int:
    need = -(-R // G)
    for r in (1, 2, 4):
        if need <= r:
            return r
    return -1


def shape_candidates(R: int, nmodes: int) -> List[Tuple[int, int]]:
    """(group, chunk) pairs with a batched kernel for rank R and N modes."""
    out = []
    for G in GROUPS:
        rpl = rank_block(R, G)
        if rpl < 0 or (G == 4 and rpl != 1) or nmodes > 4:
            continue
        # a group of G lanes with R <= G/2 leaves half its lanes idle: skip
        if rpl == 1 and G >= 2 * R and G > 4:
            continue
        out.extend((G, c) for c in CHUNKS)
    return out


_CYCLES_PER_MS: Optional[float] = None


def _hold_stream(ms: float):
    """Queue a device-side spin of about `ms` milliseconds on the current
    stream (calibrated once against HIP events)."""
    import torch
    global _CYCLES_PER_MS
    if _CYCLES_PER_MS is None:
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        torch.cuda._sleep(1_000_000)
        e1.record()
        torch.cuda.synchronize()
        _CYCLES_PER_MS = 1_000_000 / max(e0.elapsed_time(e1), 1e-3)
    torch.cuda._sleep(int(min(ms, 100.0) * _CYCLES_PER_MS))


def _enqueue_ms(fn) -> float:
    """Host time to queue one call of fn (after a warm call)."""
    import torch
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fn()
    t = time.perf_counter() - t0
    torch.cuda.synchronize()
    return t * 1e3


def _time(fn, reps: int) -> float:
    """Device time per call of fn over `reps` back-to-back calls. The stream is
    first held busy for longer than the host takes to queue the calls, so they
    run back to back on the device and the host's launch rate does not enter
    (a Phi launch on a small tensor takes a few microseconds, less than the
    host needs to issue it)."""
    import torch
    host = _enqueue_ms(fn)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    _hold_stream(2.0 * reps * host + 0.5)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def _kernel_ms(fn, reps: int) -> float:
    """Median device duration of the Phi kernel alone (the library's launch
    events bracket it) over `reps` calls of fn, queued behind a hold of the
    stream as in _time."""
    import torch
    host = _enqueue_ms(fn)
    cpapr.cpapr_prof_enable(reps)
    try:
        _hold_stream(2.0 * reps * host + 0.5)
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        recs = cpapr.cpapr_prof_read(reps)
    finally:
        cpapr.cpapr_prof_disable()
    ms = sorted(t for _, t in recs)
    return ms[len(ms) // 2]


def _reps_for(est_ms: float, min_ms: float, lo: int = 5, hi: int = 200) -> int:
    """Calls per timing: enough to cover min_ms of device time, at most `hi`
    (the calls of one timing must fit the stream's queue behind the hold)."""
    return max(lo, min(hi, int(math.ceil(min_ms / max(est_ms, 1e-4)))))


def _confirm(measure, keys: Sequence[tuple], rounds: int) -> Dict[tuple, float]:
    """Median of `rounds` timings of each finalist, taken in rotating order.
    The fastest of many single timings is biased low (it is the minimum of
    noisy draws), so the winner and the model are compared on fresh,
    interleaved timings instead."""
    samples: Dict[tuple, List[float]] = {k: [] for k in keys}
    for r in range(rounds):
        for j in range(len(keys)):
            k = keys[(j + r) % len(keys)]
            samples[k].append(measure(k))
    return {k: sorted(v)[len(v) // 2] for k, v in samples.items()}


def tune_plan(P, operands, modes: Optional[Iterable[int]] = None, min_ms: float = 1.0, rounds: int = 5,
              finalists: int = 3, candidates: Optional[Sequence[Tuple[int, int]]] = None) -> List[dict]:
    """Time the Phi kernel of each mode of one plan for every candidate
    (group, chunk) and for the library's launch-policy model. operands(n) ->
    (B, A). Each timing is the median kernel duration over enough launches to
    cover min_ms; the `finalists` fastest shapes and the model's are then
    re-timed `rounds` times, interleaved, and compared on their medians.
    Returns, per mode, the fastest shape, the model's shape and time, and
    model_vs_tuned = model time / fastest time. Leaves the plan on the model's
    shape."""
    import torch
    nm = len(P.dims)
    modes = range(nm) if modes is None else modes
    if candidates is None:
        candidates = [(g, c) for g in GROUPS for c in CHUNKS]
    P.set_shape(0, 0)
    model = tuple(P.shape())
    out = []
    for n in modes:
        B, A = operands(n)
        phi = torch.empty((P.dims[n], P.R), dtype=torch.float64, device=B.device)
        call = lambda: P.phi(n, B, A, out=phi)  # noqa: E731
        P.set_shape(*model)
        reps = _reps_for(_kernel_ms(call, 5), min_ms)

        def measure(shape):
            P.set_shape(*shape)
            return _kernel_ms(call, reps)

        first = {}
        for shape in list(candidates) + [model]:
            if shape in first:
                continue
            try:
                first[shape] = measure(shape)
            except cpapr.CpaprError:
                continue
        top = sorted(first, key=first.get)[:finalists]
        med = _confirm(measure, list(dict.fromkeys(top + [model])), rounds)
        P.set_shape(0, 0)
        best = min(med, key=med.get)
        out.append({"mode": n, "best": list(best), "best_ms": med[best], "model": list(model),
                    "model_ms": med[model], "model_vs_tuned": med[model] / med[best], "reps": reps,
                    "candidates": {f"{g},{c}": round(t, 5) for (g, c), t in sorted(first.items())},
                    "finalists": {f"{g},{c}": round(t, 5) for (g, c), t in sorted(med.items())}})
    return out


class Autotuner:
    def __init__(self, cache_path: Optional[str] = None, reps: int = 3):
        self.cache_path = cache_path
        self.reps = reps
        self.cache: Dict[str, dict] = {}
        self.log: List[dict] = []
        if cache_path and os.path.exists(cache_path):
            with open(cache_path) as f:
                self.cache = json.load(f)

    @staticmethod
    def key(nmodes: int, R: int, precision: int, mean_nnz: float) -> str:
        return f"N{nmodes}-R{R}-p{precision}-n{int(round(math.log2(max(mean_nnz, 1))))}"

    def save(self):
        if self.cache_path:
            with open(self.cache_path, "w") as f:
                json.dump(self.cache, f, indent=1, sort_keys=True)

    def tune_items(self, items: Sequence[dict]) -> Dict[str, dict]:
        """items: dicts with keys P (Plan), n (mode), B, A, Phi. Tunes each class on
        a batch of its own slots, applies the best (group, chunk) to its plans and
        returns {class key: choice}."""
        classes: Dict[str, List[dict]] = {}
        for it in items:
            P = it["P"]
            nm = len(P.dims)
            k = (nm, P.R, P.params.precision)
            classes.setdefault(k, []).append(it)
        choices = {}
        for (nm, R, prec), its in classes.items():
            mean = sum(it["P"].nnz for it in its) / len(its)
            key = self.key(nm, R, prec, mean)
            if key in self.cache:
                best = self.cache[key]
            else:
                best = self._search(its, nm, R)
                best["key"] = key
                self.cache[key] = best
            for it in its:
                it["P"].set_shape(best["group"], best["chunk"])
            choices[key] = best
            self.log.append(dict(best, key=key))
        self.save()
        return choices

    def _time_batch(self, its: Sequence[dict]) -> float:
        tiles = sum(it["P"].tiles() for it in its)
        b = cpapr.Batch(len(its), tiles + 1)
        for s, it in enumerate(its):
            b.set(s, it["P"], it["n"], it["B"], it["A"], it["Phi"])
        b.commit()
        ms = _time(lambda: b.run(use_graph=False), self.reps)
        b.close()
        return ms

    def _search(self, its: Sequence[dict], nm: int, R: int, finalists: int = 3, rounds: int = 5) -> dict:
        def measure(shape):
            for it in its:
                it["P"].set_shape(*shape)
            return self._time_batch(its)

        # the library's launch-policy model: (0, 0) gives every plan the
        # model's batch shape, timed on the same slots as the candidates
        model = (0, 0)
        first = {shape: measure(shape) for shape in shape_candidates(R, nm)}
        top = sorted(first, key=first.get)[:finalists]
        med = _confirm(measure, list(dict.fromkeys(top + [model])), rounds)
        for it in its:
            it["P"].set_shape(0, 0)
        model_shapes = sorted({it["P"].batch_shape() for it in its})
        # (0, 0) when the model's shapes are the fastest: the plans keep them
        best = min(med, key=med.get)
        G, chunk = best
        return {"group": G, "chunk": chunk, "ms": med[best],
                "model": [list(m) for m in model_shapes], "model_ms": med[model],
                "model_vs_tuned": med[model] / min(med.values()),
                "candidates": [{"group": g, "chunk": c, "ms": round(t, 4)} for (g, c), t in
                               sorted(first.items(), key=lambda kv: kv[1])]}

    def tune_sort(self, make_plan, modes: Iterable[int], operands) -> int:
        """Pick the in-row order for one tensor: make_plan(sort) builds a Plan,
        operands(n) returns (B, A) for mode n. Returns the faster CPAPR_SORT_*."""
        best = None
        for sort in (cpapr.CPAPR_SORT_ROW, cpapr.CPAPR_SORT_ROW_COL):
            P = make_plan(sort)
            total = 0.0
            for n in modes:
                B, A = operands(n)
                out = P.phi(n, B, A)
                total += _time(lambda: P.phi(n, B, A, out=out), self.reps)
            P.close()
            self.log.append(dict(sort=sort, ms=total))
            if best is None or total < best[0]:
                best = (total, sort)
        return best[1]
