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
from typing import Dict, Iterable, List, Optional, Sequence, Tuple

from . import cpapr

GROUPS = (4, 8, 16)
CHUNKS = (8, 16, 32, 64)


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


def _time(fn, reps: int) -> float:
    import torch
    fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


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

    def _search(self, its: Sequence[dict], nm: int, R: int) -> dict:
        results = []
        for G, chunk in shape_candidates(R, nm):
            for it in its:
                it["P"].set_shape(G, chunk)
            results.append((self._time_batch(its), G, chunk))
        results.sort()
        ms, G, chunk = results[0]
        # the library's launch-policy model (group by rank, chunk from precision,
        # rank and row length, per plan), timed on the same slots
        for it in its:
            it["P"].set_shape(0, 0)
        model = sorted({it["P"].shape() for it in its})
        model_ms = self._time_batch(its)
        return {"group": G, "chunk": chunk, "ms": ms,
                "model": [list(m) for m in model], "model_ms": model_ms, "model_vs_tuned": model_ms / ms,
                "candidates": [{"group": g, "chunk": c, "ms": round(t, 4)} for t, g, c in results]}

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
