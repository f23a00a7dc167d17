"""Seeded synthetic inputs for CP-APR MU: sparse count tensors and initial models.

This module only draws random inputs. It holds none of the method's
arithmetic (no Pi, Phi, MU step, KKT or likelihood), so both the FP64 CPU
oracle and the GPU library can be fed from it without sharing any code.

The paper measures on FROSTT tensors (Table 2), which are not available here.
The generators below produce stand-ins with the shapes, nonzero counts and
value/index distributions of the configured workloads:

* values are counts, 1 + Poisson(mu), optionally capped (the method targets
  count data, Section 2);
* coordinates per mode are either uniform or a bounded Zipf(s) law
  P(i) ~ i^-s on {1..I_n}, sampled by inverse CDF, shifted to 0-based and then
  relabelled by a seeded random permutation so that hot rows are scattered;
* duplicate coordinates are kept as separate entries unless ``distinct``;
* the initial model draws factors U(0,1), sets lambda_r to the product over
  modes of the column sums and divides every column by its sum, which leaves
  the represented model unchanged (the algorithm takes an initial guess
  M = [lambda; A(1..N)] as input, Algorithm 1).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np


@dataclasses.dataclass
class SparseTensor:
    """N-way COO tensor: ``idx[m, k]`` is the 0-based mode-m coordinate of nonzero k."""

    dims: tuple
    idx: np.ndarray  # int32, shape (N, nnz), C-contiguous
    vals: np.ndarray  # float64, shape (nnz,)

    @property
    def nmodes(self) -> int:
        return len(self.dims)

    @property
    def nnz(self) -> int:
        return int(self.vals.shape[0])


@dataclasses.dataclass
class Model:
    """Rank-R Kruskal model M = [lambda; A(1) .. A(N)], each A(m) row-major I_m x R."""

    lam: np.ndarray  # float64 (R,)
    factors: List[np.ndarray]  # float64 (I_m, R), C-contiguous

    @property
    def rank(self) -> int:
        return int(self.lam.shape[0])

    def copy(self) -> "Model":
        return Model(self.lam.copy(), [a.copy() for a in self.factors])


def _children(seed: int, n: int) -> List[np.random.Generator]:
    ss = np.random.SeedSequence(seed)
    return [np.random.default_rng(s) for s in ss.spawn(n)]


def zipf_coords(rng: np.random.Generator, dim: int, s: float, count: int,
                chunk: int = 1 << 24) -> np.ndarray:
    """Bounded Zipf(s) on {0..dim-1} with a seeded random relabelling of the rows."""
    w = np.arange(1, dim + 1, dtype=np.float64) ** (-s)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    cdf[-1] = 1.0
    relabel = rng.permutation(dim).astype(np.int32)
    out = np.empty(count, dtype=np.int32)
    for lo in range(0, count, chunk):
        hi = min(count, lo + chunk)
        u = rng.random(hi - lo)
        r = np.searchsorted(cdf, u, side="right")
        np.minimum(r, dim - 1, out=r)
        out[lo:hi] = relabel[r]
    return out


def uniform_coords(rng: np.random.Generator, dim: int, count: int) -> np.ndarray:
    return rng.integers(0, dim, size=count, dtype=np.int64).astype(np.int32)


def count_values(rng: np.random.Generator, mu: float, count: int,
                 cap: Optional[float] = None) -> np.ndarray:
    v = 1.0 + rng.poisson(mu, size=count).astype(np.float64)
    if cap is not None:
        np.minimum(v, cap, out=v)
    return v


def random_tensor(seed: int, dims: Sequence[int], nnz: int, *, zipf: Sequence[Optional[float]] = (),
                  mu: float = 2.0, cap: Optional[float] = None, distinct: bool = False) -> SparseTensor:
    """General recipe. ``zipf[m]`` = exponent s for mode m, or None for uniform."""
    dims = tuple(int(d) for d in dims)
    nm = len(dims)
    zipf = list(zipf) + [None] * (nm - len(zipf))
    rngs = _children(seed, nm + 2)
    if distinct:
        total = math.prod(dims)
        if nnz > total:
            raise ValueError("more distinct nonzeros than cells")
        lin = rngs[0].choice(total, size=nnz, replace=False)
        idx = np.stack(np.unravel_index(lin, dims)).astype(np.int32)
    else:
        idx = np.empty((nm, nnz), dtype=np.int32)
        for m in range(nm):
            if zipf[m] is None:
                idx[m] = uniform_coords(rngs[m + 1], dims[m], nnz)
            else:
                idx[m] = zipf_coords(rngs[m + 1], dims[m], float(zipf[m]), nnz)
    vals = count_values(rngs[nm + 1], mu, nnz, cap)
    return SparseTensor(dims, np.ascontiguousarray(idx), vals)


def random_model(seed: int, dims: Sequence[int], rank: int) -> Model:
    """U(0,1) factors; lambda_r = prod_m colsum_m(r); columns scaled to unit 1-norm."""
    rngs = _children(seed + 7919, len(dims))
    facs = [rngs[m].random((int(d), rank)) for m, d in enumerate(dims)]
    lam = np.ones(rank)
    out = []
    for u in facs:
        cs = u.sum(axis=0)
        lam = lam * cs
        out.append(np.ascontiguousarray(u / cs))
    return Model(lam, out)


# ---------------------------------------------------------------------------
# Named workloads. Each returns (tensor, model, schedule dict).
# ---------------------------------------------------------------------------

def config_small(seed: int = 0):
    """3-way 100x80x60, 10,000 distinct uniform cells, counts 1+Poisson(2), R=10,
    eps=1e-10, fixed 10 outer x 10 inner iterations."""
    X = random_tensor(seed, (100, 80, 60), 10_000, mu=2.0, distinct=True)
    M = random_model(seed, X.dims, 10)
    return X, M, dict(kmax=10, lmax=10, tau=0.0, eps=1e-10)


def config_zipf3(seed: int = 0, nnz: int = 20_000_000, dims=(200_000, 150_000, 20_000)):
    """3-way 200k x 150k x 20k, Zipf(1.1) per mode, 20M nonzeros (duplicates kept),
    counts 1+Poisson(3), R=16, fixed 5 outer x 10 inner iterations."""
    X = random_tensor(seed, dims, nnz, zipf=(1.1, 1.1, 1.1), mu=3.0)
    M = random_model(seed, X.dims, 16)
    return X, M, dict(kmax=5, lmax=10, tau=0.0, eps=1e-10)


def config_zipf4(seed: int = 0, nnz: int = 100_000_000, dims=(1_000_000, 200_000, 10_000, 500)):
    """4-way 1M x 200k x 10k x 500, Zipf(1.2) on modes 1-2, uniform on 3-4, 100M nonzeros,
    counts min(1+Poisson(1), 1000), R=32, KKT tolerance 1e-4 or 20 outer iterations."""
    X = random_tensor(seed, dims, nnz, zipf=(1.2, 1.2, None, None), mu=1.0, cap=1000.0)
    M = random_model(seed, X.dims, 32)
    return X, M, dict(kmax=20, lmax=10, tau=1e-4, eps=1e-10)


def config_batch(seed: int = 0, count: int = 512, nnz_range=(1e3, 1e6), dim_range=(50, 5000),
                 ranks=(8, 16, 32)):
    """Many independent 3-way tensors: dims U{50..5000}, nnz LogUniform[1e3, 1e6],
    uniform coordinates, counts 1+Poisson(2), R drawn from ``ranks``."""
    ss = np.random.SeedSequence(seed)
    meta_rng = np.random.default_rng(ss.spawn(1)[0])
    out = []
    for t in range(count):
        dims = tuple(int(d) for d in meta_rng.integers(dim_range[0], dim_range[1] + 1, size=3))
        nnz = int(round(math.exp(meta_rng.uniform(math.log(nnz_range[0]), math.log(nnz_range[1])))))
        R = int(meta_rng.choice(ranks))
        X = random_tensor(seed * 100003 + t + 1, dims, nnz, mu=2.0)
        M = random_model(seed * 100003 + t + 1, dims, R)
        out.append((X, M))
    return out


def serving_trace(seed: int = 0, count: int = 550, rate: float = 200.0, nnz_range=(1e4, 2e7),
                  dim_range=(1e3, 1e5), ranks=(10, 16, 32)):
    """Request descriptors of a Poisson arrival stream: arrival time (s), dims, nnz, R, seed.
    Tensors are generated lazily with :func:`request_tensor`."""
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(1)[0])
    t = 0.0
    reqs = []
    for q in range(count):
        t += rng.exponential(1.0 / rate)
        nm = int(rng.integers(3, 5))
        dims = tuple(int(d) for d in rng.integers(int(dim_range[0]), int(dim_range[1]) + 1, size=nm))
        nnz = int(round(math.exp(rng.uniform(math.log(nnz_range[0]), math.log(nnz_range[1])))))
        R = int(rng.choice(ranks))
        reqs.append(dict(id=q, arrival=t, dims=dims, nnz=nnz, rank=R, seed=seed * 1000003 + q + 1))
    return reqs


def request_tensor(req: dict):
    X = random_tensor(req["seed"], req["dims"], req["nnz"], zipf=(1.1,) * len(req["dims"]), mu=2.0)
    M = random_model(req["seed"], req["dims"], req["rank"])
    return X, M
