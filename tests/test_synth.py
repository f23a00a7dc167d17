"""Seeded generators: determinism, shapes, ranges and the distributions the
workload recipes ask for."""
import numpy as np

from paper_2307_03276_amd import synth


def test_small_config_recipe():
    X, M, sched = synth.config_small()
    assert X.dims == (100, 80, 60) and X.nnz == 10_000
    lin = np.ravel_multi_index(tuple(X.idx.astype(np.int64)), X.dims)
    assert np.unique(lin).size == 10_000  # distinct cells
    assert X.vals.min() >= 1 and np.all(X.vals == np.round(X.vals))
    assert abs(X.vals.mean() - 3.0) < 0.1  # 1 + Poisson(2)
    assert M.rank == 10 and all(np.allclose(a.sum(axis=0), 1) for a in M.factors)
    assert sched == dict(kmax=10, lmax=10, tau=0.0, eps=1e-10)
    X2, M2, _ = synth.config_small()
    assert np.array_equal(X.idx, X2.idx) and np.array_equal(M.lam, M2.lam)


def test_zipf_skew_and_relabel():
    rng = np.random.default_rng(3)
    c = synth.zipf_coords(rng, 200_000, 1.1, 1_000_000)
    assert c.min() >= 0 and c.max() < 200_000
    counts = np.bincount(c, minlength=200_000)
    top = counts.max() / c.size
    # P(1) = 1 / H_{200000, 1.1} ~ 0.10-0.15 for s = 1.1
    assert 0.08 < top < 0.2
    assert np.argmax(counts) != 0 or counts[1] > 0  # relabelled, hot rows not forced to row 0


def test_model_is_normalised_and_positive():
    M = synth.random_model(5, (7, 8, 9), 4)
    for a in M.factors:
        assert np.all(a > 0)
        np.testing.assert_allclose(a.sum(axis=0), 1.0)
    assert np.all(M.lam > 0)


def test_batch_and_trace_shapes():
    b = synth.config_batch(count=6, nnz_range=(100, 1000))
    for X, M in b:
        assert X.nmodes == 3 and 100 <= X.nnz <= 1000
        assert all(50 <= d <= 5000 for d in X.dims)
        assert M.rank in (8, 16, 32)
    tr = synth.serving_trace(count=50)
    t = [r["arrival"] for r in tr]
    assert all(b > a for a, b in zip(t, t[1:]))
    assert all(len(r["dims"]) in (3, 4) and r["rank"] in (10, 16, 32) for r in tr)
