"""Seeded generators: determinism and the stated laws."""

import numpy as np

import synth


def test_deterministic_and_thread_independent(monkeypatch):
    A1, B1 = synth.mixture(40_000, 30_000, 8, seed=3, K=5, outlier_frac=0.001)
    monkeypatch.setattr(synth, "_threads", lambda: 1)
    A2, B2 = synth.mixture(40_000, 30_000, 8, seed=3, K=5, outlier_frac=0.001)
    assert A1.dtype == np.float32 and A1.flags.c_contiguous
    assert np.array_equal(A1, A2) and np.array_equal(B1, B2)
    A3, _ = synth.mixture(40_000, 30_000, 8, seed=4, K=5)
    assert not np.array_equal(A1, A3)


def test_gauss_outliers_law():
    A, B = synth.gauss_outliers(5000, 5000, 32, seed=0)
    r = np.linalg.norm(B.astype(np.float64), axis=1)
    assert np.sum(np.abs(r - 6.0) < 1e-5) == 50        # 1 % of B on the radius-6 sphere
    assert abs(B.mean() - 0.5 * (1 - 0.01)) < 0.02      # shifted mean elsewhere
    assert abs(A.mean()) < 0.01 and abs(A.std() - 1.0) < 0.01


def test_mixture_normalised_rows():
    A, B = synth.mixture(3000, 2000, 16, seed=1, K=8, normalize=True)
    assert np.allclose(np.linalg.norm(A, axis=1), 1.0, atol=1e-6)
    assert np.allclose(np.linalg.norm(B, axis=1), 1.0, atol=1e-6)


def test_shells_are_exact_multiples():
    A, B = synth.shells(500, 7, seed=2, r1=1.0, r2=2.0)
    key = lambda X: np.lexsort(X.T[::-1])
    assert np.array_equal(np.sort(2 * A, axis=0), np.sort(B, axis=0))
    assert np.array_equal((2 * A)[key(2 * A)], B[key(B)])


def test_batch_sizes_ranges():
    nA, nB, D = synth.batch_sizes(4096, seed=0)
    assert nA.min() >= 256 and nA.max() <= 65536 and set(np.unique(D)) == {64, 128, 256}
