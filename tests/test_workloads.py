"""The seeded input generators produce the stated structures (CPU only)."""
import numpy as np
import pytest

from paper_2108_10591_amd import workloads as W


def _rows(A):
    return np.repeat(np.arange(A.n), np.diff(A.rowptr))


def test_cd2d_64_closed_form():
    A = W.cd2d(64, 10.0)
    assert A.n == 4096 and A.nnz == 5 * 4096 - 4 * 64
    h = 1.0 / 65
    d = A.to_dense()
    assert np.allclose(np.diag(d), 4.0 + 2 * 10.0 * h, rtol=0, atol=1e-15)
    i = 64 * 10 + 10  # interior node
    assert d[i, i - 1] == pytest.approx(-(1 + 10 * h)) and d[i, i - 64] == pytest.approx(-(1 + 10 * h))
    assert d[i, i + 1] == -1.0 and d[i, i + 64] == -1.0
    assert np.allclose(d @ np.ones(A.n), A.b, rtol=1e-15, atol=1e-15)
    # nonsymmetric, columns ascending within rows
    assert not np.allclose(d, d.T)
    rows = _rows(A)
    assert np.all((np.diff(A.col) > 0) | (np.diff(rows) > 0))


def test_cd3d_structure_small():
    A = W.cd3d(12, 20.0, seed=7)
    N = 12
    assert A.n == N ** 3 and A.nnz == 7 * N ** 3 - 6 * N ** 2
    d = A.to_dense()
    off = d - np.diag(np.diag(d))
    # M-matrix, weakly diagonally dominant by rows (strictly at the boundary)
    assert np.all(off <= 0)
    assert np.all(np.diag(d) >= -off.sum(1) - 1e-12)
    assert np.allclose(d.sum(1), A.b, rtol=1e-13, atol=1e-13)
    # harmonic-mean diffusion is symmetric; upwind convection makes the matrix nonsymmetric
    rng = np.random.default_rng(7)
    k = np.exp(rng.standard_normal((N, N, N))).ravel()
    i = 5 + N * 5 + N * N * 5
    kf = 2 * k[i] * k[i + 1] / (k[i] + k[i + 1])
    assert d[i, i + 1] == pytest.approx(-kf, rel=1e-14)
    assert d[i, i - 1] == pytest.approx(-(2 * k[i] * k[i - 1] / (k[i] + k[i - 1])) - 20.0 / (N + 1), rel=1e-14)


@pytest.mark.slow
def test_cd3d_128_size():
    A = W.workload("cd3d_128")
    assert A.n == 128 ** 3 and A.nnz == 14_581_760
    assert A.rowptr.dtype == np.int64 and A.col.dtype == np.int32


@pytest.mark.slow
def test_rand_band_1m_statistics():
    A = W.workload("rand_band_1m")
    L = np.diff(A.rowptr)
    assert A.n == 1_000_000
    assert L.min() >= 3 and L.max() <= 200
    assert abs(L.mean() - 27.0) < 0.1
    rows = _rows(A)
    c = A.col.astype(np.int64)
    assert np.abs(c - rows).max() <= 5000
    assert np.all((np.diff(c) > 0) | (np.diff(rows) > 0))  # sorted, distinct
    diag = A.val[c == rows]
    absoff = np.zeros(A.n)
    np.add.at(absoff, rows[c != rows], np.abs(A.val[c != rows]))
    assert np.allclose(diag, 1.1 * absoff, rtol=1e-14)
    assert np.all(np.abs(A.val[c != rows]) <= 1.0)


def test_rand_band_small_is_deterministic():
    a = W.rand_band(20_000, seed=5, band=300)
    b = W.rand_band(20_000, seed=5, band=300)
    assert np.array_equal(a.col, b.col) and np.array_equal(a.val, b.val)
    rows = _rows(a)
    assert np.abs(a.col.astype(np.int64) - rows).max() <= 300


def test_special_matrices():
    S = W.skew_blocks(8, 0)
    d = S.to_dense()
    assert np.array_equal(d, -d.T)
    r = S.b
    assert r @ (d @ r) == 0.0  # exactly, in floating point
    D = W.diag_distinct(30, [1.0, 2.0, 5.0], 0)
    assert set(np.diag(D.to_dense())) == {1.0, 2.0, 5.0}
