"""Pins for the oracle SpMM (Algorithm 1: Y starts at zero, every stored
entry (r, c, v) adds v * X[c, :] to Y[r, :]).

The oracle is checked against brute-force dense matrix products and against
identities that hold for any correct SpMM, not against itself.
"""
import numpy as np
import pytest

import oracle
import synth


def _dense(row_ptr, col, val, n_cols):
    n = len(row_ptr) - 1
    A = np.zeros((n, n_cols))
    for i in range(n):
        for p in range(row_ptr[i], row_ptr[i + 1]):
            A[i, col[p]] += 1.0 if val is None else float(val[p])
    return A


@pytest.mark.parametrize("seed", range(12))
@pytest.mark.parametrize("n,density", [(1, 1.0), (7, 0.4), (64, 0.1), (200, 0.03)])
def test_brute_force_dense(seed, n, density):
    row_ptr, col = synth.small_random_csr(n, density, seed)
    A = _dense(row_ptr, col, None, n)
    for k in (1, 3, 8):
        Xi = synth.int07(n, k, seed=seed + 100)
        assert np.array_equal(oracle.spmm(row_ptr, col, None, Xi), A @ Xi.astype(np.float64))
        Xu = synth.uniform(n, k, seed=seed + 200)
        ref = A @ Xu.astype(np.float64)
        assert np.max(np.abs(oracle.spmm(row_ptr, col, None, Xu) - ref)) <= 1e-13 * max(1.0, np.abs(ref).max())


def test_weighted_brute_force():
    row_ptr, col = synth.small_random_csr(50, 0.2, 4, symmetrize=True)
    val = synth.lognormal_weights(row_ptr, col, seed=3)
    A = _dense(row_ptr, col, val, 50)
    X = synth.uniform(50, 4, seed=9)
    np.testing.assert_allclose(oracle.spmm(row_ptr, col, val, X), A @ X.astype(np.float64), rtol=1e-14)


def test_ones_gives_out_degree(c1_graph):
    row_ptr, col = c1_graph
    n = len(row_ptr) - 1
    Y = oracle.spmm(row_ptr, col, None, np.ones((n, 1), np.float32))
    assert np.array_equal(Y[:, 0], np.diff(row_ptr).astype(np.float64))


def test_transpose_ones_gives_in_degree(c1_graph):
    row_ptr, col = c1_graph
    n = len(row_ptr) - 1
    y = oracle.spmv_t(row_ptr, col, None, np.ones(n))
    assert np.array_equal(y, np.bincount(col, minlength=n).astype(np.float64))
    t_ptr, t_col, _ = oracle.transpose_csr(row_ptr, col, None, n)
    assert np.array_equal(np.diff(t_ptr), np.bincount(col, minlength=n))


def test_unit_columns_extract_columns():
    row_ptr, col = synth.small_random_csr(40, 0.15, 8)
    A = _dense(row_ptr, col, None, 40)
    E = np.eye(40, dtype=np.float32)
    assert np.array_equal(oracle.spmm(row_ptr, col, None, E), A)


def test_linearity_integer_exact(c1_graph):
    row_ptr, col = c1_graph
    n = len(row_ptr) - 1
    X1 = synth.int07(n, 4, seed=1)
    X2 = synth.int07(n, 4, seed=2)
    Y = oracle.spmm(row_ptr, col, None, X1 + X2)
    assert np.array_equal(Y, oracle.spmm(row_ptr, col, None, X1) + oracle.spmm(row_ptr, col, None, X2))


def test_symmetric_bilinear_identity():
    row_ptr, col = synth.rmat_csr(12, 8, seed=4, symmetrize=True)
    n = 1 << 12
    x = synth.uniform(n, 1, seed=5).astype(np.float64)
    y = synth.uniform(n, 1, seed=6).astype(np.float64)
    lhs = float(x[:, 0] @ oracle.spmm(row_ptr, col, None, y)[:, 0])
    rhs = float(y[:, 0] @ oracle.spmm(row_ptr, col, None, x)[:, 0])
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_empty_rows_and_empty_matrix():
    row_ptr = np.array([0, 0, 2, 2, 3], dtype=np.int64)
    col = np.array([0, 3, 1], dtype=np.int32)
    X = synth.uniform(4, 2, seed=1)
    Y = oracle.spmm(row_ptr, col, None, X)
    assert np.all(Y[0] == 0) and np.all(Y[2] == 0)
    assert np.array_equal(Y[1], X[0].astype(np.float64) + X[3])
    Y0 = oracle.spmm(np.zeros(5, np.int64), np.zeros(0, np.int32), None, X)
    assert np.all(Y0 == 0)


def test_rows_and_sel_agree(c1_graph):
    row_ptr, col = c1_graph
    n = len(row_ptr) - 1
    X = synth.uniform(n, 3, seed=2)
    full = oracle.spmm(row_ptr, col, None, X)
    assert np.array_equal(oracle.spmm_rows(row_ptr, col, None, X, 100, 2000), full[100:2000])
    rows = np.array([0, 5, n - 1, 77, 0])
    assert np.array_equal(oracle.spmm_sel(row_ptr, col, None, X, rows), full[rows])


def test_frob_rel_err():
    a = np.array([[3.0, 4.0]])
    assert oracle.frob_rel_err(a, a) == 0
    assert abs(oracle.frob_rel_err(a * 1.1, a) - 0.1) < 1e-12


def test_threaded_leg_equals_single_threaded():
    """The CPU baseline's OpenMP leg spreads independent rows over threads:
    its result is the single-threaded oracle's, bit for bit."""
    rp, col = synth.rmat_csr(14, 16, seed=31)
    n = rp.shape[0] - 1
    val = synth.lognormal_weights(rp, col, seed=3)
    rows = np.unique(np.concatenate([np.arange(64), np.arange(100, n, 7)]))
    for v in (None, val):
        X = synth.uniform(n, 5, seed=2)
        ref = oracle.spmm_sel(rp, col, v, X, rows)
        got, used = oracle.spmm_sel_omp(rp, col, v, X, rows)
        assert used >= 1
        assert np.array_equal(got, ref)
