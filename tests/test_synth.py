"""Seeded input generators: determinism, CSR validity, R-MAT statistics."""
import numpy as np
import pytest

import synth


def _valid_csr(row_ptr, col, n):
    assert row_ptr[0] == 0 and row_ptr[-1] == col.shape[0]
    assert np.all(np.diff(row_ptr) >= 0)
    assert col.min(initial=0) >= 0 and col.max(initial=0) < n
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    # strictly increasing columns inside each row (sorted, unique)
    same = rows[1:] == rows[:-1]
    assert np.all(col[1:][same] > col[:-1][same])
    assert not np.any(rows == col), "self-loop left in"


def test_rmat_deterministic_and_valid():
    a = synth.rmat_csr(12, 8, seed=7)
    b = synth.rmat_csr(12, 8, seed=7)
    c = synth.rmat_csr(12, 8, seed=8)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert not np.array_equal(a[1][:100], c[1][:100]) or a[1].shape != c[1].shape
    _valid_csr(a[0], a[1], 1 << 12)


def test_rmat_matches_raw_samples():
    """CSR = set of raw samples minus self-loops (dedup), row = source."""
    scale, ef = 10, 4
    row_ptr, col = synth.rmat_csr(scale, ef, seed=3)
    u, v = synth.rmat_samples(scale, 0, ef << scale, seed=3)
    keep = u != v
    pairs = np.unique(u[keep].astype(np.int64) * (1 << scale) + v[keep])
    n = 1 << scale
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    got = rows.astype(np.int64) * n + col
    assert np.array_equal(np.sort(got), pairs)


def test_rmat_symmetrize():
    row_ptr, col = synth.rmat_csr(11, 8, seed=5, symmetrize=True)
    n = 1 << 11
    _valid_csr(row_ptr, col, n)
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    fwd = set(zip(rows.tolist(), col.tolist()))
    assert all((c, r) in fwd for r, c in fwd)


def test_rmat_quadrant_frequencies():
    """Top-level quadrant of each raw sample has probability a, b, c, d."""
    scale, count = 16, 1 << 20
    u, v = synth.rmat_samples(scale, 0, count, seed=11)
    top_r = (u >> (scale - 1)) & 1
    top_c = (v >> (scale - 1)) & 1
    freq = np.array([np.mean((top_r == r) & (top_c == c)) for r, c in ((0, 0), (0, 1), (1, 0), (1, 1))])
    p = np.array([0.57, 0.19, 0.19, 0.05])
    sd = np.sqrt(p * (1 - p) / count)
    assert np.all(np.abs(freq - p) < 6 * sd), (freq, p)


def test_rmat_expected_row_degree():
    """Before dedup, E[deg(u)] = E * (a+b)^(s - ones(u)) * (c+d)^ones(u)."""
    scale, count = 8, 1 << 20
    u, _ = synth.rmat_samples(scale, 0, count, seed=2)
    deg = np.bincount(u, minlength=1 << scale)
    ones = np.array([bin(i).count("1") for i in range(1 << scale)])
    expect = count * 0.76 ** (scale - ones) * 0.24 ** ones
    # aggregate by popcount class to get tight statistics
    for k in range(scale + 1):
        sel = ones == k
        got, exp = deg[sel].sum(), expect[sel].sum()
        assert abs(got - exp) < 6 * np.sqrt(exp) + 1, (k, got, exp)


def test_uniform_and_int_x():
    X = synth.uniform(1000, 5, seed=2)
    assert X.dtype == np.float32 and X.min() >= 0 and X.max() < 1
    assert np.all(X * 2 ** 24 == np.floor(X * 2 ** 24))
    assert abs(X.mean() - 0.5) < 0.02
    Xi = synth.int07(1000, 5, seed=2)
    assert set(np.unique(Xi).tolist()) == set(range(8))
    assert np.array_equal(synth.uniform(10, 3, seed=4), synth.uniform(10, 3, seed=4))


def test_lognormal_weights_symmetric():
    row_ptr, col = synth.rmat_csr(10, 8, seed=1, symmetrize=True)
    val = synth.lognormal_weights(row_ptr, col, seed=3)
    n = 1 << 10
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    d = {(r, c): w for r, c, w in zip(rows.tolist(), col.tolist(), val.tolist())}
    assert all(d[(c, r)] == w for (r, c), w in d.items())
    z = np.log(val.astype(np.float64))
    assert abs(z.mean()) < 0.05 and abs(z.std() - 1) < 0.05


# ---------------------------------------------------------------- SBM

def _cluster(x, n, c):
    return (x.astype(np.int64) * c) // n


def test_sbm_samples_follow_the_model():
    """Sources uniform; the fraction of targets in the source's cluster is
    p_in + (1 - p_in) / c (within 5 standard errors); inside targets never
    leave the cluster."""
    n, c, p_in, m = 1 << 16, 64, 0.7, 1 << 20
    u, v = synth.sbm_samples(n, c, 0, m, p_in, seed=3)
    assert u.max() < n and v.max() < n
    inside = _cluster(u, n, c) == _cluster(v, n, c)
    p = p_in + (1 - p_in) / c
    assert abs(inside.mean() - p) < 5 * np.sqrt(p * (1 - p) / m)
    counts = np.bincount(_cluster(u, n, c), minlength=c)
    assert abs(counts.mean() - m / c) < 1e-9 and counts.std() < 5 * np.sqrt(m / c)
    # p_in = 1: every target inside; p_in = 0: inside only by chance
    u1, v1 = synth.sbm_samples(n, c, 0, 1 << 16, 1.0, seed=3)
    assert np.all(_cluster(u1, n, c) == _cluster(v1, n, c))
    u0, v0 = synth.sbm_samples(n, c, 0, 1 << 16, 0.0, seed=3)
    assert (_cluster(u0, n, c) == _cluster(v0, n, c)).mean() < 3.0 / c


def test_sbm_csr_is_the_cleaned_samples_and_unclustered_is_a_relabelling():
    n, c, p_in, m = 5000, 7, 0.6, 60000          # n not a multiple of c: ragged clusters
    rp, col = synth.sbm_csr(n, c, m, p_in, clustered=True, seed=4)
    u, v = synth.sbm_samples(n, c, 0, m, p_in, seed=4)
    keep = u != v
    ref = np.unique(u[keep].astype(np.int64) * n + v[keep])
    got = np.repeat(np.arange(n, dtype=np.int64), np.diff(rp)) * n + col
    assert np.array_equal(got, ref)             # sorted rows, no duplicates, no self-loops
    rp2, col2 = synth.sbm_csr(n, c, m, p_in, clustered=False, seed=4)
    perm = synth.sbm_perm(n, seed=4).astype(np.int64)
    assert np.array_equal(np.sort(perm), np.arange(n))
    relab = np.unique(perm[got // n] * n + perm[got % n])
    got2 = np.repeat(np.arange(n, dtype=np.int64), np.diff(rp2)) * n + col2
    assert np.array_equal(got2, relab)
    again = synth.sbm_csr(n, c, m, p_in, clustered=False, seed=4)
    assert np.array_equal(again[0], rp2) and np.array_equal(again[1], col2)


def test_sbm_rejects_bad_arguments():
    import pytest
    for args in ((0, 1, 10, 0.5), (10, 0, 10, 0.5), (10, 11, 10, 0.5), (10, 2, 10, 1.5)):
        with pytest.raises(ValueError):
            synth.sbm_csr(*args)
