"""Pins for the oracle PageRank (Section 4.1), NMF (Section 4.3) and the
tile-selector MLP: closed forms, textbook solves and invariants."""
import numpy as np
import pytest

import oracle
import synth


def _csr_from_edges(n, edges):
    edges = sorted(set(edges))
    row_ptr = np.zeros(n + 1, np.int64)
    for u, _ in edges:
        row_ptr[u + 1] += 1
    row_ptr = np.cumsum(row_ptr)
    col = np.array([v for _, v in edges], np.int32)
    return row_ptr, col


# ---------------------------------------------------------------- PageRank

def test_pagerank_cycle_uniform():
    n = 9
    row_ptr, col = _csr_from_edges(n, [(i, (i + 1) % n) for i in range(n)])
    pr, res = oracle.pagerank(row_ptr, col, n, iters=30)
    assert np.allclose(pr, 1.0 / n, rtol=0, atol=1e-15)
    assert np.all(res < 1e-15)


def test_pagerank_star_closed_form():
    m = 12
    n = m + 1
    edges = [(0, i) for i in range(1, n)] + [(i, 0) for i in range(1, n)]
    row_ptr, col = _csr_from_edges(n, edges)
    d = 0.85
    pr, _ = oracle.pagerank(row_ptr, col, n, damping=d, iters=400)
    c = ((1 - d) / n + d) / (1 + d)          # PR(center) = (1-d)/N + d(1 - PR(center))
    leaf = (1 - d) / n + d * c / m
    assert abs(pr[0] - c) < 1e-13
    assert np.allclose(pr[1:], leaf, atol=1e-13)


@pytest.mark.parametrize("seed", range(5))
def test_pagerank_dense_solve(seed):
    """Converged power iteration = solution of (I - d M) PR = (1-d)/N 1,
    M column-stochastic with dangling columns uniform (textbook)."""
    n = 40
    row_ptr, col = synth.small_random_csr(n, 0.08, seed)
    d = 0.85
    A = np.zeros((n, n))
    for u in range(n):
        A[u, col[row_ptr[u]:row_ptr[u + 1]]] = 1
    deg = A.sum(axis=1)
    M = np.zeros((n, n))
    for v in range(n):
        M[:, v] = A[v] / deg[v] if deg[v] > 0 else 1.0 / n
    want = np.linalg.solve(np.eye(n) - d * M, np.full(n, (1 - d) / n))
    pr, _ = oracle.pagerank(row_ptr, col, n, damping=d, iters=300)
    assert np.allclose(pr, want, atol=1e-13)
    assert abs(pr.sum() - 1) < 1e-12


def test_pagerank_mass_and_symmetric_path():
    row_ptr, col = synth.rmat_csr(12, 8, seed=1, symmetrize=True)
    n = 1 << 12
    pr, res = oracle.pagerank(row_ptr, col, n, iters=30)
    assert abs(pr.sum() - 1) < 1e-12
    pr2, res2 = oracle.pagerank(row_ptr, col, n, iters=30, symmetric=True)
    assert np.allclose(pr, pr2, rtol=1e-13, atol=0)
    assert res[-1] < res[0]


def test_pagerank_literal_mass():
    """Without redistribution: sum PR' = (1-d) + d * sum_{L(v)>0} PR(v)."""
    row_ptr, col = synth.rmat_csr(10, 4, seed=2)
    n = 1 << 10
    pr1, _ = oracle.pagerank(row_ptr, col, n, iters=1, redistribute=False)
    deg = np.diff(row_ptr)
    assert abs(pr1.sum() - ((1 - 0.85) + 0.85 * (deg > 0).sum() / n)) < 1e-12


# --------------------------------------------------------------------- NMF

def test_nmf_objective_expansion():
    row_ptr, col = synth.small_random_csr(30, 0.2, 1)
    val = synth.lognormal_weights(row_ptr, col, seed=3)
    W = synth.uniform(30, 4, seed=4).astype(np.float64)
    H = synth.uniform(30, 4, seed=5).astype(np.float64)
    A = np.zeros((30, 30))
    for u in range(30):
        A[u, col[row_ptr[u]:row_ptr[u + 1]]] = val[row_ptr[u]:row_ptr[u + 1]]
    direct = np.sum((A - W @ H.T) ** 2)
    assert abs(oracle.nmf_objective(row_ptr, col, val, W, H) - direct) < 1e-10 * direct


def test_nmf_monotone_and_nonnegative():
    """Lee-Seung: each multiplicative update does not increase ||A - W H^T||^2.
    (eps = 0 needs every vertex to have an edge, so a ring is added.)"""
    rp, cl = synth.rmat_csr(9, 8, seed=1, symmetrize=True)
    n = 1 << 9
    rows = np.repeat(np.arange(n), np.diff(rp))
    ring = np.arange(n)
    edges = set(zip(rows.tolist(), cl.tolist())) | set(zip(ring, (ring + 1) % n)) | set(zip((ring + 1) % n, ring))
    row_ptr, col = _csr_from_edges(n, list(edges))
    W = synth.uniform(n, 8, seed=4).astype(np.float64)
    H = synth.uniform(n, 8, seed=5).astype(np.float64)
    prev = oracle.nmf_objective(row_ptr, col, None, W, H)
    for _ in range(10):
        W, H = oracle.nmf(row_ptr, col, None, W, H, iters=1, eps=0.0)
        cur = oracle.nmf_objective(row_ptr, col, None, W, H)
        assert cur <= prev * (1 + 1e-12)
        prev = cur
    assert W.min() >= 0 and H.min() >= 0


def test_nmf_fixed_point():
    """A = W0 H0^T exactly: the updates leave W0, H0 unchanged."""
    n, r = 12, 3
    W0 = (synth.int07(n, r, seed=1) + 1).astype(np.float64)
    H0 = (synth.int07(n, r, seed=2) + 1).astype(np.float64)
    A = W0 @ H0.T
    row_ptr = np.arange(0, n * n + 1, n, dtype=np.int64)
    col = np.tile(np.arange(n, dtype=np.int32), n)
    val = A.ravel().astype(np.float32)
    assert np.array_equal(val.astype(np.float64), A.ravel())
    AT = oracle.transpose_csr(row_ptr, col, val, n)
    W, H = oracle.nmf(row_ptr, col, val, W0, H0, iters=3, eps=0.0, AT=AT)
    assert np.allclose(W, W0, rtol=1e-13) and np.allclose(H, H0, rtol=1e-13)


def test_nmf_update_order_h_first():
    """One iteration equals: H from the old W, then W from the new H."""
    row_ptr, col = synth.small_random_csr(20, 0.3, 3)
    W = synth.uniform(20, 2, seed=4).astype(np.float64)
    H = synth.uniform(20, 2, seed=5).astype(np.float64)
    A = np.zeros((20, 20))
    for u in range(20):
        A[u, col[row_ptr[u]:row_ptr[u + 1]]] = 1
    AT = oracle.transpose_csr(row_ptr, col, None, 20)
    Hn = H * (A.T @ W) / (H @ (W.T @ W) + 1e-9)
    Wn = W * (A @ Hn) / (W @ (Hn.T @ Hn) + 1e-9)
    W1, H1 = oracle.nmf(row_ptr, col, None, W, H, iters=1, eps=1e-9, AT=AT)
    assert np.allclose(H1, Hn, rtol=1e-13) and np.allclose(W1, Wn, rtol=1e-13)


# --------------------------------------------------------------------- MLP

def _batch(seed, B=64, V=4):
    X = synth.uniform(B, 8, seed=seed).astype(np.float64) * 4 - 2
    y = synth.uniform(B, V, seed=seed + 1).astype(np.float64)
    mask = (synth.int07(B, V, seed=seed + 2) > 1).astype(np.float64)
    return X, y, mask


def test_mlp_gradients_finite_difference():
    p = oracle.mlp_init(8, 64, 4, seed=1)
    for k in p:
        if k.startswith("b"):
            p[k] = p[k] + 0.05   # move away from ReLU kinks
    X, y, mask = _batch(3)
    out, cache = oracle.mlp_forward(p, X)
    g = oracle.mlp_backward(p, cache, out, y, mask)
    h = 1e-6
    for name in p:
        flat = p[name].ravel()
        idx = np.linspace(0, flat.size - 1, min(flat.size, 25)).astype(int)
        for i in idx:
            old = flat[i]
            flat[i] = old + h
            lp = oracle.mse_masked(oracle.mlp_forward(p, X)[0], y, mask)
            flat[i] = old - h
            lm = oracle.mse_masked(oracle.mlp_forward(p, X)[0], y, mask)
            flat[i] = old
            fd = (lp - lm) / (2 * h)
            an = g[name].ravel()[i]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (name, i, fd, an)


def test_mlp_linear_regime_least_squares():
    """With all ReLUs active the net is affine in x; training converges to
    the least-squares affine fit (normal equations)."""
    rng_x, y, _ = _batch(5, B=256, V=2)
    X = rng_x
    target = X @ np.linspace(-1, 1, 16).reshape(8, 2) + 0.3
    p = oracle.mlp_init(8, 64, 2, seed=2)
    p["b1"] = p["b1"] + 50.0   # keep every unit in its linear region
    p["b2"] = p["b2"] + 500.0
    mask = np.ones_like(target)
    Xa = np.hstack([X, np.ones((X.shape[0], 1))])
    coef, *_ = np.linalg.lstsq(Xa, target, rcond=None)
    best = oracle.mse_masked(Xa @ coef, target, mask)
    st = {}
    for _ in range(3000):
        out, cache = oracle.mlp_forward(p, X)
        assert np.all(cache[1] > 0) and np.all(cache[3] > 0)
        g = oracle.mlp_backward(p, cache, out, target, mask)
        oracle.adam_step(p, g, st, lr=1e-3)
    final = oracle.mse_masked(oracle.mlp_forward(p, X)[0], target, mask)
    assert final <= best + 1e-3


def test_adam_first_step_is_lr_sign():
    """Step 1: m^ = g, v^ = g^2, so the update is lr * g / (|g| + eps)."""
    p = {"w": np.array([1.0, -2.0, 3.0])}
    g = {"w": np.array([0.5, -4.0, 1e-3])}
    oracle.adam_step(p, g, {}, lr=0.01)
    want = np.array([1.0, -2.0, 3.0]) - 0.01 * g["w"] / (np.abs(g["w"]) + 1e-8)
    assert np.allclose(p["w"], want, rtol=0, atol=1e-15)


# -------------------------------------------------------------- byte model

def test_scsr_dcsc_ratio_bound():
    """Section 3.2: with nnr = nnc and nnr <= nnz <= nnr t, binary tiles give
    0.4 <= S_SCSR / S_DCSC < 1."""
    for nnr in (1, 5, 100, 4096):
        for mult in (1, 2, 7, 100, 16384):
            nnz = nnr * mult
            r = oracle.scsr_bytes(nnr, nnz, 0) / oracle.dcsc_bytes(nnr, nnz, 0)
            assert 0.4 <= r < 1
    assert oracle.scsr_bytes(1, 1, 0) / oracle.dcsc_bytes(1, 1, 0) == 0.4
    assert oracle.scsr_bytes(3, 10, 4) == 2 * 3 + 6 * 10
