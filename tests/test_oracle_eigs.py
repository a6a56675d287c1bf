"""Pins for the oracle eigen-decomposition of a symmetric sparse matrix (the
quantity the eigensolver of Section 4.2 computes): closed-form spectra of
textbook graphs, trace identities against brute-force counts, and residuals
of closed-form eigenvectors."""
import math

import numpy as np
import pytest

import oracle
import synth


def _csr(n, edges, weights=None):
    """Symmetric CSR from undirected edges {u, v} (u != v)."""
    ent = {}
    for i, (u, v) in enumerate(edges):
        w = 1.0 if weights is None else weights[i]
        ent[(u, v)] = w
        ent[(v, u)] = w
    keys = sorted(ent)
    row_ptr = np.zeros(n + 1, np.int64)
    for u, _ in keys:
        row_ptr[u + 1] += 1
    row_ptr = np.cumsum(row_ptr)
    col = np.array([v for _, v in keys], np.int32)
    val = None if weights is None else np.array([ent[k] for k in keys], np.float32)
    return row_ptr, col, val


def _all(rp, col, val=None):
    n = len(rp) - 1
    w, Z = oracle.sym_eigs(rp, col, val, n, "SA")
    return w, Z


def test_cycle_spectrum():
    n = 30
    rp, col, _ = _csr(n, [(i, (i + 1) % n) for i in range(n)])
    w, Z = _all(rp, col)
    ref = np.sort([2 * math.cos(2 * math.pi * j / n) for j in range(n)])
    assert np.allclose(w, ref, atol=1e-12)
    # closed-form eigenvector cos(2 pi j i / n) for eigenvalue 2 cos(2 pi j / n)
    j = 4
    v = np.cos(2 * math.pi * j * np.arange(n) / n)[:, None]
    r = oracle.eig_residuals(rp, col, None, [2 * math.cos(2 * math.pi * j / n)], v)
    assert r[0] < 1e-12


def test_path_spectrum():
    n = 17
    rp, col, _ = _csr(n, [(i, i + 1) for i in range(n - 1)])
    w, _ = _all(rp, col)
    ref = np.sort([2 * math.cos(math.pi * j / (n + 1)) for j in range(1, n + 1)])
    assert np.allclose(w, ref, atol=1e-12)


def test_complete_graph_lm_order_and_vector():
    n = 11
    rp, col, _ = _csr(n, [(i, j) for i in range(n) for j in range(i + 1, n)])
    w, Z = oracle.sym_eigs(rp, col, None, 4, "LM")
    assert np.allclose(w, [n - 1, -1, -1, -1], atol=1e-12)
    assert np.allclose(np.abs(Z[:, 0]), 1 / math.sqrt(n), atol=1e-12)   # the all-ones direction
    w_sa, _ = oracle.sym_eigs(rp, col, None, 2, "SA")
    assert np.allclose(w_sa, [-1, -1], atol=1e-12)
    w_la, _ = oracle.sym_eigs(rp, col, None, 1, "LA")
    assert abs(w_la[0] - (n - 1)) < 1e-12


def test_star_and_complete_bipartite():
    s = 16
    rp, col, _ = _csr(s + 1, [(0, i) for i in range(1, s + 1)])
    w, _ = oracle.sym_eigs(rp, col, None, 3, "LM")
    assert np.allclose(np.sort(w[:2]), [-math.sqrt(s), math.sqrt(s)], atol=1e-12)
    assert abs(w[2]) < 1e-12
    a, b = 3, 5
    rp, col, _ = _csr(a + b, [(i, a + j) for i in range(a) for j in range(b)])
    w, _ = _all(rp, col)
    ref = np.sort([-math.sqrt(a * b), math.sqrt(a * b)] + [0.0] * (a + b - 2))
    assert np.allclose(w, ref, atol=1e-12)


def test_hypercube_multiplicities():
    d = 6
    n = 1 << d
    rp, col, _ = _csr(n, [(u, u ^ (1 << i)) for u in range(n) for i in range(d) if u < u ^ (1 << i)])
    w, _ = _all(rp, col)
    ref = np.sort(np.concatenate([[d - 2 * i] * math.comb(d, i) for i in range(d + 1)]))
    assert np.allclose(w, ref, atol=1e-11)


def test_weighted_graphs():
    # one edge of weight c: eigenvalues -c, c
    rp, col, val = _csr(2, [(0, 1)], [2.5])
    w, _ = _all(rp, col, val)
    assert np.allclose(w, [-2.5, 2.5], atol=1e-12)
    # a uniformly weighted cycle scales the cycle spectrum
    n, c = 12, 0.75
    rp, col, val = _csr(n, [(i, (i + 1) % n) for i in range(n)], [c] * n)
    w, _ = _all(rp, col, val)
    ref = np.sort([c * 2 * math.cos(2 * math.pi * j / n) for j in range(n)])
    assert np.allclose(w, ref, atol=1e-12)


def test_trace_identities_on_rmat():
    """sum(lambda) = trace A = 0, sum(lambda^2) = nnz, sum(lambda^3) = 6 x
    (triangles, counted by brute force) for a binary symmetric graph with no
    self-loops; and the eigenvectors satisfy A v = lambda v."""
    rp, col = synth.rmat_csr(7, 6, seed=3, symmetrize=True)
    n = len(rp) - 1
    w, Z = _all(rp, col)
    adj = [set(col[rp[u]:rp[u + 1]].tolist()) for u in range(n)]
    tri = sum(1 for u in range(n) for v in adj[u] if v > u for x in adj[v] if x > v and x in adj[u])
    assert abs(w.sum()) < 1e-9
    assert abs(np.sum(w ** 2) - len(col)) < 1e-8 * len(col)
    assert abs(np.sum(w ** 3) - 6 * tri) < 1e-8 * max(1, 6 * tri)
    r = oracle.eig_residuals(rp, col, None, w, Z)
    assert r.max() < 1e-10


def test_wanted_ends_and_residual_rows():
    rp, col = synth.rmat_csr(6, 5, seed=4, symmetrize=True)
    n = len(rp) - 1
    w_all, _ = _all(rp, col)
    lm, _ = oracle.sym_eigs(rp, col, None, 5, "LM")
    la, _ = oracle.sym_eigs(rp, col, None, 5, "LA")
    sa, _ = oracle.sym_eigs(rp, col, None, 5, "SA")
    assert np.allclose(la, w_all[::-1][:5])
    assert np.allclose(sa, w_all[:5])
    assert np.allclose(np.sort(np.abs(lm))[::-1], np.sort(np.abs(w_all))[::-1][:5])
    # residual of a unit coordinate vector e_u with lambda = 0 is sqrt(deg u)
    u = int(np.argmax(np.diff(rp)))
    e = np.zeros((n, 1))
    e[u, 0] = 1.0
    assert abs(oracle.eig_residuals(rp, col, None, [0.0], e)[0] - math.sqrt(rp[u + 1] - rp[u])) < 1e-12
    # restricted to rows: the full residual splits over disjoint row sets
    rows_a = np.arange(0, n, 2)
    rows_b = np.arange(1, n, 2)
    v = synth.uniform(n, 2, seed=5)
    full = oracle.eig_residuals(rp, col, None, [1.0, -2.0], v)
    part = np.hypot(oracle.eig_residuals(rp, col, None, [1.0, -2.0], v, rows_a),
                    oracle.eig_residuals(rp, col, None, [1.0, -2.0], v, rows_b))
    assert np.allclose(full, part, rtol=1e-12)


def test_rejects_non_symmetric():
    rp = np.array([0, 1, 1], np.int64)
    col = np.array([1], np.int32)
    with pytest.raises(ValueError):
        oracle.sym_eigs(rp, col, None, 1)
