"""Block Krylov-Schur eigensolver (Section 4.2) on the device against the
oracle's dense eigen-decomposition.

What is unique is compared: the wanted eigenvalues (as magnitudes for LM,
where +x and -x tie), each within the bound the residual gives; eigenvectors
are checked by their true residual ||A y - theta y|| (FP64, oracle) and
orthonormality, since repeated eigenvalues leave them free within their
eigenspace.  Tolerances: the solver stops when its residual estimate is <=
tol |theta|; with an FP32 basis the true residual can exceed the estimate by
a few units of FP32 rounding of ||A||, hence the slack terms below."""
import functools
import math

import numpy as np
import pytest

import oracle
import paper_1602_02864_amd as pk
import synth

from gpu_util import dev

pytestmark = pytest.mark.gpu


@functools.lru_cache(maxsize=None)
def _graph(scale, ef, seed):
    rp, col = synth.rmat_csr(scale, ef, seed=seed, symmetrize=True)
    return rp, col


@functools.lru_cache(maxsize=None)
def _spectrum(scale, ef, seed):
    rp, col = _graph(scale, ef, seed)
    w, _ = oracle.sym_eigs(rp, col, None, len(rp) - 1, "SA")
    return w


def _solve(h, n, nev, **kw):
    import torch
    V = torch.full((n, nev), float("nan"), device=dev())
    evals, resid, info = pk.spmm_eigs(h, nev, evecs=V, **kw)
    torch.cuda.synchronize()
    return evals, resid, info, V.cpu().numpy()


def _check_pairs(rp, col, val, evals, V, tol, lam1):
    n = V.shape[0]
    assert np.all(np.isfinite(V))
    G = V.astype(np.float64).T @ V.astype(np.float64)
    assert np.abs(G - np.eye(V.shape[1])).max() < 1e-5
    r = oracle.eig_residuals(rp, col, val, evals, V)
    bound = 4 * tol * np.abs(evals) + 2e-6 * abs(lam1)
    assert np.all(r <= bound), (r, bound)
    return r


@pytest.mark.parametrize("block", [1, 2, 4, 8, 16])
@pytest.mark.parametrize("graph", [(10, 8, 1), (12, 16, 2)])
def test_largest_magnitude_matches_oracle(graph, block):
    rp, col = _graph(*graph)
    n = len(rp) - 1
    w = _spectrum(*graph)
    nev, tol = 8, 1e-5
    h = pk.spmm_build_tiles(rp, col)
    evals, resid, info, V = _solve(h, n, nev, block=block, tol=tol, seed=11)
    h.close()
    assert info["n_converged"] == nev and info["block"] == block
    assert np.all(resid <= tol)
    ref = np.sort(np.abs(w))[::-1][:nev]
    lam1 = ref[0]
    assert np.allclose(np.sort(np.abs(evals))[::-1], ref, rtol=0, atol=2 * tol * lam1)
    # every Ritz value lies within its residual bound of a true eigenvalue
    near = np.abs(evals[:, None] - w[None, :]).min(axis=1)
    assert np.all(near <= 2 * tol * lam1)
    _check_pairs(rp, col, None, evals, V, tol, lam1)


@pytest.mark.parametrize("which", ["LA", "SA"])
def test_algebraic_ends(which):
    graph = (11, 12, 3)
    rp, col = _graph(*graph)
    n = len(rp) - 1
    w = _spectrum(*graph)
    nev, tol = 6, 1e-5
    h = pk.spmm_build_tiles(rp, col)
    evals, _, info, V = _solve(h, n, nev, block=3, max_dim=24, which=which, tol=tol)
    h.close()
    ref = w[::-1][:nev] if which == "LA" else w[:nev]
    lam1 = np.abs(w).max()
    assert info["n_converged"] == nev
    assert np.allclose(evals, ref, rtol=0, atol=2 * tol * lam1)
    _check_pairs(rp, col, None, evals, V, tol, lam1)


def test_weighted_symmetric_matrix():
    rp, col = _graph(10, 10, 4)
    n = len(rp) - 1
    rows = np.repeat(np.arange(n), np.diff(rp))
    val = (1.0 + ((rows + col) % 7) * 0.25).astype(np.float32)       # w(u, v) = w(v, u)
    w, _ = oracle.sym_eigs(rp, col, val, n, "SA")
    h = pk.spmm_build_tiles(rp, col, val)
    nev, tol = 5, 1e-5
    evals, _, info, V = _solve(h, n, nev, block=4, tol=tol)
    h.close()
    lam1 = np.abs(w).max()
    assert np.allclose(np.sort(np.abs(evals))[::-1], np.sort(np.abs(w))[::-1][:nev], atol=2 * tol * lam1)
    _check_pairs(rp, col, val, evals, V, tol, lam1)


def test_invariant_subspace_breakdown_complete_graph():
    """K_n: the Krylov space of a block has dimension b + 1, so the second
    block breaks down and is refilled with random vectors."""
    n = 200
    rows = np.repeat(np.arange(n), n - 1)
    col = np.array([j for i in range(n) for j in range(n) if j != i], np.int32)
    rp = np.arange(0, n * (n - 1) + 1, n - 1, dtype=np.int64)
    assert rows.shape == col.shape
    h = pk.spmm_build_tiles(rp, col)
    evals, _, info, V = _solve(h, n, 4, block=4, tol=1e-6)
    h.close()
    assert info["n_converged"] == 4
    assert np.allclose(evals, [n - 1, -1, -1, -1], atol=1e-4)
    _check_pairs(rp, col, None, evals, V, 1e-6, n - 1)


def test_empty_graph_all_zero():
    n = 64
    h = pk.spmm_build_tiles(np.zeros(n + 1, np.int64), np.zeros(0, np.int32))
    evals, resid, info, V = _solve(h, n, 3, block=2)
    h.close()
    assert np.array_equal(evals, np.zeros(3)) and info["n_converged"] == 3
    assert np.abs(V.astype(np.float64).T @ V - np.eye(3)).max() < 1e-5


def test_deterministic_and_seed_independent_values():
    graph = (10, 8, 1)
    rp, col = _graph(*graph)
    n = len(rp) - 1
    h = pk.spmm_build_tiles(rp, col)
    a = _solve(h, n, 6, block=4, seed=5)
    b = _solve(h, n, 6, block=4, seed=5)
    c = _solve(h, n, 6, block=4, seed=6)
    h.close()
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[3], b[3])     # same seed: same bits
    lam1 = abs(a[0][0])
    assert np.allclose(np.sort(np.abs(a[0])), np.sort(np.abs(c[0])), atol=2e-5 * lam1)


def test_not_converged_reports_current_pairs():
    rp, col = _graph(12, 16, 2)
    n = len(rp) - 1
    h = pk.spmm_build_tiles(rp, col)
    import torch
    V = torch.empty((n, 8), device=dev())
    with pytest.raises(pk.SpmmError) as ei:
        pk.spmm_eigs(h, 8, block=1, max_dim=9, tol=1e-12, max_restarts=1, evecs=V)
    assert ei.value.status == pk.SPMM_ENOTCONV
    evals, resid, info = pk.spmm_eigs(h, 8, block=1, max_dim=9, tol=1e-12, max_restarts=1, evecs=V, check=False)
    torch.cuda.synchronize()
    h.close()
    assert info["restarts"] == 1 and info["n_converged"] < 8
    assert np.all(np.isfinite(evals)) and np.all(resid > 0)
    assert torch.isfinite(V).all()


@pytest.mark.parametrize("block", [1, 4])
def test_semi_external_equals_in_hbm(block):
    """Tiles in pinned host memory, streamed per product in small transfer
    groups: the same kernels on the same work items, so the whole solve is
    bit-identical to the in-HBM one."""
    rp, col = _graph(12, 16, 2)
    n = len(rp) - 1
    hd = pk.spmm_build_tiles(rp, col)
    hs = pk.spmm_build_tiles(rp, col, place=pk.SPMM_PLACE_PINNED_HOST, stream_kib=64, ring_depth=2)
    a = _solve(hd, n, 8, block=block, seed=3)
    b = _solve(hs, n, 8, block=block, seed=3)
    hd.close()
    hs.close()
    assert a[2]["n_spmm"] == b[2]["n_spmm"] and a[2]["n_converged"] == 8
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[3], b[3])


def test_sampled_residuals_scale_20():
    """A million-vertex graph: the oracle checks the residual on sampled rows
    (hub rows plus spread blocks), the orthonormality is checked in full."""
    rp, col = synth.rmat_csr(20, 16, seed=7, symmetrize=True)
    n = len(rp) - 1
    h = pk.spmm_build_tiles(rp, col, validate=False)
    nev, tol = 8, 1e-5
    evals, resid, info, V = _solve(h, n, nev, block=4, tol=tol)
    h.close()
    assert info["n_converged"] == nev
    sel = np.unique(np.concatenate([np.arange(64)] + [np.arange(s, s + 512) for s in
                                                      np.linspace(64, n - 512, 32).astype(np.int64)]))
    r_sel = oracle.eig_residuals(rp, col, None, evals, V, sel)
    # a sampled residual is at most the full one, which the solver bounds
    assert np.all(r_sel <= 4 * tol * np.abs(evals) + 2e-6 * abs(evals[0]))
    G = V.astype(np.float64).T @ V.astype(np.float64)
    assert np.abs(G - np.eye(nev)).max() < 1e-5
    # largest eigenvalue of a graph: between the mean degree and the max degree
    deg = np.diff(rp)
    assert deg.mean() <= abs(evals[0]) <= deg.max()
    assert math.sqrt(deg.max()) <= abs(evals[0]) * (1 + 1e-6)
