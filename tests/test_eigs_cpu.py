"""CPU checks of the eigensolver's host side: the Jacobi eigen-decomposition
used for the Rayleigh-Ritz step, and the argument checks spmm_eigs makes
before any device work."""
import math

import numpy as np
import pytest

import oracle
import paper_1602_02864_amd as pk
import synth


def _err(fn, *a, **kw):
    with pytest.raises(pk.SpmmError) as ei:
        fn(*a, **kw)
    return ei.value


@pytest.mark.parametrize("n", [1, 2, 3, 8, 33, 96])
def test_jacobi_matches_definition(n):
    rng = np.random.default_rng(n)
    a = rng.standard_normal((n, n))
    a = a + a.T
    w, z = pk.spmm_sym_eig_small(a)
    assert np.all(np.diff(w) >= 0)
    assert np.abs(z.T @ z - np.eye(n)).max() < 1e-12
    assert np.abs(a @ z - z * w[None, :]).max() < 1e-11 * max(1.0, np.abs(a).max()) * n
    assert np.allclose(w, np.linalg.eigvalsh(a), atol=1e-11 * n)


def test_jacobi_closed_forms():
    # tridiagonal (path graph) matrix: 2 cos(pi j / (n + 1))
    n = 20
    a = np.diag(np.ones(n - 1), 1) + np.diag(np.ones(n - 1), -1)
    w, _ = pk.spmm_sym_eig_small(a)
    assert np.allclose(w, np.sort([2 * math.cos(math.pi * j / (n + 1)) for j in range(1, n + 1)]), atol=1e-13)
    # repeated eigenvalues: J - I (complete graph) and a diagonal matrix
    n = 9
    w, z = pk.spmm_sym_eig_small(np.ones((n, n)) - np.eye(n))
    assert np.allclose(w, [-1] * (n - 1) + [n - 1], atol=1e-13)
    assert np.allclose(np.abs(z[:, -1]), 1 / math.sqrt(n), atol=1e-13)
    d = np.array([3.0, -1.0, 3.0, 0.5])
    w, z = pk.spmm_sym_eig_small(np.diag(d))
    assert np.array_equal(w, np.sort(d))


def test_jacobi_rejects_bad_input():
    assert _err(pk.spmm_sym_eig_small, np.array([[1.0, 2.0], [2.5, 1.0]])).status == pk.SPMM_EINVAL
    assert _err(pk.spmm_sym_eig_small, np.zeros((0, 0))).status == pk.SPMM_EINVAL
    assert _err(pk.spmm_sym_eig_small, np.eye(1025)).status == pk.SPMM_EINVAL


def test_eigs_argument_checks_before_device():
    rp, col = synth.rmat_csr(8, 4, seed=1, symmetrize=True)
    n = len(rp) - 1
    h = pk.spmm_build_tiles(rp, col)
    for kw in (dict(nev=0), dict(nev=4, block=17), dict(nev=4, which="XX"), dict(nev=4, max_dim=10),
               dict(nev=8, block=4, max_dim=8), dict(nev=4, block=16, max_dim=144), dict(nev=4, tol=-1.0),
               dict(nev=4, max_restarts=-1), dict(nev=4, block=4, max_dim=n)):
        kw = dict(kw)
        nev = kw.pop("nev")
        if kw.get("which") == "XX":
            with pytest.raises(ValueError):
                pk.spmm_eigs(h, nev, **kw)
            continue
        assert _err(pk.spmm_eigs, h, nev, **kw).status == pk.SPMM_EINVAL, kw
    h.close()
    # rectangular matrix
    hr = pk.spmm_build_tiles(rp, col, n_cols=n + 7)
    assert _err(pk.spmm_eigs, hr, 2).status == pk.SPMM_EINVAL
    hr.close()
    # argument errors are reported before any device work for tiles in host memory too
    hs = pk.spmm_build_tiles(rp, col, place=pk.SPMM_PLACE_PINNED_HOST)
    assert _err(pk.spmm_eigs, hs, 4, block=4, max_dim=6).status == pk.SPMM_EINVAL
    hs.close()


def test_oracle_and_host_jacobi_agree_on_a_graph():
    """The host Jacobi (the solver's Rayleigh-Ritz step) on a whole small
    graph gives the oracle's spectrum."""
    rp, col = synth.rmat_csr(6, 4, seed=2, symmetrize=True)
    n = len(rp) - 1
    w, _ = pk.spmm_sym_eig_small(oracle.dense(rp, col, None))
    ref, _ = oracle.sym_eigs(rp, col, None, n, "SA")
    assert np.allclose(w, ref, atol=1e-11)
