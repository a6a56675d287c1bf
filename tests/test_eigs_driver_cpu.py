"""The eigensolver's host driver (csrc/eigs.cpp: expansion, projections,
SVQB, breakdown handling, Rayleigh-Ritz, residual estimates, thick restart)
compiled with g++ against plain reference kernels (tests/helpers/eigs_host)
and checked against the oracle's dense eigen-decomposition -- the whole
Krylov-Schur logic on the CPU, with the same bars as the GPU tests."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle
import synth

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HELP = os.path.join(HERE, "helpers", "eigs_host")
WHICH = {"LM": 0, "LA": 1, "SA": 2}


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("eigs_host") / "libeigs_host.so")
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-I", HELP,
                           "-I", os.path.join(ROOT, "include"),
                           "-I", os.path.join(ROOT, "paper_1602_02864_amd", "csrc"),
                           os.path.join(HELP, "reference_kernels.cpp"),
                           os.path.join(ROOT, "paper_1602_02864_amd", "csrc", "eigs.cpp"), "-o", out])
    L = ctypes.CDLL(out)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
    L.eigs_host_run.argtypes = [i64, vp, vp, vp, i32, i32, i32, i32, ctypes.c_double, i32, ctypes.c_uint64,
                                vp, vp, vp, vp]
    L.eigs_host_run.restype = i32
    L.eigs_host_error.restype = ctypes.c_char_p
    return L


def _run(L, rp, col, val, nev, block=4, max_dim=0, which="LM", tol=1e-5, max_restarts=0, seed=1):
    n = len(rp) - 1
    rp = np.ascontiguousarray(rp, np.int64)
    col = np.ascontiguousarray(col, np.int32)
    v = None if val is None else np.ascontiguousarray(val, np.float32)
    ev = np.zeros(nev)
    V = np.zeros((n, nev), np.float32)
    rs = np.zeros(nev)
    info = np.zeros(4, np.int32)
    st = L.eigs_host_run(n, rp.ctypes.data, col.ctypes.data, None if v is None else v.ctypes.data, nev, block,
                         max_dim, WHICH[which], tol, max_restarts, seed, ev.ctypes.data, V.ctypes.data,
                         rs.ctypes.data, info.ctypes.data)
    return st, ev, V, rs, info


def _check(rp, col, val, ev, V, rs, tol, which, nev):
    n = len(rp) - 1
    w, _ = oracle.sym_eigs(rp, col, val, n, "SA")
    lam1 = np.abs(w).max()
    if which == "LM":
        assert np.allclose(np.sort(np.abs(ev))[::-1], np.sort(np.abs(w))[::-1][:nev], atol=2 * tol * lam1)
    else:
        ref = w[::-1][:nev] if which == "LA" else w[:nev]
        assert np.allclose(ev, ref, atol=2 * tol * lam1)
    assert np.all(rs <= tol)
    r = oracle.eig_residuals(rp, col, val, ev, V)
    assert np.all(r <= 4 * tol * np.abs(ev) + 2e-6 * lam1)
    assert np.abs(V.astype(np.float64).T @ V - np.eye(nev)).max() < 1e-5


@pytest.mark.parametrize("block", [1, 2, 4, 8])
def test_rmat_largest_magnitude(lib, block):
    rp, col = synth.rmat_csr(10, 8, seed=1, symmetrize=True)
    st, ev, V, rs, info = _run(lib, rp, col, None, 8, block=block, seed=11)
    assert st == 0 and info[0] == 8, lib.eigs_host_error()
    _check(rp, col, None, ev, V, rs, 1e-5, "LM", 8)


@pytest.mark.parametrize("which", ["LA", "SA"])
def test_algebraic_ends_with_many_restarts(lib, which):
    rp, col = synth.rmat_csr(9, 12, seed=3, symmetrize=True)
    st, ev, V, rs, info = _run(lib, rp, col, None, 6, block=3, max_dim=24, which=which)
    assert st == 0 and info[1] >= 1, (st, info)       # the small basis forces thick restarts
    _check(rp, col, None, ev, V, rs, 1e-5, which, 6)


def test_weighted_matrix(lib):
    rp, col = synth.rmat_csr(9, 10, seed=4, symmetrize=True)
    rows = np.repeat(np.arange(len(rp) - 1), np.diff(rp))
    val = (1.0 + ((rows + col) % 7) * 0.25).astype(np.float32)
    st, ev, V, rs, _ = _run(lib, rp, col, val, 5, block=2)
    assert st == 0
    _check(rp, col, val, ev, V, rs, 1e-5, "LM", 5)


def test_breakdown_on_the_complete_graph(lib):
    n = 120
    col = np.array([j for i in range(n) for j in range(n) if j != i], np.int32)
    rp = np.arange(0, n * (n - 1) + 1, n - 1, dtype=np.int64)
    st, ev, V, rs, _ = _run(lib, rp, col, None, 4, block=4, tol=1e-6)
    assert st == 0
    assert np.allclose(ev, [n - 1, -1, -1, -1], atol=1e-4)
    assert np.abs(V.astype(np.float64).T @ V - np.eye(4)).max() < 1e-5


def test_not_converged_status(lib):
    rp, col = synth.rmat_csr(10, 8, seed=2, symmetrize=True)
    st, ev, V, rs, info = _run(lib, rp, col, None, 8, block=1, max_dim=9, tol=1e-12, max_restarts=1)
    assert st == -6 and info[1] == 1 and info[0] < 8
    assert np.all(np.isfinite(ev)) and np.all(np.isfinite(V))
