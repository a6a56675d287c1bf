"""Seeded synthetic inputs (R-MAT and stochastic-block-model graphs, dense
matrices, edge weights).

Shared by the oracle tests and the GPU path; holds none of the SpMM method's
arithmetic.  The heavy lifting is in ``synth.c`` (OpenMP), loaded through
ctypes.  Seeds used across the project: graph 1, X 2, weights 3, W 4, H 5.

The R-MAT probabilities default to the paper's evaluation setting
(a=0.57, b=0.19, c=0.19, d=0.05; Section 5, footnote to Table 1).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libsynth.so")
_SRC = os.path.join(_HERE, "synth.c")

RMAT_A, RMAT_B, RMAT_C = 0.57, 0.19, 0.19
SEED_GRAPH, SEED_X, SEED_WEIGHT, SEED_W, SEED_H = 1, 2, 3, 4, 5


def build(force: bool = False) -> str:
    """Compile libsynth.so with gcc (OpenMP)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(_SO)
        i64, u64, vp = ctypes.c_int64, ctypes.c_uint64, ctypes.c_void_p
        L.synth_rmat_begin.argtypes = [ctypes.c_int, i64, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double, u64, ctypes.c_int,
                                       ctypes.POINTER(vp), ctypes.POINTER(i64), ctypes.POINTER(i64)]
        L.synth_rmat_begin.restype = ctypes.c_int
        L.synth_rmat_finish.argtypes = [vp, vp, vp]
        L.synth_rmat_finish.restype = None
        L.synth_rmat_samples.argtypes = [ctypes.c_int, i64, i64, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_double, u64, vp, vp]
        L.synth_rmat_samples.restype = None
        for f in (L.synth_uniform, L.synth_int07):
            f.argtypes = [i64, i64, i64, u64, vp]
            f.restype = None
        L.synth_lognormal_weights.argtypes = [i64, vp, vp, u64, vp]
        L.synth_lognormal_weights.restype = None
        L.synth_stream_key.argtypes = [u64, u64]
        L.synth_stream_key.restype = u64
        L.synth_draw.argtypes = [u64, u64]
        L.synth_draw.restype = u64
        L.synth_draws.argtypes = [u64, u64, i64, vp]
        L.synth_draws.restype = None
        L.synth_sbm_begin.argtypes = [i64, i64, i64, ctypes.c_double, ctypes.c_int, u64, ctypes.c_int,
                                      ctypes.POINTER(vp), ctypes.POINTER(i64), ctypes.POINTER(i64)]
        L.synth_sbm_begin.restype = ctypes.c_int
        L.synth_sbm_samples.argtypes = [i64, i64, i64, i64, ctypes.c_double, u64, vp, vp]
        L.synth_sbm_samples.restype = None
        L.synth_set_verbose.argtypes = [ctypes.c_int]
        L.synth_set_verbose.restype = None
        L.synth_sbm_perm.argtypes = [i64, u64, vp]
        L.synth_sbm_perm.restype = None
        _lib = L
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def rmat_csr(scale: int, edge_factor: float, seed: int = SEED_GRAPH, symmetrize: bool = False,
             a: float = RMAT_A, b: float = RMAT_B, c: float = RMAT_C, progress=None):
    """R-MAT adjacency matrix as CSR (row_ptr int64[n+1], col int32[nnz]).

    ``edge_factor * 2**scale`` samples are drawn; self-loops are removed, the
    pattern is symmetrised when asked, and duplicates are removed, so the
    returned nnz is the post-dedup count.  Columns are sorted within rows.
    ``progress(msg)``, if given, is called after each of the two phases.
    """
    L = _load()
    nsamples = int(round(edge_factor * (1 << scale)))
    L.synth_set_verbose(1 if progress else 0)
    h = ctypes.c_void_p()
    n = ctypes.c_int64()
    nnz = ctypes.c_int64()
    rc = L.synth_rmat_begin(scale, nsamples, a, b, c, seed, int(bool(symmetrize)),
                            ctypes.byref(h), ctypes.byref(n), ctypes.byref(nnz))
    if rc != 0:
        raise MemoryError("synth_rmat_begin failed")
    if progress:
        progress(f"R-MAT scale {scale}: {nsamples} samples drawn and bucketed by row")
    row_ptr = np.empty(n.value + 1, dtype=np.int64)
    col = np.empty(max(nnz.value, 1), dtype=np.int32)[: nnz.value]
    L.synth_rmat_finish(h, _ptr(row_ptr), _ptr(col) if nnz.value else _ptr(np.empty(1, np.int32)))
    if progress:
        progress(f"R-MAT scale {scale}: rows sorted and deduplicated, nnz {col.shape[0]}")
    return row_ptr, col


def sbm_csr(n: int, clusters: int, edges: int, p_in: float, clustered: bool = True, seed: int = SEED_GRAPH,
            symmetrize: bool = False, progress=None):
    """Stochastic block model graph as CSR (row_ptr int64[n+1], col int32[nnz]).

    Vertices form ``clusters`` equal contiguous ranges; each of ``edges``
    samples takes a uniform source u and, with probability ``p_in``, a target
    uniform in u's cluster, else a uniform target (so the expected fraction
    of edges inside clusters is p_in + (1 - p_in) / clusters).  With
    ``clustered=False`` every vertex id is replaced by ``sbm_perm(n, seed)``
    (the same graph, randomly ordered).  Self-loops and duplicates removed,
    columns sorted within rows.
    """
    L = _load()
    h = ctypes.c_void_p()
    nn = ctypes.c_int64()
    nnz = ctypes.c_int64()
    rc = L.synth_sbm_begin(n, clusters, edges, p_in, int(bool(clustered)), seed, int(bool(symmetrize)),
                           ctypes.byref(h), ctypes.byref(nn), ctypes.byref(nnz))
    if rc != 0:
        raise ValueError("synth_sbm_begin failed (bad arguments or out of memory)")
    if progress:
        progress(f"SBM n={n} clusters={clusters} p_in={p_in} {'clustered' if clustered else 'unclustered'}: "
                 f"{edges} samples bucketed")
    row_ptr = np.empty(nn.value + 1, dtype=np.int64)
    col = np.empty(max(nnz.value, 1), dtype=np.int32)[: nnz.value]
    L.synth_rmat_finish(h, _ptr(row_ptr), _ptr(col) if nnz.value else _ptr(np.empty(1, np.int32)))
    return row_ptr, col


def sbm_samples(n: int, clusters: int, e0: int, count: int, p_in: float, seed: int = SEED_GRAPH):
    """Raw SBM samples (u, v) in cluster order for sample ids [e0, e0+count)."""
    L = _load()
    u = np.empty(count, dtype=np.uint32)
    v = np.empty(count, dtype=np.uint32)
    L.synth_sbm_samples(n, clusters, e0, count, p_in, seed, _ptr(u), _ptr(v))
    return u, v


def sbm_perm(n: int, seed: int = SEED_GRAPH) -> np.ndarray:
    """The vertex relabelling of an unclustered SBM graph (a permutation of 0..n-1)."""
    perm = np.empty(n, dtype=np.uint32)
    _load().synth_sbm_perm(n, seed, _ptr(perm))
    return perm


def rmat_samples(scale: int, e0: int, count: int, seed: int = SEED_GRAPH,
                 a: float = RMAT_A, b: float = RMAT_B, c: float = RMAT_C):
    """Raw R-MAT samples (u, v) for sample ids [e0, e0+count), before cleanup."""
    L = _load()
    u = np.empty(count, dtype=np.uint32)
    v = np.empty(count, dtype=np.uint32)
    L.synth_rmat_samples(scale, e0, count, a, b, c, seed, _ptr(u), _ptr(v))
    return u, v


def uniform(n: int, k: int, seed: int = SEED_X, ld: int | None = None) -> np.ndarray:
    """n x k float32, uniform on [0,1) on the 2^-24 grid (row-major, row stride ld)."""
    ld = k if ld is None else ld
    X = np.zeros((n, ld), dtype=np.float32)
    _load().synth_uniform(n, k, ld, seed, _ptr(X))
    return X if ld == k else X


def int07(n: int, k: int, seed: int = SEED_X, ld: int | None = None) -> np.ndarray:
    """n x k float32 holding integers in {0..7}."""
    ld = k if ld is None else ld
    X = np.zeros((n, ld), dtype=np.float32)
    _load().synth_int07(n, k, ld, seed, _ptr(X))
    return X


def lognormal_weights(row_ptr: np.ndarray, col: np.ndarray, seed: int = SEED_WEIGHT) -> np.ndarray:
    """Lognormal(0,1) float32 values for every stored entry, symmetric in (u, v)."""
    n = row_ptr.shape[0] - 1
    val = np.empty(col.shape[0], dtype=np.float32)
    if col.shape[0]:
        _load().synth_lognormal_weights(n, _ptr(row_ptr), _ptr(col), seed, _ptr(val))
    return val


def stream_key(seed: int, stream: int) -> int:
    return int(_load().synth_stream_key(seed, stream))


def draw(key: int, ctr: int) -> int:
    return int(_load().synth_draw(key, ctr))


def draws(key: int, ctr0: int, count: int) -> np.ndarray:
    out = np.empty(count, dtype=np.uint64)
    _load().synth_draws(key, ctr0, count, _ptr(out))
    return out


def small_random_csr(n: int, density: float, seed: int, symmetrize: bool = False,
                     self_loops: bool = False):
    """Tiny uniform random binary CSR (for brute-force checks), from seeded draws."""
    d = draws(stream_key(seed, 11), 0, n * n).reshape(n, n)
    dense = (d >> np.uint64(11)).astype(np.float64) * 2.0 ** -53 < density
    if not self_loops:
        np.fill_diagonal(dense, False)
    if symmetrize:
        dense |= dense.T
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    cols = []
    for i in range(n):
        c = np.nonzero(dense[i])[0]
        cols.append(c)
        row_ptr[i + 1] = row_ptr[i] + c.size
    col = np.concatenate(cols).astype(np.int32) if cols else np.zeros(0, np.int32)
    return row_ptr, col
