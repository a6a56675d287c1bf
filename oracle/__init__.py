"""ORACLE -- test infrastructure only.

A plain, slow, obviously correct CPU reference for everything the GPU path
computes.  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py`` may import it; the product package never does, and the
two share no code.  Inputs come from the seeded generators in ``synth/``.

Floating point is FP64 throughout unless a function says otherwise.

* ``spmm`` / ``spmm_rows`` / ``spmm_sel`` -- Y = A X (Algorithm 1: the
  output starts at zero and each stored entry (r, c, v) adds v * X[c, :] to
  Y[r, :]; SpMV is the one-column case).  C loop in ``oracle.c``.
* ``spmv_t`` -- y = A^T x.
* ``bf16_*``, ``e4m3_*``, ``fp8_*`` -- X quantisers from the format
  definitions (C).
* ``pagerank`` -- the PageRank update of Section 4.1 (power iteration).
* ``nmf`` -- the multiplicative updates of Section 4.3, H first, then W.
* ``sym_eigs`` / ``eig_residuals`` -- wanted eigenpairs of a symmetric A
  (Section 4.2's eigensolver) from the dense FP64 eigen-decomposition, and
  the residuals ||A v - lambda v|| of given pairs.
* ``mlp_*`` / ``adam_step`` -- the tile-selector cost model (8 -> 64 -> 64
  -> V, ReLU), masked MSE loss, its gradients and the Adam update.
* ``scsr_bytes`` / ``dcsc_bytes`` -- the per-tile storage sizes of
  Section 3.2 (byte model).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-ffp-contract=off",
                               "-fno-fast-math", "-fopenmp", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(_SO)
        i64, vp = ctypes.c_int64, ctypes.c_void_p
        for f in (L.oracle_spmm_rows_f32x, L.oracle_spmm_rows_f64x):
            f.argtypes = [i64, i64, vp, vp, vp, vp, i64, i64, vp, i64]
            f.restype = None
        L.oracle_spmm_sel_f32x.argtypes = [i64, vp, vp, vp, vp, vp, i64, i64, vp]
        L.oracle_spmm_sel_f32x.restype = None
        L.oracle_spmm_sel_f32x_omp.argtypes = [i64, vp, vp, vp, vp, vp, i64, i64, vp]
        L.oracle_spmm_sel_f32x_omp.restype = ctypes.c_int
        L.oracle_spmv_t_f64.argtypes = [i64, i64, vp, vp, vp, vp, vp]
        L.oracle_spmv_t_f64.restype = None
        for f in (L.oracle_bf16_encode, L.oracle_bf16_decode, L.oracle_e4m3_encode,
                  L.oracle_e4m3_decode):
            f.argtypes = [vp, i64, vp]
            f.restype = None
        L.oracle_fp8_colscale.argtypes = [vp, i64, i64, i64, vp]
        L.oracle_fp8_colscale.restype = None
        L.oracle_fp8_quantize.argtypes = [vp, i64, i64, i64, vp, vp, i64]
        L.oracle_fp8_quantize.restype = None
        L.oracle_bf16_quantize.argtypes = [vp, i64, i64, i64, vp, i64]
        L.oracle_bf16_quantize.restype = None
        L.oracle_e4m3_value.argtypes = [ctypes.c_uint8]
        L.oracle_e4m3_value.restype = ctypes.c_float
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data


def _c(a, dtype):
    return None if a is None else np.ascontiguousarray(a, dtype=dtype)


# ------------------------------------------------------------------ SpMM

def spmm_rows(row_ptr, col, val, X, r0: int, r1: int) -> np.ndarray:
    """(A X)[r0:r1, :] in FP64.  X is float32 or float64, shape (n_cols, k)."""
    row_ptr = _c(row_ptr, np.int64)
    col = _c(col, np.int32)
    val = _c(val, np.float32)
    k = X.shape[1]
    Y = np.zeros((r1 - r0, k), dtype=np.float64)
    if r1 <= r0:
        return Y
    if X.dtype == np.float64:
        X = np.ascontiguousarray(X)
        _load().oracle_spmm_rows_f64x(r0, r1, _p(row_ptr), _p(col), _p(val), _p(X), k, k, _p(Y), k)
    else:
        X = _c(X, np.float32)
        _load().oracle_spmm_rows_f32x(r0, r1, _p(row_ptr), _p(col), _p(val), _p(X), k, k, _p(Y), k)
    return Y


def spmm(row_ptr, col, val, X) -> np.ndarray:
    """Y = A X in FP64 (A given as CSR; ``val`` None means binary A)."""
    return spmm_rows(row_ptr, col, val, X, 0, len(row_ptr) - 1)


def spmm_sel(row_ptr, col, val, X, rows) -> np.ndarray:
    """(A X)[rows, :] in FP64, for sampled-row parity checks at full size."""
    rows = _c(rows, np.int64)
    k = X.shape[1]
    Y = np.zeros((rows.shape[0], k), dtype=np.float64)
    if rows.shape[0] == 0:
        return Y
    X = np.ascontiguousarray(X, dtype=np.float32)
    _load().oracle_spmm_sel_f32x(rows.shape[0], _p(rows), _p(_c(row_ptr, np.int64)),
                                 _p(_c(col, np.int32)), _p(_c(val, np.float32)), _p(X), k, k, _p(Y))
    return Y


def spmm_sel_omp(row_ptr, col, val, X, rows):
    """spmm_sel with the rows shared out over the host's threads (OpenMP):
    the CPU baseline's multi-threaded leg.  Returns (Y, threads used); Y is
    bit-identical to spmm_sel's."""
    rows = _c(rows, np.int64)
    k = X.shape[1]
    Y = np.zeros((rows.shape[0], k), dtype=np.float64)
    if rows.shape[0] == 0:
        return Y, 1
    X = np.ascontiguousarray(X, dtype=np.float32)
    used = _load().oracle_spmm_sel_f32x_omp(rows.shape[0], _p(rows), _p(_c(row_ptr, np.int64)),
                                            _p(_c(col, np.int32)), _p(_c(val, np.float32)), _p(X), k, k, _p(Y))
    return Y, int(used)


def spmv_t(row_ptr, col, val, x, n_cols: int | None = None) -> np.ndarray:
    """y = A^T x in FP64."""
    n_rows = len(row_ptr) - 1
    n_cols = n_rows if n_cols is None else n_cols
    x = _c(x, np.float64)
    y = np.zeros(n_cols, dtype=np.float64)
    _load().oracle_spmv_t_f64(n_rows, n_cols, _p(_c(row_ptr, np.int64)), _p(_c(col, np.int32)),
                              _p(_c(val, np.float32)), _p(x), _p(y))
    return y


def transpose_csr(row_ptr, col, val, n_cols: int):
    """CSR of A^T (columns sorted), by a counting pass over the entries."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    n_rows = len(row_ptr) - 1
    rows = np.repeat(np.arange(n_rows, dtype=np.int64), np.diff(row_ptr))
    order = np.lexsort((rows, col))
    t_ptr = np.zeros(n_cols + 1, dtype=np.int64)
    np.add.at(t_ptr, col + 1, 1)
    t_ptr = np.cumsum(t_ptr)
    t_col = rows[order].astype(np.int32)
    t_val = None if val is None else np.asarray(val, dtype=np.float32)[order]
    return t_ptr, t_col, t_val


def frob_rel_err(Y, Yref) -> float:
    """Relative Frobenius error ||Y - Yref||_F / ||Yref||_F in FP64."""
    Y = np.asarray(Y, dtype=np.float64)
    Yref = np.asarray(Yref, dtype=np.float64)
    den = np.sqrt(np.sum(Yref * Yref))
    num = np.sqrt(np.sum((Y - Yref) ** 2))
    return float(num / den) if den > 0 else float(num)


# ------------------------------------------------------------- quantisers

def bf16_encode(x) -> np.ndarray:
    x = _c(x, np.float32).ravel()
    out = np.empty(x.shape[0], dtype=np.uint16)
    _load().oracle_bf16_encode(_p(x), x.shape[0], _p(out))
    return out


def bf16_decode(h) -> np.ndarray:
    h = _c(h, np.uint16).ravel()
    out = np.empty(h.shape[0], dtype=np.float32)
    _load().oracle_bf16_decode(_p(h), h.shape[0], _p(out))
    return out


def e4m3_encode(x) -> np.ndarray:
    x = _c(x, np.float32).ravel()
    out = np.empty(x.shape[0], dtype=np.uint8)
    _load().oracle_e4m3_encode(_p(x), x.shape[0], _p(out))
    return out


def e4m3_decode(c) -> np.ndarray:
    c = _c(c, np.uint8).ravel()
    out = np.empty(c.shape[0], dtype=np.float32)
    _load().oracle_e4m3_decode(_p(c), c.shape[0], _p(out))
    return out


def fp8_colscale(X) -> np.ndarray:
    """s_j = 448 / max_i |X[i, j]| in FP32 (1 for an all-zero column)."""
    X = _c(X, np.float32)
    n, k = X.shape
    s = np.empty(k, dtype=np.float32)
    _load().oracle_fp8_colscale(_p(X), n, k, k, _p(s))
    return s


def fp8_quantize(X, s) -> np.ndarray:
    """Q[i, j] = E4M3(fp32(X[i, j] * s_j)), saturating."""
    X = _c(X, np.float32)
    s = _c(s, np.float32)
    n, k = X.shape
    Q = np.empty((n, k), dtype=np.uint8)
    _load().oracle_fp8_quantize(_p(X), n, k, k, _p(s), _p(Q), k)
    return Q


def bf16_quantize(X) -> np.ndarray:
    X = _c(X, np.float32)
    n, k = X.shape
    Q = np.empty((n, k), dtype=np.uint16)
    _load().oracle_bf16_quantize(_p(X), n, k, k, _p(Q), k)
    return Q


def dequant(Xq, dtype: str, s=None) -> np.ndarray:
    """FP64 value the kernel sees: decode(x_q), divided by s_j for FP8."""
    if dtype == "f32":
        return np.asarray(Xq, dtype=np.float64)
    if dtype == "bf16":
        return bf16_decode(Xq).reshape(Xq.shape).astype(np.float64)
    if dtype == "fp8":
        d = e4m3_decode(Xq).reshape(Xq.shape).astype(np.float64)
        return d / np.asarray(s, dtype=np.float64)[None, :]
    raise ValueError(dtype)


# --------------------------------------------------------------- PageRank

def pagerank(row_ptr, col, n: int, damping: float = 0.85, iters: int = 30,
             redistribute: bool = True, symmetric: bool = False):
    """PageRank power iteration in FP64 (Section 4.1).

    PR'(u) = (1-d)/N + d * sum_{v in B(u)} PR(v) / L(v), with B(u) the
    in-neighbours of u and L(v) the out-degree of v (row v's length).  The
    sum is A^T x with x = PR / L (0 where L = 0).  Vertices with no out-edges
    ("dangling") hold rank mass D = sum PR(v) over L(v) = 0; with
    ``redistribute`` that mass is spread evenly, adding d * D / N to every
    vertex, which keeps sum PR = 1.  Start PR = 1/N; exactly ``iters``
    iterations; residual r_t = ||PR_{t+1} - PR_t||_1.
    """
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    deg = np.diff(row_ptr).astype(np.float64)
    pr = np.full(n, 1.0 / n, dtype=np.float64)
    resid = []
    dang = deg == 0
    for _ in range(iters):
        x = np.where(dang, 0.0, pr / np.where(dang, 1.0, deg))
        D = float(pr[dang].sum()) if redistribute else 0.0
        if symmetric:
            y = spmm(row_ptr, col, None, x[:, None])[:, 0]
        else:
            y = spmv_t(row_ptr, col, None, x, n)
        new = (1.0 - damping) / n + damping * (y + D / n)
        resid.append(float(np.abs(new - pr).sum()))
        pr = new
    return pr, np.array(resid)


# -------------------------------------------------------------------- NMF

def nmf(row_ptr, col, val, W, H, iters: int, eps: float = 1e-9, AT=None):
    """Lee-Seung multiplicative updates (Section 4.3), FP64.

    Shapes: A is n x m, W is n x r, H is stored m x r (the paper's H
    transposed).  Each iteration first updates H with W fixed, then W with
    H fixed:
        H <- H * (A^T W) / (H (W^T W) + eps)
        W <- W * (A H)   / (W (H^T H) + eps)
    ``AT`` is the CSR of A^T (defaults to A, i.e. symmetric A).
    """
    W = np.array(W, dtype=np.float64)
    H = np.array(H, dtype=np.float64)
    at_ptr, at_col, at_val = AT if AT is not None else (row_ptr, col, val)
    for _ in range(iters):
        G = W.T @ W
        H = H * spmm(at_ptr, at_col, at_val, W) / (H @ G + eps)
        G2 = H.T @ H
        W = W * spmm(row_ptr, col, val, H) / (W @ G2 + eps)
    return W, H


def nmf_objective(row_ptr, col, val, W, H) -> float:
    """||A - W H^T||_F^2 = ||A||_F^2 - 2 <W, A H> + <W^T W, H^T H>."""
    a2 = float(np.sum(np.square(np.asarray(val, np.float64)))) if val is not None else float(len(col))
    AH = spmm(row_ptr, col, val, np.asarray(H, np.float64))
    W = np.asarray(W, np.float64)
    H = np.asarray(H, np.float64)
    return a2 - 2.0 * float(np.sum(W * AH)) + float(np.sum((W.T @ W) * (H.T @ H)))


# ------------------------------------------------------------ eigensolver

def _which_order(w, which: str):
    """Indices of w with the wanted end first: "LM" |w| descending (equal
    magnitudes: larger value first), "LA" descending, "SA" ascending."""
    w = np.asarray(w, dtype=np.float64)
    if which == "LM":
        return np.lexsort((-w, -np.abs(w)))
    if which == "LA":
        return np.argsort(-w, kind="stable")
    if which == "SA":
        return np.argsort(w, kind="stable")
    raise ValueError(which)


def dense(row_ptr, col, val, n_cols: int | None = None) -> np.ndarray:
    """The CSR matrix as a dense FP64 array (small matrices only)."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    n = len(row_ptr) - 1
    A = np.zeros((n, n if n_cols is None else n_cols), dtype=np.float64)
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    v = np.ones(len(col)) if val is None else np.asarray(val, dtype=np.float64)
    np.add.at(A, (rows, np.asarray(col, dtype=np.int64)), v)
    return A


def sym_eigs(row_ptr, col, val, nev: int, which: str = "LM"):
    """The nev wanted eigenpairs of a symmetric sparse A (the quantity the
    eigensolver of Section 4.2 computes), by definition: the full FP64
    eigen-decomposition of the dense matrix (numpy.linalg.eigh), ordered as
    in _which_order.  Returns (values, unit eigenvectors as columns).  Small
    n only; raises if A is not symmetric."""
    A = dense(row_ptr, col, val)
    if not np.array_equal(A, A.T):
        raise ValueError("A is not symmetric")
    w, Z = np.linalg.eigh(A)
    o = _which_order(w, which)[:nev]
    return w[o], Z[:, o]


def eig_residuals(row_ptr, col, val, lam, V, rows=None) -> np.ndarray:
    """||(A V)[rows, j] - lam_j V[rows, j]||_2 per column j, in FP64 (all
    rows if rows is None).  V: n x nev, the full vectors (A V needs every
    neighbour's entry)."""
    V = np.asarray(V)
    lam = np.asarray(lam, dtype=np.float64)
    if rows is None:
        AV = spmm(row_ptr, col, val, V)
        Vr = np.asarray(V, dtype=np.float64)
    else:
        AV = spmm_sel(row_ptr, col, val, V, rows)
        Vr = np.asarray(V[np.asarray(rows)], dtype=np.float64)
    return np.sqrt(np.sum((AV - Vr * lam[None, :]) ** 2, axis=0))


# -------------------------------------------------------------------- MLP

def mlp_init(n_in: int, hidden: int, n_out: int, seed: int):
    """He-uniform weights from seeded draws (row-major [fan_in, fan_out])."""
    import synth
    params = {}
    dims = [(n_in, hidden), (hidden, hidden), (hidden, n_out)]
    ctr = 0
    key = synth.stream_key(seed, 21)
    for li, (fi, fo) in enumerate(dims, start=1):
        d = synth.draws(key, ctr, fi * fo)
        ctr += fi * fo
        u = (d >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
        lim = np.sqrt(6.0 / fi)
        params[f"W{li}"] = ((2.0 * u - 1.0) * lim).reshape(fi, fo)
        params[f"b{li}"] = np.zeros(fo)
    return params


def mlp_forward(p, X):
    """Returns (out, cache): out = W3^T relu(W2^T relu(W1^T x + b1) + b2) + b3."""
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ p["W1"] + p["b1"]
    a1 = np.maximum(z1, 0.0)
    z2 = a1 @ p["W2"] + p["b2"]
    a2 = np.maximum(z2, 0.0)
    out = a2 @ p["W3"] + p["b3"]
    return out, (X, z1, a1, z2, a2)


def mse_masked(out, y, mask) -> float:
    """L = sum(mask * (out - y)^2) / sum(mask)."""
    m = np.asarray(mask, dtype=np.float64)
    d = np.asarray(out, np.float64) - np.asarray(y, np.float64)
    return float(np.sum(m * d * d) / max(np.sum(m), 1.0))


def mlp_backward(p, cache, out, y, mask):
    """Gradients of the masked MSE with respect to every parameter."""
    X, z1, a1, z2, a2 = cache
    m = np.asarray(mask, dtype=np.float64)
    M = max(float(np.sum(m)), 1.0)
    g_out = 2.0 * m * (np.asarray(out, np.float64) - np.asarray(y, np.float64)) / M
    g = {"W3": a2.T @ g_out, "b3": g_out.sum(axis=0)}
    g_a2 = g_out @ p["W3"].T
    g_z2 = g_a2 * (z2 > 0)
    g["W2"] = a1.T @ g_z2
    g["b2"] = g_z2.sum(axis=0)
    g_a1 = g_z2 @ p["W2"].T
    g_z1 = g_a1 * (z1 > 0)
    g["W1"] = X.T @ g_z1
    g["b1"] = g_z1.sum(axis=0)
    return g


def adam_step(p, g, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """Adam (Kingma and Ba, 2015): bias-corrected first/second moments."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for name in p:
        m = state.setdefault("m_" + name, np.zeros_like(p[name]))
        v = state.setdefault("v_" + name, np.zeros_like(p[name]))
        m[...] = b1 * m + (1 - b1) * g[name]
        v[...] = b2 * v + (1 - b2) * g[name] * g[name]
        mh = m / (1 - b1 ** t)
        vh = v / (1 - b2 ** t)
        p[name] = p[name] - lr * mh / (np.sqrt(vh) + eps)
    return p


# ---------------------------------------------------- tile storage sizes

def scsr_bytes(nnr: int, nnz: int, c: int) -> int:
    """S_SCSR = 2 nnr + (2 + c) nnz (Section 3.2)."""
    return 2 * nnr + (2 + c) * nnz


def dcsc_bytes(nnc: int, nnz: int, c: int) -> int:
    """S_DCSC = (2 + 2 + 4) nnc + (2 + c) nnz (Section 3.2)."""
    return 8 * nnc + (2 + c) * nnz
