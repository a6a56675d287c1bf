"""Python binding of libspmm.so (the C ABI declared in include/spmm.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of the library.  PyTorch tensors are accepted for device memory and
streams (their data pointers and stream handles are passed through); raw
integer device pointers work as well.  If the library has not been built,
importing the functions raises -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libspmm.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "spmm.h")

# spmm_status_t
SPMM_OK, SPMM_EINVAL, SPMM_ENOMEM, SPMM_EHIP, SPMM_EUNSUPPORTED, SPMM_ESTATE = 0, -1, -2, -3, -4, -5
SPMM_ENOTCONV = -6
# spmm_xdtype_t
SPMM_X_F32, SPMM_X_BF16, SPMM_X_FP8_E4M3 = 0, 1, 2
# spmm_variant_t
SPMM_VAR_COO, SPMM_VAR_ROW, SPMM_VAR_HYBRID, SPMM_VAR_WAVE = 0, 1, 2, 3
SPMM_NUM_VARIANTS = 4
SPMM_NUM_FEATURES = 8
VARIANT_NAMES = ("coo", "row", "hybrid", "wave")
# spmm_place_t
SPMM_PLACE_DEVICE, SPMM_PLACE_PINNED_HOST = 0, 1
SPMM_FORMAT_TILES, SPMM_FORMAT_CSR = 0, 1

SPMM_MAX_BUCKETS = 128
# cost-model parameter layout (one float array; weights row-major [in][out])
SPMM_MLP_HIDDEN = 64
SPMM_MLP_OFF_W1 = 0
SPMM_MLP_OFF_B1 = SPMM_MLP_OFF_W1 + SPMM_NUM_FEATURES * SPMM_MLP_HIDDEN
SPMM_MLP_OFF_W2 = SPMM_MLP_OFF_B1 + SPMM_MLP_HIDDEN
SPMM_MLP_OFF_B2 = SPMM_MLP_OFF_W2 + SPMM_MLP_HIDDEN * SPMM_MLP_HIDDEN
SPMM_MLP_OFF_W3 = SPMM_MLP_OFF_B2 + SPMM_MLP_HIDDEN
SPMM_MLP_OFF_B3 = SPMM_MLP_OFF_W3 + SPMM_MLP_HIDDEN * SPMM_NUM_VARIANTS
SPMM_MLP_PARAMS = SPMM_MLP_OFF_B3 + SPMM_NUM_VARIANTS

_STATUS_NAMES = {0: "SPMM_OK", -1: "SPMM_EINVAL", -2: "SPMM_ENOMEM", -3: "SPMM_EHIP",
                 -4: "SPMM_EUNSUPPORTED", -5: "SPMM_ESTATE", -6: "SPMM_ENOTCONV"}
# eigensolver: wanted end of the spectrum
SPMM_EIGS_LM, SPMM_EIGS_LA, SPMM_EIGS_SA = 0, 1, 2
_WHICH = {"LM": SPMM_EIGS_LM, "LA": SPMM_EIGS_LA, "SA": SPMM_EIGS_SA}


class SpmmError(RuntimeError):
    def __init__(self, status: int, func: str, msg: str):
        super().__init__(f"{func} -> {_STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class spmm_build_opts(ctypes.Structure):
    _fields_ = [("tile_rows", ctypes.c_uint32), ("tile_cols", ctypes.c_uint32),
                ("fixed_variant", ctypes.c_int32), ("item_nnz", ctypes.c_uint32),
                ("place", ctypes.c_uint32), ("threads", ctypes.c_uint32),
                ("validate", ctypes.c_uint32), ("max_kc", ctypes.c_uint32),
                ("keep_order", ctypes.c_uint32), ("stream_kib", ctypes.c_uint32),
                ("ring_depth", ctypes.c_uint32), ("x_stage_kib", ctypes.c_int32),
                ("transpose", ctypes.c_uint32), ("keep_row_order", ctypes.c_uint32),
                ("format", ctypes.c_uint32)]


class spmm_stats_t(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in (
        "n_rows", "n_cols", "nnz", "tile_rows", "tile_cols", "n_slabs", "n_tiles", "sum_nnr",
        "sum_nnc", "n_items", "n_parts", "blob_bytes", "desc_bytes")] + [
        ("variant_tiles", ctypes.c_uint64 * SPMM_NUM_VARIANTS),
        ("variant_nnz", ctypes.c_uint64 * SPMM_NUM_VARIANTS)]


class spmm_tune_opts(ctypes.Structure):
    _fields_ = [("min_tiles", ctypes.c_uint32), ("reps", ctypes.c_uint32)]


class spmm_train_opts(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_uint32), ("batch", ctypes.c_uint32), ("lr", ctypes.c_float),
                ("seed", ctypes.c_uint64)]


_lib = None


class spmm_eigs_opts(ctypes.Structure):
    _fields_ = [("nev", ctypes.c_int32), ("block", ctypes.c_int32), ("max_dim", ctypes.c_int32),
                ("which", ctypes.c_int32), ("max_restarts", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("tol", ctypes.c_double), ("seed", ctypes.c_uint64)]


class spmm_eigs_info(ctypes.Structure):
    _fields_ = [("n_converged", ctypes.c_int32), ("restarts", ctypes.c_int32), ("n_spmm", ctypes.c_int64),
                ("spmm_ms", ctypes.c_double), ("total_ms", ctypes.c_double), ("max_dim", ctypes.c_int32),
                ("block", ctypes.c_int32), ("dense_ms", ctypes.c_double), ("dense_bytes", ctypes.c_double),
                ("n_orth", ctypes.c_int64), ("n_reorth", ctypes.c_int64)]


def load_library():
    """Load libspmm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    # PyTorch ships its own HIP runtime under the same soname.  Loading torch
    # first makes libspmm.so bind to that one runtime, so device pointers and
    # streams from torch tensors are valid in the library; loading the
    # library first would map a second, separate runtime.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    i64, i32, vp, u64p = ctypes.c_int64, ctypes.c_int, ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64)
    L.spmm_last_error.restype = ctypes.c_char_p
    L.spmm_last_error.argtypes = []
    L.spmm_build_tiles.restype = i32
    L.spmm_build_tiles.argtypes = [i64, i64, vp, vp, vp, ctypes.POINTER(spmm_build_opts),
                                   ctypes.POINTER(vp)]
    L.spmm_build_begin.restype = i32
    L.spmm_build_begin.argtypes = [i64, i64, ctypes.POINTER(spmm_build_opts), ctypes.POINTER(vp)]
    L.spmm_build_append_rows.restype = i32
    L.spmm_build_append_rows.argtypes = [vp, i64, i64, vp, vp, vp]
    L.spmm_build_end.restype = i32
    L.spmm_build_end.argtypes = [vp]
    L.spmm_destroy.restype = None
    L.spmm_destroy.argtypes = [vp]
    L.spmm_run.restype = i32
    L.spmm_run.argtypes = [vp, vp, i32, i64, i32, vp, vp, i64, vp]
    L.spmm_run_static.restype = i32
    L.spmm_run_static.argtypes = [vp, vp, i32, i64, i32, vp, vp, i64, vp]
    L.spmm_quantize_x.restype = i32
    L.spmm_quantize_x.argtypes = [vp, i64, i32, i64, i32, vp, i64, vp, ctypes.c_uint32, vp]
    L.spmm_stream_run.restype = i32
    L.spmm_stream_run.argtypes = [vp, vp, i32, i64, i32, vp, vp, i64, vp, vp]
    L.spmm_stream_run_yhost.restype = i32
    L.spmm_stream_run_yhost.argtypes = [vp, vp, i32, i64, i32, vp, vp, i64, vp, vp, vp]
    L.spmm_pagerank.restype = i32
    L.spmm_pagerank.argtypes = [vp, ctypes.c_float, i32, ctypes.c_uint32, vp, vp, vp]
    L.spmm_nmf.restype = i32
    L.spmm_nmf.argtypes = [vp, vp, i32, i32, ctypes.c_float, vp, vp, vp]
    L.spmm_get_stats.restype = i32
    L.spmm_get_stats.argtypes = [vp, ctypes.POINTER(spmm_stats_t)]
    L.spmm_decode_tiles.restype = i32
    L.spmm_decode_tiles.argtypes = [vp, vp, vp, vp]
    L.spmm_model_tiles.restype = i32
    L.spmm_model_tiles.argtypes = [i64, i64, vp, vp, i64, u64p, u64p, u64p]
    u32, f32 = ctypes.c_uint32, ctypes.c_float
    for name, args in [
            ("spmm_tile_features", [vp, i32, i32, vp]),
            ("spmm_get_variants", [vp, vp]),
            ("spmm_set_variants", [vp, vp]),
            ("spmm_selector_collect", [vp, i32, i32, ctypes.POINTER(spmm_tune_opts), vp, vp, vp, vp]),
            ("spmm_autotune", [vp, i32, i32, ctypes.POINTER(spmm_tune_opts), vp, vp, vp]),
            ("spmm_mlp_init", [ctypes.c_uint64, vp]),
            ("spmm_mlp_predict", [vp, vp, i64, vp, vp, vp]),
            ("spmm_mlp_grad", [vp, vp, vp, vp, i64, vp, vp, vp]),
            ("spmm_mlp_adam", [vp, vp, vp, vp, i64, f32, f32, f32, f32, vp]),
            ("spmm_selector_train", [vp, vp, vp, i64, ctypes.POINTER(spmm_train_opts), vp, vp]),
            ("spmm_select_learned", [vp, vp, i32, i32]),
            ("spmm_timing_begin", [vp]),
            ("spmm_stream_run_host", [vp, vp, i32, i64, vp, i64, i32, ctypes.c_uint32]),
            ("spmm_read_probe", [vp, ctypes.c_uint64, vp, vp]),
            ("spmm_timing_end", [vp, vp, vp]),
            ("spmm_eigs", [vp, ctypes.POINTER(spmm_eigs_opts), vp, vp, i64, vp, ctypes.POINTER(spmm_eigs_info), vp]),
            ("spmm_sym_eig_small", [i32, vp, vp, vp]),
            ("spmm_dense_tn", [vp, i64, i32, vp, i64, i32, i64, vp, vp, ctypes.c_size_t, vp]),
            ("spmm_dense_nn", [vp, i64, i32, vp, i32, ctypes.c_double, ctypes.c_double, vp, i64, i64, vp])]:
        fn = getattr(L, name)
        fn.restype = i32
        fn.argtypes = args
    L.spmm_dense_tn_workspace.restype = ctypes.c_size_t
    L.spmm_dense_tn_workspace.argtypes = [i64, i32, i32]
    del u32
    _lib = L
    return L


def header_functions() -> list[str]:
    """Names of every function declared in include/spmm.h."""
    txt = open(HEADER_PATH).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(spmm_[a-z0-9_]+)\s*\(", txt)))


def spmm_last_error() -> str:
    return load_library().spmm_last_error().decode()


def _check(st: int, func: str):
    if st != SPMM_OK:
        raise SpmmError(st, func, spmm_last_error())


def _host(a, dtype):
    return None if a is None else np.ascontiguousarray(a, dtype=dtype)


def _ptr(x):
    """Device/host pointer of a torch tensor, numpy array, int or None."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if isinstance(x, np.ndarray):
        return x.ctypes.data
    return x.data_ptr()


def _stream(stream, like=None):
    if stream is None:
        if like is not None and hasattr(like, "device") and getattr(like, "is_cuda", False):
            import torch
            return torch.cuda.current_stream(like.device).cuda_stream
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


class Handle:
    """Owns an spmm_handle_t; destroyed on close() or garbage collection."""

    def __init__(self, ptr: int, n_rows: int, n_cols: int):
        self.ptr = ptr
        self.n_rows = n_rows
        self.n_cols = n_cols

    def close(self):
        if self.ptr:
            spmm_destroy(self)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def _as_parameter_(self):
        return ctypes.c_void_p(self.ptr)


def spmm_build_tiles(row_ptr, col_idx, values=None, n_cols: int | None = None, *,
                     tile_rows: int = 0, tile_cols: int = 0, fixed_variant: int = -1,
                     item_nnz: int = 0, place: int = SPMM_PLACE_DEVICE, threads: int = 0,
                     validate: bool = True, max_kc: int = 0, keep_order: bool = False,
                     stream_kib: int = 0, ring_depth: int = 0, x_stage_kib: int = 0,
                     transpose: bool = False, keep_row_order: bool = False, format: int = 0) -> Handle:
    L = load_library()
    rp = _host(row_ptr, np.int64)
    ci = _host(col_idx, np.int32)
    va = _host(values, np.float32)
    n_rows = rp.shape[0] - 1
    n_cols = n_rows if n_cols is None else int(n_cols)
    o = spmm_build_opts(tile_rows, tile_cols, fixed_variant, item_nnz, place, threads,
                        int(bool(validate)), max_kc, int(bool(keep_order)), stream_kib, ring_depth,
                        int(x_stage_kib), int(bool(transpose)), int(bool(keep_row_order)), int(format))
    out = ctypes.c_void_p()
    st = L.spmm_build_tiles(n_rows, n_cols, rp.ctypes.data, None if ci is None or ci.size == 0 else ci.ctypes.data,
                            None if va is None else va.ctypes.data, ctypes.byref(o), ctypes.byref(out))
    _check(st, "spmm_build_tiles")
    return Handle(out.value, n_cols, n_rows) if transpose else Handle(out.value, n_rows, n_cols)


def _opts(tile_rows=0, tile_cols=0, fixed_variant=-1, item_nnz=0, place=SPMM_PLACE_DEVICE, threads=0,
          validate=True, max_kc=0, keep_order=False, stream_kib=0, ring_depth=0, x_stage_kib=0,
          transpose=False, keep_row_order=False, format=0):
    return spmm_build_opts(tile_rows, tile_cols, fixed_variant, item_nnz, place, threads, int(bool(validate)),
                           max_kc, int(bool(keep_order)), stream_kib, ring_depth, int(x_stage_kib),
                           int(bool(transpose)), int(bool(keep_row_order)), int(format))


def spmm_build_begin(n_rows: int, n_cols: int | None = None, **opts) -> Handle:
    """Start a slab-wise build (options as spmm_build_tiles; columns keep
    their order, rows are ordered within each appended block)."""
    L = load_library()
    n_cols = n_rows if n_cols is None else int(n_cols)
    o = _opts(**opts)
    out = ctypes.c_void_p()
    _check(L.spmm_build_begin(int(n_rows), n_cols, ctypes.byref(o), ctypes.byref(out)), "spmm_build_begin")
    return Handle(out.value, int(n_rows), n_cols)


def spmm_build_append_rows(h: Handle, row0: int, row_ptr_local, col_idx, values=None) -> None:
    """Append rows [row0, row0 + len(row_ptr_local) - 1) (local row pointers
    starting at 0)."""
    L = load_library()
    rp = _host(row_ptr_local, np.int64)
    ci = _host(col_idx, np.int32)
    va = _host(values, np.float32)
    nrows = rp.shape[0] - 1
    st = L.spmm_build_append_rows(h.ptr, int(row0), nrows, rp.ctypes.data,
                                  None if ci is None or ci.size == 0 else ci.ctypes.data,
                                  None if va is None else va.ctypes.data)
    _check(st, "spmm_build_append_rows")


def spmm_build_end(h: Handle) -> None:
    _check(load_library().spmm_build_end(h.ptr), "spmm_build_end")


def spmm_destroy(h: Handle):
    load_library().spmm_destroy(ctypes.c_void_p(h.ptr))


def _xdtype(X, dtype):
    if dtype is not None:
        return dtype
    return _X_TORCH_DTYPES.get(str(getattr(X, "dtype", "torch.float32")), SPMM_X_F32)


# X tensor types: FP32 values, BF16 values or raw 16-bit codes, E4M3 raw 8-bit codes
_X_TORCH_DTYPES = {"torch.float32": SPMM_X_F32, "torch.bfloat16": SPMM_X_BF16, "torch.uint16": SPMM_X_BF16,
                   "torch.int16": SPMM_X_BF16, "torch.uint8": SPMM_X_FP8_E4M3, "torch.int8": SPMM_X_FP8_E4M3,
                   "torch.float8_e4m3fn": SPMM_X_FP8_E4M3}


def _check_tensors(X, Y, dtype):
    """Shape/type checks for torch tensors (raw pointers pass through)."""
    if hasattr(X, "data_ptr") and hasattr(X, "dtype"):
        name = str(X.dtype)
        if name not in _X_TORCH_DTYPES:
            raise TypeError(f"X must be float32, bfloat16 (or 16-bit codes) or 8-bit E4M3 codes, not {name}")
        if dtype is not None and _X_TORCH_DTYPES[name] != dtype:
            raise TypeError(f"X dtype {name} does not match dtype={dtype}")
        if X.dim() != 2 or X.stride(1) != 1 or not X.is_cuda:
            raise ValueError("X must be a 2-D device tensor with unit column stride")
    if hasattr(Y, "data_ptr") and hasattr(Y, "dtype"):
        if str(Y.dtype) != "torch.float32" or Y.dim() != 2 or Y.stride(1) != 1 or not Y.is_cuda:
            raise ValueError("Y must be a 2-D float32 device tensor with unit column stride")


def spmm_run(h: Handle, X, Y, k: int | None = None, ldx: int | None = None, dtype: int | None = None,
             col_scale=None, ldy: int | None = None, stream=None):
    """Y = A X on the device.  X, Y: 2-D row-major device tensors (or pointers
    with k/ldx/ldy given); X's dtype selects F32/BF16/FP8 unless ``dtype``."""
    _check_tensors(X, Y, dtype)
    L = load_library()
    if k is None:
        k = X.shape[1]
    if ldx is None:
        ldx = X.stride(0)
    if ldy is None:
        ldy = Y.stride(0)
    st = L.spmm_run(h.ptr, _ptr(X), int(k), int(ldx), _xdtype(X, dtype), _ptr(col_scale), _ptr(Y),
                    int(ldy), _stream(stream, X))
    _check(st, "spmm_run")


def spmm_run_static(h: Handle, X, Y, k: int | None = None, ldx: int | None = None, dtype: int | None = None,
                    col_scale=None, ldy: int | None = None, stream=None):
    """spmm_run without device allocation (static scratch; see spmm.h):
    the handle must keep the given order and be on the device already."""
    _check_tensors(X, Y, dtype)
    L = load_library()
    if k is None:
        k = X.shape[1]
    if ldx is None:
        ldx = X.stride(0)
    if ldy is None:
        ldy = Y.stride(0)
    st = L.spmm_run_static(h.ptr, _ptr(X), int(k), int(ldx), _xdtype(X, dtype), _ptr(col_scale), _ptr(Y),
                           int(ldy), _stream(stream, X))
    _check(st, "spmm_run_static")


SPMM_QUANT_SCALES_GIVEN = 1


def spmm_quantize_x(X, Xq, dtype: int, col_scale=None, flags: int = 0, n: int | None = None,
                    k: int | None = None, ldx: int | None = None, ldq: int | None = None,
                    stream=None):
    """Quantise FP32 X (device) into BF16 / FP8-E4M3 codes in Xq (device)."""
    L = load_library()
    n = X.shape[0] if n is None else n
    k = X.shape[1] if k is None else k
    ldx = X.stride(0) if ldx is None else ldx
    ldq = Xq.stride(0) if ldq is None else ldq
    st = L.spmm_quantize_x(_ptr(X), int(n), int(k), int(ldx), int(dtype), _ptr(Xq), int(ldq),
                           _ptr(col_scale), int(flags), _stream(stream, X))
    _check(st, "spmm_quantize_x")


def spmm_stream_run(h: Handle, X, Y, compute=None, copy=None, k: int | None = None, ldx: int | None = None,
                    dtype: int | None = None, col_scale=None, ldy: int | None = None):
    """Y = A X with A streamed from pinned host memory (see spmm.h)."""
    _check_tensors(X, Y, dtype)
    L = load_library()
    k = X.shape[1] if k is None else k
    ldx = X.stride(0) if ldx is None else ldx
    ldy = Y.stride(0) if ldy is None else ldy
    st = L.spmm_stream_run(h.ptr, _ptr(X), int(k), int(ldx), _xdtype(X, dtype), _ptr(col_scale), _ptr(Y),
                           int(ldy), _stream(compute, X), _stream(copy))
    _check(st, "spmm_stream_run")


def spmm_stream_run_yhost(h: Handle, X, Y, compute=None, copy=None, out=None, k: int | None = None,
                          ldx: int | None = None, dtype: int | None = None, col_scale=None, ldy: int | None = None):
    """Y = A X with A streamed from pinned host memory and Y streamed back to
    pinned host memory as its tile rows finish (see spmm.h).  X: device
    tensor; Y: pinned host float32 tensor.  Y is complete once ``out`` (the
    device-to-host stream) has finished."""
    _check_tensors(X, None, dtype)
    if hasattr(Y, "data_ptr") and hasattr(Y, "dtype"):
        if str(Y.dtype) != "torch.float32" or Y.dim() != 2 or Y.stride(1) != 1 or Y.is_cuda or not Y.is_pinned():
            raise ValueError("Y must be a 2-D pinned host float32 tensor with unit column stride")
    L = load_library()
    k = X.shape[1] if k is None else k
    ldx = X.stride(0) if ldx is None else ldx
    ldy = Y.stride(0) if ldy is None else ldy
    st = L.spmm_stream_run_yhost(h.ptr, _ptr(X), int(k), int(ldx), _xdtype(X, dtype), _ptr(col_scale), _ptr(Y),
                                 int(ldy), _stream(compute, X), _stream(copy), _stream(out))
    _check(st, "spmm_stream_run_yhost")


SPMM_HOSTXY_BLOCKED = 1


def spmm_stream_run_host(h: Handle, X, Y, cols_per_block: int, k: int | None = None,
                         ldx: int | None = None, ldy: int | None = None, blocked: bool = False):
    """Y = A X with A, X and Y in (pinned) host memory, X/Y columns in blocks.

    Row-major 2-D X and Y by default; with ``blocked`` X and Y are 1-D host
    arrays holding the column blocks back to back (k must be given)."""
    for name, T in (("X", X), ("Y", Y)):
        if hasattr(T, "dtype") and (str(T.dtype) not in ("torch.float32", "float32") or
                                    getattr(T, "is_cuda", False) or (T.ndim != 2 and not blocked)):
            raise ValueError(f"{name} must be a float32 host array (2-D unless blocked)")

    def lead(T):
        return T.stride(0) if hasattr(T, "stride") and callable(T.stride) else T.strides[0] // 4
    if blocked:
        if k is None:
            raise ValueError("blocked layout needs k")
        ldx = ldy = 0
    else:
        k = X.shape[1] if k is None else k
        ldx = lead(X) if ldx is None else ldx
        ldy = lead(Y) if ldy is None else ldy
    st = load_library().spmm_stream_run_host(h.ptr, _ptr(X), int(k), int(ldx), _ptr(Y), int(ldy),
                                             int(cols_per_block), SPMM_HOSTXY_BLOCKED if blocked else 0)
    _check(st, "spmm_stream_run_host")


SPMM_PR_INIT_GIVEN, SPMM_PR_NO_REDISTRIBUTE, SPMM_PR_NO_GRAPH = 1, 2, 4


def spmm_pagerank(h: Handle, pr, iters: int = 30, damping: float = 0.85, flags: int = 0, stream=None):
    """PageRank on the device; returns the FP64 residual per iteration."""
    resid = np.zeros(max(iters, 1), dtype=np.float64)
    st = load_library().spmm_pagerank(h.ptr, float(damping), int(iters), int(flags), _ptr(pr),
                                      resid.ctypes.data, _stream(stream, pr))
    _check(st, "spmm_pagerank")
    return resid[:iters]


def spmm_nmf(hA: Handle, hAT: Handle, W, H, iters: int = 10, eps: float = 1e-9, stream=None):
    """NMF multiplicative updates on the device (W: n x r, H: m x r, in place)."""
    st = load_library().spmm_nmf(hA.ptr, hAT.ptr, int(W.shape[1]), int(iters), float(eps), _ptr(W), _ptr(H),
                                 _stream(stream, W))
    _check(st, "spmm_nmf")


def spmm_read_probe(buf, sink, nbytes: int | None = None, stream=None) -> None:
    """One streaming read of a device buffer (bandwidth measurement)."""
    nbytes = buf.numel() * buf.element_size() if nbytes is None else int(nbytes)
    st = load_library().spmm_read_probe(_ptr(buf), nbytes, _ptr(sink), _stream(stream, buf))
    _check(st, "spmm_read_probe")


def spmm_timing_begin(h: Handle) -> None:
    _check(load_library().spmm_timing_begin(h.ptr), "spmm_timing_begin")


def spmm_timing_end(h: Handle):
    """(summed SpMM-launch milliseconds, runs) since spmm_timing_begin."""
    ms, runs = ctypes.c_double(), ctypes.c_uint64()
    _check(load_library().spmm_timing_end(h.ptr, ctypes.addressof(ms), ctypes.addressof(runs)),
           "spmm_timing_end")
    return ms.value, runs.value


def spmm_get_stats(h: Handle) -> dict:
    s = spmm_stats_t()
    _check(load_library().spmm_get_stats(h.ptr, ctypes.byref(s)), "spmm_get_stats")
    d = {name: getattr(s, name) for name, _ in spmm_stats_t._fields_[:-2]}
    d["variant_tiles"] = list(s.variant_tiles)
    d["variant_nnz"] = list(s.variant_nnz)
    return d


def spmm_decode_tiles(h: Handle, nnz: int, weighted: bool = False):
    """CSR (row_ptr, col[, val]) rebuilt from the encoded work items."""
    rp = np.empty(h.n_rows + 1, dtype=np.int64)
    ci = np.empty(max(nnz, 1), dtype=np.int32)
    va = np.empty(max(nnz, 1), dtype=np.float32) if weighted else None
    st = load_library().spmm_decode_tiles(h.ptr, rp.ctypes.data, ci.ctypes.data,
                                          None if va is None else va.ctypes.data)
    _check(st, "spmm_decode_tiles")
    return (rp, ci[:nnz], va[:nnz]) if weighted else (rp, ci[:nnz])


def spmm_model_tiles(row_ptr, col_idx, t: int, n_cols: int | None = None):
    """(non-empty tiles, sum nnr, sum nnc) of the paper's t x t tiling."""
    rp = _host(row_ptr, np.int64)
    ci = _host(col_idx, np.int32)
    n_rows = rp.shape[0] - 1
    n_cols = n_rows if n_cols is None else int(n_cols)
    T, R, C = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
    st = load_library().spmm_model_tiles(n_rows, n_cols, rp.ctypes.data,
                                         None if ci.size == 0 else ci.ctypes.data, int(t),
                                         ctypes.byref(T), ctypes.byref(R), ctypes.byref(C))
    _check(st, "spmm_model_tiles")
    return T.value, R.value, C.value


# ------------------------------------------------------------- selection

def spmm_tile_features(h: Handle, k: int, dtype: int = SPMM_X_F32) -> np.ndarray:
    """Features of every tile, float32 [n_tiles, 8]."""
    T = spmm_get_stats(h)["n_tiles"]
    f = np.empty((max(T, 1), SPMM_NUM_FEATURES), dtype=np.float32)
    _check(load_library().spmm_tile_features(h.ptr, int(k), int(dtype), f.ctypes.data), "spmm_tile_features")
    return f[:T]


def spmm_get_variants(h: Handle) -> np.ndarray:
    T = spmm_get_stats(h)["n_tiles"]
    v = np.empty(max(T, 1), dtype=np.uint8)
    _check(load_library().spmm_get_variants(h.ptr, v.ctypes.data), "spmm_get_variants")
    return v[:T]


def spmm_set_variants(h: Handle, variants) -> None:
    v = _host(variants, np.uint8)
    T = spmm_get_stats(h)["n_tiles"]
    if v.shape != (T,):
        raise ValueError(f"need one variant per tile ({T})")
    _check(load_library().spmm_set_variants(h.ptr, v.ctypes.data if T else None), "spmm_set_variants")


def spmm_selector_collect(h: Handle, k: int, dtype: int = SPMM_X_F32, min_tiles: int = 0, reps: int = 0,
                          stream=None):
    """(bucket of every tile uint32[T], ns per tile float32[n_buckets, V])."""
    T = spmm_get_stats(h)["n_tiles"]
    b = np.empty(max(T, 1), dtype=np.uint32)
    nb = ctypes.c_uint32()
    ns = np.zeros((SPMM_MAX_BUCKETS, SPMM_NUM_VARIANTS), dtype=np.float32)
    o = spmm_tune_opts(int(min_tiles), int(reps))
    st = load_library().spmm_selector_collect(h.ptr, int(k), int(dtype), ctypes.byref(o), b.ctypes.data,
                                              ctypes.addressof(nb), ns.ctypes.data, _stream(stream))
    _check(st, "spmm_selector_collect")
    return b[:T], ns[:nb.value]


def spmm_autotune(h: Handle, k: int, dtype: int = SPMM_X_F32, min_tiles: int = 0, reps: int = 0, stream=None):
    """Exhaustive per-bucket autotune; returns the timing table [n_buckets, V]."""
    nb = ctypes.c_uint32()
    ns = np.zeros((SPMM_MAX_BUCKETS, SPMM_NUM_VARIANTS), dtype=np.float32)
    o = spmm_tune_opts(int(min_tiles), int(reps))
    st = load_library().spmm_autotune(h.ptr, int(k), int(dtype), ctypes.byref(o), ctypes.addressof(nb),
                                      ns.ctypes.data, _stream(stream))
    _check(st, "spmm_autotune")
    return ns[:nb.value]


def spmm_mlp_init(seed: int) -> np.ndarray:
    p = np.empty(SPMM_MLP_PARAMS, dtype=np.float32)
    _check(load_library().spmm_mlp_init(ctypes.c_uint64(int(seed) & (2**64 - 1)), p.ctypes.data), "spmm_mlp_init")
    return p


def spmm_mlp_predict(params, feat, out=None, choice=None, n: int | None = None, stream=None):
    """Device inference: predicted log time per variant and/or the argmin."""
    n = int(feat.shape[0]) if n is None else int(n)
    st = load_library().spmm_mlp_predict(_ptr(params), _ptr(feat), n, _ptr(out), _ptr(choice),
                                         _stream(stream, feat))
    _check(st, "spmm_mlp_predict")


def spmm_mlp_grad(params, feat, target, mask, grad, loss=None, n: int | None = None, stream=None):
    """Device masked-MSE gradient (and loss) of the cost model."""
    n = int(feat.shape[0]) if n is None else int(n)
    st = load_library().spmm_mlp_grad(_ptr(params), _ptr(feat), _ptr(target), _ptr(mask), n, _ptr(grad),
                                      _ptr(loss), _stream(stream, feat))
    _check(st, "spmm_mlp_grad")


def spmm_mlp_adam(params, m, v, grad, t: int, lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999,
                  eps: float = 1e-8, stream=None):
    st = load_library().spmm_mlp_adam(_ptr(params), _ptr(m), _ptr(v), _ptr(grad), int(t), float(lr),
                                      float(beta1), float(beta2), float(eps), _stream(stream, params))
    _check(st, "spmm_mlp_adam")


def spmm_selector_train(feat, target, mask=None, params=None, *, epochs: int = 0, batch: int = 0,
                        lr: float = 0.0, seed: int = 0):
    """Train the cost model on the GPU; returns (params, mean loss per epoch)."""
    f = _host(feat, np.float32)
    y = _host(target, np.float32)
    m = _host(mask, np.uint8)
    p = spmm_mlp_init(seed) if params is None else np.array(params, dtype=np.float32, copy=True)
    o = spmm_train_opts(int(epochs), int(batch), float(lr), int(seed) & (2**64 - 1))
    ne = o.epochs or 30
    trace = np.zeros(ne, dtype=np.float64)
    st = load_library().spmm_selector_train(f.ctypes.data, y.ctypes.data, None if m is None else m.ctypes.data,
                                            int(f.shape[0]), ctypes.byref(o), p.ctypes.data, trace.ctypes.data)
    _check(st, "spmm_selector_train")
    return p, trace


def spmm_select_learned(h: Handle, params, k: int, dtype: int = SPMM_X_F32) -> None:
    p = _host(params, np.float32)
    _check(load_library().spmm_select_learned(h.ptr, p.ctypes.data, int(k), int(dtype)), "spmm_select_learned")


def spmm_eigs(h: Handle, nev: int, *, block: int = 4, max_dim: int = 0, which: str = "LM", tol: float = 0.0,
              max_restarts: int = 0, seed: int = 1, evecs=None, stream=None, check: bool = True):
    """Eigenpairs of a symmetric A by the block Krylov-Schur method.

    evecs: device float32 tensor n x nev (row-major) for the Ritz vectors, or
    None.  Returns (evals, resid, info): evals and resid are float64 arrays in
    the order of the wanted end ("LM", "LA" or "SA"), resid the relative
    residual estimates.  With check=False a run that stops before converging
    (SPMM_ENOTCONV) returns its current Ritz pairs instead of raising.
    """
    if which not in _WHICH:
        raise ValueError(f"which must be one of {sorted(_WHICH)}")
    o = spmm_eigs_opts(nev=int(nev), block=int(block), max_dim=int(max_dim), which=_WHICH[which],
                       max_restarts=int(max_restarts), reserved=0, tol=float(tol), seed=int(seed) & (2 ** 64 - 1))
    evals = np.zeros(max(int(nev), 0), dtype=np.float64)
    resid = np.zeros_like(evals)
    info = spmm_eigs_info()
    ldvec = 0
    if evecs is not None:
        if hasattr(evecs, "shape"):
            if tuple(evecs.shape[:1]) != (h.n_rows,) or evecs.shape[1] < nev or evecs.stride(1) != 1:
                raise ValueError("evecs must be n x (>= nev) with unit column stride")
            if str(evecs.dtype) != "torch.float32" or not evecs.is_cuda:
                raise TypeError("evecs must be a float32 device tensor")
            ldvec = int(evecs.stride(0))
        else:
            ldvec = int(nev)
    st = load_library().spmm_eigs(h.ptr, ctypes.byref(o), evals.ctypes.data, _ptr(evecs), ldvec,
                                  resid.ctypes.data, ctypes.byref(info), _stream(stream, evecs))
    if st != SPMM_OK and not (st == SPMM_ENOTCONV and not check):
        _check(st, "spmm_eigs")
    return evals, resid, {f: getattr(info, f) for f, _ in spmm_eigs_info._fields_}


def spmm_sym_eig_small(a):
    """All eigenpairs of a small dense symmetric matrix (cyclic Jacobi, host):
    (w ascending, z with unit eigenvectors in its columns)."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    n = a.shape[0]
    if a.shape != (n, n):
        raise ValueError("a must be square")
    w = np.zeros(n)
    z = np.zeros((n, n))
    _check(load_library().spmm_sym_eig_small(n, a.ctypes.data, w.ctypes.data, z.ctypes.data), "spmm_sym_eig_small")
    return w, z


def spmm_dense_tn_workspace(n: int, p: int, q: int) -> int:
    return int(load_library().spmm_dense_tn_workspace(int(n), int(p), int(q)))


def spmm_dense_tn(A, B, C, work, p: int | None = None, q: int | None = None, stream=None) -> None:
    """C = A^T B (FP64) for device FP32 row-major A (n x >= p) and B (n x >= q)."""
    p = A.shape[1] if p is None else p
    q = B.shape[1] if q is None else q
    n = A.shape[0]
    lda, ldb = (int(A.stride(0)), int(B.stride(0))) if n > 0 else (p, q)     # no rows: any stride
    st = load_library().spmm_dense_tn(_ptr(A), lda, int(p), _ptr(B), ldb, int(q), int(n),
                                      _ptr(C), _ptr(work), int(work.numel() * work.element_size()),
                                      _stream(stream, A))
    _check(st, "spmm_dense_tn")


def spmm_dense_nn(A, C, W, alpha: float = 0.0, beta: float = 1.0, p: int | None = None, q: int | None = None,
                  stream=None) -> None:
    """W = alpha W + beta A C for device FP32 A (n x >= p), FP64 C (p x q), FP32 W (n x >= q)."""
    p = A.shape[1] if p is None else p
    q = W.shape[1] if q is None else q
    lda, ldw = (int(A.stride(0)), int(W.stride(0))) if A.shape[0] > 0 else (p, q)
    st = load_library().spmm_dense_nn(_ptr(A), lda, int(p), _ptr(C), int(q), float(alpha), float(beta),
                                      _ptr(W), ldw, int(A.shape[0]), _stream(stream, A))
    _check(st, "spmm_dense_nn")
