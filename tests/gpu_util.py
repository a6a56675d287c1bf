"""Helpers shared by the GPU tests (device tensors in, numpy out)."""
import numpy as np

import paper_1602_02864_amd as pk


def dev():
    import torch
    return torch.device("cuda:0")


def run_spmm(h, X: np.ndarray, k=None, dtype=None, col_scale=None, fill=float("nan"),
             ldy=None):
    """Y = A X through the C ABI; X is a host array (any dtype the ABI takes)."""
    import torch
    Xd = torch.from_numpy(np.ascontiguousarray(X)).to(dev())
    k = X.shape[1] if k is None else k
    ldy = k if ldy is None else ldy
    Yd = torch.full((h.n_rows, ldy), fill, dtype=torch.float32, device=dev())
    sc = None if col_scale is None else torch.from_numpy(np.asarray(col_scale, np.float32)).to(dev())
    pk.spmm_run(h, Xd, Yd, k=k, ldx=X.shape[1], dtype=dtype, col_scale=sc, ldy=ldy)
    torch.cuda.synchronize()
    return Yd.cpu().numpy()


def transpose_csr(row_ptr, col, val, n_cols):
    """CSR of A^T with sorted columns (input preparation for the tests)."""
    row_ptr = np.asarray(row_ptr, np.int64)
    n_rows = row_ptr.shape[0] - 1
    rows = np.repeat(np.arange(n_rows, dtype=np.int64), np.diff(row_ptr))
    order = np.lexsort((rows, np.asarray(col, np.int64)))
    t_ptr = np.concatenate([[0], np.cumsum(np.bincount(col, minlength=n_cols))]).astype(np.int64)
    return t_ptr, rows[order].astype(np.int32), None if val is None else np.asarray(val, np.float32)[order]
