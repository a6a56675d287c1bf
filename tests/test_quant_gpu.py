"""GPU X quantisers and reduced-precision SpMM against the oracle.

Encoders must match the oracle bit for bit (exhaustively over all 2^32 FP32
inputs); FP8/BF16 SpMM must match A * deq(X_q) in FP64 within 1e-6 and the
FP32 reference within the stated dtype bars (1e-2 BF16, 6e-2 FP8)."""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
import paper_1602_02864_amd as pk
import synth
from gpu_util import run_spmm

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


def _quant_gpu(X, dt, scales=None):
    torch = _torch()
    Xd = torch.from_numpy(np.ascontiguousarray(X, np.float32)).cuda()
    n, k = X.shape
    Q = torch.empty((n, k), dtype=torch.uint16 if dt == pk.SPMM_X_BF16 else torch.uint8, device="cuda")
    sc = None
    flags = 0
    if dt == pk.SPMM_X_FP8_E4M3:
        if scales is None:
            sc = torch.full((k,), -1.0, device="cuda")
        else:
            sc = torch.from_numpy(np.asarray(scales, np.float32)).cuda()
            flags = pk.SPMM_QUANT_SCALES_GIVEN
    pk.spmm_quantize_x(Xd, Q, dt, col_scale=sc, flags=flags)
    torch.cuda.synchronize()
    return Q.cpu().numpy(), (None if sc is None else sc.cpu().numpy())


def _test_matrix(n=20000, k=7):
    X = synth.uniform(n, k, seed=3) * 8 - 4          # signs, several binades
    X[:, 2] *= 1e-3                                   # FP8 subnormal region after scaling
    X[:, 5] = 0.0                                     # zero column -> scale 1
    X[7, 1] = 2.0 ** -140                             # FP32 denormal
    X[11, 3] = -1e30
    return X


def test_bf16_quantize_bit_exact():
    X = _test_matrix()
    Q, _ = _quant_gpu(X, pk.SPMM_X_BF16)
    assert np.array_equal(Q, oracle.bf16_quantize(X))


def test_fp8_scales_and_codes_bit_exact():
    X = _test_matrix()
    Q, s = _quant_gpu(X, pk.SPMM_X_FP8_E4M3)
    s_ref = oracle.fp8_colscale(X)
    assert np.array_equal(s.view(np.uint32), s_ref.view(np.uint32))
    assert np.array_equal(Q, oracle.fp8_quantize(X, s_ref))


def test_encoders_exhaustive_all_fp32_inputs():
    """Every FP32 bit pattern through the GPU encoders (scale 1) == oracle."""
    torch = _torch()
    chunk = 1 << 27
    pool = ThreadPoolExecutor(16)

    def ref(fn, x):
        parts = np.array_split(x, 16)
        return np.concatenate(list(pool.map(fn, parts)))

    one = torch.ones(1, device="cuda")
    for start in range(0, 1 << 32, chunk):
        bits = (torch.arange(start, start + chunk, dtype=torch.int64, device="cuda") - (1 << 31)).to(torch.int32)
        xs = bits.view(torch.float32).view(chunk, 1)
        q8 = torch.empty((chunk, 1), dtype=torch.uint8, device="cuda")
        q16 = torch.empty((chunk, 1), dtype=torch.uint16, device="cuda")
        pk.spmm_quantize_x(xs, q8, pk.SPMM_X_FP8_E4M3, col_scale=one, flags=pk.SPMM_QUANT_SCALES_GIVEN)
        pk.spmm_quantize_x(xs, q16, pk.SPMM_X_BF16)
        host = (np.arange(start, start + chunk, dtype=np.int64) - (1 << 31)).astype(np.int32).view(np.float32)
        got8 = q8.cpu().numpy().ravel()
        got16 = q16.cpu().numpy().ravel()
        assert np.array_equal(got8, ref(oracle.e4m3_encode, host)), start
        assert np.array_equal(got16, ref(oracle.bf16_encode, host)), start


def _perm_csr(n, seed):
    p = synth.draws(synth.stream_key(seed, 13), 0, n).argsort().astype(np.int32)
    return np.arange(n + 1, dtype=np.int64), p


def test_fp8_and_bf16_decode_exact_through_spmm():
    """A = permutation: Y = deq(X_q) exactly, covering every finite code."""
    n = 4096
    rp, col = _perm_csr(n, 1)
    codes8 = np.array([c for c in range(256) if c not in (0x7F, 0xFF)], np.uint8)
    Xq8 = np.resize(codes8, (n, 4)).copy()
    h = pk.spmm_build_tiles(rp, col)
    Y = run_spmm(h, Xq8, dtype=pk.SPMM_X_FP8_E4M3, col_scale=np.ones(4, np.float32))
    want = oracle.e4m3_decode(Xq8.ravel()).reshape(n, 4)[col]
    assert np.array_equal(Y, want)
    # BF16 codes with exponent fields 100..149 (|x| in [2^-27, 2^23)): the
    # fixed-point accumulator represents every value within 2^54 of a
    # column's bound exactly, so the decode must come through bit-exact
    d = synth.draws(synth.stream_key(5, 14), 0, n * 4)
    sign = ((d >> np.uint64(63)) << np.uint64(15)).astype(np.uint16)
    expo = (100 + (d >> np.uint64(8)) % np.uint64(50)).astype(np.uint16) << np.uint16(7)
    frac = (d & np.uint64(0x7F)).astype(np.uint16)
    Xq16 = (sign | expo | frac).reshape(n, 4)
    Y = run_spmm(h, Xq16, dtype=pk.SPMM_X_BF16)
    want = oracle.bf16_decode(Xq16.ravel()).reshape(n, 4)[col]
    assert np.array_equal(Y, want)


def _elementwise_ok(Y, ref, rp, where):
    """Non-negative terms: any FP32 summation order of a row of L terms is
    within (L + 2) * 2^-24 of the row's exact value, relatively."""
    L = np.diff(rp).astype(np.float64)[:, None]
    bound = (L + 2.0) * 2.0 ** -24 * np.abs(ref)
    bad = np.abs(Y.astype(np.float64) - ref) > bound
    assert not bad.any(), (where, int(bad.sum()))


@pytest.mark.parametrize("item_nnz", [0, 100])
@pytest.mark.parametrize("k", [1, 4, 16, 33, 64])
def test_reduced_precision_spmm_bars(k, item_nnz):
    """BF16 and scaled FP8 X: against the oracle on the dequantised X
    (kernel error only) element by element and at 1e-6 in Frobenius norm,
    and against the FP32 X (quantisation included) at 1e-2 / 6e-2.  With
    item_nnz = 100 every row longer than 100 entries is split across work
    items, so the split-row combine and its FP8 output scaling are used."""
    rp, col = synth.rmat_csr(16, 16, seed=1, symmetrize=True)
    n = rp.shape[0] - 1
    val = synth.lognormal_weights(rp, col, seed=3)
    X = synth.uniform(n, k, seed=2)
    for weighted in (False, True):
        v = val if weighted else None
        h = pk.spmm_build_tiles(rp, col, v, item_nnz=item_nnz)
        if item_nnz:
            assert pk.spmm_get_stats(h)["n_parts"] > 0
        ref_total = oracle.spmm(rp, col, v, X)
        # BF16
        Q, _ = _quant_gpu(X, pk.SPMM_X_BF16)
        Y = run_spmm(h, Q, dtype=pk.SPMM_X_BF16)
        ref_k = oracle.spmm(rp, col, v, oracle.dequant(Q, "bf16"))
        assert oracle.frob_rel_err(Y, ref_k) <= 1e-6
        _elementwise_ok(Y, ref_k, rp, ("bf16", weighted))
        e_bf16 = oracle.frob_rel_err(Y, ref_total)
        assert e_bf16 <= 1e-2
        # FP8 with per-column scales
        Q8, s = _quant_gpu(X, pk.SPMM_X_FP8_E4M3)
        Y8 = run_spmm(h, Q8, dtype=pk.SPMM_X_FP8_E4M3, col_scale=s)
        ref_k8 = oracle.spmm(rp, col, v, oracle.dequant(Q8, "fp8", s))
        assert oracle.frob_rel_err(Y8, ref_k8) <= 1e-6
        _elementwise_ok(Y8, ref_k8, rp, ("fp8", weighted))
        e_fp8 = oracle.frob_rel_err(Y8, ref_total)
        assert e_fp8 <= 6e-2
        h.close()
