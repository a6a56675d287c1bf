"""Pins for the oracle's X quantisers (BF16, OCP FP8-E4M3 with per-column
scale).  Exhaustive over all FP32 inputs against a brute-force nearest-code
search, plus code values fixed by the OCP FP8 specification."""
import math
import os
import subprocess

import numpy as np
import pytest

import oracle
import synth

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def brute_exe(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("qb") / "quant_brute")
    odir = os.path.dirname(oracle.build())
    subprocess.check_call(["gcc", "-O2", "-fopenmp", os.path.join(HERE, "helpers", "quant_brute.c"),
                           "-o", exe, "-L", odir, "-loracle", "-Wl,-rpath," + odir, "-lm"])
    return exe


@pytest.mark.parametrize("fmt", ["bf16", "e4m3"])
def test_encoder_exhaustive(brute_exe, fmt):
    out = subprocess.run([brute_exe, fmt], capture_output=True, text=True, timeout=600, check=True)
    assert int(out.stdout.strip()) == 0


def test_e4m3_spec_values():
    """Code points fixed by the OCP 8-bit FP spec (E4M3: bias 7, no inf)."""
    v = {c: float(oracle.e4m3_decode(np.array([c], np.uint8))[0]) for c in range(256)}
    assert v[0x00] == 0.0 and math.copysign(1, v[0x80]) < 0
    assert v[0x01] == 2.0 ** -9           # smallest subnormal
    assert v[0x07] == 7 * 2.0 ** -9       # largest subnormal
    assert v[0x08] == 2.0 ** -6           # smallest normal
    assert v[0x38] == 1.0                 # exponent field 7 = bias
    assert v[0x7E] == 448.0               # largest finite
    assert v[0xFE] == -448.0
    assert math.isnan(v[0x7F]) and math.isnan(v[0xFF])
    assert v[0x77] == 240.0               # S.1110.111 = 1.875 * 2^7
    finite = [v[c] for c in range(0x7F)]
    assert all(b > a for a, b in zip(finite, finite[1:]))   # monotone codes


def test_e4m3_encode_decode_roundtrip():
    codes = np.array([c for c in range(256) if c not in (0x7F, 0xFF)], np.uint8)
    vals = oracle.e4m3_decode(codes)
    back = oracle.e4m3_encode(vals)
    # -0 and +0 both valid encodings of zero
    assert np.array_equal(back[vals != 0], codes[vals != 0])


def test_bf16_roundtrip_and_ties():
    h = np.arange(0, 0x7F80, 7, dtype=np.uint16)
    assert np.array_equal(oracle.bf16_encode(oracle.bf16_decode(h)), h)
    one_plus_half_ulp = np.frombuffer(np.uint32(0x3F808000).tobytes(), np.float32)
    assert oracle.bf16_encode(one_plus_half_ulp)[0] == 0x3F80    # tie -> even
    nxt = np.frombuffer(np.uint32(0x3F818000).tobytes(), np.float32)
    assert oracle.bf16_encode(nxt)[0] == 0x3F82                  # tie -> even (up)


def test_fp8_colscale_and_quantize():
    X = synth.uniform(1000, 6, seed=2)
    X[:, 3] = 0.0
    X[5, 1] = -3.5
    s = oracle.fp8_colscale(X)
    absmax = np.abs(X).max(axis=0)
    assert s[3] == 1.0
    for j in (0, 1, 2, 4, 5):
        assert s[j] == np.float32(448.0) / absmax[j]
    Q = oracle.fp8_quantize(X, s)
    d = oracle.dequant(Q, "fp8", s)
    # every non-zero entry within half a relative FP8 step (2^-4) of X
    rel = np.abs(d - X) / np.maximum(np.abs(X), 1e-30)
    big = np.abs(X * s[None, :]) >= 2 ** -6
    assert np.all(rel[big] <= 2.0 ** -4 + 1e-12)
    assert np.max(np.abs(d[:, 1])) == 3.5           # absmax maps to 448 exactly


def test_bf16_quantize_error_bound():
    X = synth.uniform(5000, 4, seed=7)
    d = oracle.dequant(oracle.bf16_quantize(X), "bf16")
    nz = X != 0
    # 8 significant bits: unit roundoff u = 2^-8, |x - bf16(x)| <= u/(1+u) |x|
    u = 2.0 ** -8
    assert np.all(np.abs(d - X)[nz] / X[nz] <= u / (1 + u) + 1e-15)
