"""Ordering of the streamed-SpMM transfer ring, checked on the CPU.

* The library's slot/event plan (csrc/stream_plan.h, the asynchronous read
  ahead of Algorithm 1 in Sections 3.1 and 3.5) is run against a recorder
  with vector clocks over the copy and compute streams
  (tests/helpers/stream_plan_check.cpp): over back-to-back calls every copy
  into a slot must follow every kernel that read the slot before it, and
  every kernel must follow the copy of its own group.  A plan that waits
  for a slot only from the R-th group of a call on (the ordering the ring
  had before the "slot used" state was kept across calls) must fail the
  same check as soon as two calls follow each other.
* The same with Y streamed out to host memory (a third stream copies each
  group's finished rows out of a device Y slot).
* What a kernel would gather from a slot overwritten too early: the
  library's builder, compiled with g++ (tests/helpers/stream_cross_decode.cpp),
  decodes one transfer group's work items against another group's payload;
  the X rows read then fall outside X, which on the GPU is an illegal
  memory access.  Against its own payload every gather is in range.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import synth

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1602_02864_amd", "csrc")
HELP = os.path.join(HERE, "helpers")


@pytest.fixture(scope="module")
def plan_lib(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("plan") / "libplan.so")
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-I", CSRC,
                           os.path.join(HELP, "stream_plan_check.cpp"), "-o", out])
    L = ctypes.CDLL(out)
    for f in (L.stream_plan_violations, L.legacy_plan_violations, L.yout_plan_violations,
              L.yout_nowait_plan_violations):
        f.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int]
        f.restype = ctypes.c_int
    return L


@pytest.fixture(scope="module")
def decode_lib(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("xdec") / "libxdec.so")
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-pthread",
                           "-I", os.path.join(HELP, "eigs_host"), "-I", os.path.join(ROOT, "include"), "-I", CSRC,
                           os.path.join(HELP, "stream_cross_decode.cpp"), os.path.join(CSRC, "builder.cpp"),
                           "-o", out])
    L = ctypes.CDLL(out)
    L.cross_decode.restype = ctypes.c_int64
    L.cross_decode.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32,
                               ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p]
    return L


@pytest.mark.parametrize("groups,ring", [(1, 2), (2, 2), (5, 2), (7, 3), (16, 4), (40, 16), (3, 16)])
def test_ring_plan_orders_every_copy_after_its_readers(plan_lib, groups, ring):
    for calls in (1, 2, 4):
        assert plan_lib.stream_plan_violations(groups, ring, calls) == 0, calls


@pytest.mark.parametrize("groups,ring", [(1, 2), (2, 2), (5, 2), (7, 3), (16, 4), (40, 16), (3, 16)])
def test_y_out_plan_orders_kernels_and_copy_outs(plan_lib, groups, ring):
    """Y streamed out through per-slot device buffers: kernels writing a Y
    slot follow the earlier copy-outs of that slot, and each copy-out
    follows its group's kernels -- within a call and across calls.  Without
    the wait for the previous copy-out the check fails."""
    for calls in (1, 2, 4):
        assert plan_lib.yout_plan_violations(groups, ring, calls) == 0, calls
    if groups > ring:
        assert plan_lib.yout_nowait_plan_violations(groups, ring, 1) > 0
    assert plan_lib.yout_nowait_plan_violations(groups, ring, 2) > 0


@pytest.mark.parametrize("groups,ring", [(1, 2), (2, 2), (5, 2), (7, 3), (40, 16)])
def test_per_call_ring_waits_race_across_calls(plan_lib, groups, ring):
    """Waiting on a slot only for g >= R is enough within one call, and
    lets the next call's first copies overtake the previous call's kernels."""
    assert plan_lib.legacy_plan_violations(groups, ring, 1) == 0
    assert plan_lib.legacy_plan_violations(groups, ring, 2) > 0
    assert plan_lib.legacy_plan_violations(groups, ring, 4) > 0


def test_overwritten_slot_gathers_outside_x(decode_lib):
    """The configuration of the back-to-back GPU test (scale 15, 32 KiB
    groups): each group decoded against its own payload stays inside X;
    decoded against the payload another group leaves in the slot it
    gathers X rows far outside X."""
    rp, col = synth.rmat_csr(15, 16, seed=10)
    n = rp.shape[0] - 1
    out = np.zeros(6, np.uint64)
    args = (n, rp.ctypes.data, col.ctypes.data, 32, 16384, 32 * 1024)
    ng = decode_lib.cross_decode(*args, -1, -1, out.ctypes.data)
    assert ng >= 4
    for ga, gb in ((0, 1), (1, 0), (2, ng - 1), (ng - 1, 0)):
        assert decode_lib.cross_decode(*args, ga, gb, out.ctypes.data) == ng
        assert out[0] > 0 and out[1] == 0 and out[2] == 0, (ga, out)
        assert out[4] > 0, (ga, gb, out)
