"""Host-side checks of the general parallel loop: the ParallelLoop builder's
programs, the C ABI's validation of loop bodies, and that the HIP source the
library generates for a body compiles for gfx950 with hipRTC (no GPU needed)."""
import ctypes

import numpy as np
import pytest
import torch

import paper_2211_00621_amd as mx
from test_expr_host import _hiprtc

abi, api = mx.abi, mx.api


def _every_op_loop(fdt):
    lp = api.ParallelLoop([(torch.float32, 2), (torch.int32, 1), (torch.float64, 3), (torch.int64, 1)], fdt)
    i = lp.iteration
    r, c = i // 7, i % 7
    k = lp.get(1, i)
    x = lp.get(0, r, c)
    y = lp.get(2, r, c, k % 3)
    z = lp.binary(abi.MX_X_MAX, x, y) - lp.binary(abi.MX_X_MIN, x * y, 0.5) / (x + 2.0)
    for op in (abi.MX_X_NEG, abi.MX_X_ABS, abi.MX_X_SQ, abi.MX_X_EXP):
        z = lp.unary(op, z)
    z = lp.unary(abi.MX_X_LOG, lp.unary(abi.MX_X_SQRT, z + 1.0)) + lp.unary(abi.MX_X_RSQRT, z + 1.0)
    lp.set(0, (r, c), z + (-k).to_float())
    m = lp.binary(abi.MX_L_IMAX, lp.binary(abi.MX_L_IMIN, k * 3 - 1, 100), -100)
    lp.set(3, i, m)
    lp.set(1, i, k + 1)
    return lp


@pytest.mark.parametrize("fdt", [torch.float32, torch.float64])
def test_generated_loop_source_compiles_for_gfx950(fdt):
    rtc = _hiprtc()
    src = _every_op_loop(fdt).source().encode()
    assert b"mx_loop_0" in src and b"mx_loop_1" in src and b"mx_loop_2" in src and b"atomicCAS" in src
    prog = ctypes.c_void_p()
    assert rtc.hiprtcCreateProgram(ctypes.byref(prog), src, b"mx_loop.hip", 0, None, None) == 0
    opts = [b"--offload-arch=gfx950", b"-O3", b"-ffp-contract=off", b"-Xclang", b"-target-feature", b"-Xclang",
            b"-packed-fp32-ops"]
    arr = (ctypes.c_char_p * len(opts))(*opts)
    rc = rtc.hiprtcCompileProgram(prog, len(opts), arr)
    size = ctypes.c_size_t()
    rtc.hiprtcGetProgramLogSize(prog, ctypes.byref(size))
    log = ctypes.create_string_buffer(size.value + 1)
    rtc.hiprtcGetProgramLog(prog, log)
    assert rc == 0, log.value.decode(errors="replace")
    rtc.hiprtcGetCodeSize(prog, ctypes.byref(size))
    assert size.value > 1000
    rtc.hiprtcDestroyProgram(ctypes.byref(prog))


def L(op, dst=0, a=0, b=0, c=0, src=0, tensor=0, iimm=0, fimm=0.0):
    return (op, dst, a, b, c, src, tensor, iimm, fimm)


def test_loop_create_rejects_malformed_bodies():
    f1 = [(abi.MX_F32, 1)]
    good = [L(abi.MX_L_ITER, 0), L(abi.MX_L_FGET, 0, a=0, tensor=0), L(abi.MX_L_FSET, a=0, src=0, tensor=0)]
    abi.mx_loop_create(good, f1, abi.MX_F32)
    bad = [
        ([L(99)], f1, abi.MX_F32),                                              # unknown op
        ([L(abi.MX_L_ITER, 64)], f1, abi.MX_F32),                               # register out of range
        ([L(abi.MX_L_FGET, 0, tensor=1)], f1, abi.MX_F32),                      # no such tensor
        ([L(abi.MX_L_IGET, 0, tensor=0)], f1, abi.MX_F32),                      # int get of a float tensor
        ([L(abi.MX_L_FSET, src=70, tensor=0)], f1, abi.MX_F32),                 # bad src
        (good, [(abi.MX_F32, 4)], abi.MX_F32),                                  # rank 4
        (good, f1, abi.MX_I32),                                                 # float type
        ([L(abi.MX_X_IN, 0)], f1, abi.MX_F32),                                  # map-body input op
        ([L(abi.MX_L_ITER, 0)] * 257, f1, abi.MX_F32),                          # too long
    ]
    for prog, types, fdt in bad:
        with pytest.raises(abi.MxError):
            abi.mx_loop_create(prog, types, fdt)


def test_builder_rejects_kind_mixing_and_rank_mismatch():
    lp = api.ParallelLoop([(torch.float32, 2), (torch.int64, 1)])
    i = lp.iteration
    with pytest.raises(TypeError):
        _ = i + lp.get(0, i, i)
    with pytest.raises(ValueError):
        lp.get(0, i)
    with pytest.raises(TypeError):
        lp.set(1, i, lp.get(0, i, i))
    with pytest.raises(TypeError):
        _ = i / 2
