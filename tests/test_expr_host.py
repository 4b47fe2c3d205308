"""User-defined map bodies, host side (no GPU): program checks at creation,
the lowering of written expressions to register programs, and the generated
HIP source compiling for gfx950 with hipRTC (the same compiler the library
calls at run time)."""
import ctypes
import os

import numpy as np
import pytest

import oracle as O
from paper_2211_00621_amd import abi, api

X = abi


def IN(d, k): return (X.MX_X_IN, d, k, 0, 0.0)
def CONST(d, v): return (X.MX_X_CONST, d, 0, 0, v)
def OP(op, d, a, b=0): return (op, d, a, b, 0.0)


ALL_OPS = [IN(0, 0), IN(1, 1), IN(2, 2), OP(X.MX_X_SUB, 3, 0, 1), OP(X.MX_X_SQ, 3, 3), OP(X.MX_X_NEG, 3, 3),
           OP(X.MX_X_EXP, 3, 3), CONST(4, 0.5), OP(X.MX_X_MUL, 3, 3, 4), OP(X.MX_X_DIV, 5, 0, 2),
           OP(X.MX_X_SQRT, 6, 2), OP(X.MX_X_RSQRT, 7, 2), OP(X.MX_X_LOG, 8, 2), OP(X.MX_X_ABS, 9, 5),
           OP(X.MX_X_MIN, 10, 9, 6), OP(X.MX_X_MAX, 10, 10, 7), OP(X.MX_X_ADD, 3, 3, 10), OP(X.MX_X_ADD, 3, 3, 8)]


@pytest.mark.parametrize("prog,nin,out,dtype,status", [
    ([], 1, 0, abi.MX_F32, abi.MX_ERR_INVALID),                                   # empty
    ([IN(0, 0), OP(X.MX_X_ADD, 1, 0, 2)], 1, 1, abi.MX_F32, abi.MX_ERR_INVALID),  # r2 read before written
    ([IN(0, 1)], 1, 0, abi.MX_F32, abi.MX_ERR_INVALID),                           # input 1 of 1
    ([IN(0, 0)], 1, 3, abi.MX_F32, abi.MX_ERR_INVALID),                           # out_reg never written
    ([IN(16, 0)], 1, 0, abi.MX_F32, abi.MX_ERR_INVALID),                          # register out of range
    ([(15, 0, 0, 0, 0.0)], 1, 0, abi.MX_F32, abi.MX_ERR_INVALID),                 # unknown op
    ([IN(0, 0)], 5, 0, abi.MX_F32, abi.MX_ERR_INVALID),                           # too many inputs
    ([IN(0, 0)], 1, 0, abi.MX_I32, abi.MX_ERR_DTYPE),                             # integer element type
    ([IN(0, 0)] * 65, 1, 0, abi.MX_F32, abi.MX_ERR_INVALID),                      # too long
])
def test_create_rejects_bad_programs(prog, nin, out, dtype, status):
    with pytest.raises(abi.MxError) as e:
        abi.mx_expr_create(prog, nin, out, dtype)
    assert e.value.status == status


def test_lowering_reuses_registers_and_keeps_the_value():
    a, b, c = api.body_inputs(3)
    t = a * b
    f = api.exp(-(a - b) ** 2) * 0.5 + t / (c + 1.0) - abs(t) + api.sqrt(c) * api.rsqrt(c) + api.log(c)
    f = api.minimum(f, 100.0) + api.maximum(a, b)
    prog, out = api.lower_body(f)
    assert max(p[1] for p in prog) < 16
    rng = np.random.default_rng(1)
    xa, xb, xc = rng.uniform(-1, 1, 50), rng.uniform(-1, 1, 50), rng.uniform(0.5, 2, 50)
    ref = (np.exp(-(xa - xb) ** 2) * 0.5 + xa * xb / (xc + 1.0) - np.abs(xa * xb) + np.sqrt(xc) / np.sqrt(xc)
           + np.log(xc))
    ref = np.minimum(ref, 100.0) + np.maximum(xa, xb)
    assert np.allclose(O.expr_map(prog, out, xa, xb, xc), ref, rtol=1e-14, atol=1e-14)
    abi.mx_expr_create(prog, 3, out, abi.MX_F32)  # accepted by the library's checks


def test_lowering_deep_chain_fits_the_registers():
    (a,) = api.body_inputs(1)
    v = a
    for i in range(21):
        v = v * 0.99 + a
    prog, out = api.lower_body(v)
    assert len(prog) == 64 and max(p[1] for p in prog) < 16
    abi.mx_expr_create(prog, 1, out, abi.MX_F32)
    with pytest.raises(abi.MxError):
        api.Body((v * 0.99 + a), 1)  # 67 instructions


def _hiprtc():
    for path in ("/opt/rocm/lib/libhiprtc.so", "libhiprtc.so"):
        try:
            return ctypes.CDLL(path)
        except OSError:
            continue
    pytest.skip("libhiprtc is not available")


@pytest.mark.parametrize("dtype", [abi.MX_F32, abi.MX_F64])
def test_generated_source_compiles_for_gfx950(dtype):
    rtc = _hiprtc()
    e = abi.mx_expr_create(ALL_OPS, 3, 3, dtype)
    src = abi.mx_expr_source(e).encode()
    assert b"mx_xmap" in src and b"mx_xvjp" in src and b"mx_xred_max" in src and b"mx_xseg_min" in src
    prog = ctypes.c_void_p()
    assert rtc.hiprtcCreateProgram(ctypes.byref(prog), src, b"mx_expr.hip", 0, None, None) == 0
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


def test_constants_are_rounded_to_the_element_type_in_the_source():
    e32 = abi.mx_expr_create([CONST(0, 0.1)], 1, 0, abi.MX_F32)
    e64 = abi.mx_expr_create([CONST(0, 0.1)], 1, 0, abi.MX_F64)
    def lit(src):
        i = src.index("v0 = ((T)") + len("v0 = ((T)")
        return float.fromhex(src[i:src.index(")", i)])
    assert lit(abi.mx_expr_source(e32)) == float(np.float32(0.1))
    assert lit(abi.mx_expr_source(e64)) == 0.1
