"""Thin Python binding of the C ABI in include/mx.h.

Each function has the name of the C entry point and does argument marshalling
only: it takes torch tensors (device memory) or numpy arrays (host memory),
passes their addresses, sizes and the stream to libmx.so, and raises MxError if
the call returns a non-zero status.  All computation happens in the library.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib

# ---------------------------------------------------------------- enums (values of mx.h)
MX_OK, MX_ERR_INVALID, MX_ERR_SHAPE, MX_ERR_DTYPE, MX_ERR_UNSUPPORTED, MX_ERR_HIP, MX_ERR_WORKSPACE = \
    0, -1, -2, -3, -4, -5, -6
MX_F32, MX_F64, MX_I32, MX_I64 = 0, 1, 2, 3
MX_ADD, MX_MUL, MX_MIN, MX_MAX = 0, 1, 2, 3
(MX_U_ID, MX_U_NEG, MX_U_ABS, MX_U_SQ, MX_U_AFFINE, MX_U_EXP, MX_U_LOG, MX_U_SQRT,
 MX_U_RSQRT) = range(9)
MX_B_ADD, MX_B_SUB, MX_B_MUL, MX_B_DIV, MX_B_MIN, MX_B_MAX = range(6)
MX_WS_REDUCE, MX_WS_SCAN, MX_WS_HISTOGRAM, MX_WS_SEGMENTED = 0, 1, 2, 3
(MX_X_IN, MX_X_CONST, MX_X_ADD, MX_X_SUB, MX_X_MUL, MX_X_DIV, MX_X_MIN, MX_X_MAX, MX_X_NEG, MX_X_ABS, MX_X_SQ,
 MX_X_EXP, MX_X_LOG, MX_X_SQRT, MX_X_RSQRT) = range(15)

DTYPE_OF = {torch.float32: MX_F32, torch.float64: MX_F64, torch.int32: MX_I32, torch.int64: MX_I64}
ACC_OF = {torch.float32: torch.float32, torch.float64: torch.float64, torch.int32: torch.int64,
          torch.int64: torch.int64}


class MxError(RuntimeError):
    """A libmx entry point returned a non-zero status."""

    def __init__(self, status: int, message: str):
        super().__init__(f"[{status}] {message}")
        self.status = status


def _L():
    return _lib.load()


def _check(status: int, name: str) -> None:
    if status != MX_OK:
        msg = _L().mx_last_error().decode(errors="replace")
        raise MxError(status, f"{name}: {msg}")


def _stream(stream) -> int:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, torch.cuda.Stream):
        return stream.cuda_stream
    return int(stream)


def _dptr(t):
    """Device address of a contiguous tensor (None -> NULL)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return t.data_ptr() if t.numel() else (t.data_ptr() or None)


def _nbytes(t) -> int:
    return 0 if t is None else t.numel() * t.element_size()


def _dtype(t) -> int:
    try:
        return DTYPE_OF[t.dtype]
    except KeyError:
        raise MxError(MX_ERR_DTYPE, f"unsupported dtype {t.dtype}") from None


def _acc_scalar(value, dtype: torch.dtype):
    """A host scalar of the accumulator type of `dtype` (for ne / params)."""
    acc = ACC_OF[dtype]
    if acc == torch.float32:
        return ctypes.c_float(float(value))
    if acc == torch.float64:
        return ctypes.c_double(float(value))
    return ctypes.c_int64(int(value))


# ---------------------------------------------------------------- runtime
def mx_init(device: int = 0) -> None:
    _check(_L().mx_init(int(device)), "mx_init")


def mx_last_error() -> str:
    return _L().mx_last_error().decode(errors="replace")


def mx_version() -> str:
    return _L().mx_version().decode()


def mx_set_debug(on: bool) -> None:
    _check(_L().mx_set_debug(1 if on else 0), "mx_set_debug")


def mx_get_debug() -> bool:
    return bool(_L().mx_get_debug())


def mx_workspace_bytes(kind: int, n: int, aux: int = 0) -> int:
    return int(_L().mx_workspace_bytes(int(kind), int(n), int(aux)))


def mx_copy32(src, dst, stream=None) -> None:
    n = src.numel() * src.element_size() // 4
    _check(_L().mx_copy32(_dptr(src), _dptr(dst), n, _stream(stream)), "mx_copy32")


MX_STREAM_READ_SLOTS = 16384


def mx_stream_read(src, xor_slots, stream=None) -> None:
    """Read-only pass over src (16-byte aligned, 4-byte elements); the XOR of its words is XORed, block by
    block, into its own word of the MX_STREAM_READ_SLOTS words of xor_slots (the XOR of the slots is the XOR
    of src)."""
    if src.element_size() != 4:
        raise MxError(MX_ERR_INVALID, "mx_stream_read: 4-byte elements expected")
    if xor_slots.numel() * xor_slots.element_size() < 4 * MX_STREAM_READ_SLOTS:
        raise MxError(MX_ERR_INVALID, "mx_stream_read: xor_slots needs MX_STREAM_READ_SLOTS words")
    _check(_L().mx_stream_read(_dptr(src), src.numel(), _dptr(xor_slots), _stream(stream)), "mx_stream_read")


# ---------------------------------------------------------------- marshaling
def mx_lengths_to_offsets(lengths, offsets, ws, stream=None) -> None:
    _check(_L().mx_lengths_to_offsets(_dptr(lengths), lengths.numel(), _dptr(offsets), _dptr(ws),
                                      _nbytes(ws), _stream(stream)), "mx_lengths_to_offsets")


def mx_marshal_rows(rows, staging, values, lengths_dev, offsets, ws, stream=None) -> None:
    """rows: list of contiguous numpy arrays of one dtype; staging: pinned uint8 tensor."""
    nseg = len(rows)
    elem = rows[0].dtype.itemsize if nseg else values.element_size()
    for r in rows:
        if not r.flags["C_CONTIGUOUS"]:
            raise ValueError("rows must be C-contiguous")
    ptrs = (ctypes.c_void_p * max(nseg, 1))(*[r.ctypes.data if r.size else None for r in rows])
    lengths = np.ascontiguousarray([r.size for r in rows], dtype=np.int64)
    if not staging.is_pinned():
        raise ValueError("staging must be pinned host memory")
    _check(_L().mx_marshal_rows(ptrs, lengths.ctypes.data, nseg, elem, staging.data_ptr(),
                                _nbytes(staging), _dptr(values), _dptr(lengths_dev), _dptr(offsets),
                                _dptr(ws), _nbytes(ws), _stream(stream)), "mx_marshal_rows")


def mx_unmarshal_rows(values, offsets_host: np.ndarray, staging, rows, stream=None) -> None:
    """Synchronous: fills the numpy arrays in `rows` (preallocated, row r of the right length)."""
    off = np.ascontiguousarray(offsets_host, dtype=np.int64)
    nseg = off.size - 1
    ptrs = (ctypes.c_void_p * max(nseg, 1))(*[r.ctypes.data if r.size else None for r in rows])
    elem = values.element_size()
    _check(_L().mx_unmarshal_rows(_dptr(values), off.ctypes.data, nseg, elem, staging.data_ptr(),
                                  _nbytes(staging), ptrs, _stream(stream)), "mx_unmarshal_rows")


def mx_records_to_fields(aos, fields, stream=None) -> None:
    """aos: device tensor [n, f]; fields: list of f device tensors [n] of the same element size."""
    n, f = aos.shape
    ptrs = (ctypes.c_void_p * f)(*[_dptr(t) for t in fields])
    _check(_L().mx_records_to_fields(_dptr(aos), n, f, aos.element_size(), ptrs, _stream(stream)),
           "mx_records_to_fields")


def mx_fields_to_records(fields, aos, stream=None) -> None:
    n, f = aos.shape
    ptrs = (ctypes.c_void_p * f)(*[_dptr(t) for t in fields])
    _check(_L().mx_fields_to_records(ptrs, n, f, aos.element_size(), _dptr(aos), _stream(stream)),
           "mx_fields_to_records")


def mx_compose_offsets(outer, inner, out, stream=None) -> None:
    _check(_L().mx_compose_offsets(_dptr(outer), outer.numel() - 1, _dptr(inner), _dptr(out),
                                   _stream(stream)), "mx_compose_offsets")


def mx_offsets_regular(offsets, stream=None) -> int:
    """Common row length of a regular nesting level (MxError MX_ERR_SHAPE if ragged)."""
    r = ctypes.c_int64()
    _check(_L().mx_offsets_regular(_dptr(offsets), offsets.numel() - 1, ctypes.byref(r), _stream(stream)),
           "mx_offsets_regular")
    return r.value


# ---------------------------------------------------------------- map / map2
def mx_map(f: int, x, params, out, stream=None) -> None:
    dt = x.dtype
    pbuf = None
    if params is not None:
        acc = ACC_OF[dt]
        ctype = {torch.float32: ctypes.c_float, torch.float64: ctypes.c_double}.get(acc, ctypes.c_int64)
        pbuf = (ctype * 2)(*(float(p) if acc.is_floating_point else int(p) for p in params))
    _check(_L().mx_map(int(f), _dtype(x), _dptr(x), x.numel(),
                       ctypes.cast(pbuf, ctypes.c_void_p) if pbuf is not None else None,
                       _dptr(out), _stream(stream)), "mx_map")


def mx_map2(f: int, a, b, out, stream=None) -> None:
    if a.numel() != b.numel() or a.dtype != b.dtype:
        raise MxError(MX_ERR_SHAPE, "mx_map2: operands differ in length or dtype")
    _check(_L().mx_map2(int(f), _dtype(a), _dptr(a), _dptr(b), a.numel(), _dptr(out),
                        _stream(stream)), "mx_map2")


# ---------------------------------------------------------------- reduce
def mx_reduce(op: int, x, ne, out, ws, stream=None) -> None:
    nb = _acc_scalar(ne, x.dtype)
    _check(_L().mx_reduce(int(op), _dtype(x), _dptr(x), x.numel(), ctypes.byref(nb), _dptr(out),
                          _dptr(ws), _nbytes(ws), _stream(stream)), "mx_reduce")


def mx_map2_reduce(f: int, op: int, a, b, ne, out, ws, stream=None) -> None:
    if a.numel() != b.numel() or a.dtype != b.dtype:
        raise MxError(MX_ERR_SHAPE, "mx_map2_reduce: operands differ in length or dtype")
    nb = _acc_scalar(ne, a.dtype)
    _check(_L().mx_map2_reduce(int(f), int(op), _dtype(a), _dptr(a), _dptr(b), a.numel(),
                               ctypes.byref(nb), _dptr(out), _dptr(ws), _nbytes(ws), _stream(stream)),
           "mx_map2_reduce")


def mx_dot_adjoint_f32(a, b, gout, ga, gb, stream=None) -> None:
    n = a.numel() if a is not None else b.numel()
    _check(_L().mx_dot_adjoint_f32(_dptr(a), _dptr(b), n, _dptr(gout), _dptr(ga), _dptr(gb),
                                   _stream(stream)), "mx_dot_adjoint_f32")


# ---------------------------------------------------------------- ragged
def mx_segmented_reduce(op: int, values, offsets, ne, out, ws, stream=None) -> None:
    """ws: a zero-filled workspace of mx_workspace_bytes(MX_WS_SEGMENTED, values.numel()) bytes (None when
    values has at most 2048 elements)."""
    nb = _acc_scalar(ne, values.dtype)
    _check(_L().mx_segmented_reduce(int(op), _dtype(values), _dptr(values), values.numel(), _dptr(offsets),
                                    offsets.numel() - 1, ctypes.byref(nb), _dptr(out), _dptr(ws), _nbytes(ws),
                                    _stream(stream)), "mx_segmented_reduce")


def mx_segmented_reduce_noalloc(op: int, values, offsets, ne, out, stream=None) -> None:
    """mx_segmented_reduce with the library's built-in scratch instead of a workspace (no allocation)."""
    nb = _acc_scalar(ne, values.dtype)
    _check(_L().mx_segmented_reduce_noalloc(int(op), _dtype(values), _dptr(values), values.numel(), _dptr(offsets),
                                            offsets.numel() - 1, ctypes.byref(nb), _dptr(out), _stream(stream)),
           "mx_segmented_reduce_noalloc")


def mx_segmented_noalloc_max_values() -> int:
    return int(_L().mx_segmented_noalloc_max_values())


def mx_segmented_reduce_plain(op: int, values, offsets, ne, out, stream=None) -> None:
    nb = _acc_scalar(ne, values.dtype)
    _check(_L().mx_segmented_reduce_plain(int(op), _dtype(values), _dptr(values), values.numel(), _dptr(offsets),
                                          offsets.numel() - 1, ctypes.byref(nb), _dptr(out),
                                          _stream(stream)), "mx_segmented_reduce_plain")


def mx_segmented_sum_adjoint_f32(gout, offsets, gvalues, stream=None) -> None:
    _check(_L().mx_segmented_sum_adjoint_f32(_dptr(gout), _dptr(offsets), offsets.numel() - 1,
                                             _dptr(gvalues), gvalues.numel(), _stream(stream)),
           "mx_segmented_sum_adjoint_f32")


def mx_reduce_adjoint_f32(op: int, x, ne, gout, gx, ws=None, stream=None) -> None:
    """Reverse of reduce op ne x (ADD, MIN, MAX); gout: one device float."""
    nb = ctypes.c_float(float(ne))
    _check(_L().mx_reduce_adjoint_f32(int(op), _dptr(x), x.numel(), ctypes.byref(nb), _dptr(gout), _dptr(gx),
                                      _dptr(ws), _nbytes(ws), _stream(stream)), "mx_reduce_adjoint_f32")


def mx_segmented_reduce_adjoint_f32(op: int, values, offsets, ne, gout, gvalues, stream=None) -> None:
    """Reverse of map (reduce op ne) over ragged rows; gout: device float[nseg]."""
    nb = ctypes.c_float(float(ne))
    _check(_L().mx_segmented_reduce_adjoint_f32(int(op), _dptr(values), gvalues.numel(), _dptr(offsets),
                                                offsets.numel() - 1, ctypes.byref(nb), _dptr(gout), _dptr(gvalues),
                                                _stream(stream)),
           "mx_segmented_reduce_adjoint_f32")


# ---------------------------------------------------------------- dense
def _mmr_dims(ta, tb, A, B):
    M, K = (A.shape[1], A.shape[0]) if ta else (A.shape[0], A.shape[1])
    N, Kb = (B.shape[0], B.shape[1]) if tb else (B.shape[1], B.shape[0])
    if K != Kb:
        raise MxError(MX_ERR_SHAPE, f"inner dimensions differ: {K} vs {Kb}")
    return M, N, K


def mx_map_map_reduce_f32(ta: int, tb: int, A, B, C, stream=None) -> None:
    M, N, K = _mmr_dims(ta, tb, A, B)
    _check(_L().mx_map_map_reduce_f32(int(ta), int(tb), M, N, K, _dptr(A), _dptr(B), _dptr(C),
                                      _stream(stream)), "mx_map_map_reduce_f32")


def mx_map_map_reduce_plain_f32(ta: int, tb: int, A, B, C, stream=None) -> None:
    M, N, K = _mmr_dims(ta, tb, A, B)
    _check(_L().mx_map_map_reduce_plain_f32(int(ta), int(tb), M, N, K, _dptr(A), _dptr(B), _dptr(C),
                                            _stream(stream)), "mx_map_map_reduce_plain_f32")


# ---------------------------------------------------------------- N-body loop
def _n4(t):
    """Number of float4 records in a [n, 4] float32 tensor."""
    if t.dtype != torch.float32 or t.dim() != 2 or t.shape[1] != 4:
        raise MxError(MX_ERR_SHAPE, "expected a float32 tensor of shape [n, 4]")
    return t.shape[0]


def mx_nbody_pair_workspace_bytes(n: int) -> int:
    return int(_L().mx_nbody_pair_workspace_bytes(int(n)))


def mx_nbody_accel_f32(pos4, eps2, G, acc4, ws, stream=None) -> None:
    _check(_L().mx_nbody_accel_f32(_dptr(pos4), _n4(pos4), eps2, G, _dptr(acc4), _dptr(ws), _nbytes(ws),
                                   _stream(stream)), "mx_nbody_accel_f32")


def mx_nbody_step_f32(pos4, vel4, eps2, G, dt, pos4_out, vel4_out, ws, stream=None) -> None:
    _check(_L().mx_nbody_step_f32(_dptr(pos4), _dptr(vel4), _n4(pos4), eps2, G, dt, _dptr(pos4_out),
                                  _dptr(vel4_out), _dptr(ws), _nbytes(ws), _stream(stream)), "mx_nbody_step_f32")


def mx_nbody_step_plain_f32(pos4, vel4, eps2, G, dt, acc4, pos4_out, vel4_out, stream=None) -> None:
    _check(_L().mx_nbody_step_plain_f32(_dptr(pos4), _dptr(vel4), _n4(pos4), eps2, G, dt, _dptr(acc4),
                                        _dptr(pos4_out), _dptr(vel4_out), _stream(stream)),
           "mx_nbody_step_plain_f32")


def mx_nbody_accel_vjp_f32(pos4, abar4, eps2, G, out4, ws, stream=None) -> None:
    _check(_L().mx_nbody_accel_vjp_f32(_dptr(pos4), _dptr(abar4), _n4(pos4), eps2, G, _dptr(out4), _dptr(ws),
                                       _nbytes(ws), _stream(stream)), "mx_nbody_accel_vjp_f32")


def mx_nbody_adjoint_step_f32(pos4, xbar4, vbar4, eps2, G, dt, xbar4_out, vbar4_out, ws, stream=None) -> None:
    _check(_L().mx_nbody_adjoint_step_f32(_dptr(pos4), _dptr(xbar4), _dptr(vbar4), _n4(pos4), eps2, G, dt,
                                          _dptr(xbar4_out), _dptr(vbar4_out), _dptr(ws), _nbytes(ws),
                                          _stream(stream)), "mx_nbody_adjoint_step_f32")


def mx_nbody_kinetic_f32(pos4, vel4, ke, stream=None) -> None:
    _check(_L().mx_nbody_kinetic_f32(_dptr(pos4), _dptr(vel4), _n4(pos4), _dptr(ke), _stream(stream)),
           "mx_nbody_kinetic_f32")


def mx_nbody_workspace_bytes(n: int, nsteps: int, ckpt_every: int) -> int:
    return int(_L().mx_nbody_workspace_bytes(int(n), int(nsteps), int(ckpt_every)))


def mx_nbody_ke_grad_f32(pos4, vel4, eps2, G, dt, nsteps, ckpt_every, ke, gx4, gv4, ws, stream=None) -> None:
    _check(_L().mx_nbody_ke_grad_f32(_dptr(pos4), _dptr(vel4), _n4(pos4), eps2, G, dt, int(nsteps),
                                     int(ckpt_every), _dptr(ke), _dptr(gx4), _dptr(gv4), _dptr(ws), _nbytes(ws),
                                     _stream(stream)), "mx_nbody_ke_grad_f32")


def mx_nbody_ke_f32(pos4, vel4, eps2, G, dt, nsteps, ckpt_every, ke, ws, stream=None) -> None:
    _check(_L().mx_nbody_ke_f32(_dptr(pos4), _dptr(vel4), _n4(pos4), eps2, G, dt, int(nsteps), int(ckpt_every),
                                _dptr(ke), _dptr(ws), _nbytes(ws), _stream(stream)), "mx_nbody_ke_f32")


def mx_nbody_ke_vjp_f32(pos4, vel4, eps2, G, dt, nsteps, ckpt_every, gscale, gx4, gv4, ws, stream=None) -> None:
    _check(_L().mx_nbody_ke_vjp_f32(_dptr(pos4), _dptr(vel4), _n4(pos4), eps2, G, dt, int(nsteps),
                                    int(ckpt_every), _dptr(gscale), _dptr(gx4), _dptr(gv4), _dptr(ws),
                                    _nbytes(ws), _stream(stream)), "mx_nbody_ke_vjp_f32")


# ---------------------------------------------------------------- k-means
def _nd(X):
    if X.dtype != torch.float32 or X.dim() != 2:
        raise MxError(MX_ERR_SHAPE, "expected a float32 matrix [n, d]")
    return X.shape[0], X.shape[1]


def mx_kmeans_workspace_bytes(n: int, d: int, k: int) -> int:
    return int(_L().mx_kmeans_workspace_bytes(int(n), int(d), int(k)))


def mx_kmeans_step_f32(X, C, labels, counts, C_out, ws, stream=None) -> None:
    n, d = _nd(X)
    _check(_L().mx_kmeans_step_f32(_dptr(X), n, d, _dptr(C), C.shape[0], _dptr(labels), _dptr(counts),
                                   _dptr(C_out), _dptr(ws), _nbytes(ws), _stream(stream)), "mx_kmeans_step_f32")


def mx_kmeans_debug_fallbacks() -> int:
    return int(_L().mx_kmeans_debug_fallbacks())


def mx_kmeans_step_plain_f32(X, C, labels, counts, C_out, ws, stream=None) -> None:
    n, d = _nd(X)
    _check(_L().mx_kmeans_step_plain_f32(_dptr(X), n, d, _dptr(C), C.shape[0], _dptr(labels), _dptr(counts),
                                         _dptr(C_out), _dptr(ws), _nbytes(ws), _stream(stream)),
           "mx_kmeans_step_plain_f32")


def mx_kmeans_sse_f32(X, C, labels, sse, ws, stream=None) -> None:
    n, d = _nd(X)
    _check(_L().mx_kmeans_sse_f32(_dptr(X), n, d, _dptr(C), _dptr(labels), _dptr(sse), _dptr(ws), _nbytes(ws),
                                  _stream(stream)), "mx_kmeans_sse_f32")


def mx_kmeans_sse_grad_f32(X, C, labels, gscale, G, stream=None) -> None:
    n, d = _nd(X)
    _check(_L().mx_kmeans_sse_grad_f32(_dptr(X), n, d, _dptr(C), _dptr(labels), _dptr(gscale), _dptr(G),
                                       _stream(stream)), "mx_kmeans_sse_grad_f32")


# ---------------------------------------------------------------- batches
class BatchConfig(ctypes.Structure):
    _fields_ = [("tile_elems", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 2)]


class BatchPlan:
    """Owns an mx_batch_plan handle."""

    def __init__(self, handle: int, ntasks: int):
        self.handle = handle
        self.ntasks = ntasks

    def __del__(self):
        if getattr(self, "handle", None):
            _L().mx_batch_plan_destroy(self.handle)
            self.handle = None


def mx_batch_plan_create(table: np.ndarray, cfg: tuple | None = None) -> BatchPlan:
    tb = np.ascontiguousarray(table, dtype=np.int64).reshape(-1, 6)
    h = ctypes.c_void_p()
    c = BatchConfig(cfg[0], cfg[1]) if cfg else None
    _check(_L().mx_batch_plan_create(tb.ctypes.data, tb.shape[0], ctypes.byref(c) if c else None,
                                     ctypes.byref(h)), "mx_batch_plan_create")
    return BatchPlan(h.value, tb.shape[0])


def mx_batch_plan_destroy(plan: BatchPlan) -> None:
    if plan.handle:
        _check(_L().mx_batch_plan_destroy(plan.handle), "mx_batch_plan_destroy")
        plan.handle = None


def mx_batch_workspace_bytes(plan: BatchPlan) -> int:
    return int(_L().mx_batch_workspace_bytes(plan.handle))


def mx_batch_get_config(plan: BatchPlan) -> tuple:
    c = BatchConfig()
    _check(_L().mx_batch_get_config(plan.handle, ctypes.byref(c)), "mx_batch_get_config")
    return (c.tile_elems, c.blocks_per_cu)


def mx_batch_set_config(plan: BatchPlan, cfg: tuple) -> None:
    c = BatchConfig(cfg[0], cfg[1])
    _check(_L().mx_batch_set_config(plan.handle, ctypes.byref(c)), "mx_batch_set_config")


def mx_batch_forward(plan: BatchPlan, A, B, out, ws, stream=None) -> None:
    _check(_L().mx_batch_forward(plan.handle, _dptr(A), _dptr(B), _dptr(out), _dptr(ws), _nbytes(ws),
                                 _stream(stream)), "mx_batch_forward")


def mx_batch_backward(plan: BatchPlan, A, B, gout, gA, gB, ws, stream=None) -> None:
    _check(_L().mx_batch_backward(plan.handle, _dptr(A), _dptr(B), _dptr(gout), _dptr(gA), _dptr(gB), _dptr(ws),
                                  _nbytes(ws), _stream(stream)), "mx_batch_backward")


def mx_batch_forward_plain(plan: BatchPlan, A, B, out, stream=None) -> None:
    _check(_L().mx_batch_forward_plain(plan.handle, _dptr(A), _dptr(B), _dptr(out), _stream(stream)),
           "mx_batch_forward_plain")


def mx_batch_backward_plain(plan: BatchPlan, A, B, gout, gA, gB, stream=None) -> None:
    _check(_L().mx_batch_backward_plain(plan.handle, _dptr(A), _dptr(B), _dptr(gout), _dptr(gA), _dptr(gB),
                                        _stream(stream)), "mx_batch_backward_plain")


def mx_batch_autotune(plan: BatchPlan, A, B, out, gout, gA, gB, ws, cache_path: str | None = None,
                      stream=None) -> tuple:
    c = BatchConfig()
    _check(_L().mx_batch_autotune(plan.handle, _dptr(A), _dptr(B), _dptr(out), _dptr(gout), _dptr(gA), _dptr(gB),
                                  _dptr(ws), _nbytes(ws), cache_path.encode() if cache_path else None,
                                  _stream(stream), ctypes.byref(c)), "mx_batch_autotune")
    return (c.tile_elems, c.blocks_per_cu)


# ---------------------------------------------------------------- graphs
# ---------------------------------------------------------------- Parboil-shaped kernels
def mx_histogram_u32(keys, nbins: int, counts, ws=None, stream=None) -> None:
    _check(_L().mx_histogram_u32(_dptr(keys), keys.numel(), int(nbins), _dptr(counts),
                                 None if ws is None else _dptr(ws), 0 if ws is None else ws.numel(),
                                 _stream(stream)), "mx_histogram_u32")


def mx_stencil7_f32(grid_in, grid_out, c0: float, c1: float, stream=None) -> None:
    nz, ny, nx = grid_in.shape
    _check(_L().mx_stencil7_f32(_dptr(grid_in), _dptr(grid_out), nx, ny, nz, float(c0), float(c1), _stream(stream)),
           "mx_stencil7_f32")


def mx_mriq_f32(kx, ky, kz, phi, x, y, z, qr, qi, stream=None) -> None:
    _check(_L().mx_mriq_f32(_dptr(kx), _dptr(ky), _dptr(kz), _dptr(phi), kx.numel(), _dptr(x), _dptr(y), _dptr(z),
                            x.numel(), _dptr(qr), _dptr(qi), _stream(stream)), "mx_mriq_f32")


def mx_tpacf_f32(p1, p2, edges, counts, self_pairs: bool = False, stream=None) -> None:
    """p1, p2: (3, n) float32 device tensors of unit vectors (p2 ignored for self pairs)."""
    q = p1 if self_pairs else p2
    _check(_L().mx_tpacf_f32(_dptr(p1[0]), _dptr(p1[1]), _dptr(p1[2]), p1.shape[1], _dptr(q[0]), _dptr(q[1]),
                             _dptr(q[2]), q.shape[1], int(bool(self_pairs)), _dptr(edges), edges.numel(),
                             _dptr(counts), _stream(stream)), "mx_tpacf_f32")


# ---------------------------------------------------------------- user-defined map bodies
class XInsn(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int32), ("dst", ctypes.c_int32), ("a", ctypes.c_int32), ("b", ctypes.c_int32),
                ("imm", ctypes.c_double)]


class Expr:
    """Owning handle of an mx_expr (destroyed with the object)."""

    def __init__(self, handle: int, nin: int, dtype: int):
        self.handle, self.nin, self.dtype = handle, nin, dtype

    def __del__(self):
        if getattr(self, "handle", None):
            try:
                _L().mx_expr_destroy(self.handle)
            except Exception:  # interpreter shutdown: the library may already be gone
                pass
            self.handle = None


def _ptr_list(ts):
    arr = (ctypes.c_void_p * max(1, len(ts)))()
    for i, t in enumerate(ts):
        arr[i] = _dptr(t)
    return arr


def mx_expr_create(prog, nin: int, out_reg: int, dtype: int) -> Expr:
    """prog: sequence of (op, dst, a, b, imm)."""
    ins = (XInsn * max(1, len(prog)))()
    for i, (op, dst, a, b, imm) in enumerate(prog):
        ins[i] = XInsn(int(op), int(dst), int(a), int(b), float(imm))
    h = ctypes.c_void_p()
    _check(_L().mx_expr_create(ins, len(prog), int(nin), int(out_reg), int(dtype), ctypes.byref(h)),
           "mx_expr_create")
    return Expr(h.value, nin, dtype)


def mx_expr_destroy(e: Expr) -> None:
    if e.handle:
        _check(_L().mx_expr_destroy(e.handle), "mx_expr_destroy")
        e.handle = None


def mx_expr_prepare(e: Expr) -> None:
    _check(_L().mx_expr_prepare(e.handle), "mx_expr_prepare")


def mx_expr_source(e: Expr) -> str:
    return _L().mx_expr_source(e.handle).decode()


def mx_expr_map(e: Expr, inputs, out, stream=None) -> None:
    _check(_L().mx_expr_map(e.handle, _ptr_list(inputs), out.numel(), _dptr(out), _stream(stream)), "mx_expr_map")


def mx_expr_workspace_bytes(e: Expr, n: int) -> int:
    return int(_L().mx_expr_workspace_bytes(e.handle, int(n)))


def mx_expr_map_reduce(e: Expr, op: int, inputs, n: int, ne, out, ws, stream=None) -> None:
    nb = ctypes.c_float(ne) if e.dtype == MX_F32 else ctypes.c_double(ne)
    _check(_L().mx_expr_map_reduce(e.handle, int(op), _ptr_list(inputs), int(n), ctypes.byref(nb), _dptr(out),
                                   _dptr(ws), _nbytes(ws), _stream(stream)), "mx_expr_map_reduce")


def mx_expr_segmented_reduce(e: Expr, op: int, inputs, offsets, ne, out, stream=None) -> None:
    nb = ctypes.c_float(ne) if e.dtype == MX_F32 else ctypes.c_double(ne)
    _check(_L().mx_expr_segmented_reduce(e.handle, int(op), _ptr_list(inputs), _dptr(offsets), offsets.numel() - 1,
                                         ctypes.byref(nb), _dptr(out), _stream(stream)), "mx_expr_segmented_reduce")


def mx_expr_loop_workspace_bytes(out_len: int) -> int:
    return int(_L().mx_expr_loop_workspace_bytes(int(out_len)))


def mx_expr_loop_scatter(e: Expr, inputs, index, out, ws=None, stream=None) -> None:
    _check(_L().mx_expr_loop_scatter(e.handle, _ptr_list(inputs), index.numel(), _dptr(index), _dptr(out),
                                     out.numel(), _dptr(ws), _nbytes(ws), _stream(stream)), "mx_expr_loop_scatter")


def mx_expr_vjp(e: Expr, inputs, n: int, gout, gscale, grads, stream=None) -> None:
    _check(_L().mx_expr_vjp(e.handle, _ptr_list(inputs), int(n), _dptr(gout), _dptr(gscale), _ptr_list(grads),
                            _stream(stream)), "mx_expr_vjp")


class Graph:
    """An instantiated capture of library launches (opaque mx_graph handle)."""

    def __init__(self, handle: int):
        self.handle = handle

    def launch(self, stream=None) -> None:
        mx_graph_launch(self, stream)

    def __del__(self):
        if getattr(self, "handle", None):
            _L().mx_graph_destroy(self.handle)
            self.handle = None


def mx_graph_begin(stream=None) -> None:
    _check(_L().mx_graph_begin(_stream(stream)), "mx_graph_begin")


def mx_graph_end(stream=None) -> Graph:
    h = ctypes.c_void_p()
    _check(_L().mx_graph_end(_stream(stream), ctypes.byref(h)), "mx_graph_end")
    return Graph(h.value)


def mx_graph_launch(graph: Graph, stream=None) -> None:
    _check(_L().mx_graph_launch(graph.handle, _stream(stream)), "mx_graph_launch")


def mx_graph_destroy(graph: Graph) -> None:
    if graph.handle:
        _check(_L().mx_graph_destroy(graph.handle), "mx_graph_destroy")
        graph.handle = None


# ---------------------------------------------------------------- the general parallel loop
(MX_L_ITER, MX_L_ICONST, MX_L_IADD, MX_L_ISUB, MX_L_IMUL, MX_L_IDIV, MX_L_IMOD, MX_L_IMIN, MX_L_IMAX, MX_L_INEG,
 MX_L_I2F) = range(32, 43)
MX_L_FGET, MX_L_IGET, MX_L_FSET, MX_L_ISET = 48, 49, 50, 51


class LInsn(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int32), ("dst", ctypes.c_int32), ("a", ctypes.c_int32), ("b", ctypes.c_int32),
                ("c", ctypes.c_int32), ("src", ctypes.c_int32), ("tensor", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("iimm", ctypes.c_int64), ("fimm", ctypes.c_double)]


class LType(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int), ("rank", ctypes.c_int32)]


class LTensor(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("dims", ctypes.c_int64 * 3)]


class Loop:
    """Owning handle of an mx_loop (destroyed with the object)."""

    def __init__(self, handle: int, types):
        self.handle, self.types = handle, list(types)

    def __del__(self):
        if getattr(self, "handle", None):
            try:
                _L().mx_loop_destroy(self.handle)
            except Exception:  # interpreter shutdown: the library may already be gone
                pass
            self.handle = None


def mx_loop_create(prog, types, float_dtype: int) -> Loop:
    """prog: tuples (op, dst, a, b, c, src, tensor, iimm, fimm); types: (dtype, rank) per tensor."""
    ins = (LInsn * max(1, len(prog)))()
    for i, q in enumerate(prog):
        op, dst, a, b, c, src, tensor, iimm, fimm = q
        ins[i] = LInsn(int(op), int(dst), int(a), int(b), int(c), int(src), int(tensor), 0, int(iimm), float(fimm))
    tt = (LType * max(1, len(types)))()
    for i, (dt, rank) in enumerate(types):
        tt[i] = LType(int(dt), int(rank))
    h = ctypes.c_void_p()
    _check(_L().mx_loop_create(ins, len(prog), tt, len(types), int(float_dtype), ctypes.byref(h)), "mx_loop_create")
    return Loop(h.value, types)


def mx_loop_destroy(lp: Loop) -> None:
    if lp.handle:
        _check(_L().mx_loop_destroy(lp.handle), "mx_loop_destroy")
        lp.handle = None


def _ltensors(tensors):
    arr = (LTensor * max(1, len(tensors)))()
    for i, t in enumerate(tensors):
        dims = list(t.shape) + [1] * (3 - t.dim())
        arr[i] = LTensor(_dptr(t), (ctypes.c_int64 * 3)(*dims))
    return arr


def mx_loop_prepare(lp: Loop) -> None:
    _check(_L().mx_loop_prepare(lp.handle), "mx_loop_prepare")


def mx_loop_source(lp: Loop) -> str:
    return _L().mx_loop_source(lp.handle).decode()


def mx_loop_workspace_bytes(lp: Loop, tensors) -> int:
    return int(_L().mx_loop_workspace_bytes(lp.handle, _ltensors(tensors)))


def mx_loop_run(lp: Loop, n: int, tensors, ws=None, stream=None) -> None:
    """tensors: contiguous device tensors of rank 1..3, in the loop's order."""
    if len(tensors) != len(lp.types):
        raise MxError(MX_ERR_INVALID, "mx_loop_run: wrong number of tensors")
    for t, (dt, rank) in zip(tensors, lp.types):
        if t.dim() != rank or _dtype(t) != dt:
            raise MxError(MX_ERR_SHAPE, "mx_loop_run: tensor rank or dtype differs from the loop's")
    _check(_L().mx_loop_run(lp.handle, int(n), _ltensors(tensors), _dptr(ws), _nbytes(ws), _stream(stream)),
           "mx_loop_run")


# ---------------------------------------------------------------- records whose fields are sequences
MX_FIELD_SCALAR, MX_FIELD_SEQ = 0, 1


class HSeq(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("len", ctypes.c_int64)]


class Field(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("elem_bytes", ctypes.c_int32), ("offset", ctypes.c_int64),
                ("values_dev", ctypes.c_void_p), ("lengths_dev", ctypes.c_void_p), ("offsets_dev", ctypes.c_void_p)]


def _fields(desc):
    """desc: (kind, elem_bytes, offset, values, lengths, offsets) with device tensors or None."""
    arr = (Field * max(1, len(desc)))()
    for i, (kind, eb, off, vals, lens, offs) in enumerate(desc):
        arr[i] = Field(int(kind), int(eb), int(off), _dptr(vals), _dptr(lens), _dptr(offs))
    return arr


def mx_records_layout(recs: np.ndarray, desc):
    """(element counts per field, staging bytes) for host records `recs` (a numpy structured array)."""
    counts = np.zeros(max(1, len(desc)), dtype=np.int64)
    staging = ctypes.c_size_t()
    _check(_L().mx_records_layout(recs.ctypes.data if recs.size else None, recs.size, recs.dtype.itemsize,
                                  _fields(desc), len(desc), counts.ctypes.data, ctypes.byref(staging)),
           "mx_records_layout")
    return counts[:len(desc)], staging.value


def mx_marshal_records(recs: np.ndarray, desc, staging, ws, stream=None) -> None:
    _check(_L().mx_marshal_records(recs.ctypes.data if recs.size else None, recs.size, recs.dtype.itemsize,
                                   _fields(desc), len(desc), staging.data_ptr() if staging is not None else None,
                                   _nbytes(staging), _dptr(ws), _nbytes(ws), _stream(stream)), "mx_marshal_records")


def mx_unmarshal_records(desc, recs: np.ndarray, staging, stream=None) -> None:
    _check(_L().mx_unmarshal_records(_fields(desc), len(desc), recs.size, recs.ctypes.data if recs.size else None,
                                     recs.dtype.itemsize, staging.data_ptr() if staging is not None else None,
                                     _nbytes(staging), _stream(stream)), "mx_unmarshal_records")
