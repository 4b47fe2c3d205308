"""Oracle -- TEST INFRASTRUCTURE ONLY.

A plain, slow, sequential CPU reference for what the accelerated-expression
primitives compute (the parallel keywords of Appendix A: map, map2, reduce,
flatten, loop; marshaling of Section 4.3), in binary64 / int64.  The
arithmetic lives in ``oracle.c`` (sequential left folds, no blocking, no
reordering); this module only converts numpy arrays to float64 / int64 and
calls it, plus the pure-Python marshaling of nested sequences and records.

Only ``tests/``, the smoke check and the bench's CPU-baseline leg may import
this package.  It shares no code with the GPU library, and the GPU library
never calls it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# operator numbering (same integers as the public C enums)
ADD, MUL, MIN, MAX = 0, 1, 2, 3
U_ID, U_NEG, U_ABS, U_SQ, U_AFFINE, U_EXP, U_LOG, U_SQRT, U_RSQRT = range(9)
B_ADD, B_SUB, B_MUL, B_DIV, B_MIN, B_MAX = range(6)
(X_IN, X_CONST, X_ADD, X_SUB, X_MUL, X_DIV, X_MIN, X_MAX, X_NEG, X_ABS, X_SQ, X_EXP, X_LOG, X_SQRT,
 X_RSQRT) = range(15)


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so with gcc (-O2, no fast-math, no contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
                               "-fno-fast-math", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _L():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        _declare(_lib)
    return _lib


_d = ctypes.c_double
_i64 = ctypes.c_int64
_int = ctypes.c_int
_p = ctypes.c_void_p


def _declare(lib):
    sig = {
        "or_map_f64": (None, [_int, _d, _d, _p, _i64, _p]),
        "or_map_i64": (None, [_int, _i64, _i64, _p, _i64, _p]),
        "or_map2_f64": (None, [_int, _p, _p, _i64, _p]),
        "or_map2_i64": (None, [_int, _p, _p, _i64, _p]),
        "or_foldl_f64": (_d, [_int, _d, _p, _i64]),
        "or_foldl_i64": (_i64, [_int, _i64, _p, _i64]),
        "or_map2_foldl_f64": (_d, [_int, _int, _d, _p, _p, _i64]),
        "or_map2_foldl_i64": (_i64, [_int, _int, _i64, _p, _p, _i64]),
        "or_offsets_from_lengths": (None, [_p, _i64, _p]),
        "or_segmented_foldl_f64": (None, [_int, _d, _p, _p, _i64, _p]),
        "or_segmented_foldl_i64": (None, [_int, _i64, _p, _p, _i64, _p]),
        "or_segmented_sum_adjoint_f64": (None, [_p, _p, _i64, _p]),
        "or_reduce_adjoint_f64": (_int, [_int, _d, _p, _i64, _d, _p]),
        "or_loop_run": (_int, [_p, _p, _p, _int, _int, _p, _p, _p, _p, _p, _i64, _p]),
        "or_loop_check": (_int, [_p, _p, _p, _int, _int, _p, _p, _p, _p, _p, _i64]),
        "or_segmented_reduce_adjoint_f64": (_int, [_int, _d, _p, _p, _i64, _p, _p]),
        "or_matmul_f64": (None, [_p, _p, _p, _i64, _i64, _i64, _int, _int]),
        "or_nbody_accel": (None, [_p, _p, _i64, _d, _d, _p]),
        "or_nbody_step": (None, [_p, _p, _p, _i64, _d, _d, _d, _p, _p]),
        "or_nbody_kinetic": (_d, [_p, _p, _i64]),
        "or_nbody_forward": (None, [_p, _p, _p, _i64, _d, _d, _d, _i64, _p, _p, _p]),
        "or_nbody_accel_vjp": (None, [_p, _p, _i64, _d, _d, _p, _p]),
        "or_nbody_ke_grad_tape": (_d, [_p, _p, _p, _i64, _d, _d, _d, _i64, _p, _p]),
        "or_nbody_ke_grad_ckpt": (_d, [_p, _p, _p, _i64, _d, _d, _d, _i64, _i64, _p, _p]),
        "or_sqdist": (_d, [_p, _p, _i64]),
        "or_kmeans_assign": (None, [_p, _i64, _i64, _p, _i64, _p]),
        "or_kmeans_update": (None, [_p, _i64, _i64, _p, _i64, _p, _p, _p, _p]),
        "or_kmeans_sse": (_d, [_p, _i64, _i64, _p, _p]),
        "or_kmeans_sse_grad": (None, [_p, _i64, _i64, _p, _p, _d, _p]),
        "or_batch_forward": (None, [_p, _i64, _p, _p, _p]),
        "or_batch_backward": (None, [_p, _i64, _p, _p, _p, _p, _p]),
        "or_expr_map_f64": (None, [_p, _p, _int, _int, _p, _i64, _p]),
        "or_expr_map_foldl_f64": (_d, [_int, _d, _p, _p, _int, _int, _p, _i64]),
        "or_expr_vjp_f64": (None, [_p, _p, _int, _int, _int, _p, _i64, _p, _p, _p]),
        "or_expr_loop_scatter_f64": (None, [_p, _p, _int, _int, _p, _i64, _p, _p, _i64]),
        "or_histogram_u32": (None, [_p, _i64, _i64, _p]),
        "or_stencil7": (None, [_p, _i64, _i64, _i64, _d, _d, _p]),
        "or_mriq": (None, [_p, _p, _p, _p, _i64, _p, _p, _p, _i64, _p, _p]),
        "or_tpacf": (None, [_p, _p, _p, _i64, _p, _p, _p, _i64, _int, _p, _int, _p]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args


def _f64(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64))


def _i64a(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.int64))


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _is_int(x) -> bool:
    return np.issubdtype(np.asarray(x).dtype, np.integer)


# ---------------------------------------------------------------- map / map2
def map(f: int, s, params=(0, 0)) -> np.ndarray:  # noqa: A001 - the paper's keyword
    """map f s: float inputs evaluated in binary64, integer inputs in int64."""
    if _is_int(s):
        x = _i64a(s)
        out = np.empty_like(x)
        _L().or_map_i64(f, int(params[0]), int(params[1]), _ptr(x), x.size, _ptr(out))
    else:
        x = _f64(s)
        out = np.empty_like(x)
        _L().or_map_f64(f, float(params[0]), float(params[1]), _ptr(x), x.size, _ptr(out))
    return out


def map2(f: int, s1, s2) -> np.ndarray:
    if len(s1) != len(s2):
        raise ValueError("map2: sequences of different lengths")
    if _is_int(s1) and _is_int(s2):
        a, b = _i64a(s1), _i64a(s2)
        out = np.empty_like(a)
        _L().or_map2_i64(f, _ptr(a), _ptr(b), a.size, _ptr(out))
    else:
        a, b = _f64(s1), _f64(s2)
        out = np.empty_like(a)
        _L().or_map2_f64(f, _ptr(a), _ptr(b), a.size, _ptr(out))
    return out


# ---------------------------------------------------------------- reduce
def reduce(op: int, ne, s):
    """reduce op ne s, evaluated as foldl op ne s."""
    if _is_int(s):
        x = _i64a(s)
        return int(_L().or_foldl_i64(op, int(ne), _ptr(x), x.size))
    x = _f64(s)
    return float(_L().or_foldl_f64(op, float(ne), _ptr(x), x.size))


foldl = reduce


def map2_reduce(f: int, op: int, ne, a, b):
    """reduce op ne (map2 f a b)."""
    if len(a) != len(b):
        raise ValueError("map2: sequences of different lengths")
    if _is_int(a) and _is_int(b):
        x, y = _i64a(a), _i64a(b)
        return int(_L().or_map2_foldl_i64(f, op, int(ne), _ptr(x), _ptr(y), x.size))
    x, y = _f64(a), _f64(b)
    return float(_L().or_map2_foldl_f64(f, op, float(ne), _ptr(x), _ptr(y), x.size))


def dot(a, b):
    return map2_reduce(B_MUL, ADD, 0, a, b)


# ---------------------------------------------------------------- marshaling
def offsets_from_lengths(lengths) -> np.ndarray:
    L = _i64a(lengths)
    out = np.empty(L.size + 1, dtype=np.int64)
    _L().or_offsets_from_lengths(_ptr(L), L.size, _ptr(out))
    return out


def marshal_nested(seq, depth: int):
    """Flatten a nested Python sequence of the given depth (depth 1 = [T]).

    Returns (values, [offsets_0, ..., offsets_{depth-2}]): values is the
    depth-first concatenation of the innermost elements; offsets_l[i] ..
    offsets_l[i+1] delimits the children of the i-th sequence at level l,
    counted in sequences of level l+1 (the last level counts values).
    Pure Python, for small cases.
    """
    if depth == 1:
        return list(seq), []
    offsets = [[0] for _ in range(depth - 1)]
    values = []

    def walk(node, lvl):
        if lvl == depth - 2:
            values.extend(node)
            offsets[lvl].append(len(values))
        else:
            for child in node:
                walk(child, lvl + 1)
            offsets[lvl].append(len(offsets[lvl + 1]) - 1)

    for node in seq:
        walk(node, 0)
    return values, [np.asarray(o, dtype=np.int64) for o in offsets]


def unmarshal_nested(values, offsets_levels):
    """Inverse of marshal_nested: rebuild nested Python lists."""
    vals = list(values)
    if not offsets_levels:
        return vals

    def build(level, i):
        lo, hi = int(offsets_levels[level][i]), int(offsets_levels[level][i + 1])
        if level == len(offsets_levels) - 1:
            return vals[lo:hi]
        return [build(level + 1, j) for j in range(lo, hi)]

    return [build(0, i) for i in range(len(offsets_levels[0]) - 1)]


def marshal_rows(rows):
    """Marshal a ragged sequence of numpy rows: (flat values, offsets)."""
    lengths = np.array([len(r) for r in rows], dtype=np.int64)
    offsets = offsets_from_lengths(lengths)
    dt = rows[0].dtype if len(rows) else np.float32
    values = np.empty(int(offsets[-1]), dtype=dt)
    for r, row in enumerate(rows):
        values[offsets[r]:offsets[r + 1]] = row
    return values, offsets


def marshal_records(records, fields):
    """A sequence of records {l_i = e_i} -> one flat array per field (SoA)."""
    return {f: np.array([rec[f] for rec in records]) for f in fields}


def unmarshal_records(soa, fields):
    n = len(soa[fields[0]]) if fields else 0
    return [{f: soa[f][i].item() for f in fields} for i in range(n)]


def marshal_record_seqs(records, schema):
    """A sequence of records whose fields are scalars or sequences (Appendix
    A: record types {l_i : T_i} with T_i possibly [T]; Section 4.3) -> one
    flat layout per field: a scalar field becomes one array of len(records)
    values; a sequence field becomes (values, offsets), its values the
    records' sequences concatenated in record order and offsets[r] ..
    offsets[r + 1] delimiting record r's.  schema: (name, "scalar" | "seq",
    numpy dtype) triples.  Pure Python loops, for small cases."""
    out = {}
    for name, kind, dt in schema:
        if kind == "scalar":
            out[name] = np.array([rec[name] for rec in records], dtype=dt)
            continue
        values, offsets = [], [0]
        for rec in records:
            for x in rec[name]:
                values.append(x)
            offsets.append(len(values))
        out[name] = (np.array(values, dtype=dt), np.array(offsets, dtype=np.int64))
    return out


def unmarshal_record_seqs(layout, schema):
    """Inverse of marshal_record_seqs: a list of dicts, sequence fields as lists."""
    n = None
    for name, kind, _ in schema:
        m = len(layout[name]) if kind == "scalar" else len(layout[name][1]) - 1
        n = m if n is None else n
    recs = [dict() for _ in range(n or 0)]
    for name, kind, _ in schema:
        for r in range(n or 0):
            if kind == "scalar":
                recs[r][name] = layout[name][r].item()
            else:
                vals, off = layout[name]
                recs[r][name] = [v.item() for v in vals[off[r]:off[r + 1]]]
    return recs


def flatten(values, offsets_levels):
    """flatten [[T]] -> [T] on a marshalled value: drop the outermost offsets.

    For depth >= 3 the remaining levels describe the concatenated inner sequences.
    """
    return values, list(offsets_levels[1:])


# ---------------------------------------------------------------- segmented
def segmented_reduce(op: int, ne, values, offsets) -> np.ndarray:
    off = _i64a(offsets)
    nseg = off.size - 1
    if _is_int(values):
        v = _i64a(values)
        out = np.empty(nseg, dtype=np.int64)
        _L().or_segmented_foldl_i64(op, int(ne), _ptr(v), _ptr(off), nseg, _ptr(out))
    else:
        v = _f64(values)
        out = np.empty(nseg, dtype=np.float64)
        _L().or_segmented_foldl_f64(op, float(ne), _ptr(v), _ptr(off), nseg, _ptr(out))
    return out


def segmented_sum_adjoint(gout, offsets) -> np.ndarray:
    off = _i64a(offsets)
    g = _f64(gout)
    out = np.empty(int(off[-1]), dtype=np.float64)
    _L().or_segmented_sum_adjoint_f64(_ptr(g), _ptr(off), off.size - 1, _ptr(out))
    return out


def reduce_adjoint(op: int, ne, s, g) -> np.ndarray:
    """Gradient of foldl op ne s with respect to s, times g (op = ADD, MIN, MAX):
    a broadcast of g for ADD; g at the element the fold ends on (the lowest
    index attaining the extreme, none when ne is not improved upon) for MIN /
    MAX."""
    x = _f64(s).ravel()
    out = np.empty_like(x)
    if _L().or_reduce_adjoint_f64(op, float(ne), _ptr(x), x.size, float(g), _ptr(out)):
        raise ValueError("no reverse mode for this operator")
    return out


def segmented_reduce_adjoint(op: int, ne, values, offsets, gout) -> np.ndarray:
    """Row by row reduce_adjoint of map (reduce op ne) over a ragged sequence."""
    off = _i64a(offsets)
    v = _f64(values).ravel()
    g = _f64(gout).ravel()
    out = np.empty_like(v)
    if _L().or_segmented_reduce_adjoint_f64(op, float(ne), _ptr(v), _ptr(off), off.size - 1, _ptr(g), _ptr(out)):
        raise ValueError("no reverse mode for this operator")
    return out


# ---------------------------------------------------------------- dense
def matmul(A, B, ta: bool = False, tb: bool = False) -> np.ndarray:
    """C = op(A) op(B) with op the identity or the transpose (stored row-major)."""
    a, b = _f64(A), _f64(B)
    M = a.shape[1] if ta else a.shape[0]
    K = a.shape[0] if ta else a.shape[1]
    N = b.shape[0] if tb else b.shape[1]
    Kb = b.shape[1] if tb else b.shape[0]
    if K != Kb:
        raise ValueError("inner dimensions differ")
    C = np.empty((M, N), dtype=np.float64)
    _L().or_matmul_f64(_ptr(a), _ptr(b), _ptr(C), M, N, K, int(ta), int(tb))
    return C


# ---------------------------------------------------------------- N-body loop
def nbody_accel(x, m, eps2: float, G: float = 1.0) -> np.ndarray:
    x, m = _f64(x), _f64(m)
    out = np.empty_like(x)
    _L().or_nbody_accel(_ptr(x), _ptr(m), m.size, eps2, G, _ptr(out))
    return out


def nbody_step(x, v, m, eps2: float, G: float, dt: float):
    x, v, m = _f64(x), _f64(v), _f64(m)
    xo, vo = np.empty_like(x), np.empty_like(v)
    _L().or_nbody_step(_ptr(x), _ptr(v), _ptr(m), m.size, eps2, G, dt, _ptr(xo), _ptr(vo))
    return xo, vo


def nbody_forward(x0, v0, m, eps2: float, G: float, dt: float, nsteps: int, traj: bool = False):
    x0, v0, m = _f64(x0), _f64(v0), _f64(m)
    xo, vo = np.empty_like(x0), np.empty_like(v0)
    tr = np.empty((nsteps + 1,) + x0.shape, dtype=np.float64) if traj else None
    _L().or_nbody_forward(_ptr(x0), _ptr(v0), _ptr(m), m.size, eps2, G, dt, nsteps,
                          _ptr(xo), _ptr(vo), _ptr(tr) if traj else None)
    return (xo, vo, tr) if traj else (xo, vo)


def nbody_kinetic(v, m) -> float:
    v, m = _f64(v), _f64(m)
    return float(_L().or_nbody_kinetic(_ptr(v), _ptr(m), m.size))


def nbody_accel_vjp(x, m, abar, eps2: float, G: float = 1.0) -> np.ndarray:
    x, m, ab = _f64(x), _f64(m), _f64(abar)
    out = np.empty_like(x)
    _L().or_nbody_accel_vjp(_ptr(x), _ptr(m), m.size, eps2, G, _ptr(ab), _ptr(out))
    return out


def nbody_ke_grad(x0, v0, m, eps2: float, G: float, dt: float, nsteps: int,
                  ckpt_every: int | None = None):
    """(KE at t = nsteps, dKE/dx0, dKE/dv0); checkpointed if ckpt_every is given."""
    x0, v0, m = _f64(x0), _f64(v0), _f64(m)
    gx, gv = np.empty_like(x0), np.empty_like(v0)
    if ckpt_every is None:
        ke = _L().or_nbody_ke_grad_tape(_ptr(x0), _ptr(v0), _ptr(m), m.size, eps2, G, dt,
                                        nsteps, _ptr(gx), _ptr(gv))
    else:
        ke = _L().or_nbody_ke_grad_ckpt(_ptr(x0), _ptr(v0), _ptr(m), m.size, eps2, G, dt,
                                        nsteps, ckpt_every, _ptr(gx), _ptr(gv))
    return float(ke), gx, gv


# ---------------------------------------------------------------- k-means
def sqdist(x, c) -> float:
    x, c = _f64(x), _f64(c)
    return float(_L().or_sqdist(_ptr(x), _ptr(c), x.size))


def kmeans_assign(X, C) -> np.ndarray:
    X, C = _f64(X), _f64(C)
    n, d = X.shape
    labels = np.empty(n, dtype=np.int32)
    _L().or_kmeans_assign(_ptr(X), n, d, _ptr(C), C.shape[0], _ptr(labels))
    return labels


def kmeans_update(X, labels, C_old):
    X, C_old = _f64(X), _f64(C_old)
    lab = np.ascontiguousarray(labels, dtype=np.int32)
    n, d = X.shape
    k = C_old.shape[0]
    counts = np.empty(k, dtype=np.int64)
    sums = np.empty((k, d), dtype=np.float64)
    C_new = np.empty((k, d), dtype=np.float64)
    _L().or_kmeans_update(_ptr(X), n, d, _ptr(lab), k, _ptr(C_old), _ptr(counts), _ptr(sums),
                          _ptr(C_new))
    return counts, sums, C_new


def kmeans_step(X, C):
    labels = kmeans_assign(X, C)
    counts, sums, C_new = kmeans_update(X, labels, C)
    return labels, counts, C_new


def kmeans_sse(X, C, labels) -> float:
    X, C = _f64(X), _f64(C)
    lab = np.ascontiguousarray(labels, dtype=np.int32)
    return float(_L().or_kmeans_sse(_ptr(X), X.shape[0], X.shape[1], _ptr(C), _ptr(lab)))


def kmeans_sse_grad(X, C, labels, gscale: float = 1.0) -> np.ndarray:
    X, C = _f64(X), _f64(C)
    lab = np.ascontiguousarray(labels, dtype=np.int32)
    G = np.empty_like(X)
    _L().or_kmeans_sse_grad(_ptr(X), X.shape[0], X.shape[1], _ptr(C), _ptr(lab), gscale, _ptr(G))
    return G


# ---------------------------------------------------------------- batched
def batch_forward(table, A, B, out_len: int) -> np.ndarray:
    tb = _i64a(table).reshape(-1, 6)
    a, b = _f64(A), _f64(B)
    out = np.zeros(out_len, dtype=np.float64)
    _L().or_batch_forward(_ptr(tb), tb.shape[0], _ptr(a), _ptr(b), _ptr(out))
    return out


def batch_backward(table, A, B, gout):
    tb = _i64a(table).reshape(-1, 6)
    a, b, g = _f64(A), _f64(B), _f64(gout)
    gA = np.zeros_like(a)
    gB = np.zeros_like(b)
    _L().or_batch_backward(_ptr(tb), tb.shape[0], _ptr(a), _ptr(b), _ptr(g), _ptr(gA), _ptr(gB))
    return gA, gB


# ---------------------------------------------------------------- user-defined map bodies
def _prog(prog):
    """prog: sequence of (op, dst, a, b, imm) -> int32 code [ninsn x 4], float64 imm [ninsn]."""
    code = np.ascontiguousarray(np.array([[int(p[0]), int(p[1]), int(p[2]), int(p[3])] for p in prog],
                                         dtype=np.int32).reshape(-1, 4))
    imm = np.ascontiguousarray(np.array([float(p[4]) for p in prog], dtype=np.float64))
    return code, imm


def _inputs(inputs):
    X = np.ascontiguousarray(np.stack([_f64(x).ravel() for x in inputs]))
    return X, X.shape[1]


def expr_map(prog, out_reg: int, *inputs) -> np.ndarray:
    """map of the straight-line body `prog` over the inputs (binary64)."""
    code, imm = _prog(prog)
    X, n = _inputs(inputs)
    out = np.zeros(n, dtype=np.float64)
    _L().or_expr_map_f64(_ptr(code), _ptr(imm), code.shape[0], out_reg, _ptr(X), n, _ptr(out))
    return out


def expr_map_reduce(op: int, ne, prog, out_reg: int, *inputs) -> float:
    """foldl op ne (map body inputs) (binary64)."""
    code, imm = _prog(prog)
    X, n = _inputs(inputs)
    return _L().or_expr_map_foldl_f64(op, float(ne), _ptr(code), _ptr(imm), code.shape[0], out_reg, _ptr(X), n)


def expr_vjp(prog, out_reg: int, inputs, gout=None, gscale=None):
    """Per-element reverse mode of the body: list of d body / d input_k times the seed."""
    code, imm = _prog(prog)
    X, n = _inputs(inputs)
    G = np.zeros_like(X)
    g = _f64(gout).ravel() if gout is not None else None
    s = np.array([float(gscale)], dtype=np.float64) if gscale is not None else None
    _L().or_expr_vjp_f64(_ptr(code), _ptr(imm), code.shape[0], X.shape[0], out_reg, _ptr(X), n,
                         _ptr(g) if g is not None else None, _ptr(s) if s is not None else None, _ptr(G))
    return [G[k] for k in range(X.shape[0])]


def expr_loop_scatter(prog, out_reg: int, inputs, idx, out_init):
    """loop over i ascending: out[idx[i]] = body(inputs at i) (binary64); out
    starts as a copy of out_init; indices outside the output are skipped."""
    code, imm = _prog(prog)
    X, n = _inputs(inputs)
    ix = _i64a(idx)
    out = _f64(out_init).copy()
    _L().or_expr_loop_scatter_f64(_ptr(code), _ptr(imm), code.shape[0], out_reg, _ptr(X), n, _ptr(ix), _ptr(out),
                                  out.size)
    return out


# ---------------------------------------------------------------- the general parallel loop
(L_ITER, L_ICONST, L_IADD, L_ISUB, L_IMUL, L_IDIV, L_IMOD, L_IMIN, L_IMAX, L_INEG, L_I2F) = range(32, 43)
L_FGET, L_IGET, L_FSET, L_ISET = 48, 49, 50, 51


def _loop_prog(prog):
    """prog: tuples (op, dst, a, b, c, src, tensor, iimm, fimm)."""
    m = len(prog)
    code = np.zeros((max(m, 1), 8), dtype=np.int32)
    iimm = np.zeros(max(m, 1), dtype=np.int64)
    fimm = np.zeros(max(m, 1), dtype=np.float64)
    for k, q in enumerate(prog):
        code[k, :7] = q[:7]
        iimm[k] = int(q[7])
        fimm[k] = float(q[8])
    return code, iimm, fimm, m


def _loop_tensors(tensors):
    """Working copies: float tensors as float64, integer tensors as int64."""
    arrs, is_int, is32, rank, dims = [], [], [], [], []
    for t in tensors:
        t = np.asarray(t)
        if t.ndim < 1 or t.ndim > 3:
            raise ValueError("tensors have rank 1..3")
        integer = np.issubdtype(t.dtype, np.integer)
        arrs.append(np.ascontiguousarray(t, dtype=np.int64 if integer else np.float64).copy())
        is_int.append(int(integer))
        is32.append(int(t.dtype == np.int32))
        rank.append(t.ndim)
        dims.extend(list(t.shape) + [1] * (3 - t.ndim))
    k = len(arrs)
    ptrs = (ctypes.c_void_p * max(k, 1))(*[a.ctypes.data for a in arrs])
    return (arrs, np.array(is_int or [0], np.int32), np.array(is32 or [0], np.int32), np.array(rank or [1], np.int32),
            np.array(dims or [0, 0, 0], np.int64), ptrs)


def loop_run(prog, tensors, n: int, order=None):
    """loop n f over copies of the tensors, iterations in `order` (default
    ascending).  Returns (tensors after the loop, flags; bit 0: an index was
    out of range)."""
    code, iimm, fimm, m = _loop_prog(prog)
    arrs, is_int, is32, rank, dims, ptrs = _loop_tensors(tensors)
    o = None if order is None else _i64a(order)
    flags = _L().or_loop_run(_ptr(code), _ptr(iimm), _ptr(fimm), m, len(arrs), _ptr(is_int), _ptr(is32), _ptr(rank),
                             _ptr(dims), ptrs, int(n), _ptr(o) if o is not None else None)
    return arrs, int(flags)


def loop_check(prog, tensors, n: int) -> int:
    """The debug-mode verdict: bit 0 an index out of range, bit 1 a slot set by
    two iterations, bit 2 a slot set by one iteration and read by another."""
    code, iimm, fimm, m = _loop_prog(prog)
    arrs, is_int, is32, rank, dims, ptrs = _loop_tensors(tensors)
    return int(_L().or_loop_check(_ptr(code), _ptr(iimm), _ptr(fimm), m, len(arrs), _ptr(is_int), _ptr(is32),
                                  _ptr(rank), _ptr(dims), ptrs, int(n)))


# ---------------------------------------------------------------- Parboil-shaped kernels (Table 1)
def histogram(keys, nbins: int) -> np.ndarray:
    """counts[k] = #{i : keys[i] = k} (int64); keys >= nbins fall in no bin."""
    k = np.ascontiguousarray(np.asarray(keys, dtype=np.uint32))
    counts = np.zeros(int(nbins), dtype=np.int64)
    _L().or_histogram_u32(_ptr(k), k.size, int(nbins), _ptr(counts))
    return counts


def stencil7(grid, c0: float, c1: float) -> np.ndarray:
    """One 7-point Jacobi sweep of a (nz, ny, nx) grid (binary64); boundary copied."""
    g = _f64(grid)
    nz, ny, nx = g.shape
    out = np.empty_like(g)
    _L().or_stencil7(_ptr(g), nx, ny, nz, float(c0), float(c1), _ptr(out))
    return out


def mriq(kx, ky, kz, phi, x, y, z):
    """(Qr, Qi) of the mri-q computation (binary64)."""
    kx, ky, kz, phi = _f64(kx), _f64(ky), _f64(kz), _f64(phi)
    x, y, z = _f64(x), _f64(y), _f64(z)
    qr = np.empty(x.size)
    qi = np.empty(x.size)
    _L().or_mriq(_ptr(kx), _ptr(ky), _ptr(kz), _ptr(phi), kx.size, _ptr(x), _ptr(y), _ptr(z), x.size, _ptr(qr),
                 _ptr(qi))
    return qr, qi


def tpacf(p1, p2, edges, self_pairs: bool) -> np.ndarray:
    """Angular pair counts (int64, len(edges) + 1 bins); points (3, n) binary32
    unit vectors; the dot product and the comparisons in binary32."""
    f = lambda a: np.ascontiguousarray(np.asarray(a, dtype=np.float32))  # noqa: E731
    x1, y1, z1 = (f(c) for c in p1)
    x2, y2, z2 = (f(c) for c in (p1 if self_pairs else p2))
    e = f(edges)
    counts = np.zeros(e.size + 1, dtype=np.int64)
    _L().or_tpacf(_ptr(x1), _ptr(y1), _ptr(z1), x1.size, _ptr(x2), _ptr(y2), _ptr(z2), x2.size, int(self_pairs),
                  _ptr(e), e.size, _ptr(counts))
    return counts
