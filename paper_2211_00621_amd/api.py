"""Convenience layer over the C ABI: output allocation, cached workspaces and
torch.autograd.Function wrappers whose backward calls the library's adjoint
entry points.  Every numeric step runs in libmx.so.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

from . import abi
from .abi import (MX_ADD, MX_MIN, MX_MAX, MX_B_MUL, MX_WS_REDUCE, MX_WS_SCAN, ACC_OF)

# ---------------------------------------------------------------- workspaces
_WS: dict = {}


def workspace(kind: int, n: int, aux: int = 0, device=None, stream=None) -> torch.Tensor:
    """A zero-initialised device workspace for (device, stream, kind), grown on demand.

    The library leaves its counters at zero after each call, so the buffer is
    reused as is; calls sharing it are ordered on the one stream.
    """
    device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    sid = abi._stream(stream)
    need = abi.mx_workspace_bytes(kind, n, aux)
    key = (device.index, sid, kind)
    buf = _WS.get(key)
    if buf is None or buf.numel() < need:
        buf = torch.zeros(max(need, 256), dtype=torch.uint8, device=device)
        _WS[key] = buf
    return buf


# ---------------------------------------------------------------- map / map2 / reduce
def map(f: int, x: torch.Tensor, params=None) -> torch.Tensor:  # noqa: A001 - the paper's keyword
    out = torch.empty(x.shape, dtype=ACC_OF[x.dtype], device=x.device)
    abi.mx_map(f, x.contiguous(), params, out)
    return out


def map2(f: int, a: torch.Tensor, b: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
    if out is None:
        out = torch.empty(a.shape, dtype=ACC_OF[a.dtype], device=a.device)
    abi.mx_map2(f, a.contiguous(), b.contiguous(), out)
    return out


def _reduce(op: int, x: torch.Tensor, ne) -> torch.Tensor:
    out = torch.empty((), dtype=ACC_OF[x.dtype], device=x.device)
    abi.mx_reduce(op, x, ne, out, workspace(MX_WS_REDUCE, x.numel(), device=x.device))
    return out


class _Reduce(torch.autograd.Function):
    """reduce op ne x for float32 x and op in (+, min, max); backward is the
    library's reverse of reduce (a broadcast, or the arg element's scatter)."""

    @staticmethod
    def forward(ctx, x, op, ne):
        ctx.save_for_backward(x)
        ctx.op, ctx.ne = op, ne
        return _reduce(op, x, ne)

    @staticmethod
    def backward(ctx, g):
        (x,) = ctx.saved_tensors
        gx = torch.empty_like(x)
        abi.mx_reduce_adjoint_f32(ctx.op, x, ctx.ne, g.contiguous().view(1), gx,
                                  workspace(MX_WS_REDUCE, x.numel(), device=x.device))
        return gx, None, None


def reduce(op: int, x: torch.Tensor, ne) -> torch.Tensor:
    """reduce op ne x; differentiable for float32 x with op in (+, min, max)."""
    x = x.contiguous().view(-1)
    if x.dtype == torch.float32 and x.requires_grad and op in (MX_ADD, MX_MIN, MX_MAX):
        return _Reduce.apply(x, op, ne)
    return _reduce(op, x, ne)


def map2_reduce(f: int, op: int, a: torch.Tensor, b: torch.Tensor, ne) -> torch.Tensor:
    a, b = a.contiguous().view(-1), b.contiguous().view(-1)
    out = torch.empty((), dtype=ACC_OF[a.dtype], device=a.device)
    abi.mx_map2_reduce(f, op, a, b, ne, out, workspace(MX_WS_REDUCE, a.numel(), device=a.device))
    return out


class _Dot(torch.autograd.Function):
    @staticmethod
    def forward(ctx, a, b):
        ctx.save_for_backward(a, b)
        return map2_reduce(MX_B_MUL, MX_ADD, a, b, 0)

    @staticmethod
    def backward(ctx, g):
        a, b = ctx.saved_tensors
        ga = torch.empty_like(a) if ctx.needs_input_grad[0] else None
        gb = torch.empty_like(b) if ctx.needs_input_grad[1] else None
        abi.mx_dot_adjoint_f32(a, b, g.contiguous().view(1), ga, gb)
        return ga, gb


def dot(a: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
    """reduce (+) 0 (map2 (*) a b); differentiable for float32."""
    a, b = a.contiguous().view(-1), b.contiguous().view(-1)
    if a.dtype == torch.float32 and (a.requires_grad or b.requires_grad):
        return _Dot.apply(a, b)
    return map2_reduce(MX_B_MUL, MX_ADD, a, b, 0)


# ---------------------------------------------------------------- ragged sequences
@dataclass
class Ragged:
    """A marshalled ragged sequence [[T]]: flat values plus int64 offsets (device)."""
    values: torch.Tensor
    offsets: torch.Tensor

    @property
    def nseg(self) -> int:
        return self.offsets.numel() - 1

    def flatten(self) -> torch.Tensor:
        """flatten [[T]] -> [T]: the values themselves (no copy)."""
        return self.values


def offsets_from_lengths(lengths: torch.Tensor) -> torch.Tensor:
    lengths = lengths.contiguous()
    off = torch.empty(lengths.numel() + 1, dtype=torch.int64, device=lengths.device)
    abi.mx_lengths_to_offsets(lengths, off, workspace(MX_WS_SCAN, lengths.numel(), device=lengths.device))
    return off


def ragged_from_lengths(values: torch.Tensor, lengths: torch.Tensor) -> Ragged:
    return Ragged(values, offsets_from_lengths(lengths))


def marshal_rows(rows, device="cuda") -> Ragged:
    """Marshal a list of numpy rows (one dtype) into a device Ragged."""
    nseg = len(rows)
    dt = rows[0].dtype if nseg else np.dtype(np.float32)
    total = int(sum(r.size for r in rows))
    elem = dt.itemsize
    staging = torch.empty(((total * elem + 255) // 256) * 256 + 8 * max(nseg, 1), dtype=torch.uint8,
                          pin_memory=True)
    values = torch.empty(total, dtype=torch.from_numpy(np.zeros(0, dt)).dtype, device=device)
    lengths = torch.empty(nseg, dtype=torch.int64, device=device)
    offsets = torch.empty(nseg + 1, dtype=torch.int64, device=device)
    rows = [np.ascontiguousarray(r) for r in rows]
    abi.mx_marshal_rows(rows, staging, values, lengths, offsets, workspace(MX_WS_SCAN, nseg, device=device))
    torch.cuda.current_stream().synchronize()  # staging is local to this call
    return Ragged(values, offsets)


def unmarshal_rows(r: Ragged):
    off = r.offsets.cpu().numpy()
    np_dt = torch.empty(0, dtype=r.values.dtype).numpy().dtype
    rows = [np.empty(int(off[i + 1] - off[i]), dtype=np_dt) for i in range(r.nseg)]
    staging = torch.empty(max(r.values.numel() * r.values.element_size(), 1), dtype=torch.uint8,
                          pin_memory=True)
    abi.mx_unmarshal_rows(r.values, off, staging, rows)
    return rows


@dataclass
class Nested:
    """A marshalled nested sequence of depth len(offsets) + 1: flat values in
    depth-first order and one int64 offsets array per level, outermost first
    (level l counts the sequences of level l + 1; the last level counts
    values), all on the device."""
    values: torch.Tensor
    offsets: list

    @property
    def depth(self) -> int:
        return len(self.offsets) + 1


def marshal_nested(seq, depth: int, dtype=np.float32, device="cuda") -> Nested:
    """Marshal a nested Python sequence (depth 1..4; depth 1 = [T]) of scalars:
    the innermost sequences go through mx_marshal_rows (host gather, one copy,
    device scan), the upper levels' lengths through mx_lengths_to_offsets."""
    if depth < 1 or depth > 4:
        raise ValueError("depth must be 1..4")
    if depth == 1:
        rows = [np.asarray(seq, dtype=dtype)]
        return Nested(marshal_rows(rows, device).values, [])
    lengths = [[] for _ in range(depth - 2)]   # per upper level, children counts
    leaves = []

    def walk(node, lvl):
        if lvl == depth - 2:
            leaves.append(np.asarray(node, dtype=dtype).ravel())
        else:
            lengths[lvl].append(len(node))
            for child in node:
                walk(child, lvl + 1)

    top = list(seq)
    for node in top:
        walk(node, 0)
    inner = marshal_rows(leaves, device) if leaves else Ragged(
        torch.empty(0, dtype=torch.from_numpy(np.zeros(0, dtype)).dtype, device=device),
        torch.zeros(1, dtype=torch.int64, device=device))
    offsets = []
    for lvl in range(depth - 2):
        L = torch.from_numpy(np.asarray(lengths[lvl], dtype=np.int64)).to(device)
        offsets.append(offsets_from_lengths(L) if L.numel() else torch.zeros(1, dtype=torch.int64,
                                                                               device=device))
    return Nested(inner.values, offsets + [inner.offsets])


def unmarshal_nested(nd: Nested):
    """Inverse of marshal_nested: nested lists whose innermost sequences are
    numpy arrays (mx_unmarshal_rows copies the values back row by row)."""
    if not nd.offsets:
        return unmarshal_rows(Ragged(nd.values, torch.tensor([0, nd.values.numel()], dtype=torch.int64,
                                                               device=nd.values.device)))[0]
    rows = unmarshal_rows(Ragged(nd.values, nd.offsets[-1]))
    levels = [o.cpu().numpy() for o in nd.offsets[:-1]]

    def build(level, i):
        lo, hi = int(levels[level][i]), int(levels[level][i + 1])
        if level == len(levels) - 1:
            return rows[lo:hi]
        return [build(level + 1, j) for j in range(lo, hi)]

    if not levels:
        return rows
    return [build(0, i) for i in range(len(levels[0]) - 1)]


def flatten(nd: Nested, level: int = 0) -> Nested:
    """flatten at nesting level `level` (0 = outermost): the sequences of that
    level are concatenated, so level and level + 1 merge (mx_compose_offsets)."""
    if level < 0 or level >= len(nd.offsets):
        raise ValueError("no such level to flatten")
    if level == 0:
        return Nested(nd.values, nd.offsets[1:])
    outer, inner = nd.offsets[level - 1], nd.offsets[level]
    merged = torch.empty_like(outer)
    abi.mx_compose_offsets(outer, inner, merged)
    return Nested(nd.values, nd.offsets[:level - 1] + [merged] + nd.offsets[level + 1:])


def to_tensor(nd: Nested) -> torch.Tensor:
    """A regular nesting as a dense tensor of rank depth (the rows of every
    level must have equal lengths: mx_offsets_regular)."""
    shape = [nd.offsets[0].numel() - 1] if nd.offsets else []
    for o in nd.offsets:
        shape.append(abi.mx_offsets_regular(o))
    if not nd.offsets:
        shape = [nd.values.numel()]
    return nd.values.view(*shape)


@dataclass
class RecordSeqs:
    """A marshalled sequence of records whose fields are scalars or sequences:
    scalar fields as one device tensor each, sequence fields as Ragged."""
    fields: dict
    nrec: int
    schema: list


def _record_dtype(schema):
    """C layout of a host record: scalar fields in their dtype, sequence fields
    as the C ABI's mx_hseq (data pointer, int64 length)."""
    hseq = np.dtype([("data", np.uint64), ("len", np.int64)], align=True)
    return np.dtype({"names": [n for n, _, _ in schema],
                     "formats": [np.dtype(dt) if kind == "scalar" else hseq for _, kind, dt in schema]}, align=True)


def _field_desc(schema, rdt, tensors=None):
    desc = []
    for name, kind, dt in schema:
        k = abi.MX_FIELD_SCALAR if kind == "scalar" else abi.MX_FIELD_SEQ
        vals, lens, offs = tensors[name] if tensors else (None, None, None)
        desc.append((k, np.dtype(dt).itemsize, rdt.fields[name][1], vals, lens, offs))
    return desc


def marshal_record_seqs(records, schema, device="cuda") -> RecordSeqs:
    """Marshal a list of dict records through the C ABI (mx_marshal_records).
    schema: (name, "scalar" | "seq", numpy dtype) triples."""
    rdt = _record_dtype(schema)
    n = len(records)
    recs = np.zeros(n, dtype=rdt)
    keep = []
    for name, kind, dt in schema:
        if kind == "scalar":
            recs[name] = np.array([r[name] for r in records], dtype=dt) if n else np.zeros(0, dt)
            continue
        for i, r in enumerate(records):
            a = np.ascontiguousarray(np.asarray(r[name], dtype=dt))
            keep.append(a)
            recs[name]["data"][i] = a.ctypes.data if a.size else 0
            recs[name]["len"][i] = a.size
    counts, staging_bytes = abi.mx_records_layout(recs, _field_desc(schema, rdt))
    tensors, out = {}, {}
    for (name, kind, dt), cnt in zip(schema, counts):
        tdt = torch.from_numpy(np.zeros(0, dt)).dtype
        vals = torch.empty(int(cnt), dtype=tdt, device=device)
        if kind == "scalar":
            tensors[name] = (vals, None, None)
            out[name] = vals
        else:
            lens = torch.empty(n, dtype=torch.int64, device=device)
            offs = torch.empty(n + 1, dtype=torch.int64, device=device)
            tensors[name] = (vals, lens, offs)
            out[name] = Ragged(vals, offs)
    staging = torch.empty(max(staging_bytes, 256), dtype=torch.uint8, pin_memory=True)
    abi.mx_marshal_records(recs, _field_desc(schema, rdt, tensors), staging,
                           workspace(MX_WS_SCAN, n, device=device))
    torch.cuda.current_stream().synchronize()  # staging and the host sequences are local to this call
    del keep
    return RecordSeqs(out, n, list(schema))


def unmarshal_record_seqs(rs: RecordSeqs):
    """Back to a list of dict records (mx_unmarshal_records): scalar fields as
    Python scalars, sequence fields as numpy arrays."""
    rdt = _record_dtype(rs.schema)
    n = rs.nrec
    recs = np.zeros(n, dtype=rdt)
    tensors, seqs = {}, {}
    for name, kind, dt in rs.schema:
        f = rs.fields[name]
        if kind == "scalar":
            tensors[name] = (f, None, None)
            continue
        off = f.offsets.cpu().numpy()
        arrs = [np.empty(int(off[i + 1] - off[i]), dtype=dt) for i in range(n)]
        seqs[name] = arrs
        for i, a in enumerate(arrs):
            recs[name]["data"][i] = a.ctypes.data if a.size else 0
            recs[name]["len"][i] = a.size
        tensors[name] = (f.values, None, f.offsets)
    _, staging_bytes = abi.mx_records_layout(recs, _field_desc(rs.schema, rdt))
    staging = torch.empty(max(staging_bytes, 256), dtype=torch.uint8, pin_memory=True)
    abi.mx_unmarshal_records(_field_desc(rs.schema, rdt, tensors), recs, staging)
    out = []
    for i in range(n):
        rec = {}
        for name, kind, _ in rs.schema:
            rec[name] = recs[name][i].item() if kind == "scalar" else seqs[name][i]
        out.append(rec)
    return out


def records_to_fields(aos: torch.Tensor):
    fields = [torch.empty(aos.shape[0], dtype=aos.dtype, device=aos.device) for _ in range(aos.shape[1])]
    abi.mx_records_to_fields(aos.contiguous(), fields)
    return fields


def fields_to_records(fields) -> torch.Tensor:
    aos = torch.empty((fields[0].numel(), len(fields)), dtype=fields[0].dtype, device=fields[0].device)
    abi.mx_fields_to_records([f.contiguous() for f in fields], aos)
    return aos


def _segmented_reduce(op: int, r: Ragged, ne, plain: bool = False) -> torch.Tensor:
    out = torch.empty(r.nseg, dtype=ACC_OF[r.values.dtype], device=r.values.device)
    if plain:
        abi.mx_segmented_reduce_plain(op, r.values, r.offsets, ne, out)
    else:
        ws = workspace(abi.MX_WS_SEGMENTED, r.values.numel(), device=r.values.device)
        abi.mx_segmented_reduce(op, r.values, r.offsets, ne, out, ws)
    return out


class _SegReduce(torch.autograd.Function):
    @staticmethod
    def forward(ctx, values, offsets, op, ne):
        ctx.save_for_backward(values, offsets)
        ctx.op, ctx.ne = op, ne
        return _segmented_reduce(op, Ragged(values, offsets), ne)

    @staticmethod
    def backward(ctx, g):
        values, offsets = ctx.saved_tensors
        gv = torch.empty_like(values)
        abi.mx_segmented_reduce_adjoint_f32(ctx.op, values, offsets, ctx.ne, g.contiguous(), gv)
        return gv, None, None, None


def segmented_reduce(op: int, r: Ragged, ne, plain: bool = False) -> torch.Tensor:
    """map (reduce op ne) over the rows; differentiable for float32 values with
    op in (+, min, max)."""
    if (not plain and r.values.dtype == torch.float32 and r.values.requires_grad
            and op in (MX_ADD, MX_MIN, MX_MAX)):
        return _SegReduce.apply(r.values, r.offsets, op, ne)
    return _segmented_reduce(op, r, ne, plain)


class _SegSum(torch.autograd.Function):
    @staticmethod
    def forward(ctx, values, offsets):
        ctx.save_for_backward(offsets)
        ctx.n = values.numel()
        out = torch.empty(offsets.numel() - 1, dtype=values.dtype, device=values.device)
        ws = workspace(abi.MX_WS_SEGMENTED, values.numel(), device=values.device)
        abi.mx_segmented_reduce(MX_ADD, values, offsets, 0.0, out, ws)
        return out

    @staticmethod
    def backward(ctx, g):
        (offsets,) = ctx.saved_tensors
        gv = torch.empty(ctx.n, dtype=g.dtype, device=g.device)
        abi.mx_segmented_sum_adjoint_f32(g.contiguous(), offsets, gv)
        return gv, None


def segmented_sum(r: Ragged) -> torch.Tensor:
    """map (reduce (+) 0) over the rows; differentiable for float32 values."""
    if r.values.dtype == torch.float32 and r.values.requires_grad:
        return _SegSum.apply(r.values, r.offsets)
    return _segmented_reduce(MX_ADD, r, 0)


# ---------------------------------------------------------------- dense
class _MapMapReduce(torch.autograd.Function):
    @staticmethod
    def forward(ctx, A, B):
        ctx.save_for_backward(A, B)
        C = torch.empty((A.shape[0], B.shape[1]), dtype=torch.float32, device=A.device)
        abi.mx_map_map_reduce_f32(0, 0, A, B, C)
        return C

    @staticmethod
    def backward(ctx, gC):
        A, B = ctx.saved_tensors
        gC = gC.contiguous()
        gA = gB = None
        if ctx.needs_input_grad[0]:
            gA = torch.empty_like(A)
            abi.mx_map_map_reduce_f32(0, 1, gC, B, gA)  # dC B^T
        if ctx.needs_input_grad[1]:
            gB = torch.empty_like(B)
            abi.mx_map_map_reduce_f32(1, 0, A, gC, gB)  # A^T dC
        return gA, gB


def matmul(A: torch.Tensor, B: torch.Tensor, plain: bool = False) -> torch.Tensor:
    """C[i][j] = reduce (+) 0 (map2 (*) A[i,:] B[:,j]) in FP32 on the matrix cores."""
    A, B = A.contiguous(), B.contiguous()
    if not plain and (A.requires_grad or B.requires_grad):
        return _MapMapReduce.apply(A, B)
    C = torch.empty((A.shape[0], B.shape[1]), dtype=torch.float32, device=A.device)
    (abi.mx_map_map_reduce_plain_f32 if plain else abi.mx_map_map_reduce_f32)(0, 0, A, B, C)
    return C


# ---------------------------------------------------------------- N-body loop
_BYTES_WS: dict = {}


def bytes_workspace(nbytes: int, tag: str, device=None, stream=None) -> torch.Tensor:
    """A zero-initialised device workspace of at least nbytes for (device, stream, tag)."""
    device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    key = (device.index, abi._stream(stream), tag)
    buf = _BYTES_WS.get(key)
    if buf is None or buf.numel() < nbytes:
        buf = torch.zeros(max(nbytes, 256), dtype=torch.uint8, device=device)
        _BYTES_WS[key] = buf
    return buf


def bodies(pos: torch.Tensor, mass: torch.Tensor) -> torch.Tensor:
    """The record {x, y, z, m} of each body as one float4 row (marshalling on the device)."""
    return fields_to_records([pos[:, 0].contiguous(), pos[:, 1].contiguous(), pos[:, 2].contiguous(),
                              mass.contiguous()])


def vec4(v: torch.Tensor) -> torch.Tensor:
    out = torch.zeros((v.shape[0], 4), dtype=torch.float32, device=v.device)
    out[:, :3] = v
    return out


def nbody_accel(pos4: torch.Tensor, eps2: float, G: float = 1.0) -> torch.Tensor:
    acc = torch.empty_like(pos4)
    ws = bytes_workspace(abi.mx_nbody_pair_workspace_bytes(pos4.shape[0]), "nbody_pair", pos4.device)
    abi.mx_nbody_accel_f32(pos4, eps2, G, acc, ws)
    return acc


def nbody_step(pos4, vel4, eps2, G, dt, plain: bool = False):
    xo, vo = torch.empty_like(pos4), torch.empty_like(vel4)
    if plain:
        acc = torch.empty_like(pos4)
        abi.mx_nbody_step_plain_f32(pos4, vel4, eps2, G, dt, acc, xo, vo)
    else:
        ws = bytes_workspace(abi.mx_nbody_pair_workspace_bytes(pos4.shape[0]), "nbody_pair", pos4.device)
        abi.mx_nbody_step_f32(pos4, vel4, eps2, G, dt, xo, vo, ws)
    return xo, vo


def nbody_accel_vjp(pos4, abar4, eps2, G=1.0):
    out = torch.empty_like(pos4)
    ws = bytes_workspace(abi.mx_nbody_pair_workspace_bytes(pos4.shape[0]), "nbody_pair", pos4.device)
    abi.mx_nbody_accel_vjp_f32(pos4, abar4, eps2, G, out, ws)
    return out


def nbody_ke_grad(pos4, vel4, eps2, G, dt, nsteps, ckpt_every):
    """(KE at t = nsteps, dKE/dx0 [n,4], dKE/dv0 [n,4]) with checkpointed reverse."""
    n = pos4.shape[0]
    ke = torch.empty((), dtype=torch.float32, device=pos4.device)
    gx, gv = torch.empty_like(pos4), torch.empty_like(pos4)
    ws = bytes_workspace(abi.mx_nbody_workspace_bytes(n, nsteps, ckpt_every), "nbody_loop", pos4.device)
    abi.mx_nbody_ke_grad_f32(pos4, vel4, eps2, G, dt, nsteps, ckpt_every, ke, gx, gv, ws)
    return ke, gx, gv


class _NBodyKE(torch.autograd.Function):
    """KE after an Euler loop as a differentiable function of (x0, v0).

    forward runs the loop and keeps its checkpoints in a workspace of its own;
    backward runs the checkpointed reverse sweep from them, seeded on the
    device with the upstream gradient."""

    @staticmethod
    def forward(ctx, pos, vel, mass, eps2, G, dt, nsteps, ckpt_every):
        p4 = bodies(pos, mass)
        v4 = vec4(vel)
        n = p4.shape[0]
        ke = torch.empty((), dtype=torch.float32, device=p4.device)
        ws = torch.zeros(max(abi.mx_nbody_workspace_bytes(n, nsteps, ckpt_every), 256), dtype=torch.uint8,
                         device=p4.device)
        abi.mx_nbody_ke_f32(p4, v4, eps2, G, dt, nsteps, ckpt_every, ke, ws)
        ctx.save_for_backward(p4, v4, ws)
        ctx.args = (eps2, G, dt, nsteps, ckpt_every)
        return ke

    @staticmethod
    def backward(ctx, g):
        p4, v4, ws = ctx.saved_tensors
        eps2, G, dt, nsteps, ckpt_every = ctx.args
        gx, gv = torch.empty_like(p4), torch.empty_like(p4)
        gs = g.detach().to(torch.float32).contiguous().view(1)
        abi.mx_nbody_ke_vjp_f32(p4, v4, eps2, G, dt, nsteps, ckpt_every, gs, gx, gv, ws)
        return (gx[:, :3], gv[:, :3], None, None, None, None, None, None)


def nbody_kinetic_energy(pos, vel, mass, eps2, G, dt, nsteps, ckpt_every=5):
    """KE(t = nsteps) of the Euler loop; backward runs the checkpointed reverse sweep."""
    return _NBodyKE.apply(pos, vel, mass, eps2, G, dt, nsteps, ckpt_every)


# ---------------------------------------------------------------- k-means
def kmeans_step(X: torch.Tensor, C: torch.Tensor, plain: bool = False):
    """(labels int32[n], counts int64[k], C' float32[k, d]) of one k-means step."""
    n, d = X.shape
    k = C.shape[0]
    labels = torch.empty(n, dtype=torch.int32, device=X.device)
    counts = torch.empty(k, dtype=torch.int64, device=X.device)
    C_out = torch.empty_like(C)
    ws = bytes_workspace(abi.mx_kmeans_workspace_bytes(n, d, k), "kmeans", X.device)
    (abi.mx_kmeans_step_plain_f32 if plain else abi.mx_kmeans_step_f32)(X, C, labels, counts, C_out, ws)
    return labels, counts, C_out


class _KMeansSSE(torch.autograd.Function):
    @staticmethod
    def forward(ctx, X, C, labels):
        ctx.save_for_backward(X, C, labels)
        out = torch.empty((), dtype=torch.float32, device=X.device)
        abi.mx_kmeans_sse_f32(X, C, labels, out, bytes_workspace(256 + 4096, "kmeans_sse", X.device))
        return out

    @staticmethod
    def backward(ctx, g):
        X, C, labels = ctx.saved_tensors
        G = torch.empty_like(X)
        abi.mx_kmeans_sse_grad_f32(X, C, labels, g.contiguous().view(1), G)
        return G, None, None


def kmeans_sse(X: torch.Tensor, C: torch.Tensor, labels: torch.Tensor) -> torch.Tensor:
    """Within-cluster sum of squares; differentiable with respect to X."""
    return _KMeansSSE.apply(X, C, labels)


# ---------------------------------------------------------------- batches
class Batch:
    """A plan for many uneven dot / matvec expressions and its workspace."""

    def __init__(self, table, cfg=None, device=None):
        self.plan = abi.mx_batch_plan_create(np.asarray(table), cfg)
        device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        self.ws = torch.zeros(max(abi.mx_batch_workspace_bytes(self.plan), 256), dtype=torch.uint8, device=device)

    @property
    def config(self):
        return abi.mx_batch_get_config(self.plan)

    def forward(self, A, B, out, plain=False, stream=None):
        if plain:
            abi.mx_batch_forward_plain(self.plan, A, B, out, stream)
        else:
            abi.mx_batch_forward(self.plan, A, B, out, self.ws, stream)
        return out

    def backward(self, A, B, gout, gA, gB, plain=False, stream=None):
        if plain:
            abi.mx_batch_backward_plain(self.plan, A, B, gout, gA, gB, stream)
        else:
            abi.mx_batch_backward(self.plan, A, B, gout, gA, gB, self.ws, stream)
        return gA, gB

    def autotune(self, A, B, out, gout, gA, gB, cache_path=None, stream=None):
        return abi.mx_batch_autotune(self.plan, A, B, out, gout, gA, gB, self.ws, cache_path, stream)


# ---------------------------------------------------------------- user-defined map bodies
class Var:
    """A value of a map body under construction: the body is written with the
    usual operators on the results of ``body_inputs`` and lowered to the C
    ABI's straight-line register program by ``Body``."""

    def __init__(self, op: int, args=(), imm: float = 0.0, index: int = 0):
        self.op, self.args, self.imm, self.index = op, tuple(args), float(imm), index

    @staticmethod
    def of(x) -> "Var":
        return x if isinstance(x, Var) else Var(abi.MX_X_CONST, imm=float(x))

    def _bin(self, op, other, swap=False):
        a, b = (Var.of(other), self) if swap else (self, Var.of(other))
        return Var(op, (a, b))

    def __add__(self, o): return self._bin(abi.MX_X_ADD, o)
    def __radd__(self, o): return self._bin(abi.MX_X_ADD, o, True)
    def __sub__(self, o): return self._bin(abi.MX_X_SUB, o)
    def __rsub__(self, o): return self._bin(abi.MX_X_SUB, o, True)
    def __mul__(self, o): return self._bin(abi.MX_X_MUL, o)
    def __rmul__(self, o): return self._bin(abi.MX_X_MUL, o, True)
    def __truediv__(self, o): return self._bin(abi.MX_X_DIV, o)
    def __rtruediv__(self, o): return self._bin(abi.MX_X_DIV, o, True)
    def __neg__(self): return Var(abi.MX_X_NEG, (self,))
    def __abs__(self): return Var(abi.MX_X_ABS, (self,))

    def __pow__(self, p):
        if p != 2:
            raise ValueError("only x ** 2 is a body operation")
        return Var(abi.MX_X_SQ, (self,))


def body_inputs(n: int):
    return tuple(Var(abi.MX_X_IN, index=k) for k in range(n))


def exp(x): return Var(abi.MX_X_EXP, (Var.of(x),))
def log(x): return Var(abi.MX_X_LOG, (Var.of(x),))
def sqrt(x): return Var(abi.MX_X_SQRT, (Var.of(x),))
def rsqrt(x): return Var(abi.MX_X_RSQRT, (Var.of(x),))
def minimum(a, b): return Var(abi.MX_X_MIN, (Var.of(a), Var.of(b)))
def maximum(a, b): return Var(abi.MX_X_MAX, (Var.of(a), Var.of(b)))


def lower_body(out: Var, nregs: int = 16):
    """Straight-line program (op, dst, a, b, imm) and output register for the
    expression `out`: nodes in post order (shared nodes once), a register
    freed after the last read of its value."""
    order, seen = [], {}

    def visit(v):
        if id(v) in seen:
            return
        for a in v.args:
            visit(a)
        seen[id(v)] = len(order)
        order.append(v)

    visit(out)
    last_use = {}
    for pos, v in enumerate(order):
        for a in v.args:
            last_use[id(a)] = pos
    free, reg, prog = list(range(nregs - 1, -1, -1)), {}, []
    for pos, v in enumerate(order):
        srcs = [reg[id(a)] for a in v.args]
        # operands read for the last time give their registers back (the
        # instruction reads them before it writes its result)
        for a in {id(a): a for a in v.args}.values():
            if last_use.get(id(a)) == pos and id(a) != id(out):
                free.append(reg[id(a)])
        if not free:
            raise ValueError(f"the body needs more than {nregs} live values")
        dst = free.pop()
        reg[id(v)] = dst
        a = srcs[0] if srcs else (v.index if v.op == abi.MX_X_IN else 0)
        b = srcs[1] if len(srcs) > 1 else 0
        prog.append((v.op, dst, a, b, v.imm))
    return prog, reg[id(out)]


class Body:
    """A user-defined map body compiled by the library (hipRTC) into fused
    map, map + reduce and reverse-mode kernels."""

    def __init__(self, out: Var, nin: int, dtype=torch.float32):
        self.prog, self.out_reg = lower_body(out)
        self.nin, self.torch_dtype = nin, dtype
        self.e = abi.mx_expr_create(self.prog, nin, self.out_reg, abi.DTYPE_OF[dtype])
        self._ws = {}

    def _args(self, xs):
        if len(xs) != self.nin:
            raise ValueError(f"the body takes {self.nin} inputs")
        xs = [x.contiguous().view(-1) for x in xs]
        n = xs[0].numel()
        if any(x.numel() != n or x.dtype != self.torch_dtype for x in xs):
            raise abi.MxError(abi.MX_ERR_SHAPE, "inputs differ in length or dtype")
        return xs, n

    def _map(self, *xs) -> torch.Tensor:
        xs, n = self._args(xs)
        out = torch.empty(n, dtype=self.torch_dtype, device=xs[0].device)
        abi.mx_expr_map(self.e, xs, out)
        return out

    def _grad(self, xs) -> bool:
        return self.torch_dtype == torch.float32 and torch.is_grad_enabled() and any(x.requires_grad for x in xs)

    def map(self, *xs) -> torch.Tensor:
        """map body xs (flat); differentiable for float32 (reverse mode of the body)."""
        if self._grad(xs):
            return _BodyMap.apply(self, *xs)
        return self._map(*xs)

    def map_reduce(self, op: int, *xs, ne=0.0) -> torch.Tensor:
        """reduce op ne (map body xs); differentiable for float32 with op in (+, min, max)."""
        if self._grad(xs) and op in (MX_ADD, MX_MIN, MX_MAX):
            return _BodyMapReduce.apply(self, op, ne, *xs)
        return self._map_reduce(op, *xs, ne=ne)

    def _map_reduce(self, op: int, *xs, ne=0.0) -> torch.Tensor:
        xs, n = self._args(xs)
        out = torch.empty((), dtype=self.torch_dtype, device=xs[0].device)
        key = xs[0].device.index
        ws = self._ws.get(key)
        need = abi.mx_expr_workspace_bytes(self.e, n)
        if ws is None or ws.numel() < need:
            ws = self._ws[key] = torch.zeros(need, dtype=torch.uint8, device=xs[0].device)
        abi.mx_expr_map_reduce(self.e, op, xs, n, ne, out, ws)
        return out

    def segmented_reduce(self, op: int, offsets: torch.Tensor, *xs, ne=0.0) -> torch.Tensor:
        """out[r] = ne op body(x_i) ... over the elements i of ragged row r;
        differentiable for float32 with op in (+, min, max)."""
        if self._grad(xs) and op in (MX_ADD, MX_MIN, MX_MAX):
            return _BodySegReduce.apply(self, op, ne, offsets, *xs)
        return self._segmented_reduce(op, offsets, *xs, ne=ne)

    def _segmented_reduce(self, op: int, offsets: torch.Tensor, *xs, ne=0.0) -> torch.Tensor:
        xs, n = self._args(xs)
        out = torch.empty(offsets.numel() - 1, dtype=self.torch_dtype, device=xs[0].device)
        abi.mx_expr_segmented_reduce(self.e, op, xs, offsets, ne, out)
        return out

    def vjp(self, *xs, gout=None, gscale=None):
        xs, n = self._args(xs)
        grads = [torch.empty_like(x) for x in xs]
        abi.mx_expr_vjp(self.e, xs, n, None if gout is None else gout.contiguous().view(-1),
                        None if gscale is None else gscale.contiguous().view(1), grads)
        return grads

    def sum(self, *xs) -> torch.Tensor:
        """reduce (+) 0 (map body xs), differentiable."""
        return _BodySum.apply(self, *xs)


class _BodySum(torch.autograd.Function):
    @staticmethod
    def forward(ctx, body, *xs):
        ctx.body = body
        ctx.save_for_backward(*xs)
        return body._map_reduce(MX_ADD, *xs, ne=0.0)

    @staticmethod
    def backward(ctx, g):
        xs = ctx.saved_tensors
        grads = ctx.body.vjp(*xs, gscale=g.contiguous().to(ctx.body.torch_dtype))
        return (None, *[gr.view(x.shape) for gr, x in zip(grads, xs)])


def _shaped(grads, xs):
    return [gr.view(x.shape) for gr, x in zip(grads, xs)]


class _BodyMap(torch.autograd.Function):
    """map body xs; backward: the body's reverse mode seeded with the
    upstream gradient of every element."""

    @staticmethod
    def forward(ctx, body, *xs):
        ctx.body = body
        ctx.save_for_backward(*xs)
        return body._map(*xs)

    @staticmethod
    def backward(ctx, g):
        xs = ctx.saved_tensors
        return (None, *_shaped(ctx.body.vjp(*xs, gout=g.contiguous()), xs))


class _BodyMapReduce(torch.autograd.Function):
    """reduce op ne (map body xs): the reverse of the reduce (broadcast for +,
    the arg element for min / max) over the body's values, then the body's
    reverse mode with that as the per-element seed."""

    @staticmethod
    def forward(ctx, body, op, ne, *xs):
        ctx.body, ctx.op, ctx.ne = body, op, ne
        ctx.save_for_backward(*xs)
        return body._map_reduce(op, *xs, ne=ne)

    @staticmethod
    def backward(ctx, g):
        xs = ctx.saved_tensors
        body = ctx.body
        g = g.contiguous().view(1)
        if ctx.op == MX_ADD:
            grads = body.vjp(*xs, gscale=g)
        else:
            vals = body._map(*xs)
            seed = torch.empty_like(vals)
            abi.mx_reduce_adjoint_f32(ctx.op, vals, ctx.ne, g, seed,
                                      workspace(MX_WS_REDUCE, vals.numel(), device=vals.device))
            grads = body.vjp(*xs, gout=seed)
        return (None, None, None, *_shaped(grads, xs))


class _BodySegReduce(torch.autograd.Function):
    """map (reduce op ne . map body) over ragged rows: the reverse of each
    row's reduce over the body's values, then the body's reverse mode."""

    @staticmethod
    def forward(ctx, body, op, ne, offsets, *xs):
        ctx.body, ctx.op, ctx.ne = body, op, ne
        ctx.save_for_backward(offsets, *xs)
        return body._segmented_reduce(op, offsets, *xs, ne=ne)

    @staticmethod
    def backward(ctx, g):
        offsets, *xs = ctx.saved_tensors
        body = ctx.body
        n = xs[0].numel()
        seed = torch.empty(n, dtype=torch.float32, device=g.device)
        vals = body._map(*xs) if ctx.op != MX_ADD else None
        abi.mx_segmented_reduce_adjoint_f32(ctx.op, vals, offsets, ctx.ne, g.contiguous(), seed)
        return (None, None, None, None, *_shaped(body.vjp(*xs, gout=seed), xs))


# ---------------------------------------------------------------- the general parallel loop
class _LVal:
    """A value of a loop body under construction (integer or float register)."""

    def __init__(self, lp: "ParallelLoop", reg: int, is_int: bool):
        self.lp, self.reg, self.is_int = lp, reg, is_int

    def _other(self, o):
        if isinstance(o, _LVal):
            if o.is_int != self.is_int:
                raise TypeError("integer and float values do not mix; use .to_float()")
            return o
        return self.lp.const(o, self.is_int)

    def _bin(self, iop, fop, o, swap=False):
        o = self._other(o)
        a, b = (o, self) if swap else (self, o)
        return self.lp._emit(iop if self.is_int else fop, self.is_int, a=a.reg, b=b.reg)

    def __add__(self, o): return self._bin(abi.MX_L_IADD, abi.MX_X_ADD, o)
    def __radd__(self, o): return self._bin(abi.MX_L_IADD, abi.MX_X_ADD, o, True)
    def __sub__(self, o): return self._bin(abi.MX_L_ISUB, abi.MX_X_SUB, o)
    def __rsub__(self, o): return self._bin(abi.MX_L_ISUB, abi.MX_X_SUB, o, True)
    def __mul__(self, o): return self._bin(abi.MX_L_IMUL, abi.MX_X_MUL, o)
    def __rmul__(self, o): return self._bin(abi.MX_L_IMUL, abi.MX_X_MUL, o, True)

    def __truediv__(self, o):
        if self.is_int:
            raise TypeError("integer division is //")
        return self._bin(None, abi.MX_X_DIV, o)

    def __floordiv__(self, o):
        """Integer division truncating toward zero (C semantics; 0 for a zero divisor)."""
        if not self.is_int:
            raise TypeError("// is integer division")
        return self._bin(abi.MX_L_IDIV, None, o)

    def __mod__(self, o):
        if not self.is_int:
            raise TypeError("% is the integer remainder")
        return self._bin(abi.MX_L_IMOD, None, o)

    def __neg__(self):
        return self.lp._emit(abi.MX_L_INEG if self.is_int else abi.MX_X_NEG, self.is_int, a=self.reg)

    def to_float(self):
        if not self.is_int:
            return self
        return self.lp._emit(abi.MX_L_I2F, False, a=self.reg)


class ParallelLoop:
    """`loop n f` with tensorGet / tensorSet: the body is written imperatively
    against an iteration value, compiled by the library (hipRTC) on first run.

        lp = ParallelLoop([(torch.float32, 1), (torch.float32, 1)])
        i = lp.iteration
        lp.set(0, i, lp.get(0, i) + 2.0 * lp.get(1, i))     # Listing 1's axpy
        lp.run(n, t1, t2)
    """

    def __init__(self, types, float_dtype=torch.float32):
        self.types = [(abi.DTYPE_OF[dt], int(rank)) for dt, rank in types]
        self.float_dtype = abi.DTYPE_OF[float_dtype]
        self.prog = []
        self._next = [0, 0]  # float, int registers
        self._handle = None
        self.iteration = self._emit(abi.MX_L_ITER, True)

    def _reg(self, is_int):
        r = self._next[is_int]
        if r >= 64:
            raise ValueError("the loop body needs more than 64 registers of one kind")
        self._next[is_int] += 1
        return r

    def _emit(self, op, is_int, a=0, b=0, iimm=0, fimm=0.0):
        dst = self._reg(is_int)
        self.prog.append((op, dst, a, b, 0, 0, 0, iimm, fimm))
        self._handle = None
        return _LVal(self, dst, is_int)

    def const(self, v, is_int=None):
        if is_int is None:
            is_int = isinstance(v, (int, np.integer))
        if is_int:
            return self._emit(abi.MX_L_ICONST, True, iimm=int(v))
        return self._emit(abi.MX_X_CONST, False, fimm=float(v))

    def _index(self, t, idx):
        rank = self.types[t][1]
        idx = list(idx)
        if len(idx) != rank:
            raise ValueError(f"tensor {t} has rank {rank}")
        regs = [(x if isinstance(x, _LVal) else self.const(int(x), True)) for x in idx]
        if any(not r.is_int for r in regs):
            raise TypeError("indices are integer values")
        regs = [r.reg for r in regs] + [0] * (3 - rank)
        return regs

    def get(self, t: int, *idx) -> _LVal:
        a, b, c = self._index(t, idx)
        is_int = self.types[t][0] in (abi.MX_I32, abi.MX_I64)
        dst = self._reg(is_int)
        self.prog.append((abi.MX_L_IGET if is_int else abi.MX_L_FGET, dst, a, b, c, 0, t, 0, 0.0))
        self._handle = None
        return _LVal(self, dst, is_int)

    def set(self, t: int, idx, value) -> None:
        if not isinstance(idx, (tuple, list)):
            idx = (idx,)
        a, b, c = self._index(t, idx)
        is_int = self.types[t][0] in (abi.MX_I32, abi.MX_I64)
        if not isinstance(value, _LVal):
            value = self.const(value, is_int)
        if value.is_int != is_int:
            raise TypeError("the value's kind differs from the tensor's element kind")
        self.prog.append((abi.MX_L_ISET if is_int else abi.MX_L_FSET, 0, a, b, c, value.reg, t, 0, 0.0))
        self._handle = None

    def unary(self, xop: int, x: _LVal) -> _LVal:
        """f(x) for a float map-body operator (MX_X_NEG .. MX_X_RSQRT)."""
        return self._emit(xop, False, a=x.reg)

    def binary(self, op: int, x: _LVal, y) -> _LVal:
        """min / max (MX_X_MIN / MX_X_MAX, or MX_L_IMIN / MX_L_IMAX) and the other binary codes."""
        y = x._other(y)
        return self._emit(op, x.is_int, a=x.reg, b=y.reg)

    @property
    def handle(self):
        if self._handle is None:
            self._handle = abi.mx_loop_create(self.prog, self.types, self.float_dtype)
        return self._handle

    def source(self) -> str:
        return abi.mx_loop_source(self.handle)

    def run(self, n: int, *tensors, stream=None) -> None:
        ts = [t if t.is_contiguous() else t.contiguous() for t in tensors]
        if any(a is not b for a, b in zip(ts, tensors)):
            raise ValueError("loop tensors must be contiguous (they are written in place)")
        ws = None
        if abi.mx_get_debug():
            ws = torch.zeros(max(abi.mx_loop_workspace_bytes(self.handle, ts), 256), dtype=torch.uint8,
                             device=ts[0].device if ts else None)
        abi.mx_loop_run(self.handle, n, ts, ws, stream)
