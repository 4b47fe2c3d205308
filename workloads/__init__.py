"""Seeded synthetic inputs shared by the oracle tests, the GPU parity tests and the bench.

This module only draws random numbers and lays them out (lengths, offsets into
pools, task tables).  It holds none of the primitives' arithmetic: no map body,
no reduction, no update step.  Everything is drawn with numpy's PCG64
(``numpy.random.default_rng(seed)``), in float64 and then cast to float32
(integers are drawn directly as int32).

Workload shapes follow the paper's evaluation programs (Section 5) as
synthetic stand-ins, since the paper's datasets (Parboil inputs, MNIST,
CIFAR-10, the ODE model) are not available:

* ``dot``      -- two vectors for ``reduce (+) 0 (map2 (*) a b)``
* ``ragged``   -- a ragged sequence of rows for a nested ``map (reduce)``
* ``dense``    -- two matrices for the nested ``map (map (reduce (map2)))``
                  (the sgemm pattern of Table 1)
* ``nbody``    -- bodies for a sequential loop around a pairwise map(reduce)
                  (the ODE-solver pattern of Table 2)
* ``kmeans``   -- Gaussian blobs for map(argmin-reduce) + reduce-by-key
                  (the histo reduce-by-key pattern of Table 1)
* ``batched``  -- many uneven dot / matvec expressions (the neural-network
                  matvec pattern of Table 2, many accelerate uses)
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "dot_f32", "dot_i32", "ragged_lengths", "ragged_f32", "dense_f32",
    "nbody", "kmeans_blobs", "batched_tasks", "BatchedTasks",
    "TASK_DOT", "TASK_MATVEC",
]

TASK_DOT = 0
TASK_MATVEC = 1


def _rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def _uniform_f32(rng: np.random.Generator, lo: float, hi: float, size) -> np.ndarray:
    return rng.uniform(lo, hi, size).astype(np.float32)


def dot_f32(n: int, seed: int = 0):
    """Two float32 vectors of length n, uniform in [-1, 1]."""
    rng = _rng(seed)
    a = _uniform_f32(rng, -1.0, 1.0, n)
    b = _uniform_f32(rng, -1.0, 1.0, n)
    return a, b


def dot_i32(n: int, seed: int = 0):
    """Two int32 vectors of length n, uniform on the integers [-1000, 1000]."""
    rng = _rng(seed)
    a = rng.integers(-1000, 1001, n, dtype=np.int32)
    b = rng.integers(-1000, 1001, n, dtype=np.int32)
    return a, b


def ragged_lengths(nseg: int, seed: int = 0, lmax: int = 4096, lmin: int = 1) -> np.ndarray:
    """Row lengths L = floor(exp(U[ln lmin, ln(lmax+1)))), so L lies in [lmin, lmax].

    P(L = k) is proportional to ln((k+1)/k): log-uniform over [1, lmax].
    """
    rng = _rng(seed)
    u = rng.uniform(math.log(lmin), math.log(lmax + 1), nseg)
    lengths = np.floor(np.exp(u)).astype(np.int64)
    return np.clip(lengths, lmin, lmax)


def ragged_f32(nseg: int, seed: int = 0, lmax: int = 4096, empty_rows: int = 0):
    """Ragged float32 rows, values uniform in [-1, 1].

    Returns (lengths int64[nseg], values float32[sum L]).  If ``empty_rows`` is
    positive, that many seeded rows are set to length zero (edge cases).
    """
    lengths = ragged_lengths(nseg, seed, lmax)
    if empty_rows:
        rng = _rng(seed + 7919)
        idx = rng.choice(nseg, size=min(empty_rows, nseg), replace=False)
        lengths[idx] = 0
    rng = _rng(seed + 1)
    values = _uniform_f32(rng, -1.0, 1.0, int(lengths.sum()))
    return lengths, values


def dense_f32(m: int, n: int, k: int, seed: int = 0):
    """Row-major float32 A[m,k] and B[k,n], uniform in [-1, 1]."""
    rng = _rng(seed)
    a = _uniform_f32(rng, -1.0, 1.0, (m, k))
    b = _uniform_f32(rng, -1.0, 1.0, (k, n))
    return a, b


def nbody(n: int, seed: int = 0):
    """N bodies: positions uniform in the unit cube, masses uniform in [0.5, 1.5].

    Returns (pos float32[n,3], mass float32[n], vel float32[n,3] = 0).
    """
    rng = _rng(seed)
    pos = _uniform_f32(rng, 0.0, 1.0, (n, 3))
    mass = _uniform_f32(rng, 0.5, 1.5, n)
    vel = np.zeros((n, 3), dtype=np.float32)
    return pos, mass, vel


def kmeans_blobs(n: int, d: int, nblobs: int, seed: int = 0, spread: float = 10.0,
                 sigma: float = 1.0):
    """Points drawn from ``nblobs`` isotropic Gaussian blobs.

    Blob centres are uniform in [-spread, spread]^d; each point picks its blob
    i.i.d. uniformly (so blob membership is in random order) and adds N(0, sigma^2)
    noise.  Returns (X float32[n,d], blob_id int64[n], centres float32[nblobs,d]).
    """
    rng = _rng(seed)
    centres = rng.uniform(-spread, spread, (nblobs, d))
    blob = rng.integers(0, nblobs, n)
    x = centres[blob] + rng.normal(0.0, sigma, (n, d))
    return x.astype(np.float32), blob.astype(np.int64), centres.astype(np.float32)


@dataclass
class BatchedTasks:
    """A table of independent expressions laid out in three float32 pools.

    Task t of kind TASK_DOT reads a = A[a_off : a_off+cols], b = B[b_off : b_off+cols]
    and writes one scalar out[out_off].  Task t of kind TASK_MATVEC reads the
    row-major matrix A[a_off : a_off+rows*cols] and vector x = B[b_off : b_off+cols]
    and writes y = out[out_off : out_off+rows].
    """
    kind: np.ndarray      # int32[ntasks]
    rows: np.ndarray      # int64[ntasks] (1 for dot)
    cols: np.ndarray      # int64[ntasks]
    a_off: np.ndarray     # int64[ntasks]
    b_off: np.ndarray     # int64[ntasks]
    out_off: np.ndarray   # int64[ntasks]
    A: np.ndarray         # float32 pool
    B: np.ndarray         # float32 pool
    out_len: int          # length of the output pool
    gout: np.ndarray      # float32[out_len] upstream gradient

    @property
    def ntasks(self) -> int:
        return len(self.kind)

    def table(self) -> np.ndarray:
        """int64[ntasks, 6] rows of (kind, rows, cols, a_off, b_off, out_off)."""
        return np.stack([self.kind.astype(np.int64), self.rows, self.cols,
                         self.a_off, self.b_off, self.out_off], axis=1)


def batched_tasks(ntasks: int, seed: int = 0, smin: float = 1e2, smax: float = 1e6,
                  max_total: int | None = None, pad: int = 4) -> BatchedTasks:
    """Uneven batch: even task index = dot, odd = matvec.

    Sizes s = floor(exp(U[ln smin, ln smax))).  A dot has s elements per operand;
    a matvec has rows r = floor(sqrt(s)) and cols c = ceil(s / r).  Values are
    uniform in [-1, 1]; the upstream gradient is 1.0 for every dot output and
    uniform in [-1, 1] for matvec outputs.  ``max_total`` (optional) rescales
    nothing: it only asserts that the A pool stays below that many elements.
    ``pad``: operand lengths are rounded up to a multiple of ``pad`` floats in
    the pools (4: every operand starts on a 16-byte boundary; 1: operands are
    packed back to back at arbitrary offsets).
    """
    rng = _rng(seed)
    s = np.floor(np.exp(rng.uniform(math.log(smin), math.log(smax), ntasks))).astype(np.int64)
    kind = (np.arange(ntasks) % 2).astype(np.int32)
    rows = np.ones(ntasks, dtype=np.int64)
    cols = s.copy()
    mv = kind == TASK_MATVEC
    r = np.floor(np.sqrt(s[mv].astype(np.float64))).astype(np.int64)
    r = np.maximum(r, 1)
    c = (s[mv] + r - 1) // r
    rows[mv] = r
    cols[mv] = c
    a_len = rows * cols
    b_len = cols.copy()
    o_len = np.where(mv, rows, 1).astype(np.int64)
    # with pad = 4, operands start on 16-byte boundaries (lengths padded to
    # multiples of 4 floats; the padding belongs to no task)
    a_pad = (a_len + pad - 1) // pad * pad
    b_pad = (b_len + pad - 1) // pad * pad
    a_off = np.zeros(ntasks, dtype=np.int64)
    b_off = np.zeros(ntasks, dtype=np.int64)
    out_off = np.zeros(ntasks, dtype=np.int64)
    a_off[1:] = np.cumsum(a_pad)[:-1]
    b_off[1:] = np.cumsum(b_pad)[:-1]
    out_off[1:] = np.cumsum(o_len)[:-1]
    a_total = int(a_pad.sum())
    if max_total is not None:
        assert a_total <= max_total, (a_total, max_total)
    A = _uniform_f32(rng, -1.0, 1.0, a_total)
    B = _uniform_f32(rng, -1.0, 1.0, int(b_pad.sum()))
    out_len = int(o_len.sum())
    gout = _uniform_f32(rng, -1.0, 1.0, out_len)
    for t in np.nonzero(~mv)[0]:
        gout[out_off[t]] = 1.0
    return BatchedTasks(kind, rows, cols, a_off, b_off, out_off, A, B, out_len, gout)
