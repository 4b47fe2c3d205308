"""GPU parity of the reverse of reduce (+, min, max), flat and per ragged row,
and of the autograd wrappers built on it (reduce, segmented reduce, and the
user-defined body's map, map + reduce and nested map(reduce)), against the
oracle.

The arg element of min / max is an index decided by comparisons of the
float32 inputs; the oracle widens the same float32 values exactly to binary64,
so both sides take every comparison on the same numbers and the gradients
(g at one element, 0 elsewhere) are compared bit for bit.  For bodies, the
inputs are small integers, so the body's values are exact in float32 and
binary64 alike and the decisions again coincide.
"""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from parity import check_vector, say

import paper_2211_00621_amd as mx  # noqa: E402

pytestmark = pytest.mark.gpu
abi, api = mx.abi, mx.api
X = abi
DEV = "cuda"
NE = {abi.MX_MIN: np.inf, abi.MX_MAX: -np.inf, abi.MX_ADD: 0.0}


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def flat_adjoint(op, x, ne, g, shift=0):
    """Run mx_reduce_adjoint_f32 on x placed at element offset `shift` of a buffer."""
    n = x.size
    buf = dev(np.concatenate([np.zeros(shift, np.float32), x]))
    xv = buf[shift:]
    gx = torch.full((n + shift,), np.nan, device=DEV)[shift:]
    ws = api.workspace(abi.MX_WS_REDUCE, n)
    abi.mx_reduce_adjoint_f32(op, xv, ne, dev(np.array([g], np.float32)), gx, ws)
    return host(gx)


@pytest.mark.parametrize("op", [abi.MX_MIN, abi.MX_MAX, abi.MX_ADD])
@pytest.mark.parametrize("n", [1, 3, 63, 64, 65, 1025, (1 << 20) + 3, (1 << 24) + 5])
@pytest.mark.parametrize("shift", [0, 1])
def test_reduce_adjoint_vs_oracle(op, n, shift):
    say("reduce adjoint", op, n, shift)
    rng = np.random.default_rng(n + 3 * op + shift)
    x = rng.uniform(-1, 1, n).astype(np.float32)
    g = np.float32(-1.75)
    got = flat_adjoint(op, x, NE[op], g, shift)
    ref = O.reduce_adjoint(op, NE[op], x, g)
    assert np.array_equal(got, ref.astype(np.float32))


@pytest.mark.parametrize("op", [abi.MX_MIN, abi.MX_MAX])
def test_reduce_adjoint_ties_ne_and_nan(op):
    say("reduce adjoint ties", op)
    rng = np.random.default_rng(5)
    n = 300001
    x = rng.integers(-20, 21, n).astype(np.float32)          # every value many times over
    for ne in (NE[op], 20.0 if op == abi.MX_MAX else -20.0, 21.0 if op == abi.MX_MAX else -21.0,
               5.0, np.nan):
        got = flat_adjoint(op, x, ne, 2.0)
        ref = O.reduce_adjoint(op, ne, x, 2.0)
        assert np.array_equal(got, ref.astype(np.float32)), ne
    # the extreme first appears late, and NaN elements are skipped
    y = rng.uniform(0, 1, n).astype(np.float32)
    y[::7] = np.nan
    y[n - 2] = -3.0 if op == abi.MX_MIN else 3.0
    y[n - 1] = y[n - 2]
    got = flat_adjoint(op, y, NE[op], 1.0, shift=1)
    assert np.array_equal(got, O.reduce_adjoint(op, NE[op], y, 1.0).astype(np.float32))
    assert got[n - 2] == 1.0 and got.sum() == 1.0
    # signed zeros compare equal: the first of them
    z = np.zeros(1000, np.float32)
    z[1::2] = -0.0
    got = flat_adjoint(op, z, NE[op], 1.0)
    assert got[0] == 1.0 and got[1:].sum() == 0


def test_reduce_adjoint_errors_and_empty():
    say("reduce adjoint errors")
    x = torch.zeros(10, device=DEV)
    g = torch.ones(1, device=DEV)
    with pytest.raises(abi.MxError):
        abi.mx_reduce_adjoint_f32(abi.MX_MUL, x, 1.0, g, torch.empty_like(x), api.workspace(abi.MX_WS_REDUCE, 10))
    with pytest.raises(abi.MxError):  # MIN without a workspace
        abi.mx_reduce_adjoint_f32(abi.MX_MIN, x, np.inf, g, torch.empty_like(x), None)
    e = torch.zeros(0, device=DEV)
    abi.mx_reduce_adjoint_f32(abi.MX_MIN, e, np.inf, g, e, None)


@pytest.mark.parametrize("op", [abi.MX_MIN, abi.MX_MAX, abi.MX_ADD])
@pytest.mark.parametrize("kind", ["config", "empty_and_short", "ties"])
def test_segmented_reduce_adjoint_vs_oracle(op, kind):
    say("segmented reduce adjoint", op, kind)
    if kind == "config":
        L, v = W.ragged_f32(65536, seed=4)
    elif kind == "empty_and_short":
        L, v = W.ragged_f32(5000, seed=5, lmax=70, empty_rows=900)
    else:
        L = W.ragged_lengths(3000, seed=6, lmax=500)
        v = np.random.default_rng(6).integers(-3, 4, int(L.sum())).astype(np.float32)
    off = O.offsets_from_lengths(L)
    g = np.random.default_rng(7).uniform(-1, 1, len(L)).astype(np.float32)
    gv = torch.full((v.size,), np.nan, device=DEV)
    abi.mx_segmented_reduce_adjoint_f32(op, dev(v), dev(off), NE[op], dev(g), gv)
    ref = O.segmented_reduce_adjoint(op, NE[op], v, off, g)
    assert np.array_equal(host(gv), ref.astype(np.float32))


def test_autograd_reduce_and_segmented_reduce():
    say("autograd reduce")
    rng = np.random.default_rng(8)
    x = rng.uniform(-1, 1, 100003).astype(np.float32)
    for op in (abi.MX_ADD, abi.MX_MIN, abi.MX_MAX):
        t = dev(x).requires_grad_(True)
        y = api.reduce(op, t, NE[op])
        (3.0 * y).backward()
        assert np.array_equal(host(t.grad), O.reduce_adjoint(op, NE[op], x, 3.0).astype(np.float32)), op
    L, v = W.ragged_f32(2000, seed=9, empty_rows=50)
    off = O.offsets_from_lengths(L)
    g = rng.uniform(-1, 1, len(L)).astype(np.float32)
    for op in (abi.MX_ADD, abi.MX_MIN, abi.MX_MAX):
        t = dev(v).requires_grad_(True)
        y = api.segmented_reduce(op, api.Ragged(t, dev(off)), NE[op])
        y.backward(dev(g))
        ref = O.segmented_reduce_adjoint(op, NE[op], v, off, g)
        assert np.array_equal(host(t.grad), ref.astype(np.float32)), op


# ---------------------------------------------------------------- bodies
def _body():
    a, b = api.body_inputs(2)
    return api.Body(a * b - b, 2)


def _int_inputs(n, seed):
    rng = np.random.default_rng(seed)
    return [rng.integers(-30, 31, n).astype(np.float32) for _ in range(2)]


def _vjp_close(got, ref, what):
    ref = np.asarray(ref, np.float64)
    scale = np.linalg.norm(ref) / np.sqrt(max(ref.size, 1)) + 1e-30
    assert np.all(np.abs(np.asarray(got, np.float64) - ref) <= 2e-6 * (np.abs(ref) + scale)), what


def test_autograd_body_map():
    say("autograd body map")
    body = _body()
    xs = _int_inputs(50003, 10)
    ts = [dev(x).requires_grad_(True) for x in xs]
    y = body.map(*ts)
    gout = np.random.default_rng(11).uniform(-1, 1, xs[0].size).astype(np.float32)
    y.backward(dev(gout))
    assert np.array_equal(host(y.detach()), O.expr_map(body.prog, body.out_reg, *xs).astype(np.float32))
    ref = O.expr_vjp(body.prog, body.out_reg, xs, gout=gout)
    for t, r, k in zip(ts, ref, "ab"):
        _vjp_close(host(t.grad), r, f"d/d{k}")


@pytest.mark.parametrize("op", [abi.MX_ADD, abi.MX_MIN, abi.MX_MAX])
def test_autograd_body_map_reduce(op):
    say("autograd body map reduce", op)
    body = _body()
    xs = _int_inputs(70001, 12)
    ts = [dev(x).requires_grad_(True) for x in xs]
    y = body.map_reduce(op, *ts, ne=NE[op])
    (0.5 * y).backward()
    vals = O.expr_map(body.prog, body.out_reg, *xs)
    seed = O.reduce_adjoint(op, NE[op], vals, 0.5)
    ref = O.expr_vjp(body.prog, body.out_reg, xs, gout=seed)
    for t, r, k in zip(ts, ref, "ab"):
        _vjp_close(host(t.grad), r, f"d/d{k}")


@pytest.mark.parametrize("op", [abi.MX_ADD, abi.MX_MIN, abi.MX_MAX])
def test_autograd_body_segmented_reduce(op):
    say("autograd body segmented", op)
    body = _body()
    L = W.ragged_lengths(4000, seed=13, lmax=2000)
    L[::37] = 0
    off = O.offsets_from_lengths(L)
    xs = _int_inputs(int(off[-1]), 14)
    g = np.random.default_rng(15).uniform(-1, 1, len(L)).astype(np.float32)
    ts = [dev(x).requires_grad_(True) for x in xs]
    y = body.segmented_reduce(op, dev(off), *ts, ne=NE[op])
    y.backward(dev(g))
    vals = O.expr_map(body.prog, body.out_reg, *xs)
    assert np.array_equal(host(y.detach()), O.segmented_reduce(op, NE[op], vals, off).astype(np.float32)) \
        or op == abi.MX_ADD
    seed = O.segmented_reduce_adjoint(op, NE[op], vals, off, g)
    ref = O.expr_vjp(body.prog, body.out_reg, xs, gout=seed)
    for t, r, k in zip(ts, ref, "ab"):
        _vjp_close(host(t.grad), r, f"d/d{k}")
