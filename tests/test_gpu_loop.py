"""GPU parity of the general parallel loop (`loop n f` with tensorGet /
tensorSet on rank 1-3 tensors) against the oracle's interpreter, through the C
ABI: the paper's loop programs, transposes of rank-2 and rank-3 tensors,
gathers and scatters through index tensors with two sets per iteration,
integer semantics, float bodies over every operator, a get after a set in the
same iteration, out-of-range indices, the debug-mode conflict check, graph
replay and a 2^24-iteration in-place update.

Integer results and moved values are bit-exact.  Float bodies compute in the
loop's float type against the oracle's binary64: relative 4e-6 (float32) or
1e-13 (float64) of the value's magnitude plus one, over at most a dozen
correctly rounded operations and library exp / log / sqrt.
"""
import numpy as np
import pytest
import torch

import oracle as O
from parity import say

import paper_2211_00621_amd as mx  # noqa: E402

pytestmark = pytest.mark.gpu
abi, api = mx.abi, mx.api
DEV = "cuda"


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def run_both(lp, n, arrays):
    """The loop on the GPU and in the oracle, from the same arrays."""
    ts = [dev(a) for a in arrays]
    lp.run(n, *ts)
    got = [host(t) for t in ts]
    ref, flags = O.loop_run(lp.prog, arrays, n)
    return got, ref, flags


def test_paper_double_and_axpy_int():
    say("loop paper programs")
    # b[i] = 2 a[i] (int tensors) and Listing 1's t1[i] <- t1[i] + 2 t2[i] in place
    n = 100003
    rng = np.random.default_rng(1)
    a = rng.integers(-1000, 1001, n).astype(np.int64)
    lp = api.ParallelLoop([(torch.int64, 1), (torch.int64, 1)])
    i = lp.iteration
    lp.set(1, i, lp.get(0, i) * 2)
    got, ref, _ = run_both(lp, n, [a, np.zeros(n, np.int64)])
    assert np.array_equal(got[1], 2 * a) and np.array_equal(got[1], ref[1])
    t1, t2 = rng.integers(-50, 50, n).astype(np.int32), rng.integers(-50, 50, n).astype(np.int32)
    lp = api.ParallelLoop([(torch.int32, 1), (torch.int32, 1)])
    i = lp.iteration
    lp.set(0, i, lp.get(0, i) + lp.get(1, i) * 2)
    got, ref, _ = run_both(lp, n, [t1, t2])
    assert np.array_equal(got[0], t1 + 2 * t2) and np.array_equal(got[0], ref[0]) and np.array_equal(got[1], t2)


@pytest.mark.parametrize("fdt", [torch.float32, torch.float64])
def test_float_axpy_in_place_2e24(fdt):
    n = (1 << 24) + 7
    say("loop axpy", fdt, n)
    rng = np.random.default_rng(2)
    npd = np.float32 if fdt == torch.float32 else np.float64
    x, y = rng.uniform(-1, 1, n).astype(npd), rng.uniform(-1, 1, n).astype(npd)
    lp = api.ParallelLoop([(fdt, 1), (fdt, 1)], fdt)
    i = lp.iteration
    lp.set(0, i, lp.get(0, i) + 0.375 * lp.get(1, i))
    got, ref, _ = run_both(lp, n, [x, y])
    if fdt == torch.float64:
        # the oracle's binary64 operations, uncontracted, are the loop's own
        assert np.array_equal(got[0], ref[0])
    else:
        # 0.375 y can need 26 significant bits, so the float32 body rounds
        # twice (product, then sum; no contraction): the same two correctly
        # rounded float32 operations in numpy give every bit, and the oracle's
        # binary64 value is within those two roundings
        emu = (x + (np.float32(0.375) * y).astype(np.float32)).astype(np.float32)
        assert np.array_equal(got[0], emu)
        assert np.all(np.abs(got[0] - ref[0]) <= 2.0 ** -23 * (np.abs(ref[0]) + 1))


def test_rank2_and_rank3_transposes():
    say("loop transposes")
    rng = np.random.default_rng(3)
    A = rng.uniform(-1, 1, (1000, 777)).astype(np.float32)
    lp = api.ParallelLoop([(torch.float32, 2), (torch.float32, 2)])
    i = lp.iteration
    r, c = i // 777, i % 777
    lp.set(1, (c, r), lp.get(0, r, c))
    got, ref, _ = run_both(lp, A.size, [A, np.zeros((777, 1000), np.float32)])
    assert np.array_equal(got[1], A.T) and np.array_equal(got[1], ref[1].astype(np.float32))
    B = rng.uniform(-1, 1, (37, 41, 53))
    lp = api.ParallelLoop([(torch.float64, 3), (torch.float64, 3)], torch.float64)
    i = lp.iteration
    a0, rest = i // (41 * 53), i % (41 * 53)
    a1, a2 = rest // 53, rest % 53
    lp.set(1, (a2, a0, a1), lp.get(0, a0, a1, a2))
    got, ref, _ = run_both(lp, B.size, [B, np.zeros((53, 37, 41))])
    assert np.array_equal(got[1], np.transpose(B, (2, 0, 1))) and np.array_equal(got[1], ref[1])


def test_gather_scatter_two_sets_per_iteration():
    n, m = (1 << 20) + 17, 3 << 20
    say("loop gather scatter", n)
    rng = np.random.default_rng(4)
    idx = rng.permutation(m)[:n].astype(np.int64)
    src = rng.uniform(-1, 1, m).astype(np.float32)
    lp = api.ParallelLoop([(torch.int64, 1), (torch.float32, 1), (torch.float32, 1), (torch.int32, 1)])
    i = lp.iteration
    j = lp.get(0, i)
    lp.set(2, i, lp.get(1, j))      # out[i] = src[idx[i]]
    lp.set(3, j, i)                 # inv[idx[i]] = i
    got, ref, flags = run_both(lp, n, [idx, src, np.zeros(n, np.float32), np.full(m, -1, np.int32)])
    assert flags == 0
    assert np.array_equal(got[2], src[idx]) and np.array_equal(got[3], ref[3].astype(np.int32))


def test_integer_semantics():
    say("loop integer semantics")
    rng = np.random.default_rng(5)
    n = 50000
    a = rng.integers(-2 ** 62, 2 ** 62, n, dtype=np.int64)
    b = rng.integers(-9, 10, n, dtype=np.int64)
    a[:4] = [np.iinfo(np.int64).min, np.iinfo(np.int64).min, 7, -7]
    b[:4] = [-1, 0, 0, -1]
    lp = api.ParallelLoop([(torch.int64, 1), (torch.int64, 1), (torch.int64, 2), (torch.int32, 1)])
    i = lp.iteration
    x, y = lp.get(0, i), lp.get(1, i)
    outs = [x // y, x % y, x * y, x - y, -x, lp.binary(abi.MX_L_IMIN, x, y), lp.binary(abi.MX_L_IMAX, x, y)]
    for k, v in enumerate(outs):
        lp.set(2, (i, k), v)
    lp.set(3, i, x + y)             # wraps to 32 bits
    got, ref, _ = run_both(lp, n, [a, b, np.zeros((n, 7), np.int64), np.zeros(n, np.int32)])
    assert np.array_equal(got[2], ref[2]) and np.array_equal(got[3], ref[3].astype(np.int32))


@pytest.mark.parametrize("fdt", [torch.float32, torch.float64])
def test_float_body_every_operator(fdt):
    say("loop float body", fdt)
    rng = np.random.default_rng(6)
    n = 30011
    npd = np.float32 if fdt == torch.float32 else np.float64
    x, y = rng.uniform(0.1, 2, n).astype(npd), rng.uniform(-2, 2, n).astype(npd)
    k = rng.integers(-5, 6, n).astype(np.int32)
    lp = api.ParallelLoop([(fdt, 1), (fdt, 1), (torch.int32, 1), (fdt, 2)], fdt)
    i = lp.iteration
    a, b, kk = lp.get(0, i), lp.get(1, i), lp.get(2, i).to_float()
    vals = [a + b, a - b, a * b, b / a, lp.binary(abi.MX_X_MIN, a, b), lp.binary(abi.MX_X_MAX, a, b), -b,
            lp.unary(abi.MX_X_ABS, b), lp.unary(abi.MX_X_SQ, b), lp.unary(abi.MX_X_EXP, b),
            lp.unary(abi.MX_X_LOG, a), lp.unary(abi.MX_X_SQRT, a), lp.unary(abi.MX_X_RSQRT, a), kk * a + b]
    for c, v in enumerate(vals):
        lp.set(3, (i, c), v)
    got, ref, _ = run_both(lp, n, [x, y, k, np.zeros((n, len(vals)), npd)])
    tol = 4e-6 if fdt == torch.float32 else 1e-13
    err = np.abs(got[3].astype(np.float64) - ref[3])
    assert np.all(err <= tol * (np.abs(ref[3]) + 1.0)), np.argwhere(err > tol * (np.abs(ref[3]) + 1.0))[:5]


def test_get_after_set_sees_the_stored_value():
    say("loop get after set")
    n = 4099
    lp = api.ParallelLoop([(torch.float32, 1), (torch.float32, 1)])
    i = lp.iteration
    lp.set(0, i, i.to_float() * 0.5)
    lp.set(1, i, lp.get(0, i) + 1.0)
    got, ref, _ = run_both(lp, n, [np.full(n, 7, np.float32), np.zeros(n, np.float32)])
    assert np.array_equal(got[1], np.arange(n, dtype=np.float32) * 0.5 + 1) and np.array_equal(got[1], ref[1])


def _shift_loop(target):
    """x[i] -> tensor `target`[i], reading x[i + 3]: out of range at the tail."""
    lp = api.ParallelLoop([(torch.float32, 1), (torch.float32, 1)])
    i = lp.iteration
    lp.set(target, i, lp.get(0, i + 3))
    return lp


def test_out_of_range_fast_mode_and_debug_mode():
    say("loop out of range")
    n = 1000
    x = np.arange(n, dtype=np.float32)
    lp = _shift_loop(1)
    got, ref, flags = run_both(lp, n, [x, np.full(n, -1, np.float32)])
    assert flags == 1 and np.array_equal(got[1], ref[1]) and np.all(got[1][-3:] == 0)
    abi.mx_set_debug(True)
    try:
        t = [dev(x), dev(np.full(n, -1, np.float32))]
        with pytest.raises(abi.MxError, match="outside"):
            lp.run(n, *t)
        assert np.all(host(t[1]) == -1)         # nothing written
        lp.run(n - 3, *t)                       # in range: runs
        assert np.array_equal(host(t[1])[:n - 3], x[3:])
    finally:
        abi.mx_set_debug(False)


def test_debug_mode_flags_conflicts_and_writes_nothing():
    say("loop debug conflicts")
    n = 5000
    x = np.random.default_rng(7).uniform(-1, 1, n + 3).astype(np.float32)
    abi.mx_set_debug(True)
    try:
        # x[i] = x[i + 3]: iteration i reads the slot iteration i + 3 sets
        rw = _shift_loop(0)
        t = [dev(x), dev(np.zeros(n + 3, np.float32))]
        with pytest.raises(abi.MxError, match="read by another"):
            rw.run(n, *t)
        assert np.array_equal(host(t[0]), x)
        assert O.loop_check(rw.prog, [x, np.zeros(n + 3, np.float32)], n) == 4
        # every iteration sets slot i // 2: write-write
        ww = api.ParallelLoop([(torch.float32, 1)])
        i = ww.iteration
        ww.set(0, i // 2, i.to_float())
        t = [dev(np.zeros(n, np.float32))]
        with pytest.raises(abi.MxError, match="two iterations"):
            ww.run(n, *t)
        assert np.all(host(t[0]) == 0)
        # conflict free (into the other tensor): passes and matches the oracle
        ok = _shift_loop(1)
        t = [dev(x), dev(np.zeros(n + 3, np.float32))]
        ok.run(n, *t)
        ref, _ = O.loop_run(ok.prog, [x, np.zeros(n + 3, np.float32)], n)
        assert np.array_equal(host(t[1]), ref[1].astype(np.float32))
    finally:
        abi.mx_set_debug(False)


def test_graph_replay_of_a_loop():
    say("loop graph")
    rng = np.random.default_rng(8)
    A = rng.uniform(-1, 1, (513, 257)).astype(np.float32)
    lp = api.ParallelLoop([(torch.float32, 2), (torch.float32, 2)])
    i = lp.iteration
    r, c = i // 257, i % 257
    lp.set(1, (c, r), lp.unary(abi.MX_X_SQ, lp.get(0, r, c)))
    ta, tb = dev(A), torch.zeros((257, 513), device=DEV)
    abi.mx_loop_prepare(lp.handle)
    lp.run(A.size, ta, tb)
    eager = host(tb).copy()
    side = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(side):
        abi.mx_graph_begin(side)
        abi.mx_loop_run(lp.handle, A.size, [ta, tb], None, side)
        graph = abi.mx_graph_end(side)
    for rep in range(3):
        tb.zero_()
        torch.cuda.synchronize()
        graph.launch(side)
        side.synchronize()
        assert host(tb).tobytes() == eager.tobytes(), rep
    abi.mx_graph_destroy(graph)
    assert np.array_equal(eager, (A * A).T)
