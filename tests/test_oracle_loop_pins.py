"""Pins for the oracle's interpreter of the general parallel loop (`loop n f`
with tensorGet / tensorSet, Appendix A): the paper's own loop programs on the
hand-computed golden values, numpy library routines on special cases
(transposes of rank-2 and rank-3 tensors, fancy-index gathers and scatters,
C integer division), order independence of conflict-free loops, and the
debug-mode verdict on loops whose conflicts are known by construction.
"""
import json
import os

import numpy as np
import pytest

import oracle as O

RNG = np.random.default_rng(31)


def L(op, dst=0, a=0, b=0, c=0, src=0, tensor=0, iimm=0, fimm=0.0):
    return (op, dst, a, b, c, src, tensor, iimm, fimm)


ITER = lambda d: L(O.L_ITER, d)                       # noqa: E731
ICONST = lambda d, v: L(O.L_ICONST, d, iimm=v)       # noqa: E731
FCONST = lambda d, v: L(O.X_CONST, d, fimm=v)        # noqa: E731


@pytest.fixture(scope="module")
def gold(golden_dir):
    with open(os.path.join(golden_dir, "paper_examples.json")) as f:
        return json.load(f)


def test_golden_loop_double(gold):
    # f i = tensorSet b [i] (muli 2 (tensorGet a i)), integer tensors
    g = gold["loop_double"]
    a = np.array(g["a"], dtype=np.int64)
    prog = [ITER(0), L(O.L_IGET, 1, a=0, tensor=0), ICONST(2, 2), L(O.L_IMUL, 3, 1, 2),
            L(O.L_ISET, a=0, src=3, tensor=1)]
    (a_out, b_out), flags = O.loop_run(prog, [a, np.zeros_like(a)], a.size)
    assert flags == 0 and b_out.tolist() == g["b"] and a_out.tolist() == g["a"]


def test_golden_listing1_axpy_in_place(gold):
    # axpy c i: t1[i] <- addi (tensorGet t1 [i]) (muli c (tensorGet t2 [i])), c = 2
    g = gold["listing1_small"]
    prog = [ITER(0), L(O.L_IGET, 1, a=0, tensor=0), L(O.L_IGET, 2, a=0, tensor=1), ICONST(3, 2),
            L(O.L_IMUL, 4, 3, 2), L(O.L_IADD, 5, 1, 4), L(O.L_ISET, a=0, src=5, tensor=0)]
    (t1, t2), flags = O.loop_run(prog, [np.array(g["t1"]), np.array(g["t2"])], 3)
    assert flags == 0 and t1.tolist() == g["t1_after"] and t2.tolist() == g["t2"]
    assert O.loop_check(prog, [np.array(g["t1"]), np.array(g["t2"])], 3) == 0
    gl = gold["listing1_large"]
    n = gl["n"]
    (t1, _), _ = O.loop_run(prog, [np.arange(n), np.ones(n, dtype=np.int64)], n)
    assert int(t1.sum()) == gl["sum"]


def test_float_axpy_closed_form():
    x, y = RNG.uniform(-1, 1, 500), RNG.uniform(-1, 1, 500)
    prog = [ITER(0), L(O.L_FGET, 1, a=0, tensor=0), L(O.L_FGET, 2, a=0, tensor=1), FCONST(3, 0.375),
            L(O.X_MUL, 4, 3, 2), L(O.X_ADD, 5, 1, 4), L(O.L_FSET, a=0, src=5, tensor=0)]
    (t1, _), _ = O.loop_run(prog, [x, y], 500)
    assert np.array_equal(t1, x + 0.375 * y)   # one product and one sum per element, as numpy rounds them


def test_rank2_transpose_is_numpy_transpose():
    # B[j][i] = A[i][j] with (i, j) = divmod(iteration, cols)
    A = RNG.uniform(-1, 1, (7, 13))
    prog = [ITER(0), ICONST(1, 13), L(O.L_IDIV, 2, 0, 1), L(O.L_IMOD, 3, 0, 1),
            L(O.L_FGET, 0, a=2, b=3, tensor=0), L(O.L_FSET, a=3, b=2, src=0, tensor=1)]
    (_, B), flags = O.loop_run(prog, [A, np.zeros((13, 7))], 7 * 13)
    assert flags == 0 and np.array_equal(B, A.T)
    assert O.loop_check(prog, [A, np.zeros((13, 7))], 91) == 0


def test_rank3_axis_permutation_is_numpy_transpose():
    A = RNG.uniform(-1, 1, (3, 4, 5))
    # iteration -> (i, j, k) of A; out[k][i][j] = A[i][j][k]
    prog = [ITER(0), ICONST(1, 20), ICONST(2, 5), L(O.L_IDIV, 3, 0, 1), L(O.L_IMOD, 4, 0, 1),
            L(O.L_IDIV, 5, 4, 2), L(O.L_IMOD, 6, 4, 2), L(O.L_FGET, 0, a=3, b=5, c=6, tensor=0),
            L(O.L_FSET, a=6, b=3, c=5, src=0, tensor=1)]
    (_, out), flags = O.loop_run(prog, [A, np.zeros((5, 3, 4))], 60)
    assert flags == 0 and np.array_equal(out, np.transpose(A, (2, 0, 1)))


def test_gather_and_scatter_through_an_index_tensor_and_two_sets():
    n, m = 300, 1000
    idx = RNG.permutation(m)[:n]
    src = RNG.uniform(-1, 1, m)
    # out[i] = src[idx[i]] (gather) and out2[idx[i]] = i (scatter): two sets per iteration
    prog = [ITER(0), L(O.L_IGET, 1, a=0, tensor=0), L(O.L_FGET, 0, a=1, tensor=1),
            L(O.L_FSET, a=0, src=0, tensor=2), L(O.L_ISET, a=1, src=0, tensor=3)]
    ts = [idx, src, np.zeros(n), np.full(m, -1, dtype=np.int64)]
    (_, _, out, out2), flags = O.loop_run(prog, ts, n)
    ref2 = np.full(m, -1)
    ref2[idx] = np.arange(n)
    assert flags == 0 and np.array_equal(out, src[idx]) and np.array_equal(out2, ref2)
    assert O.loop_check(prog, ts, n) == 0


def test_integer_division_and_wrap_semantics():
    vals = np.array([7, -7, 7, -7, 0, 5, np.iinfo(np.int64).min, 9], dtype=np.int64)
    divs = np.array([2, 2, -2, -2, 3, 0, -1, 4], dtype=np.int64)
    prog = [ITER(0), L(O.L_IGET, 1, a=0, tensor=0), L(O.L_IGET, 2, a=0, tensor=1), L(O.L_IDIV, 3, 1, 2),
            L(O.L_IMOD, 4, 1, 2), L(O.L_ISET, a=0, src=3, tensor=2), L(O.L_ISET, a=0, src=4, tensor=3)]
    (_, _, q, r), _ = O.loop_run(prog, [vals, divs, np.zeros(8, np.int64), np.zeros(8, np.int64)], 8)
    ref_q, ref_r = [], []
    for a, b in zip(vals.tolist(), divs.tolist()):   # C semantics written with Python integers
        if b == 0:
            ref_q.append(0), ref_r.append(0)
            continue
        qq = abs(a) // abs(b) * (1 if (a >= 0) == (b > 0) else -1)
        qq = (qq + 2 ** 63) % 2 ** 64 - 2 ** 63      # INT64_MIN / -1 wraps
        ref_q.append(qq)
        ref_r.append(0 if b == -1 else a - qq * b)
    assert q.tolist() == ref_q and r.tolist() == ref_r
    # an int32 tensor keeps its stores wrapped to 32 bits; arithmetic wraps mod 2^64
    big = np.array([2 ** 31 - 1, -2 ** 31, 12345], dtype=np.int32)
    prog = [ITER(0), L(O.L_IGET, 1, a=0, tensor=0), ICONST(2, 3), L(O.L_IMUL, 3, 1, 2),
            L(O.L_ISET, a=0, src=3, tensor=0)]
    (out,), _ = O.loop_run(prog, [big], 3)
    assert out.tolist() == (big.astype(np.int64) * 3).astype(np.int32).tolist()


def test_get_after_set_in_the_same_iteration_sees_the_stored_value():
    # t[i] = 5; x = t[i]; u[i] = x + 1 -- program order within an iteration
    prog = [ITER(0), ICONST(1, 5), L(O.L_ISET, a=0, src=1, tensor=0), L(O.L_IGET, 2, a=0, tensor=0),
            ICONST(3, 1), L(O.L_IADD, 4, 2, 3), L(O.L_ISET, a=0, src=4, tensor=1)]
    ts = [np.zeros(10, np.int64), np.zeros(10, np.int64)]
    (t, u), _ = O.loop_run(prog, ts, 10)
    assert t.tolist() == [5] * 10 and u.tolist() == [6] * 10
    assert O.loop_check(prog, ts, 10) == 0
    # the check sees the stored value too: the index written here comes from it
    prog2 = [ITER(0), L(O.L_ISET, a=0, src=0, tensor=0), L(O.L_IGET, 1, a=0, tensor=0),
             ICONST(2, 100), L(O.L_IADD, 3, 1, 2), L(O.L_ISET, a=3, src=0, tensor=0)]
    ts2 = [np.zeros(200, np.int64)]
    assert O.loop_check(prog2, ts2, 100) == 0          # slots i and i + 100: disjoint
    # iteration 100 sets slot 100, which iteration 0 sets (2), and reads it back (4)
    assert O.loop_check(prog2, [np.zeros(300, np.int64)], 101) == 6
    assert O.loop_check(prog2, ts2, 101) == 7          # ... and its second set falls outside (1)


def test_out_of_range_gets_give_zero_and_sets_write_nothing():
    x = np.arange(10, dtype=np.int64)
    prog = [ITER(0), ICONST(1, 3), L(O.L_IADD, 2, 0, 1), L(O.L_IGET, 3, a=2, tensor=0),
            L(O.L_ISET, a=0, src=3, tensor=1), L(O.L_ISET, a=2, src=3, tensor=2)]
    ts = [x, np.full(10, -1, np.int64), np.full(10, -1, np.int64)]
    (_, y, z), flags = O.loop_run(prog, ts, 10)
    assert flags == 1
    assert y.tolist() == [3, 4, 5, 6, 7, 8, 9, 0, 0, 0]
    assert z.tolist() == [-1, -1, -1, 3, 4, 5, 6, 7, 8, 9]
    assert O.loop_check(prog, ts, 10) & 1


def test_conflict_free_loops_give_the_same_result_in_any_order():
    A = RNG.uniform(-1, 1, (9, 11))
    prog = [ITER(0), ICONST(1, 11), L(O.L_IDIV, 2, 0, 1), L(O.L_IMOD, 3, 0, 1),
            L(O.L_FGET, 0, a=2, b=3, tensor=0), L(O.X_SQ, 1, 0), L(O.L_FSET, a=3, b=2, src=1, tensor=1),
            L(O.L_FSET, a=2, b=3, src=0, tensor=0)]
    ts = [A, np.zeros((11, 9))]
    ref, _ = O.loop_run(prog, ts, 99)
    for order in (np.arange(98, -1, -1), RNG.permutation(99)):
        got, _ = O.loop_run(prog, ts, 99, order=order)
        assert all(np.array_equal(a, b) for a, b in zip(got, ref))


def test_check_flags_write_write_and_read_write_conflicts():
    n = 50
    # every iteration sets slot 0: a write-write conflict
    ww = [ICONST(0, 0), ITER(1), L(O.L_ISET, a=0, src=1, tensor=0)]
    assert O.loop_check(ww, [np.zeros(4, np.int64)], n) == 2
    assert O.loop_check(ww, [np.zeros(4, np.int64)], 1) == 0
    # out[i] = out[i + 1]: iteration i reads the slot iteration i + 1 sets
    rw = [ITER(0), ICONST(1, 1), L(O.L_IADD, 2, 0, 1), L(O.L_FGET, 0, a=2, tensor=0),
          L(O.L_FSET, a=0, src=0, tensor=0)]
    assert O.loop_check(rw, [np.zeros(n + 1)], n) == 4
    # the same shift into another tensor is conflict free
    ok = [ITER(0), ICONST(1, 1), L(O.L_IADD, 2, 0, 1), L(O.L_FGET, 0, a=2, tensor=0),
          L(O.L_FSET, a=0, src=0, tensor=1)]
    assert O.loop_check(ok, [np.zeros(n + 1), np.zeros(n)], n) == 0
    # the tensors are not modified by the check
    t = np.arange(5, dtype=np.int64)
    O.loop_check([ITER(0), ICONST(1, 7), L(O.L_ISET, a=0, src=1, tensor=0)], [t], 5)
    assert t.tolist() == [0, 1, 2, 3, 4]
