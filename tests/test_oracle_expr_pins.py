"""Pins for the oracle's interpreter of user-defined map bodies (straight-line
register programs): each test checks it against something other than itself --
the operator tables of the fixed map / map2 bodies (pinned on their own),
library routines on special cases (numpy.polyval, numpy.dot), closed-form
derivatives, and central finite differences of the interpreter's own forward
evaluation for the reverse mode.
"""
import numpy as np
import pytest

import oracle as O

RNG = np.random.default_rng(11)

UNARY = [(O.X_NEG, O.U_NEG), (O.X_ABS, O.U_ABS), (O.X_SQ, O.U_SQ), (O.X_EXP, O.U_EXP), (O.X_LOG, O.U_LOG),
         (O.X_SQRT, O.U_SQRT), (O.X_RSQRT, O.U_RSQRT)]
BINARY = [(O.X_ADD, O.B_ADD), (O.X_SUB, O.B_SUB), (O.X_MUL, O.B_MUL), (O.X_DIV, O.B_DIV), (O.X_MIN, O.B_MIN),
          (O.X_MAX, O.B_MAX)]


def IN(dst, k):
    return (O.X_IN, dst, k, 0, 0.0)


def CONST(dst, v):
    return (O.X_CONST, dst, 0, 0, v)


def OP(op, dst, a, b=0):
    return (op, dst, a, b, 0.0)


# the example body used across tests: exp(-(a - b)^2) * 0.5 + a * b
GAUSS_DOT = [IN(0, 0), IN(1, 1), OP(O.X_SUB, 2, 0, 1), OP(O.X_SQ, 2, 2), OP(O.X_NEG, 2, 2), OP(O.X_EXP, 2, 2),
             CONST(3, 0.5), OP(O.X_MUL, 2, 2, 3), OP(O.X_MUL, 4, 0, 1), OP(O.X_ADD, 2, 2, 4)]


@pytest.mark.parametrize("xop,uop", UNARY)
def test_single_unary_instruction_is_the_fixed_map_body(xop, uop):
    x = RNG.uniform(0.1, 3.0, 257) * RNG.choice([-1, 1], 257)
    if uop in (O.U_LOG, O.U_SQRT, O.U_RSQRT):
        x = np.abs(x)
    got = O.expr_map([IN(5, 0), OP(xop, 9, 5)], 9, x)
    assert np.array_equal(got, O.map(uop, x))


@pytest.mark.parametrize("xop,bop", BINARY)
def test_single_binary_instruction_is_the_fixed_map2_body(xop, bop):
    a = RNG.uniform(-2, 2, 300)
    b = RNG.uniform(-2, 2, 300)
    b[:20] = a[:20]  # ties for min / max
    got = O.expr_map([IN(3, 1), IN(7, 0), OP(xop, 1, 7, 3)], 1, a, b)
    assert np.array_equal(got, O.map2(bop, a, b))


def test_registers_overwrite_and_reuse_give_horner_polyval():
    c = [0.75, -1.5, 2.0, 0.25]            # c3 x^3 + c2 x^2 + c1 x + c0, highest first
    prog = [IN(0, 0), CONST(1, c[0])]
    for ci in c[1:]:                       # r1 = r1 * x + ci, reusing r1 and r2
        prog += [OP(O.X_MUL, 1, 1, 0), CONST(2, ci), OP(O.X_ADD, 1, 1, 2)]
    x = RNG.uniform(-3, 3, 101)
    assert np.array_equal(O.expr_map(prog, 1, x), np.polyval(c, x))


def test_map_reduce_of_the_product_body_is_the_dot_product():
    a = RNG.uniform(-1, 1, 1000)
    b = RNG.uniform(-1, 1, 1000)
    prog = [IN(0, 0), IN(1, 1), OP(O.X_MUL, 2, 0, 1)]
    assert O.expr_map_reduce(O.ADD, 0.0, prog, 2, a, b) == O.dot(a, b)
    assert abs(O.expr_map_reduce(O.ADD, 0.0, prog, 2, a, b) - float(np.dot(a, b))) <= 1000 * 2 ** -53 * np.abs(a * b).sum()


def test_map_reduce_min_max_mul_and_neutral_element():
    x = RNG.uniform(0.5, 1.5, 64)
    prog = [IN(0, 0), OP(O.X_SQ, 1, 0)]
    sq = x * x
    assert O.expr_map_reduce(O.MIN, np.inf, prog, 1, x) == sq.min()
    assert O.expr_map_reduce(O.MAX, -np.inf, prog, 1, x) == sq.max()
    assert O.expr_map_reduce(O.MIN, -5.0, prog, 1, x) == -5.0
    assert O.expr_map_reduce(O.ADD, 7.0, prog, 1, x[:0]) == 7.0
    assert abs(O.expr_map_reduce(O.MUL, 1.0, prog, 1, x) - np.prod(sq)) <= 64 * 2 ** -52 * np.prod(sq)


def test_unused_instructions_do_not_change_value_or_gradient():
    x = RNG.uniform(-1, 1, 50)
    # r3 = log(-1) is NaN but the output never reads it
    prog = [IN(0, 0), CONST(1, -1.0), OP(O.X_LOG, 3, 1), OP(O.X_SQ, 2, 0)]
    assert np.array_equal(O.expr_map(prog, 2, x), x * x)
    (g,) = O.expr_vjp(prog, 2, [x])
    assert np.array_equal(g, x + x)


def test_vjp_closed_forms():
    x = RNG.uniform(0.2, 2.0, 200)
    for xop, d in [(O.X_EXP, np.exp(x)), (O.X_LOG, 1 / x), (O.X_SQ, 2 * x), (O.X_NEG, -np.ones_like(x)),
                   (O.X_SQRT, 0.5 / np.sqrt(x)), (O.X_RSQRT, -0.5 * x ** -1.5)]:
        (g,) = O.expr_vjp([IN(0, 0), OP(xop, 1, 0)], 1, [x])
        assert np.allclose(g, d, rtol=4e-16 * 8, atol=0), xop
    a, b = RNG.uniform(-1, 1, 100), RNG.uniform(0.5, 1, 100)
    ga, gb = O.expr_vjp([IN(0, 0), IN(1, 1), OP(O.X_MUL, 2, 0, 1)], 2, [a, b])
    assert np.array_equal(ga, b) and np.array_equal(gb, a)
    ga, gb = O.expr_vjp([IN(0, 0), IN(1, 1), OP(O.X_DIV, 2, 0, 1)], 2, [a, b])
    assert np.allclose(ga, 1 / b, rtol=1e-15) and np.allclose(gb, -a / b ** 2, rtol=1e-15, atol=1e-300)


def test_vjp_min_max_abs_pass_to_the_branch_taken():
    a = np.array([1.0, 2.0, 3.0, -1.0, 0.0])
    b = np.array([2.0, 1.0, 3.0, -2.0, 0.0])
    ga, gb = O.expr_vjp([IN(0, 0), IN(1, 1), OP(O.X_MIN, 2, 0, 1)], 2, [a, b])
    assert ga.tolist() == [1, 0, 1, 0, 1] and gb.tolist() == [0, 1, 0, 1, 0]   # ties go to a
    ga, gb = O.expr_vjp([IN(0, 0), IN(1, 1), OP(O.X_MAX, 2, 0, 1)], 2, [a, b])
    assert ga.tolist() == [0, 1, 1, 1, 1] and gb.tolist() == [1, 0, 0, 0, 0]
    (g,) = O.expr_vjp([IN(0, 0), OP(O.X_ABS, 1, 0)], 1, [a])
    assert g.tolist() == [1, 1, 1, -1, 1]


def test_vjp_min_max_do_not_reach_the_operand_not_returned():
    # min / max equal the operand they return on a neighbourhood of any point
    # where the operands differ, so the derivative is that operand's alone;
    # the other subtree is not reached even where its own partials are not
    # finite (log c and 1 / c at c = 0 -- a zero term pushed through them
    # would give 0 * inf = NaN).
    x = np.array([-0.75, 0.0, 0.5, 1.0])
    c = np.zeros(4)
    # max(x, log c): log 0 = -inf < x, so d/dx = 1 and d/dc = 0
    gx, gc = O.expr_vjp([IN(0, 0), IN(1, 1), OP(O.X_LOG, 2, 1), OP(O.X_MAX, 3, 0, 2)], 3, [x, c])
    assert gx.tolist() == [1, 1, 1, 1] and gc.tolist() == [0, 0, 0, 0]
    # min(x, 1 / c): 1 / +0 = +inf > x
    gx, gc = O.expr_vjp([IN(0, 0), IN(1, 1), CONST(2, 1.0), OP(O.X_DIV, 2, 2, 1), OP(O.X_MIN, 3, 0, 2)], 3,
                        [x, c])
    assert gx.tolist() == [1, 1, 1, 1] and gc.tolist() == [0, 0, 0, 0]
    # max(x, sqrt c): the branch taken is x where x > 0 = sqrt 0; at x <= 0 it
    # is sqrt c (ties go to the first operand only when equal: x = 0 here)
    x2, c2 = np.array([0.5, 2.0]), np.zeros(2)
    gx, gc = O.expr_vjp([IN(0, 0), IN(1, 1), OP(O.X_SQRT, 2, 1), OP(O.X_MAX, 3, 0, 2)], 3, [x2, c2])
    assert gx.tolist() == [1, 1] and gc.tolist() == [0, 0]
    # the safe-division clamp min(1, x / y) at y = 0 (x > 0): constant 1 there
    xs, ys = np.array([0.5, 3.0]), np.zeros(2)
    gx, gy = O.expr_vjp([IN(0, 0), IN(1, 1), CONST(2, 1.0), OP(O.X_DIV, 3, 0, 1), OP(O.X_MIN, 4, 2, 3)], 4,
                        [xs, ys])
    assert gx.tolist() == [0, 0] and gy.tolist() == [0, 0]
    # an operand not returned here but used elsewhere still gets that use's
    # term: max(x, log c) + c at c = 0 has d/dc = 1
    gx, gc = O.expr_vjp([IN(0, 0), IN(1, 1), OP(O.X_LOG, 2, 1), OP(O.X_MAX, 3, 0, 2), OP(O.X_ADD, 3, 3, 1)], 3,
                        [x, c])
    assert gx.tolist() == [1, 1, 1, 1] and gc.tolist() == [1, 1, 1, 1]
    # and where the branch flips, the gradient follows it: max(x, log c) at
    # c = e^2 > e^x for x < 2 gives d/dc = 1 / c
    ce = np.full(4, np.exp(2.0))
    gx, gc = O.expr_vjp([IN(0, 0), IN(1, 1), OP(O.X_LOG, 2, 1), OP(O.X_MAX, 3, 0, 2)], 3, [x, ce])
    assert gx.tolist() == [0, 0, 0, 0] and np.array_equal(gc, 1.0 / ce)


def test_vjp_of_a_value_used_twice_adds_both_terms():
    x = RNG.uniform(-2, 2, 60)
    (g,) = O.expr_vjp([IN(0, 0), OP(O.X_MUL, 1, 0, 0), IN(2, 0), OP(O.X_ADD, 1, 1, 2)], 1, [x])
    assert np.allclose(g, 2 * x + 1, rtol=1e-15, atol=1e-15)


@pytest.mark.parametrize("seeded", [False, True])
def test_vjp_matches_central_differences(seeded):
    n = 40
    a, b = RNG.uniform(-1, 1, n), RNG.uniform(-1, 1, n)
    c = RNG.uniform(0.5, 2.0, n)
    # gauss-dot body plus a tail through every remaining unary and binary op
    prog = list(GAUSS_DOT) + [IN(5, 2), OP(O.X_DIV, 6, 2, 5), OP(O.X_SQRT, 7, 5), OP(O.X_RSQRT, 8, 5),
                              OP(O.X_LOG, 9, 5), OP(O.X_ABS, 10, 6), OP(O.X_MIN, 11, 10, 7),
                              OP(O.X_MAX, 12, 11, 8), OP(O.X_ADD, 13, 12, 9), OP(O.X_MUL, 13, 13, 6)]
    gout = RNG.uniform(-1, 1, n) if seeded else None
    gscale = 0.625 if seeded else None
    grads = O.expr_vjp(prog, 13, [a, b, c], gout=gout, gscale=gscale)
    seed = (gout if seeded else 1.0) * (gscale if seeded else 1.0)
    ins = [a, b, c]
    for k in range(3):
        h = 1e-6 * np.maximum(1.0, np.abs(ins[k]))
        up = [x.copy() for x in ins]
        dn = [x.copy() for x in ins]
        up[k] += h
        dn[k] -= h
        fd = (O.expr_map(prog, 13, *up) - O.expr_map(prog, 13, *dn)) / (2 * h) * seed
        assert np.allclose(grads[k], fd, rtol=2e-6, atol=2e-7), k


def test_loop_scatter_identity_and_permutation_and_skips():
    a, b = RNG.uniform(-1, 1, 77), RNG.uniform(-1, 1, 77)
    vals = O.expr_map(GAUSS_DOT, 2, a, b)
    ident = np.arange(77)
    assert np.array_equal(O.expr_loop_scatter(GAUSS_DOT, 2, [a, b], ident, np.zeros(77)), vals)
    perm = RNG.permutation(100)[:77]
    ref = np.full(100, -5.0)
    ref[perm] = vals                          # numpy fancy-index assignment
    assert np.array_equal(O.expr_loop_scatter(GAUSS_DOT, 2, [a, b], perm, np.full(100, -5.0)), ref)
    idx = ident.copy()
    idx[3], idx[5] = -1, 77                   # outside the output: not written
    got = O.expr_loop_scatter(GAUSS_DOT, 2, [a, b], idx, np.full(77, 9.0))
    assert got[3] == 9.0 and got[5] == 9.0 and np.array_equal(np.delete(got, [3, 5]), np.delete(vals, [3, 5]))


def test_min_max_return_the_first_operand_on_ties():
    # min a b = (b < a ? b : a) and max a b = (b > a ? b : a): on equal
    # values (here +0 and -0) the first operand comes back, sign included
    a = np.array([0.0, -0.0, 1.0], dtype=np.float64)
    b = np.array([-0.0, 0.0, 1.0], dtype=np.float64)
    for xop in (O.X_MIN, O.X_MAX):
        got = O.expr_map([IN(0, 0), IN(1, 1), OP(xop, 2, 0, 1)], 2, a, b)
        assert np.array_equal(np.signbit(got), np.signbit(a)) and np.array_equal(got, a)
