"""Pins for the oracle: each test checks it against something other than itself.

Sources of truth used here: the worked instances of the paper's own programs
(tests/golden/paper_examples.json, hand computed), closed forms, algebraic
invariants, IEEE facts (a binary32 op equals the binary64 result rounded once,
since binary64 has more than 2p+2 bits), textbook error bounds for recursive
summation, exact scaling laws, brute force on tiny inputs, library routines on
special cases, and central finite differences of the oracle's own forward
functions for every adjoint.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest

import oracle as O
import workloads as W

U64 = 2 ** 64
RNG_ADJ = np.random.default_rng(2211)
EPS64 = 2.0 ** -53


def _wrap(x):
    x %= U64
    return x - U64 if x >= 2 ** 63 else x


# ------------------------------------------------------------------ golden
@pytest.fixture(scope="module")
def gold(golden_dir):
    with open(os.path.join(golden_dir, "paper_examples.json")) as f:
        return json.load(f)


def test_golden_map2_addi(gold):
    g = gold["map2_addi"]
    assert O.map2(O.B_ADD, np.array(g["s1"]), np.array(g["s2"])).tolist() == g["out"]


def test_golden_reduce_muli(gold):
    g = gold["reduce_muli"]
    assert O.reduce(O.MUL, g["ne"], np.array(g["s"])) == g["out"]


def test_golden_loop_double(gold):
    g = gold["loop_double"]
    a = np.array(g["a"])
    assert O.map(O.U_AFFINE, a, (2, 0)).tolist() == g["b"]


def test_golden_listing1(gold):
    g = gold["listing1_small"]
    t1 = np.array(g["t1"])
    t2 = np.array(g["t2"])
    two_t2 = O.map(O.U_AFFINE, t2, (2, 0))
    t1 = O.map2(O.B_ADD, t1, two_t2)
    assert t1.tolist() == g["t1_after"]
    assert O.foldl(O.ADD, 0, t1) == g["sum"]
    gl = gold["listing1_large"]
    n = gl["n"]
    t1 = O.map2(O.B_ADD, np.arange(n), O.map(O.U_AFFINE, np.ones(n, dtype=np.int64), (2, 0)))
    assert O.reduce(O.ADD, 0, t1) == gl["sum"]


def test_golden_listing2(gold):
    g = gold["listing2"]
    c = g["c"]
    mapped = O.map(O.U_AFFINE, np.array(g["s"]), (c, c))  # c * (x + 1)
    assert mapped.tolist() == g["mapped"]
    assert O.reduce(O.ADD, 0, mapped) == g["sum"]


def test_golden_flatten(gold):
    g = gold["flatten"]
    values, offs = O.marshal_nested(g["nested"], 2)
    assert values == g["out"]
    assert offs[0].tolist() == g["offsets"]
    v2, rest = O.flatten(values, offs)
    assert v2 == g["out"] and rest == []


# ------------------------------------------------------------------ reduce (integer)
@pytest.mark.parametrize("n", [0, 1, 2, 99, 100, 101, 4097, 100000])
def test_sum_closed_form(n):
    assert O.reduce(O.ADD, 0, np.arange(1, n + 1, dtype=np.int64)) == n * (n + 1) // 2


@pytest.mark.parametrize("n", [0, 1, 5, 12, 20])
def test_product_is_factorial(n):
    assert O.reduce(O.MUL, 1, np.arange(1, n + 1, dtype=np.int64)) == math.factorial(n)


def test_product_wraps_mod_2_64():
    n = 25
    assert O.reduce(O.MUL, 1, np.arange(1, n + 1, dtype=np.int64)) == _wrap(math.factorial(n))


def test_listing2_closed_form():
    rng = np.random.default_rng(3)
    s = rng.integers(-10 ** 6, 10 ** 6, 5000)
    for c in (10, 13, 20):
        mapped = O.map(O.U_AFFINE, s, (c, c))
        assert O.reduce(O.ADD, 0, mapped) == c * (int(s.sum()) + len(s))


def _tree(op, xs, rng):
    if len(xs) == 1:
        return xs[0]
    cut = int(rng.integers(1, len(xs)))
    left, right = _tree(op, xs[:cut], rng), _tree(op, xs[cut:], rng)
    if op == O.ADD:
        return _wrap(left + right)
    if op == O.MUL:
        return _wrap(left * right)
    if op == O.MIN:
        return min(left, right)
    return max(left, right)


@pytest.mark.parametrize("op", [O.ADD, O.MUL, O.MIN, O.MAX])
def test_integer_reduce_bracketing_invariant(op):
    rng = np.random.default_rng(op)
    for trial in range(20):
        n = int(rng.integers(1, 200))
        xs = [int(v) for v in rng.integers(-2 ** 62, 2 ** 62, n)]
        ne = {O.ADD: 0, O.MUL: 1, O.MIN: 2 ** 63 - 1, O.MAX: -2 ** 63}[op]
        expect = _tree(op, xs, rng)
        assert O.reduce(op, ne, np.array(xs, dtype=np.int64)) == expect


def test_reduce_empty_is_ne():
    assert O.reduce(O.ADD, 7, np.zeros(0, dtype=np.int64)) == 7
    assert O.reduce(O.MAX, -3.5, np.zeros(0)) == -3.5


def test_reduce_nonneutral_ne_is_left_fold():
    s = np.array([4, 5, 6])
    # foldl (+) 10 [4,5,6] = 25 and foldl (-)-like checks are covered by min/max below
    assert O.reduce(O.ADD, 10, s) == 25
    assert O.reduce(O.MIN, 2, s) == 2
    assert O.reduce(O.MAX, 2, s) == 6


def test_min_max_match_builtins():
    rng = np.random.default_rng(11)
    x = rng.normal(size=1001)
    assert O.reduce(O.MIN, np.inf, x) == min(x.tolist())
    assert O.reduce(O.MAX, -np.inf, x) == max(x.tolist())


# ------------------------------------------------------------------ reduce (float)
@pytest.mark.parametrize("n", [1, 1000, 2 ** 20])
def test_float_fold_within_recursive_summation_bound(n):
    a, _ = W.dot_f32(n, seed=5)
    x = a.astype(np.float64)
    got = O.reduce(O.ADD, 0.0, x)
    exact = math.fsum(x.tolist())
    bound = (n - 1) * EPS64 * float(np.abs(x).sum()) * 1.01
    assert abs(got - exact) <= bound


def test_dot_of_dyadic_constants_exact():
    for n in (1, 3, 1000, 2 ** 20):
        a = np.full(n, 0.5, dtype=np.float32)
        b = np.full(n, 0.25, dtype=np.float32)
        assert O.dot(a, b) == n / 8


def test_dot_int_matches_exact_python():
    a, b = W.dot_i32(5000, seed=2)
    assert O.dot(a, b) == sum(int(x) * int(y) for x, y in zip(a.tolist(), b.tolist()))


def test_dot_float_near_exact():
    a, b = W.dot_f32(4096, seed=1)
    prods = [float(x) * float(y) for x, y in zip(a.tolist(), b.tolist())]  # exact in binary64
    exact = math.fsum(prods)
    got = O.dot(a, b)
    assert abs(got - exact) <= 4096 * EPS64 * sum(abs(p) for p in prods)


# ------------------------------------------------------------------ map / map2
def test_map_preserves_length():
    for n in (0, 1, 17):
        assert O.map(O.U_NEG, np.arange(n)).shape == (n,)
        assert O.map2(O.B_ADD, np.arange(n), np.arange(n)).shape == (n,)


def test_map2_length_mismatch_rejected():
    with pytest.raises(ValueError):
        O.map2(O.B_ADD, np.arange(3), np.arange(4))


@pytest.mark.parametrize("f,npop", [(O.B_ADD, np.add), (O.B_SUB, np.subtract),
                                    (O.B_MUL, np.multiply), (O.B_DIV, np.divide),
                                    (O.B_MIN, np.minimum), (O.B_MAX, np.maximum)])
def test_map2_binary32_single_rounding(f, npop):
    a, b = W.dot_f32(20000, seed=9)
    got = O.map2(f, a, b).astype(np.float32)
    want = npop(a, b)  # IEEE binary32, one rounding
    assert np.array_equal(got, want)


def test_map2_int_ops():
    a, b = W.dot_i32(1000, seed=4)
    ai, bi = a.astype(np.int64).tolist(), b.astype(np.int64).tolist()
    assert O.map2(O.B_SUB, a, b).tolist() == [x - y for x, y in zip(ai, bi)]
    assert O.map2(O.B_MUL, a, b).tolist() == [x * y for x, y in zip(ai, bi)]
    assert O.map2(O.B_MIN, a, b).tolist() == [min(x, y) for x, y in zip(ai, bi)]


def test_map_unary_identities():
    rng = np.random.default_rng(0)
    x = rng.uniform(0.1, 10.0, 1000)
    assert np.array_equal(O.map(O.U_NEG, O.map(O.U_NEG, x)), x)
    assert np.allclose(O.map(O.U_EXP, O.map(O.U_LOG, x)), x, rtol=4e-15)
    r = O.map(O.U_SQRT, x)
    assert np.allclose(r * r, x, rtol=4e-16)
    assert np.allclose(O.map(O.U_RSQRT, x) * r, 1.0, rtol=4e-16)
    y = rng.normal(size=1000)
    ab = O.map(O.U_ABS, y)
    assert np.all(ab >= 0) and np.all((ab == y) | (ab == -y))
    assert O.map(O.U_SQ, np.array([3.0, -0.5]))[0] == 9.0
    assert O.map(O.U_EXP, np.array([0.0]))[0] == 1.0 and O.map(O.U_LOG, np.array([1.0]))[0] == 0.0
    # exp(a + b) = exp(a) exp(b)
    a, b = rng.uniform(-3, 3, 200), rng.uniform(-3, 3, 200)
    assert np.allclose(O.map(O.U_EXP, a + b), O.map(O.U_EXP, a) * O.map(O.U_EXP, b), rtol=1e-14)


# ------------------------------------------------------------------ marshaling
def _random_nested(rng, depth, maxlen=4):
    if depth == 1:
        return [int(v) for v in rng.integers(-50, 50, int(rng.integers(0, maxlen + 1)))]
    return [_random_nested(rng, depth - 1, maxlen) for _ in range(int(rng.integers(0, maxlen + 1)))]


@pytest.mark.parametrize("depth", [1, 2, 3])
def test_marshal_roundtrip(depth):
    rng = np.random.default_rng(depth)
    for _ in range(50):
        x = _random_nested(rng, depth)
        values, offs = O.marshal_nested(x, depth)
        assert O.unmarshal_nested(values, offs) == x
        for lvl in offs:
            assert lvl[0] == 0 and np.all(np.diff(lvl) >= 0)


def test_marshal_flatten_is_concat():
    rng = np.random.default_rng(7)
    x = _random_nested(rng, 2, 8)
    values, offs = O.marshal_nested(x, 2)
    assert values == list(itertools.chain.from_iterable(x))
    assert np.array_equal(np.diff(offs[0]), [len(r) for r in x])
    x3 = _random_nested(rng, 3, 5)
    v3, o3 = O.marshal_nested(x3, 3)
    vf, of = O.flatten(v3, o3)
    assert O.unmarshal_nested(vf, of) == list(itertools.chain.from_iterable(x3))


def test_offsets_from_lengths():
    L = W.ragged_lengths(10000, seed=3)
    off = O.offsets_from_lengths(L)
    assert off[0] == 0 and off[-1] == int(L.sum())
    assert np.array_equal(np.diff(off), L)
    assert O.offsets_from_lengths(np.zeros(0, dtype=np.int64)).tolist() == [0]


def test_marshal_rows_and_records():
    rng = np.random.default_rng(1)
    rows = [rng.normal(size=int(n)).astype(np.float32) for n in rng.integers(0, 9, 30)]
    values, off = O.marshal_rows(rows)
    for r, row in enumerate(rows):
        assert np.array_equal(values[off[r]:off[r + 1]], row)
    recs = [{"x": float(i), "y": -float(i), "m": 0.5 * i} for i in range(7)]
    soa = O.marshal_records(recs, ["x", "y", "m"])
    assert soa["y"].tolist() == [-float(i) for i in range(7)]
    assert O.unmarshal_records(soa, ["x", "y", "m"]) == recs


RECORD_SCHEMA = [("id", "scalar", np.int64), ("xs", "seq", np.float32), ("w", "scalar", np.float64),
                 ("tags", "seq", np.int32), ("k", "scalar", np.int16)]


def _records(n, seed):
    rng = np.random.default_rng(seed)
    recs = []
    for r in range(n):
        lx, lt = int(rng.integers(0, 7)), int(rng.integers(0, 4))
        recs.append({"id": int(rng.integers(-2 ** 40, 2 ** 40)), "xs": rng.uniform(-1, 1, lx).astype(np.float32).tolist(),
                     "w": float(rng.normal()), "tags": rng.integers(-100, 100, lt).tolist(),
                     "k": int(rng.integers(-300, 300))})
    return recs


def test_marshal_record_seqs_fieldwise_layout():
    recs = _records(40, 3)
    lay = O.marshal_record_seqs(recs, RECORD_SCHEMA)
    # scalar fields: the column in record order (numpy's own array of the column)
    assert np.array_equal(lay["id"], np.array([r["id"] for r in recs]))
    assert lay["k"].dtype == np.int16 and lay["k"].tolist() == [r["k"] for r in recs]
    for name in ("xs", "tags"):
        vals, off = lay[name]
        # offsets: the running sum of the sequence lengths (numpy cumsum); values: numpy concatenate
        assert np.array_equal(off, np.concatenate([[0], np.cumsum([len(r[name]) for r in recs])]))
        parts = [np.asarray(r[name]) for r in recs]
        assert np.array_equal(vals, np.concatenate(parts).astype(vals.dtype))
    assert O.unmarshal_record_seqs(lay, RECORD_SCHEMA) == [
        {k: (v if not isinstance(v, list) else [type(x)(x) for x in v]) for k, v in r.items()} for r in recs]


def test_marshal_record_seqs_empty_cases():
    lay = O.marshal_record_seqs([], RECORD_SCHEMA)
    assert lay["id"].size == 0 and lay["xs"][1].tolist() == [0]
    recs = [{"id": 1, "xs": [], "w": 0.5, "tags": [], "k": 0}] * 3
    lay = O.marshal_record_seqs(recs, RECORD_SCHEMA)
    assert lay["xs"][1].tolist() == [0, 0, 0, 0] and lay["tags"][0].size == 0
    assert O.unmarshal_record_seqs(lay, RECORD_SCHEMA) == recs


def test_ragged_lengths_distribution():
    L = W.ragged_lengths(65536, seed=0)
    assert L.min() >= 1 and L.max() <= 4096
    # E[L] for P(L=k) proportional to ln((k+1)/k) on [1, 4096]
    ks = np.arange(1, 4097, dtype=np.float64)
    p = np.log((ks + 1) / ks)
    mean = float((ks * p).sum() / p.sum())
    assert abs(L.mean() - mean) < 0.03 * mean


# ------------------------------------------------------------------ segmented
def test_segmented_rows_of_ones_give_lengths():
    L = W.ragged_lengths(3000, seed=1)
    off = O.offsets_from_lengths(L)
    out = O.segmented_reduce(O.ADD, 0, np.ones(int(off[-1]), dtype=np.int64), off)
    assert np.array_equal(out, L)


def test_segmented_int_brute_force_and_flatten_total():
    rng = np.random.default_rng(2)
    L = W.ragged_lengths(500, seed=2, lmax=300)
    L[::17] = 0
    off = O.offsets_from_lengths(L)
    v = rng.integers(-1000, 1001, int(off[-1]))
    out = O.segmented_reduce(O.ADD, 0, v, off)
    vl = v.tolist()
    assert out.tolist() == [sum(vl[off[r]:off[r + 1]]) for r in range(len(L))]
    assert int(out.sum()) == O.reduce(O.ADD, 0, v)
    mx = O.segmented_reduce(O.MAX, -10 ** 9, v, off)
    assert mx.tolist() == [max(vl[off[r]:off[r + 1]], default=-10 ** 9) for r in range(len(L))]


def test_segmented_float_within_bound():
    L, v = W.ragged_f32(400, seed=4, lmax=2000, empty_rows=5)
    off = O.offsets_from_lengths(L)
    out = O.segmented_reduce(O.ADD, 0.0, v, off)
    for r in range(len(L)):
        seg = v[off[r]:off[r + 1]].astype(np.float64)
        assert abs(out[r] - math.fsum(seg.tolist())) <= max(len(seg), 1) * EPS64 * np.abs(seg).sum()
        if len(seg) == 0:
            assert out[r] == 0.0


def test_segmented_sum_adjoint_by_finite_differences():
    rng = np.random.default_rng(5)
    L = np.array([3, 0, 1, 5, 2])
    off = O.offsets_from_lengths(L)
    v = rng.normal(size=int(off[-1]))
    g = rng.normal(size=len(L))
    adj = O.segmented_sum_adjoint(g, off)
    h = 1e-6
    for e in range(len(v)):
        vp, vm = v.copy(), v.copy()
        vp[e] += h
        vm[e] -= h
        fd = (np.dot(g, O.segmented_reduce(O.ADD, 0.0, vp, off))
              - np.dot(g, O.segmented_reduce(O.ADD, 0.0, vm, off))) / (2 * h)
        assert abs(fd - adj[e]) <= 1e-8 * (1 + abs(adj[e]))


# ------------------------------------------------------------------ dense
# ------------------------------------------------------------------ reverse of reduce (min / max / +)
def test_reduce_min_max_adjoint_is_the_library_argmin():
    # values distinct: the fold ends on numpy's argmin / argmax
    x = RNG_ADJ.permutation(1000).astype(np.float64) * 0.5 - 100
    for op, arg in ((O.MIN, np.argmin(x)), (O.MAX, np.argmax(x))):
        ne = np.inf if op == O.MIN else -np.inf
        g = O.reduce_adjoint(op, ne, x, 3.0)
        ref = np.zeros_like(x)
        ref[arg] = 3.0
        assert np.array_equal(g, ref)


def test_reduce_min_max_adjoint_by_finite_differences():
    # on distinct values min / max are locally one of the elements: the central
    # difference of the oracle's own fold is 1 there and 0 elsewhere
    x = RNG_ADJ.uniform(-1, 1, 40)
    for op in (O.MIN, O.MAX):
        ne = np.inf if op == O.MIN else -np.inf
        g = O.reduce_adjoint(op, ne, x, 1.0)
        fd = np.empty_like(x)
        for i in range(x.size):
            h = 1e-7
            up, dn = x.copy(), x.copy()
            up[i] += h
            dn[i] -= h
            fd[i] = (O.reduce(op, ne, up) - O.reduce(op, ne, dn)) / (2 * h)
        assert np.allclose(g, fd, rtol=1e-8, atol=1e-8), op


def test_reduce_min_max_adjoint_ties_and_neutral_element():
    # equal values: the lowest index (numpy's argmin also returns the first)
    x = np.array([3.0, 1.0, 2.0, 1.0, 1.0])
    assert O.reduce_adjoint(O.MIN, np.inf, x, 1.0).tolist() == [0, 1, 0, 0, 0]
    assert O.reduce_adjoint(O.MAX, -np.inf, -x, 1.0).tolist() == [0, 1, 0, 0, 0]
    # +0 and -0 compare equal: the first of them
    z = np.array([1.0, 0.0, -0.0])
    assert O.reduce_adjoint(O.MIN, np.inf, z, 1.0).tolist() == [0, 1, 0]
    # ne at or beyond the extreme: y = ne does not depend on the elements
    assert O.reduce_adjoint(O.MIN, 1.0, x, 1.0).tolist() == [0] * 5
    assert O.reduce_adjoint(O.MIN, 0.5, x, 1.0).tolist() == [0] * 5
    assert O.reduce_adjoint(O.MAX, 3.0, x, 1.0).tolist() == [0] * 5
    # a finite ne that the elements improve on: the arg as before
    assert O.reduce_adjoint(O.MAX, 2.5, x, 2.0).tolist() == [2, 0, 0, 0, 0]
    assert O.reduce_adjoint(O.MIN, 7.0, np.zeros(0), 1.0).size == 0
    # NaN elements never replace the accumulator of the fold
    y = np.array([np.nan, 2.0, np.nan, 1.5])
    assert O.reduce_adjoint(O.MIN, np.inf, y, 1.0).tolist() == [0, 0, 0, 1]
    with pytest.raises(ValueError):
        O.reduce_adjoint(O.MUL, 1.0, x, 1.0)


def test_reduce_add_adjoint_is_a_broadcast():
    x = RNG_ADJ.uniform(-1, 1, 17)
    assert np.array_equal(O.reduce_adjoint(O.ADD, 0.0, x, -1.25), np.full(17, -1.25))


def test_segmented_reduce_adjoint_row_by_row():
    L = np.array([0, 3, 1, 0, 5, 2])
    off = O.offsets_from_lengths(L)
    v = RNG_ADJ.permutation(int(off[-1])).astype(np.float64)
    g = np.arange(1, len(L) + 1, dtype=np.float64)
    for op in (O.MIN, O.MAX):
        ne = np.inf if op == O.MIN else -np.inf
        got = O.segmented_reduce_adjoint(op, ne, v, off, g)
        ref = np.zeros_like(v)
        for r in range(len(L)):
            row = v[off[r]:off[r + 1]]
            if row.size:
                ref[off[r] + (np.argmin(row) if op == O.MIN else np.argmax(row))] = g[r]
        assert np.array_equal(got, ref)
    assert np.array_equal(O.segmented_reduce_adjoint(O.ADD, 0.0, v, off, g), O.segmented_sum_adjoint(g, off))


def test_matmul_rank_one_closed_form():
    M, N, K = 7, 5, 33
    u = np.arange(1, M + 1) * 0.25
    v = np.arange(1, N + 1) * -0.5
    A = np.outer(u, np.ones(K))
    B = np.outer(np.ones(K), v)
    assert np.array_equal(O.matmul(A, B), K * np.outer(u, v))


def test_matmul_identity_and_library():
    rng = np.random.default_rng(0)
    A = rng.uniform(-1, 1, (9, 13))
    B = rng.uniform(-1, 1, (13, 6))
    assert np.array_equal(O.matmul(A, np.eye(13)), A)
    assert np.array_equal(O.matmul(np.eye(9), A), A)
    ref = A @ B
    assert np.allclose(O.matmul(A, B), ref, rtol=0, atol=1e-14 * 13)


def test_matmul_transposed_operands():
    rng = np.random.default_rng(1)
    A = rng.uniform(-1, 1, (6, 11))
    B = rng.uniform(-1, 1, (11, 4))
    C = O.matmul(A, B)
    assert np.array_equal(O.matmul(A.T.copy(), B, ta=True), C)
    assert np.array_equal(O.matmul(A, B.T.copy(), tb=True), C)
    assert np.array_equal(O.matmul(A.T.copy(), B.T.copy(), ta=True, tb=True), C)
    assert np.allclose(O.matmul(B, A, ta=True, tb=True), (A @ B).T, atol=1e-14)


# ------------------------------------------------------------------ N-body
EPS2 = 1e-6


def test_two_body_inverse_square_law():
    x = np.array([[0.0, 0.0, 0.0], [2.0, 0.0, 0.0]])
    m = np.array([3.0, 5.0])
    a = O.nbody_accel(x, m, eps2=1e-30, G=1.0)
    assert abs(a[0, 0] - 5.0 / 4.0) < 1e-14 and abs(a[1, 0] + 3.0 / 4.0) < 1e-14
    assert np.all(a[:, 1:] == 0.0)


def test_three_body_symmetric_middle_feels_nothing():
    x = np.array([[-1.0, 0.5, 0.25], [0.0, 0.5, 0.25], [1.0, 0.5, 0.25]])
    m = np.array([2.0, 7.0, 2.0])
    a = O.nbody_accel(x, m, EPS2)
    assert np.all(a[1] == 0.0)
    assert a[0, 0] > 0 and a[2, 0] < 0 and a[0, 0] == -a[2, 0]


def test_momentum_conservation_and_exact_scaling():
    pos, mass, _ = W.nbody(64, seed=3)
    x, m = pos.astype(np.float64), mass.astype(np.float64)
    a = O.nbody_accel(x, m, EPS2)
    p = (m[:, None] * a).sum(0)
    assert np.all(np.abs(p) <= 1e-12 * np.abs(m[:, None] * a).sum(0))
    # x -> 2x, eps -> 2 eps: every distance doubles, so a -> a / 4 exactly
    assert np.array_equal(O.nbody_accel(2 * x, m, 4 * EPS2), a / 4)
    # m -> 2m: a -> 2a exactly; G -> 2G likewise
    assert np.array_equal(O.nbody_accel(x, 2 * m, EPS2), 2 * a)
    # translation invariance up to rounding of the differences
    assert np.allclose(O.nbody_accel(x + 0.125, m, EPS2), a, rtol=1e-9, atol=1e-9)


def test_nbody_permutation_equivariance():
    pos, mass, _ = W.nbody(40, seed=4)
    x, m = pos.astype(np.float64), mass.astype(np.float64)
    perm = np.random.default_rng(0).permutation(40)
    a = O.nbody_accel(x, m, EPS2)
    ap = O.nbody_accel(x[perm], m[perm], EPS2)
    assert np.allclose(ap, a[perm], rtol=1e-12, atol=1e-12)


def test_euler_free_particle_and_rest_start():
    x0 = np.array([[0.5, 0.25, -1.0]])
    v0 = np.array([[1.0, -2.0, 0.5]])
    xT, vT = O.nbody_forward(x0, v0, np.array([1.0]), EPS2, 1.0, 0.125, 8)
    assert np.array_equal(xT, x0 + v0) and np.array_equal(vT, v0)
    pos, mass, vel = W.nbody(16, seed=1)
    x1, v1 = O.nbody_step(pos, vel, mass, EPS2, 1.0, 1e-3)
    assert np.array_equal(x1, pos.astype(np.float64))
    assert np.array_equal(v1, 1e-3 * O.nbody_accel(pos, mass, EPS2))


def test_total_momentum_stays_zero():
    pos, mass, vel = W.nbody(32, seed=2)
    xT, vT = O.nbody_forward(pos, vel, mass, 1e-4, 1.0, 1e-3, 10)
    p = (mass.astype(np.float64)[:, None] * vT).sum(0)
    assert np.all(np.abs(p) <= 1e-10 * np.abs(mass[:, None] * vT).sum(0) + 1e-15)


def test_accel_vjp_by_finite_differences():
    rng = np.random.default_rng(8)
    x = rng.uniform(0, 1, (5, 3))
    m = rng.uniform(0.5, 1.5, 5)
    abar = rng.normal(size=(5, 3))
    eps2 = 1e-2
    vjp = O.nbody_accel_vjp(x, m, abar, eps2, G=1.3)
    h = 1e-6
    for k in range(5):
        for c in range(3):
            xp, xm = x.copy(), x.copy()
            xp[k, c] += h
            xm[k, c] -= h
            fd = (np.sum(abar * O.nbody_accel(xp, m, eps2, 1.3))
                  - np.sum(abar * O.nbody_accel(xm, m, eps2, 1.3))) / (2 * h)
            assert abs(fd - vjp[k, c]) <= 1e-6 * (1 + abs(vjp[k, c]))


def test_ke_gradient_by_finite_differences():
    rng = np.random.default_rng(9)
    N, T, dt, eps2 = 6, 4, 2e-2, 1e-2
    x0 = rng.uniform(0, 1, (N, 3))
    v0 = rng.normal(scale=0.1, size=(N, 3))
    m = rng.uniform(0.5, 1.5, N)
    ke, gx, gv = O.nbody_ke_grad(x0, v0, m, eps2, 1.0, dt, T)
    xT, vT = O.nbody_forward(x0, v0, m, eps2, 1.0, dt, T)
    assert ke == O.nbody_kinetic(vT, m)
    h = 1e-6
    for i in range(N):
        for c in range(3):
            for arr, g in ((x0, gx), (v0, gv)):
                p, q = arr.copy(), arr.copy()
                p[i, c] += h
                q[i, c] -= h
                args_p = (p, v0) if arr is x0 else (x0, p)
                args_q = (q, v0) if arr is x0 else (x0, q)
                fp = O.nbody_kinetic(O.nbody_forward(*args_p, m, eps2, 1.0, dt, T)[1], m)
                fq = O.nbody_kinetic(O.nbody_forward(*args_q, m, eps2, 1.0, dt, T)[1], m)
                fd = (fp - fq) / (2 * h)
                assert abs(fd - g[i, c]) <= 1e-6 * (1 + abs(g[i, c]))


@pytest.mark.parametrize("k", [1, 2, 3, 5, 7])
def test_checkpointed_reverse_equals_full_tape(k):
    pos, mass, vel = W.nbody(12, seed=6)
    ke1, gx1, gv1 = O.nbody_ke_grad(pos, vel, mass, EPS2, 1.0, 1e-3, 7)
    ke2, gx2, gv2 = O.nbody_ke_grad(pos, vel, mass, EPS2, 1.0, 1e-3, 7, ckpt_every=k)
    assert ke1 == ke2 and np.array_equal(gx1, gx2) and np.array_equal(gv1, gv2)


# ------------------------------------------------------------------ k-means
def test_kmeans_assign_brute_force_and_validity():
    X, blob, centres = W.kmeans_blobs(2000, 8, 6, seed=1)
    C = X[:6].astype(np.float64)
    lab = O.kmeans_assign(X, C)
    D = ((X.astype(np.float64)[:, None, :] - C[None]) ** 2).sum(-1)
    assert np.array_equal(lab, np.argmin(D, axis=1))
    for i in range(0, 2000, 97):
        di = [O.sqdist(X[i], C[j]) for j in range(6)]
        assert all(di[lab[i]] <= dj for dj in di)


def test_kmeans_ties_take_lowest_index():
    X = np.array([[0.0, 0.0], [1.0, 1.0], [-3.0, 2.0]])
    C = np.array([[5.0, 5.0], [0.5, 0.5], [0.5, 0.5], [-3.0, 2.0], [-3.0, 2.0]])
    assert O.kmeans_assign(X, C).tolist() == [1, 1, 3]


def test_sqdist_within_bound():
    rng = np.random.default_rng(2)
    x, c = rng.normal(size=32), rng.normal(size=32)
    terms = (x - c) ** 2
    assert abs(O.sqdist(x, c) - math.fsum(terms.tolist())) <= 32 * 3 * EPS64 * terms.sum()


def test_kmeans_update_counts_sums_and_empty_cluster():
    X, blob, centres = W.kmeans_blobs(3000, 5, 4, seed=2)
    C = np.vstack([X[:4].astype(np.float64), [[1e6] * 5]])  # cluster 4 stays empty
    lab = O.kmeans_assign(X, C)
    counts, sums, C_new = O.kmeans_update(X, lab, C)
    assert np.array_equal(counts, np.bincount(lab, minlength=5)) and counts.sum() == 3000
    assert counts[4] == 0 and np.array_equal(C_new[4], C[4])
    ref = np.zeros((5, 5))
    np.add.at(ref, lab, X.astype(np.float64))
    assert np.allclose(sums, ref, rtol=1e-12, atol=1e-9)
    for j in range(4):
        assert np.allclose(C_new[j], X[lab == j].astype(np.float64).mean(0), rtol=1e-12, atol=1e-12)


def test_kmeans_blobs_separate_after_iterations():
    X, blob, centres = W.kmeans_blobs(4000, 8, 5, seed=3, spread=30.0)
    C = centres.astype(np.float64) + 0.5
    for _ in range(3):
        lab, counts, C = O.kmeans_step(X, C)
    for b in range(5):
        assert len(set(lab[blob == b].tolist())) == 1


def test_kmeans_sse_gradient_by_finite_differences():
    X, _, _ = W.kmeans_blobs(30, 4, 3, seed=4)
    X = X.astype(np.float64)
    C = X[:3].copy()
    lab = O.kmeans_assign(X, C)
    G = O.kmeans_sse_grad(X, C, lab, 0.5)
    h = 1e-5
    for i in range(0, 30, 7):
        for t in range(4):
            Xp, Xm = X.copy(), X.copy()
            Xp[i, t] += h
            Xm[i, t] -= h
            fd = 0.5 * (O.kmeans_sse(Xp, C, lab) - O.kmeans_sse(Xm, C, lab)) / (2 * h)
            assert abs(fd - G[i, t]) <= 1e-6 * (1 + abs(G[i, t]))


# ------------------------------------------------------------------ batched
def _small_batch():
    return W.batched_tasks(24, seed=5, smin=10, smax=3000)


def test_batch_forward_matches_library_per_task():
    bt = _small_batch()
    out = O.batch_forward(bt.table(), bt.A, bt.B, bt.out_len)
    for t in range(bt.ntasks):
        r, c = int(bt.rows[t]), int(bt.cols[t])
        a = bt.A[bt.a_off[t]: bt.a_off[t] + r * c].astype(np.float64)
        b = bt.B[bt.b_off[t]: bt.b_off[t] + c].astype(np.float64)
        if bt.kind[t] == W.TASK_DOT:
            ref = np.array([np.dot(a, b)])
        else:
            ref = a.reshape(r, c) @ b
        got = out[bt.out_off[t]: bt.out_off[t] + len(ref)]
        assert np.allclose(got, ref, rtol=1e-12, atol=1e-12 * c)


def test_batch_backward_by_finite_differences():
    bt = W.batched_tasks(6, seed=6, smin=10, smax=60)
    tb = bt.table()
    A, B, g = bt.A.astype(np.float64), bt.B.astype(np.float64), bt.gout.astype(np.float64)
    gA, gB = O.batch_backward(tb, A, B, g)
    h = 1e-3  # the forward is bilinear, so central differences are exact up to rounding
    rng = np.random.default_rng(0)
    for pool, grad, which in ((A, gA, 0), (B, gB, 1)):
        for e in rng.choice(len(pool), size=min(40, len(pool)), replace=False):
            p, q = pool.copy(), pool.copy()
            p[e] += h
            q[e] -= h
            fp = O.batch_forward(tb, p, B, bt.out_len) if which == 0 else O.batch_forward(tb, A, p, bt.out_len)
            fq = O.batch_forward(tb, q, B, bt.out_len) if which == 0 else O.batch_forward(tb, A, q, bt.out_len)
            fd = np.dot(g, fp - fq) / (2 * h)
            assert abs(fd - grad[e]) <= 1e-9 * (1 + abs(grad[e]))


def test_batch_permutation_invariance():
    bt = _small_batch()
    tb = bt.table()
    out = O.batch_forward(tb, bt.A, bt.B, bt.out_len)
    perm = np.random.default_rng(1).permutation(bt.ntasks)
    assert np.array_equal(O.batch_forward(tb[perm], bt.A, bt.B, bt.out_len), out)
