"""GPU parity of map, map2, reduce, the fused dot, marshaling and ragged /
dense nested map(reduce) against the oracle, through the C ABI."""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from parity import check_scalar, check_vector, say, ulp_diff_f32

pytestmark = pytest.mark.gpu

import paper_2211_00621_amd as mx  # noqa: E402  (no skip: a missing library must fail)
abi = mx.abi
api = mx.api

DEV = "cuda"


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


SIZES = [0, 1, 3, 63, 64, 65, 255, 256, 257, 1000, 4095, 4097, 65537, (1 << 20) + 3]


# ------------------------------------------------------------------ map / map2
@pytest.mark.parametrize("f,np_op", [(abi.MX_B_ADD, np.add), (abi.MX_B_SUB, np.subtract),
                                     (abi.MX_B_MUL, np.multiply), (abi.MX_B_DIV, np.divide),
                                     (abi.MX_B_MIN, np.minimum), (abi.MX_B_MAX, np.maximum)])
@pytest.mark.parametrize("n", [1, 5, 4099, 1 << 18])
def test_map2_f32_bit_exact(f, np_op, n):
    say("map2 f32", f, n)
    a, b = W.dot_f32(n, seed=n)
    out = api.map2(f, dev(a), dev(b))
    ref = O.map2(f, a, b).astype(np.float32)  # one IEEE binary32 rounding of the exact value
    assert np.array_equal(host(out), ref)


@pytest.mark.parametrize("dt", [np.int32, np.int64])
@pytest.mark.parametrize("f", [abi.MX_B_ADD, abi.MX_B_SUB, abi.MX_B_MUL, abi.MX_B_MIN, abi.MX_B_MAX])
def test_map2_int_exact(dt, f):
    say("map2 int", dt, f)
    rng = np.random.default_rng(f)
    n = 10007
    hi = 2 ** 31 - 1 if dt == np.int32 else 2 ** 62
    a = rng.integers(-hi, hi, n).astype(dt)
    b = rng.integers(-hi, hi, n).astype(dt)
    out = api.map2(f, dev(a), dev(b))
    assert np.array_equal(host(out), O.map2(f, a, b))


def test_map2_unaligned_views_and_inplace():
    say("map2 views")
    a, b = W.dot_f32(5001, seed=3)
    ta, tb = dev(a), dev(b)
    out = api.map2(abi.MX_B_ADD, ta[1:], tb[1:])  # offset by 4 bytes: scalar path
    assert np.array_equal(host(out), (a[1:] + b[1:]))
    # Listing 1's axpy loop as an in-place map2: t1 <- t1 + 2 t2
    t1 = dev(np.arange(1000, dtype=np.int64))
    t2 = dev(np.ones(1000, dtype=np.int64))
    two_t2 = api.map(abi.MX_U_AFFINE, t2, (2, 0))
    abi.mx_map2(abi.MX_B_ADD, t1, two_t2, t1)
    assert np.array_equal(host(t1), np.arange(1000) + 2)


@pytest.mark.parametrize("f", [abi.MX_U_ID, abi.MX_U_NEG, abi.MX_U_ABS, abi.MX_U_SQ])
@pytest.mark.parametrize("dt", [np.float32, np.float64, np.int32, np.int64])
def test_map_exact_bodies(f, dt):
    say("map", f, dt)
    rng = np.random.default_rng(1)
    x = (rng.uniform(-1000, 1000, 3001)).astype(dt)
    out = host(api.map(f, dev(x)))
    ref = O.map(f, x)
    if dt == np.float32:
        ref = ref.astype(np.float32)
    assert np.array_equal(out, ref)


def test_map_affine_listing2_int():
    say("map affine int")
    s = np.arange(-5000, 5000, dtype=np.int32)
    c = 13
    out = host(api.map(abi.MX_U_AFFINE, dev(s), (c, c)))
    assert out.dtype == np.int64
    assert np.array_equal(out, O.map(O.U_AFFINE, s, (c, c)))


@pytest.mark.parametrize("f,maxulp", [(abi.MX_U_EXP, 2), (abi.MX_U_LOG, 2), (abi.MX_U_SQRT, 1),
                                      (abi.MX_U_RSQRT, 2), (abi.MX_U_AFFINE, 2)])
def test_map_float_bodies_within_ulps(f, maxulp):
    say("map float", f)
    x = np.random.default_rng(2).uniform(0.01, 20.0, 20000).astype(np.float32)
    params = (1.5, 0.25) if f == abi.MX_U_AFFINE else None
    out = host(api.map(f, dev(x), params))
    ref = O.map(f, x, params or (0, 0)).astype(np.float32)
    assert ulp_diff_f32(out, ref).max() <= maxulp


# ------------------------------------------------------------------ reduce / fused dot
@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("op", [abi.MX_ADD, abi.MX_MUL, abi.MX_MIN, abi.MX_MAX])
def test_reduce_int64_exact(n, op):
    say("reduce i64", n, op)
    rng = np.random.default_rng(n + op)
    x = rng.integers(-2 ** 40, 2 ** 40, n).astype(np.int64)
    ne = {abi.MX_ADD: 0, abi.MX_MUL: 1, abi.MX_MIN: 2 ** 63 - 1, abi.MX_MAX: -2 ** 63}[op]
    got = int(host(api.reduce(op, dev(x), ne)))
    assert got == O.reduce(op, ne, x)


@pytest.mark.parametrize("n", SIZES)
def test_reduce_int32_widens(n):
    say("reduce i32", n)
    a, _ = W.dot_i32(n, seed=n)
    got = api.reduce(abi.MX_ADD, dev(a), 0)
    assert got.dtype == torch.int64 and int(host(got)) == O.reduce(O.ADD, 0, a)


def test_reduce_nonneutral_ne_is_left_fold():
    say("reduce ne")
    x = np.arange(1, 101, dtype=np.int64)
    assert int(host(api.reduce(abi.MX_ADD, dev(x), 1000))) == 1000 + 5050
    assert int(host(api.reduce(abi.MX_MAX, dev(x), 7000))) == 7000


@pytest.mark.parametrize("n", SIZES)
def test_reduce_f32_within_tolerance(n):
    say("reduce f32", n)
    a, _ = W.dot_f32(n, seed=n + 1)
    got = float(host(api.reduce(abi.MX_ADD, dev(a), 0.0)))
    R = O.reduce(O.ADD, 0.0, a)
    check_scalar(got, R, float(np.abs(a.astype(np.float64)).sum()), n, what=f"sum n={n}")
    mn = float(host(api.reduce(abi.MX_MIN, dev(a), np.inf)))
    assert mn == (O.reduce(O.MIN, np.inf, a) if n else np.inf)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_dot_f32_config(seed):
    """map2 (*) + reduce (+), two float32 vectors of 2^20, uniform [-1, 1]."""
    n = 1 << 20
    say("dot f32 2^20 seed", seed)
    a, b = W.dot_f32(n, seed)
    got = float(host(api.dot(dev(a), dev(b))))
    R = O.dot(a, b)
    S = O.map2_reduce(O.B_MUL, O.ADD, 0, np.abs(a), np.abs(b))
    check_scalar(got, R, S, n, what="dot")


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_dot_i32_config_exact(seed):
    """int32 variant, values in [-1000, 1000], products and sum in int64: bit-exact."""
    n = 1 << 20
    say("dot i32 2^20 seed", seed)
    a, b = W.dot_i32(n, seed)
    got = int(host(api.map2_reduce(abi.MX_B_MUL, abi.MX_ADD, dev(a), dev(b), 0)))
    assert got == O.dot(a, b)
    assert int(host(api.reduce(abi.MX_ADD, dev(a), 0))) == O.reduce(O.ADD, 0, a)


@pytest.mark.parametrize("k", [10, 14, 18, 22, 24])
def test_dot_f32_accuracy_sweep(k):
    n = (1 << k) + 7
    say("dot sweep", n)
    a, b = W.dot_f32(n, seed=k)
    got = float(host(api.dot(dev(a), dev(b))))
    R = O.dot(a, b)
    S = O.map2_reduce(O.B_MUL, O.ADD, 0, np.abs(a), np.abs(b))
    check_scalar(got, R, S, n, what=f"dot n={n}")


def test_dot_dyadic_constants_exact():
    n = 1 << 24
    say("dot dyadic")
    a = torch.full((n,), 0.5, device=DEV)
    b = torch.full((n,), 0.25, device=DEV)
    assert float(host(api.dot(a, b))) == n / 8


def test_reduce_deterministic_and_unaligned():
    say("reduce determinism")
    a, b = W.dot_f32((1 << 22) + 1, seed=9)
    ta, tb = dev(a), dev(b)
    r1 = host(api.dot(ta, tb))
    r2 = host(api.dot(ta, tb))
    assert r1.tobytes() == r2.tobytes()
    r3 = float(host(api.dot(ta[1:], tb[1:])))
    R = O.dot(a[1:], b[1:])
    check_scalar(r3, R, O.map2_reduce(O.B_MUL, O.ADD, 0, np.abs(a[1:]), np.abs(b[1:])), a.size - 1)


def test_dot_gradient_closed_form():
    say("dot adjoint")
    a, b = W.dot_f32(100003, seed=4)
    ta = dev(a).requires_grad_()
    tb = dev(b).requires_grad_()
    y = api.dot(ta, tb)
    (3.0 * y).backward()
    assert np.array_equal(host(ta.grad), (np.float32(3.0) * b).astype(np.float32))
    assert np.array_equal(host(tb.grad), (np.float32(3.0) * a).astype(np.float32))


# ------------------------------------------------------------------ marshaling
@pytest.mark.parametrize("nseg", [0, 1, 1023, 1024, 1025, 4095, 4096, 4097, 65536, 9_000_001])
def test_lengths_to_offsets_exact(nseg):
    say("offsets", nseg)
    L = W.ragged_lengths(nseg, seed=3, lmax=100) if nseg else np.zeros(0, dtype=np.int64)
    off = host(api.offsets_from_lengths(dev(L)))
    assert np.array_equal(off, O.offsets_from_lengths(L))


def test_lengths_to_offsets_reuse_and_wide_values():
    """Consecutive scans of different sizes share one workspace (the look-back
    status words must come back cleared), and sums beyond 32 bits stay exact."""
    say("offsets reuse")
    ws = api.workspace(abi.MX_WS_SCAN, 9_000_001)
    for nseg, lmax in ((65536, 4096), (4097, 10), (9_000_001, 100), (8193, 1 << 40), (65536, 4096)):
        L = W.ragged_lengths(nseg, seed=nseg, lmax=lmax)
        off = torch.empty(nseg + 1, dtype=torch.int64, device=DEV)
        abi.mx_lengths_to_offsets(dev(L), off, ws)
        assert np.array_equal(host(off), O.offsets_from_lengths(L)), nseg
    assert not host(ws).any(), "scan workspace not left zero"


def test_marshal_rows_roundtrip_and_flatten():
    say("marshal rows")
    L, v = W.ragged_f32(3000, seed=5, lmax=700, empty_rows=40)
    offs = O.offsets_from_lengths(L)
    rows = [v[offs[r]:offs[r + 1]] for r in range(len(L))]
    rg = api.marshal_rows(rows)
    values_o, offsets_o = O.marshal_rows(rows)
    assert np.array_equal(host(rg.offsets), offsets_o)
    assert np.array_equal(host(rg.flatten()), values_o)
    back = api.unmarshal_rows(rg)
    assert all(np.array_equal(x, y) for x, y in zip(back, rows))


def test_records_fields_roundtrip():
    say("records")
    rng = np.random.default_rng(0)
    recs = [{"x": float(rng.normal()), "y": float(rng.normal()), "z": float(rng.normal()),
             "m": float(rng.uniform(0.5, 1.5))} for _ in range(1001)]
    fields = ["x", "y", "z", "m"]
    aos = np.array([[r[f] for f in fields] for r in recs], dtype=np.float32)
    soa = api.records_to_fields(dev(aos))
    ref = O.marshal_records([{f: np.float32(r[f]) for f in fields} for r in recs], fields)
    for f, t in zip(fields, soa):
        assert np.array_equal(host(t), ref[f])
    assert np.array_equal(host(api.fields_to_records(soa)), aos)
    aos3 = np.arange(3 * 77, dtype=np.int64).reshape(77, 3)
    soa3 = api.records_to_fields(dev(aos3))
    assert np.array_equal(host(soa3[2]), aos3[:, 2])
    assert np.array_equal(host(api.fields_to_records(soa3)), aos3)


def test_compose_offsets_map_flatten():
    say("compose offsets")
    rng = np.random.default_rng(4)
    nested = [[list(rng.integers(0, 9, int(rng.integers(0, 4)))) for _ in range(int(rng.integers(0, 5)))]
              for _ in range(200)]
    values, (o1, o2) = O.marshal_nested(nested, 3)
    out = host(_compose(o1, o2))
    flat_rows = [[v for inner in outer for v in inner] for outer in nested]
    _, ref = O.marshal_nested(flat_rows, 2)
    assert np.array_equal(out, ref[0])


def _compose(o1, o2):
    out = torch.empty(len(o1), dtype=torch.int64, device=DEV)
    abi.mx_compose_offsets(dev(o1), dev(o2), out)
    return out


# ------------------------------------------------------------------ ragged nested map(reduce)
def _ragged(nseg, seed, lmax=4096, empty_rows=0):
    L, v = W.ragged_f32(nseg, seed, lmax, empty_rows)
    return L, v, O.offsets_from_lengths(L)


@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("plain", [False, True])
def test_segmented_sum_config(seed, plain):
    """65536 float32 rows, lengths log-uniform in [1, 4096]: every row vs the oracle."""
    say("segmented config seed", seed, "plain", plain)
    L, v, off = _ragged(65536, seed)
    rg = api.Ragged(dev(v), dev(off))
    got = host(api.segmented_reduce(abi.MX_ADD, rg, 0.0, plain=plain))
    R = O.segmented_reduce(O.ADD, 0.0, v, off)
    S = O.segmented_reduce(O.ADD, 0.0, np.abs(v), off)
    check_vector(got, R, S, L, what="row sums")


@pytest.mark.parametrize("op", [abi.MX_ADD, abi.MX_MUL, abi.MX_MIN, abi.MX_MAX])
@pytest.mark.parametrize("dt", [np.int32, np.int64])
def test_segmented_int_exact_with_empty_rows(op, dt):
    say("segmented int", op, dt)
    L = W.ragged_lengths(5000, seed=op, lmax=3000)
    L[::13] = 0
    off = O.offsets_from_lengths(L)
    rng = np.random.default_rng(op)
    v = rng.integers(-3, 4, int(off[-1])).astype(dt) if op == abi.MX_MUL else \
        rng.integers(-10 ** 6, 10 ** 6, int(off[-1])).astype(dt)
    ne = {abi.MX_ADD: 0, abi.MX_MUL: 1, abi.MX_MIN: 2 ** 63 - 1, abi.MX_MAX: -2 ** 63}[op]
    rg = api.Ragged(dev(v), dev(off))
    for plain in (False, True):
        got = host(api.segmented_reduce(op, rg, ne, plain=plain))
        assert np.array_equal(got, O.segmented_reduce(op, ne, v, off)), plain


def test_segmented_unaligned_values_view():
    say("segmented view")
    L, v, off = _ragged(777, 8, lmax=300)
    full = dev(np.concatenate([[np.float32(7.0)], v]))
    rg = api.Ragged(full[1:], dev(off))
    got = host(api.segmented_reduce(abi.MX_ADD, rg, 0.0))
    check_vector(got, O.segmented_reduce(O.ADD, 0.0, v, off),
                 O.segmented_reduce(O.ADD, 0.0, np.abs(v), off), L)


@pytest.mark.parametrize("lengths", [
    [0], [1], [5, 0, 3], [100000, 0, 250001],            # few rows: one row per block, many rounds
    [4096] * 17, [0] * 40 + [9000] + [0] * 40,            # full and ragged last block, empty runs
], ids=lambda L: f"n{len(L)}")
@pytest.mark.parametrize("dt", [np.float32, np.float64, np.int32])
def test_segmented_shapes(lengths, dt):
    """Row counts and lengths around the rows-per-block split, each dtype."""
    say("segmented shapes", len(lengths), dt)
    L = np.array(lengths, dtype=np.int64)
    off = O.offsets_from_lengths(L)
    rng = np.random.default_rng(len(L))
    if dt == np.int32:
        v = rng.integers(-1000, 1001, int(off[-1])).astype(dt)
    else:
        v = rng.uniform(-1, 1, int(off[-1])).astype(dt)
    for shift in (0, 1):  # aligned values and a view one element in
        full = dev(np.concatenate([np.zeros(shift, dtype=dt), v]))
        rg = api.Ragged(full[shift:], dev(off))
        got = host(api.segmented_reduce(abi.MX_ADD, rg, 0))
        R = O.segmented_reduce(O.ADD, 0, v, off)
        if dt == np.int32:
            assert np.array_equal(got, R), shift
        else:
            check_vector(got, R, O.segmented_reduce(O.ADD, 0.0, np.abs(v), off), L, what=f"shift {shift}")
    if dt == np.float32 and off[-1] > 0:
        g = rng.uniform(-1, 1, len(L)).astype(np.float32)
        gv = torch.full((int(off[-1]) + 1,), 5.0, device=DEV)
        abi.mx_segmented_sum_adjoint_f32(dev(g), dev(off), gv[1:])
        assert np.array_equal(host(gv[1:]), O.segmented_sum_adjoint(g, off).astype(np.float32))
        assert host(gv[:1])[0] == 5.0


def _chunk_case(case, dt):
    """Row lengths that stress the 16 KB chunks (S = 4096 four-byte or 2048
    eight-byte elements)."""
    S = 4096 if np.dtype(dt).itemsize == 4 else 2048
    rng = np.random.default_rng(hash(case) % 1000)
    if case == "tiny_rows":        # thousands of rows per chunk: several row batches each
        L = rng.integers(0, 4, 200000)
    elif case == "chunk_edges":    # rows ending and starting on chunk boundaries, empty rows there
        pat = [S, 0, 0, S - 1, 1, 0, S + 1, S - 1, 2 * S, 0, 1, S - 2, 1, 0, 3 * S, 0]
        L = np.array(pat * 7)
    elif case == "one_long_row":   # one row over ~1000-2000 chunks: the finish folds many head parts
        L = np.array([0, 3, (1 << 22) + 5, 0, 7, 0])
    else:                          # mixed: log-uniform up to 5 S, every seventh row empty
        L = np.floor(np.exp(rng.uniform(0, np.log(5 * S + 1), 3000))).astype(np.int64)
        L[::7] = 0
    return np.asarray(L, dtype=np.int64), S


@pytest.mark.parametrize("case", ["tiny_rows", "chunk_edges", "one_long_row", "mixed"])
@pytest.mark.parametrize("dt", [np.float32, np.float64, np.int32, np.int64])
def test_segmented_chunk_boundaries(case, dt):
    """Every row against the oracle for layouts around the chunk boundaries
    (integers bit-exact for every operator); a second call gives the same bits
    and the workspace is left zero-filled."""
    say("segmented chunks", case, np.dtype(dt).name)
    L, S = _chunk_case(case, dt)
    off = O.offsets_from_lengths(L)
    nv = int(off[-1])
    rng = np.random.default_rng(7)
    ops = [abi.MX_ADD]
    if np.issubdtype(dt, np.integer):
        v = rng.integers(-10 ** 6, 10 ** 6, nv).astype(dt)
        ops = [abi.MX_ADD, abi.MX_MIN, abi.MX_MAX, abi.MX_MUL]
    else:
        v = rng.uniform(-1, 1, nv).astype(dt)
    tv, toff = dev(v), dev(off)
    ws = torch.zeros(abi.mx_workspace_bytes(abi.MX_WS_SEGMENTED, nv), dtype=torch.uint8, device=DEV)
    for op in ops:
        ne = {abi.MX_ADD: 0, abi.MX_MUL: 1, abi.MX_MIN: 2 ** 63 - 1, abi.MX_MAX: -2 ** 63}[op]
        vin = v
        if op == abi.MX_MUL:  # small factors keep products in range of the exact check
            vin = rng.integers(-2, 3, nv).astype(dt)
            tv = dev(vin)
        out = torch.empty(len(L), dtype=api.ACC_OF[tv.dtype], device=DEV)
        abi.mx_segmented_reduce(op, tv, toff, ne if np.issubdtype(dt, np.integer) else 0.0, out, ws)
        got = host(out).copy()
        assert not np.any(host(ws)), "workspace left non-zero"
        out2 = torch.full_like(out, 3)
        abi.mx_segmented_reduce(op, tv, toff, ne if np.issubdtype(dt, np.integer) else 0.0, out2, ws)
        assert got.tobytes() == host(out2).tobytes(), "second call differs"
        if np.issubdtype(dt, np.integer):
            assert np.array_equal(got, O.segmented_reduce(op, ne, vin, off)), op
        else:
            check_vector(got, O.segmented_reduce(O.ADD, 0.0, vin, off),
                         O.segmented_reduce(O.ADD, 0.0, np.abs(vin), off), L, what=case)
    if dt == np.float32:
        g = rng.uniform(-1, 1, len(L)).astype(np.float32)
        gv = torch.full((nv + 1,), 5.0, device=DEV)
        abi.mx_segmented_sum_adjoint_f32(dev(g), toff, gv[1:])      # misaligned destination
        assert np.array_equal(host(gv[1:]), O.segmented_sum_adjoint(g, off).astype(np.float32))
        gv2 = torch.empty(nv, device=DEV)
        abi.mx_segmented_sum_adjoint_f32(dev(g), toff, gv2)         # aligned destination
        assert np.array_equal(host(gv2), O.segmented_sum_adjoint(g, off).astype(np.float32))


def _span_case(case):
    """Row layouts for the row-span path (enough rows, short on average)."""
    rng = np.random.default_rng(11)
    if case == "log_uniform_empty":   # log-uniform up to 3000, every 13th row empty
        L = W.ragged_lengths(20000, seed=4, lmax=3000)
        L[::13] = 0
    elif case == "few_giant_rows":    # mostly short rows, ten of 200 000 values
        L = rng.integers(0, 40, 12000)
        L[rng.choice(12000, 10, replace=False)] = 200000
    else:                             # runs of empty rows between blocks of long ones
        L = np.zeros(16384, dtype=np.int64)
        L[::3] = rng.integers(1000, 9000, len(L[::3]))
    return np.asarray(L, dtype=np.int64)


@pytest.mark.parametrize("case", ["log_uniform_empty", "few_giant_rows", "empty_runs"])
@pytest.mark.parametrize("dt", [np.float32, np.float64, np.int32, np.int64])
def test_segmented_row_span_path(case, dt):
    """The row-span kernels (many rows of ordinary mean length): every row
    against the oracle, integers bit-exact for every operator, aligned and
    misaligned value views, the broadcast into aligned and misaligned
    destinations."""
    say("segmented row-span", case, np.dtype(dt).name)
    L = _span_case(case)
    off = O.offsets_from_lengths(L)
    nv = int(off[-1])
    rng = np.random.default_rng(5)
    toff = dev(off)
    ws = torch.zeros(abi.mx_workspace_bytes(abi.MX_WS_SEGMENTED, nv), dtype=torch.uint8, device=DEV)
    integer = np.issubdtype(dt, np.integer)
    ops = [abi.MX_ADD, abi.MX_MIN, abi.MX_MAX, abi.MX_MUL] if integer else [abi.MX_ADD]
    for op in ops:
        if op == abi.MX_MUL:
            v = rng.integers(-2, 3, nv).astype(dt)
        elif integer:
            v = rng.integers(-10 ** 6, 10 ** 6, nv).astype(dt)
        else:
            v = rng.uniform(-1, 1, nv).astype(dt)
        ne = {abi.MX_ADD: 0, abi.MX_MUL: 1, abi.MX_MIN: 2 ** 63 - 1, abi.MX_MAX: -2 ** 63}[op]
        for shift in (0, 1):
            full = dev(np.concatenate([np.zeros(shift, dtype=dt), v]))
            out = torch.empty(len(L), dtype=api.ACC_OF[full.dtype], device=DEV)
            abi.mx_segmented_reduce(op, full[shift:], toff, ne if integer else 0.0, out, ws)
            got = host(out)
            if integer:
                assert np.array_equal(got, O.segmented_reduce(op, ne, v, off)), (op, shift)
            else:
                check_vector(got, O.segmented_reduce(O.ADD, 0.0, v, off),
                             O.segmented_reduce(O.ADD, 0.0, np.abs(v), off), L, what=f"{case} shift {shift}")
    if dt == np.float32:
        g = rng.uniform(-1, 1, len(L)).astype(np.float32)
        ref = O.segmented_sum_adjoint(g, off).astype(np.float32)
        gv = torch.full((nv + 1,), 5.0, device=DEV)
        abi.mx_segmented_sum_adjoint_f32(dev(g), toff, gv[1:])
        assert np.array_equal(host(gv[1:]), ref) and host(gv[:1])[0] == 5.0
        gv2 = torch.empty(nv, device=DEV)
        abi.mx_segmented_sum_adjoint_f32(dev(g), toff, gv2)
        assert np.array_equal(host(gv2), ref)


def test_segmented_all_rows_empty_and_single_chunk():
    """No values at all (every row gives ne), and one chunk or less (no
    workspace needed)."""
    say("segmented empty / single chunk")
    out = torch.full((5,), 9.0, device=DEV)
    abi.mx_segmented_reduce(abi.MX_MAX, torch.empty(0, device=DEV), dev(np.zeros(6, np.int64)), -3.5, out, None)
    assert np.array_equal(host(out), np.full(5, -3.5, np.float32))
    for L in ([4096], [1, 4094, 1], [0, 4096, 0], [5, 0, 7]):
        L = np.array(L, np.int64)
        off = O.offsets_from_lengths(L)
        v = np.random.default_rng(1).integers(-9, 10, int(off[-1])).astype(np.int32)
        out = torch.empty(len(L), dtype=torch.int64, device=DEV)
        abi.mx_segmented_reduce(abi.MX_ADD, dev(v), dev(off), 0, out, None)
        assert np.array_equal(host(out), O.segmented_reduce(O.ADD, 0, v, off)), L


def test_segmented_graph_replay():
    """The chunked reduce and broadcast captured in a HIP graph: every replay
    (with eager work between them) equals the eager result bit for bit."""
    say("segmented graph")
    L, v, off = _ragged(20000, 5, lmax=6000, empty_rows=50)
    tv, toff = dev(v), dev(off)
    ws = torch.zeros(abi.mx_workspace_bytes(abi.MX_WS_SEGMENTED, v.size), dtype=torch.uint8, device=DEV)
    out = torch.empty(len(L), device=DEV)
    g = dev(np.random.default_rng(2).uniform(-1, 1, len(L)).astype(np.float32))
    gv = torch.empty(v.size, device=DEV)
    abi.mx_segmented_reduce(abi.MX_ADD, tv, toff, 0.0, out, ws)
    abi.mx_segmented_sum_adjoint_f32(g, toff, gv)
    ref = (host(out).copy(), host(gv).copy())
    side = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(side):
        abi.mx_graph_begin(side)
        abi.mx_segmented_reduce(abi.MX_ADD, tv, toff, 0.0, out, ws, stream=side)
        abi.mx_segmented_sum_adjoint_f32(g, toff, gv, stream=side)
        graph = abi.mx_graph_end(side)
    for rep in range(3):
        out.fill_(float("nan"))
        gv.fill_(float("nan"))
        torch.cuda.synchronize()
        graph.launch(side)
        side.synchronize()
        assert host(out).tobytes() == ref[0].tobytes() and host(gv).tobytes() == ref[1].tobytes(), rep
        abi.mx_segmented_reduce(abi.MX_ADD, tv, toff, 0.0, out, ws)  # eager work between replays
        torch.cuda.synchronize()
    abi.mx_graph_destroy(graph)


def test_segmented_sum_adjoint_broadcast_exact():
    say("segmented adjoint")
    L, v, off = _ragged(4000, 3, lmax=2000, empty_rows=30)
    g = np.random.default_rng(0).uniform(-1, 1, len(L)).astype(np.float32)
    vals = dev(v).requires_grad_()
    out = api.segmented_sum(api.Ragged(vals, dev(off)))
    out.backward(dev(g))
    assert np.array_equal(host(vals.grad), O.segmented_sum_adjoint(g, off).astype(np.float32))


def test_debug_mode_rejects_bad_offsets():
    say("debug offsets")
    bad = dev(np.array([0, 5, 3, 9], dtype=np.int64))
    vals = dev(np.zeros(9, dtype=np.float32))
    out = torch.empty(3, device=DEV)
    abi.mx_set_debug(True)
    try:
        with pytest.raises(abi.MxError) as e:
            abi.mx_segmented_reduce(abi.MX_ADD, vals, bad, 0.0, out, None)
        assert e.value.status == abi.MX_ERR_SHAPE
        # offsets[nseg] must equal the number of values
        with pytest.raises(abi.MxError) as e:
            abi.mx_segmented_reduce(abi.MX_ADD, vals, dev(np.array([0, 3, 5, 8], dtype=np.int64)), 0.0, out, None)
        assert e.value.status == abi.MX_ERR_SHAPE and "number of values" in str(e.value)
        with pytest.raises(abi.MxError):
            abi.mx_segmented_sum_adjoint_f32(dev(np.zeros(3, np.float32)), dev(np.array([0, 3, 5, 8], np.int64)),
                                             torch.empty(9, device=DEV))
        with pytest.raises(abi.MxError):
            api.offsets_from_lengths(dev(np.array([3, -1, 2], dtype=np.int64)))
    finally:
        abi.mx_set_debug(False)
    # accelerate mode does not check: the call is accepted
    abi.mx_segmented_reduce(abi.MX_ADD, vals, dev(np.array([0, 3, 5, 9], dtype=np.int64)), 0.0, out, None)
    assert np.array_equal(host(out), np.zeros(3, dtype=np.float32))


@pytest.mark.parametrize("n", [1, 3, 4, 5, 4099, 4096 * 1024 + 7, 1 << 24,
                               16384 * 4096 + 5 * 4096 + 3])  # the last: blocks loop over chunks
def test_stream_read_xor(n):
    """The read-only ceiling kernel reads every word exactly once: its XOR
    against numpy's."""
    say("stream read", n)
    w = np.random.default_rng(n).integers(0, 2 ** 32, n, dtype=np.uint64).astype(np.uint32)
    x = torch.zeros(abi.MX_STREAM_READ_SLOTS, dtype=torch.int32, device=DEV)
    abi.mx_stream_read(dev(w.view(np.int32)), x)
    assert int(np.bitwise_xor.reduce(host(x).view(np.uint32))) == int(np.bitwise_xor.reduce(w))


# ------------------------------------------------------------------ dense map-map-reduce
def _abs_prod_sum(A, B):
    return O.matmul(np.abs(A), np.abs(B))


@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (128, 128, 32), (200, 130, 70), (257, 511, 33),
                                   (64, 300, 1000), (129, 127, 129), (3, 1025, 5),
                                   # K a multiple of 64: interior tiles take the pipelined loop
                                   (256, 192, 128), (300, 200, 64), (513, 257, 320)])
@pytest.mark.parametrize("ta,tb", [(0, 0), (0, 1), (1, 0), (1, 1)])
def test_mmr_shapes_vs_oracle(M, N, K, ta, tb):
    say("mmr", M, N, K, ta, tb)
    A, B = W.dense_f32(M, N, K, seed=M + N + K)
    As = A.T.copy() if ta else A
    Bs = B.T.copy() if tb else B
    C = torch.empty((M, N), device=DEV)
    abi.mx_map_map_reduce_f32(ta, tb, dev(As), dev(Bs), C)
    R = O.matmul(A, B)
    check_vector(host(C).ravel(), R.ravel(), _abs_prod_sum(A, B).ravel(), K, what="C")
    Cp = torch.empty((M, N), device=DEV)
    abi.mx_map_map_reduce_plain_f32(ta, tb, dev(As), dev(Bs), Cp)
    check_vector(host(Cp).ravel(), R.ravel(), _abs_prod_sum(A, B).ravel(), K, what="C plain")


def test_mmr_rank_one_exact():
    say("mmr rank one")
    M, N, K = 256, 384, 512
    u = (np.arange(M) % 7 - 3).astype(np.float32) * 0.25
    v = (np.arange(N) % 5 - 2).astype(np.float32) * 0.5
    A = np.outer(u, np.ones(K, dtype=np.float32))
    B = np.outer(np.ones(K, dtype=np.float32), v)
    C = api.matmul(dev(A), dev(B))
    assert np.array_equal(host(C), (K * np.outer(u, v)).astype(np.float32))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_mmr_config_2048_sampled(seed):
    """2048 x 2048 x 2048, uniform [-1, 1]: 512 sampled elements vs the oracle one by one."""
    say("mmr 2048 seed", seed)
    M = N = K = 2048
    A, B = W.dense_f32(M, N, K, seed)
    C = host(api.matmul(dev(A), dev(B)))
    rng = np.random.default_rng(seed)
    ii = rng.integers(0, M, 512)
    jj = rng.integers(0, N, 512)
    ii[:4] = [0, M - 1, 0, M - 1]
    jj[:4] = [0, 0, N - 1, N - 1]
    for i, j in zip(ii, jj):
        R = O.dot(A[i], B[:, j])
        S = O.dot(np.abs(A[i]), np.abs(B[:, j]))
        check_scalar(C[i, j], R, S, K, what=f"C[{i},{j}]")


TILES = ["128x64", "128x128", "128x64w8", "128x128w8", "64x64", "128x128w8b", "128x128w16"]


@pytest.mark.parametrize("tile", TILES)
@pytest.mark.parametrize("ta,tb", [(0, 0), (0, 1), (1, 0), (1, 1)])
def test_mmr_every_tile_vs_oracle(tile, ta, tb, monkeypatch):
    """Every tile configuration (forced through MX_GEMM_TILE, read per call) on
    shapes with edge tiles, ragged K and K a multiple of 64 (interior tiles on
    the pipelined loop): the whole C against the oracle."""
    monkeypatch.setenv("MX_GEMM_TILE", tile)
    # K = 512: sixteen slices through the pipelined loop
    for M, N, K in [(300, 200, 128), (257, 385, 100), (512, 256, 192), (384, 260, 512)]:
        say("mmr tile", tile, ta, tb, M, N, K)
        A, B = W.dense_f32(M, N, K, seed=M + K + 7 * ta + 3 * tb)
        As = A.T.copy() if ta else A
        Bs = B.T.copy() if tb else B
        C = torch.empty((M, N), device=DEV)
        abi.mx_map_map_reduce_f32(ta, tb, dev(As), dev(Bs), C)
        check_vector(host(C).ravel(), O.matmul(A, B).ravel(), _abs_prod_sum(A, B).ravel(), K,
                     what=f"C {tile} {ta}{tb}")


def _rows_cols_check(C, A, B, seed, what):
    """64 whole rows and 64 whole columns of C = A B against the oracle
    (including the first and last of each)."""
    M, K = A.shape
    N = B.shape[1]
    rng = np.random.default_rng(seed)
    rows = np.unique(np.concatenate([[0, M - 1], rng.choice(M, 62, replace=False)]))
    cols = np.unique(np.concatenate([[0, N - 1], rng.choice(N, 62, replace=False)]))
    Bt = B.T.copy()  # the oracle reads B^T row by row: same fold, contiguous access
    R = O.matmul(A[rows], Bt, tb=True)
    S = O.matmul(np.abs(A[rows]), np.abs(Bt), tb=True)
    check_vector(C[rows].ravel(), R.ravel(), S.ravel(), K, what=f"{what} rows")
    Bc = B[:, cols].copy()
    R = O.matmul(A, Bc)
    S = O.matmul(np.abs(A), np.abs(Bc))
    check_vector(C[:, cols].ravel(), R.ravel(), S.ravel(), K, what=f"{what} cols")


@pytest.mark.parametrize("ta,tb", [(0, 0), (0, 1), (1, 0), (1, 1)])
def test_mmr_config_2048_every_transpose_rows_and_cols(ta, tb):
    """2048^3 with the default tile choice (256 tiles of 128 x 128, 16 waves):
    64 whole rows and 64 whole columns."""
    say("mmr 2048 transposes", ta, tb)
    M = N = K = 2048
    A, B = W.dense_f32(M, N, K, seed=10 + 2 * ta + tb)
    As = A.T.copy() if ta else A
    Bs = B.T.copy() if tb else B
    C = torch.empty((M, N), device=DEV)
    abi.mx_map_map_reduce_f32(ta, tb, dev(As), dev(Bs), C)
    _rows_cols_check(host(C), A, B, seed=ta * 2 + tb, what=f"C {ta}{tb}")


def test_mmr_config_2048_backward_rows_and_cols():
    """The benchmark's products through autograd: C = A B, then dA = dC B^T
    and dB = A^T dC (128 x 128 tiles of 16 waves each), at 2048^3."""
    say("mmr 2048 backward")
    M = N = K = 2048
    A, B = W.dense_f32(M, N, K, seed=0)
    G = np.random.default_rng(42).uniform(-1, 1, (M, N)).astype(np.float32)
    tA, tB = dev(A).requires_grad_(), dev(B).requires_grad_()
    C = api.matmul(tA, tB)
    C.backward(dev(G))
    _rows_cols_check(host(C.detach()), A, B, seed=1, what="C")
    _rows_cols_check(host(tA.grad), G, B.T.copy(), seed=2, what="dA")
    _rows_cols_check(host(tB.grad), A.T.copy(), G, seed=3, what="dB")


def test_mmr_deterministic_and_gradients():
    say("mmr grad")
    M, N, K = 192, 160, 96
    A, B = W.dense_f32(M, N, K, seed=5)
    G = np.random.default_rng(1).uniform(-1, 1, (M, N)).astype(np.float32)
    tA, tB = dev(A).requires_grad_(), dev(B).requires_grad_()
    C = api.matmul(tA, tB)
    C2 = api.matmul(tA.detach(), tB.detach())
    assert host(C.detach()).tobytes() == host(C2).tobytes()
    C.backward(dev(G))
    gA_ref = O.matmul(G, B.T)
    gB_ref = O.matmul(A.T, G)
    check_vector(host(tA.grad).ravel(), gA_ref.ravel(), O.matmul(np.abs(G), np.abs(B.T)).ravel(), N)
    check_vector(host(tB.grad).ravel(), gB_ref.ravel(), O.matmul(np.abs(A.T), np.abs(G)).ravel(), M)
