"""GPU parity of the nested marshaling surface against the oracle: nested
sequences of depth 1-4 (with empty sequences at every level) marshalled to
values + one offsets array per level, unmarshalled back, flattened at every
level, regular nestings turned into tensors (ragged ones rejected), and the
innermost rows reduced -- map (map (reduce (+))) -- all bit-exact."""
import numpy as np
import pytest
import torch

import oracle as O
from parity import say

import paper_2211_00621_amd as mx  # noqa: E402

pytestmark = pytest.mark.gpu
abi, api = mx.abi, mx.api


def random_nested(rng, depth, width=5, leaf=9, p_empty=0.2):
    if depth == 1:
        n = 0 if rng.random() < p_empty else int(rng.integers(1, leaf))
        return [float(np.float32(v)) for v in rng.uniform(-1, 1, n)]
    n = 0 if rng.random() < p_empty else int(rng.integers(1, width))
    return [random_nested(rng, depth - 1, width, leaf, p_empty) for _ in range(n)]


def as_lists(x):
    if isinstance(x, np.ndarray):
        return [float(v) for v in x]
    return [as_lists(c) for c in x]


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("depth", [1, 2, 3, 4])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_marshal_unmarshal_matches_oracle(depth, seed):
    say("nested marshal", depth, seed)
    rng = np.random.default_rng(seed)
    seq = [random_nested(rng, depth - 1) for _ in range(int(rng.integers(0, 12)))] if depth > 1 else \
        random_nested(rng, 1, leaf=40, p_empty=0.0)
    nd = api.marshal_nested(seq, depth)
    values, offs = O.marshal_nested(seq, depth)
    assert np.array_equal(host(nd.values), np.asarray(values, dtype=np.float32))
    assert len(nd.offsets) == len(offs)
    for got, ref in zip(nd.offsets, offs):
        assert np.array_equal(host(got), ref)
    back = api.unmarshal_nested(nd)
    assert as_lists(back) == seq if depth > 1 else [float(v) for v in back] == seq


@pytest.mark.parametrize("depth,level", [(2, 0), (3, 0), (3, 1), (4, 0), (4, 1), (4, 2)])
def test_flatten_every_level(depth, level):
    say("nested flatten", depth, level)
    rng = np.random.default_rng(depth * 10 + level)
    seq = [random_nested(rng, depth - 1) for _ in range(9)]
    nd = api.flatten(api.marshal_nested(seq, depth), level)

    def flat_at(s, lvl):  # the Python definition: concatenate the sequences of that level
        if lvl == 0:
            return [x for child in s for x in child]
        return [flat_at(child, lvl - 1) for child in s]

    ref_values, ref_offs = O.marshal_nested(flat_at(seq, level), depth - 1)
    assert np.array_equal(host(nd.values), np.asarray(ref_values, dtype=np.float32))
    for got, ref in zip(nd.offsets, ref_offs):
        assert np.array_equal(host(got), ref)
    if level == 0:
        v0, rest = O.flatten(*O.marshal_nested(seq, depth))
        for got, ref in zip(nd.offsets, rest):
            assert np.array_equal(host(got), ref)


@pytest.mark.parametrize("shape", [(7,), (5, 3), (4, 3, 2), (2, 3, 1, 4), (3, 0), (2, 1, 0)])
def test_regular_nesting_is_a_tensor(shape):
    say("nested tensor", shape)
    arr = np.random.default_rng(3).uniform(-1, 1, shape).astype(np.float32)
    nd = api.marshal_nested(arr.tolist(), len(shape))
    t = api.to_tensor(nd)
    assert tuple(t.shape) == shape and np.array_equal(host(t), arr)


def test_ragged_nesting_is_not_a_tensor():
    say("nested ragged")
    nd = api.marshal_nested([[1.0, 2.0], [3.0]], 2)
    with pytest.raises(abi.MxError) as e:
        api.to_tensor(nd)
    assert e.value.status == abi.MX_ERR_SHAPE
    bad = torch.tensor([0, 5, 3], dtype=torch.int64, device="cuda")
    with pytest.raises(abi.MxError) as e:
        abi.mx_offsets_regular(bad)
    assert e.value.status == abi.MX_ERR_SHAPE
    assert abi.mx_offsets_regular(torch.zeros(1, dtype=torch.int64, device="cuda")) == 0


def test_innermost_row_sums_of_a_depth3_nesting():
    """map (map (reduce (+) 0)) over a depth-3 nesting = row sums of the innermost offsets."""
    say("nested inner reduce")
    rng = np.random.default_rng(5)
    seq = [random_nested(rng, 2, width=6, leaf=50) for _ in range(40)]
    nd = api.marshal_nested(seq, 3)
    values, (o1, o2) = O.marshal_nested(seq, 3)
    sums = api.segmented_reduce(abi.MX_ADD, api.Ragged(nd.values, nd.offsets[1]), 0.0)
    ref = O.segmented_reduce(O.ADD, 0.0, np.asarray(values, np.float64), o2)
    S = O.segmented_reduce(O.ADD, 0.0, np.abs(np.asarray(values, np.float64)), o2)
    L = np.diff(o2)
    assert np.all(np.abs(host(sums) - ref) <= 1e-4 * np.maximum(np.abs(ref), S / np.sqrt(np.maximum(L, 1))))


# ---------------------------------------------------------------- integer nested values
def random_nested_int(rng, depth, width=5, leaf=9, p_empty=0.2, lo=-2 ** 31, hi=2 ** 31):
    if depth == 1:
        n = 0 if rng.random() < p_empty else int(rng.integers(1, leaf))
        return [int(v) for v in rng.integers(lo, hi, n)]
    n = 0 if rng.random() < p_empty else int(rng.integers(1, width))
    return [random_nested_int(rng, depth - 1, width, leaf, p_empty, lo, hi) for _ in range(n)]


def as_int_lists(x):
    if isinstance(x, np.ndarray):
        return [int(v) for v in x]
    return [as_int_lists(c) for c in x]


@pytest.mark.parametrize("dtype", [np.int32, np.int64])
@pytest.mark.parametrize("depth", [2, 3])
def test_marshal_integer_nested_values(dtype, depth):
    say("nested int marshal", dtype.__name__, depth)
    rng = np.random.default_rng(depth + 7)
    hi = 2 ** 31 if dtype == np.int32 else 2 ** 62
    seq = [random_nested_int(rng, depth - 1, lo=-hi, hi=hi) for _ in range(40)]
    nd = api.marshal_nested(seq, depth, dtype=dtype)
    values, offs = O.marshal_nested(seq, depth)
    assert nd.values.dtype == torch.from_numpy(np.zeros(0, dtype)).dtype
    assert np.array_equal(host(nd.values), np.asarray(values, dtype=dtype))
    for got, ref in zip(nd.offsets, offs):
        assert np.array_equal(host(got), ref)
    assert as_int_lists(api.unmarshal_nested(nd)) == seq
    # the innermost rows reduced on the device: integer sums, bit-exact
    inner = api.Ragged(nd.values, nd.offsets[-1])
    got = host(api.segmented_reduce(abi.MX_ADD, inner, 0))
    assert np.array_equal(got, O.segmented_reduce(O.ADD, 0, np.asarray(values, dtype=np.int64), offs[-1]))


# ---------------------------------------------------------------- records whose fields are sequences
SCHEMA = [("id", "scalar", np.int64), ("xs", "seq", np.float32), ("w", "scalar", np.float64),
          ("tags", "seq", np.int32), ("k", "scalar", np.int16), ("b", "seq", np.int8)]


def make_records(n, seed, p_empty=0.2):
    rng = np.random.default_rng(seed)
    recs = []
    for _ in range(n):
        def ln(m):
            return 0 if rng.random() < p_empty else int(rng.integers(1, m))
        recs.append({"id": int(rng.integers(-2 ** 62, 2 ** 62)),
                     "xs": rng.uniform(-1, 1, ln(300)).astype(np.float32).tolist(),
                     "w": float(rng.normal()), "tags": rng.integers(-2 ** 31, 2 ** 31, ln(20)).tolist(),
                     "k": int(rng.integers(-2 ** 15, 2 ** 15)), "b": rng.integers(-128, 128, ln(5)).tolist()})
    return recs


@pytest.mark.parametrize("n", [0, 1, 7, 5000])
def test_marshal_record_seqs_matches_oracle(n):
    say("records of sequences", n)
    recs = make_records(n, n + 1)
    rs = api.marshal_record_seqs(recs, SCHEMA)
    ref = O.marshal_record_seqs(recs, SCHEMA)
    for name, kind, dt in SCHEMA:
        if kind == "scalar":
            assert rs.fields[name].dtype == torch.from_numpy(np.zeros(0, dt)).dtype
            assert np.array_equal(host(rs.fields[name]), ref[name]), name
        else:
            vals, off = ref[name]
            assert np.array_equal(host(rs.fields[name].values), vals), name
            assert np.array_equal(host(rs.fields[name].offsets), off), name
    back = api.unmarshal_record_seqs(rs)
    assert len(back) == n
    for got, want in zip(back, recs):
        for name, kind, dt in SCHEMA:
            if kind == "scalar":
                assert got[name] == want[name], name
            else:
                assert np.array_equal(got[name], np.asarray(want[name], dtype=dt)), name


def test_record_seqs_feed_the_nested_reduce():
    """map (reduce) over every record's sequence field, on the marshalled layout."""
    say("records of sequences reduced")
    recs = make_records(3000, 11)
    rs = api.marshal_record_seqs(recs, SCHEMA)
    lay = O.marshal_record_seqs(recs, SCHEMA)
    vals, off = lay["tags"]
    got = host(api.segmented_reduce(abi.MX_ADD, rs.fields["tags"], 0))
    assert np.array_equal(got, O.segmented_reduce(O.ADD, 0, vals.astype(np.int64), off))
    got = host(api.segmented_reduce(abi.MX_MAX, rs.fields["xs"], -np.inf))
    assert np.array_equal(got, O.segmented_reduce(O.MAX, -np.inf, lay["xs"][0], lay["xs"][1]).astype(np.float32))


def test_unmarshal_record_seqs_rejects_a_length_mismatch():
    say("records length mismatch")
    recs = make_records(50, 3, p_empty=0.0)
    rs = api.marshal_record_seqs(recs, SCHEMA)
    rdt = api._record_dtype(SCHEMA)
    host_recs = np.zeros(50, dtype=rdt)
    bufs = []
    for name, kind, dt in SCHEMA:
        if kind == "seq":
            for i, r in enumerate(recs):
                a = np.empty(len(r[name]) + (1 if (name == "xs" and i == 17) else 0), dtype=dt)
                bufs.append(a)
                host_recs[name]["data"][i] = a.ctypes.data
                host_recs[name]["len"][i] = a.size
    tensors = {name: (rs.fields[name], None, None) if kind == "scalar" else
               (rs.fields[name].values, None, rs.fields[name].offsets) for name, kind, _ in SCHEMA}
    desc = api._field_desc(SCHEMA, rdt, tensors)
    _, nbytes = abi.mx_records_layout(host_recs, desc)
    staging = torch.empty(nbytes, dtype=torch.uint8, pin_memory=True)
    with pytest.raises(abi.MxError, match="length differs"):
        abi.mx_unmarshal_records(desc, host_recs, staging)
    assert all(host_recs["id"] == 0)     # nothing written
