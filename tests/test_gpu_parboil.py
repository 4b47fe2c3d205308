"""GPU parity of the Parboil-shaped kernels against the oracle: histogram
counts bit-exact (LDS, bucketed and global paths, skewed and uniform keys,
keys past the last bin, one repeated key, misaligned and empty inputs, 2^24
keys, up to 2^27 bins); one 7-point stencil sweep
within a bound derived from its six additions and three roundings; mri-q
within a bound from the rounding of t, the sin / cos error (4 units of 2^-24
per sample, checked on its own) and the FP32 sums.  Inputs are seeded synthetic stand-ins for the Parboil datasets."""
import numpy as np
import pytest
import torch

import oracle as O
from parity import say

import paper_2211_00621_amd as mx  # noqa: E402

pytestmark = pytest.mark.gpu
abi, api = mx.abi, mx.api
DEV = "cuda"
U32 = 2.0 ** -24


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def keys_for(kind, n, nbins, seed):
    rng = np.random.default_rng(seed)
    if kind == "uniform":
        k = rng.integers(0, nbins + max(1, nbins // 50), n)        # about 2 % past the last bin
    else:                                                           # image-like: concentrated
        k = np.clip(np.rint(rng.normal(nbins * 0.4, max(1.0, nbins / 20), n)), 0, 2 ** 32 - 1)
    return k.astype(np.uint32)


def hist_ws(n, nbins):
    nbytes = abi.mx_workspace_bytes(abi.MX_WS_HISTOGRAM, n, nbins)
    return torch.zeros(max(nbytes, 256), dtype=torch.uint8, device=DEV) if nbytes else None


@pytest.mark.parametrize("nbins", [1, 7, 4096, 32768, 32769, 1 << 20])
@pytest.mark.parametrize("kind", ["uniform", "skewed"])
@pytest.mark.parametrize("n", [0, 3, 100001])
@pytest.mark.parametrize("with_ws", [False, True])
def test_histogram(nbins, kind, n, with_ws):
    say("histogram", nbins, kind, n, with_ws)
    keys = keys_for(kind, n, nbins, nbins + n)
    counts = torch.full((nbins,), 7, dtype=torch.int32, device=DEV)   # overwritten, not added to
    abi.mx_histogram_u32(dev(keys).view(torch.int32), nbins, counts, hist_ws(n, nbins) if with_ws else None)
    assert np.array_equal(host(counts).astype(np.int64), O.histogram(keys, nbins))


@pytest.mark.parametrize("nbins", [256, 1 << 20])
@pytest.mark.parametrize("with_ws", [False, True])
def test_histogram_misaligned_and_large(nbins, with_ws):
    say("histogram large", nbins, with_ws)
    n = (1 << 24) + 3
    keys = keys_for("skewed", n + 1, nbins, 5)
    counts = torch.empty(nbins, dtype=torch.int32, device=DEV)
    abi.mx_histogram_u32(dev(keys).view(torch.int32)[1:], nbins, counts, hist_ws(n, nbins) if with_ws else None)
    assert np.array_equal(host(counts).astype(np.int64), O.histogram(keys[1:], nbins))


@pytest.mark.parametrize("nbins", [32769, 65543, 3_000_001, 1 << 24, 1 << 27])
@pytest.mark.parametrize("kind", ["uniform", "skewed", "one_key", "past_end"])
def test_histogram_bucketed(nbins, kind):
    # bucket widths 2^11 .. 2^15 and up to 4096 buckets; one key repeated
    # (every key in one bucket and one bin); keys mostly past the last bin
    n = 300_007
    say("histogram bucketed", nbins, kind, n)
    if kind == "one_key":
        keys = np.full(n, nbins - 1, np.uint32)
    elif kind == "past_end":
        keys = np.random.default_rng(3).integers(nbins - 50, nbins + 50, n).astype(np.uint32)
    else:
        keys = keys_for(kind, n, nbins, 11)
    ws = hist_ws(n, nbins)
    assert ws is not None
    counts = torch.full((nbins,), 7, dtype=torch.int32, device=DEV)
    abi.mx_histogram_u32(dev(keys).view(torch.int32), nbins, counts, ws)
    got = host(counts).astype(np.int64)
    ref = O.histogram(keys, nbins)
    assert np.array_equal(got, ref)


def test_histogram_bucketed_reuses_workspace():
    # the same workspace for a large call then a smaller one: its scan
    # counters are back at zero after each call
    nbins = 1 << 20
    ws = hist_ws(1 << 22, nbins)
    for n, seed in ((1 << 22, 1), (70_001, 2), (1 << 22, 3)):
        keys = keys_for("skewed", n, nbins, seed)
        counts = torch.empty(nbins, dtype=torch.int32, device=DEV)
        abi.mx_histogram_u32(dev(keys).view(torch.int32), nbins, counts, ws)
        assert np.array_equal(host(counts).astype(np.int64), O.histogram(keys, nbins)), n


def test_histogram_bucketed_graph_replay():
    # the four bucketed passes captured in one HIP graph: every replay, with
    # eager work between them, gives the eager counts (the scan's counters
    # and status words are back at zero after each call, no memset nodes)
    nbins, n = 1 << 20, 1 << 21
    say("histogram graph", nbins, n)
    keys_np = keys_for("skewed", n, nbins, 21)
    keys = dev(keys_np).view(torch.int32)
    ws = hist_ws(n, nbins)
    counts = torch.empty(nbins, dtype=torch.int32, device=DEV)
    abi.mx_histogram_u32(keys, nbins, counts, ws)
    eager = host(counts).copy()
    assert np.array_equal(eager.astype(np.int64), O.histogram(keys_np, nbins))
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        abi.mx_graph_begin(s)
        abi.mx_histogram_u32(keys, nbins, counts, ws, stream=s)
        g = abi.mx_graph_end(s)
    other = torch.empty(nbins, dtype=torch.int32, device=DEV)
    for rep in range(3):
        counts.fill_(-1)
        abi.mx_histogram_u32(keys[: n // 2], nbins, other, ws)   # eager use of the same workspace
        torch.cuda.synchronize()
        abi.mx_graph_launch(g, s)
        s.synchronize()
        assert np.array_equal(host(counts), eager), rep
    abi.mx_graph_destroy(g)


def test_histogram_rejects_small_workspace():
    nbins, n = 1 << 20, 4096
    ws = torch.zeros(abi.mx_workspace_bytes(abi.MX_WS_HISTOGRAM, n, nbins) - 256, dtype=torch.uint8, device=DEV)
    keys = dev(np.zeros(n, np.uint32)).view(torch.int32)
    with pytest.raises(abi.MxError) as err:
        abi.mx_histogram_u32(keys, nbins, torch.empty(nbins, dtype=torch.int32, device=DEV), ws)
    assert err.value.status == abi.MX_ERR_WORKSPACE


def stencil_bound(g, c0, c1):
    """8 u (|c1| sum|neighbours| + |c0| |centre|) at interior points."""
    return 8 * U32 * O.stencil7(np.abs(g.astype(np.float64)), -abs(c0), abs(c1))


@pytest.mark.parametrize("shape", [(3, 3, 3), (7, 9, 11), (40, 64, 64), (17, 1, 5), (64, 512, 512)])
def test_stencil(shape):
    say("stencil", shape)
    rng = np.random.default_rng(sum(shape))
    g = rng.uniform(-1, 1, shape).astype(np.float32)
    c0, c1 = np.float32(1.0 / 6.0), np.float32(0.125)
    out = torch.full(shape, np.nan, device=DEV)
    abi.mx_stencil7_f32(dev(g), out, float(c0), float(c1))
    got = host(out).astype(np.float64)
    ref = O.stencil7(g, float(c0), float(c1))
    interior = np.zeros(shape, bool)
    if min(shape) >= 3:
        interior[1:-1, 1:-1, 1:-1] = True
    assert np.array_equal(got[~interior], g.astype(np.float64)[~interior])
    bound = stencil_bound(g, float(c0), float(c1))
    assert np.all(np.abs(got - ref)[interior] <= bound[interior])


def mriq_inputs(nk, nv, seed):
    rng = np.random.default_rng(seed)
    k = [rng.uniform(-16, 16, nk).astype(np.float32) for _ in range(3)]
    phi = rng.uniform(0, 1, nk).astype(np.float32)
    x = [rng.uniform(-0.5, 0.5, nv).astype(np.float32) for _ in range(3)]
    return k, phi, x


def mriq_bound(k, phi, x, idx):
    """sum_k phi_k (2 pi 3u T_ik + 4u) + nk u sum_k phi_k, T_ik = sum |k_c x_c|."""
    T = sum(np.abs(np.outer(xc[idx].astype(np.float64), kc.astype(np.float64))) for kc, xc in zip(k, x))
    phi64 = phi.astype(np.float64)
    return (2 * np.pi * 3 * U32 * T + 4 * U32) @ phi64 + len(phi) * U32 * phi64.sum()


@pytest.mark.parametrize("nk,nv", [(1, 1), (100, 513), (2048, 4096), (3000, 1000)])
def test_mriq(nk, nv):
    say("mriq", nk, nv)
    k, phi, x = mriq_inputs(nk, nv, nk + nv)
    qr, qi = torch.empty(nv, device=DEV), torch.empty(nv, device=DEV)
    abi.mx_mriq_f32(*[dev(a) for a in k], dev(phi), *[dev(a) for a in x], qr, qi)
    rr, ri = O.mriq(*k, phi, *x)
    b = mriq_bound(k, phi, x, np.arange(nv))
    assert np.all(np.abs(host(qr) - rr) <= b) and np.all(np.abs(host(qi) - ri) <= b)


def test_mriq_trig_error_per_sample():
    # one sample k = (1, 0, 0), phi = 1: t = x exactly, so Qr, Qi are the
    # kernel's cos(2 pi x), sin(2 pi x) alone; each within the 4 units of
    # 2^-24 per sample that mriq_bound allows, over |x| <= 24 and near the
    # multiples of 1/4 where one of them passes through zero
    rng = np.random.default_rng(9)
    near = (np.arange(-96, 97) / 4.0)[:, None] + rng.uniform(-1e-3, 1e-3, (193, 256))
    xs = np.concatenate([rng.uniform(-24, 24, 1 << 20), near.ravel()]).astype(np.float32)
    nv = xs.size
    say("mriq trig", nv)
    one, zero = np.ones(1, np.float32), np.zeros(1, np.float32)
    zv = np.zeros(nv, np.float32)
    qr, qi = torch.empty(nv, device=DEV), torch.empty(nv, device=DEV)
    abi.mx_mriq_f32(dev(one), dev(zero), dev(zero), dev(one), dev(xs), dev(zv), dev(zv), qr, qi)
    ang = 2 * np.pi * xs.astype(np.float64)
    assert np.max(np.abs(host(qr) - np.cos(ang))) <= 4 * U32
    assert np.max(np.abs(host(qi) - np.sin(ang))) <= 4 * U32


def test_mriq_full_size_sampled():
    nk, nv = 2048, 1 << 18
    say("mriq full size", nk, nv)
    k, phi, x = mriq_inputs(nk, nv, 0)
    qr, qi = torch.empty(nv, device=DEV), torch.empty(nv, device=DEV)
    abi.mx_mriq_f32(*[dev(a) for a in k], dev(phi), *[dev(a) for a in x], qr, qi)
    idx = np.concatenate([np.arange(256), np.random.default_rng(1).integers(0, nv, 512), np.arange(nv - 256, nv)])
    rr, ri = O.mriq(*k, phi, *[xc[idx] for xc in x])
    b = mriq_bound(k, phi, x, idx)
    assert np.all(np.abs(host(qr)[idx] - rr) <= b) and np.all(np.abs(host(qi)[idx] - ri) <= b)


# ---------------------------------------------------------------- tpacf
def sphere(n, seed):
    v = np.random.default_rng(seed).normal(size=(3, n))
    return (v / np.linalg.norm(v, axis=0)).astype(np.float32)


def edges_of(m):
    return np.cos(np.radians(np.logspace(-1, 2.2, m))).astype(np.float32) if m else np.zeros(0, np.float32)


@pytest.mark.parametrize("n1,n2", [(1, 1), (300, 700), (4096, 4096), (1000, 0), (5000, 257)])
@pytest.mark.parametrize("self_pairs", [False, True])
@pytest.mark.parametrize("m", [0, 1, 20, 32])
def test_tpacf_counts_bit_exact(n1, n2, self_pairs, m):
    say("tpacf", n1, n2, self_pairs, m)
    p1, p2 = sphere(n1, n1 + 7), sphere(n2, n2 + 11)
    e = edges_of(m)
    counts = torch.full((m + 1,), -1, dtype=torch.int64, device=DEV)
    abi.mx_tpacf_f32(dev(p1), dev(p2), dev(e) if m else torch.empty(0, device=DEV), counts, self_pairs)
    ref = O.tpacf(p1, p2, e, self_pairs)
    assert np.array_equal(host(counts), ref)
    assert ref.sum() == (n1 * (n1 - 1) // 2 if self_pairs else n1 * n2)


@pytest.mark.parametrize("n1,n2", [(300, 701), (4096, 4093)])
@pytest.mark.parametrize("self_pairs", [False, True])
@pytest.mark.parametrize("m", [3, 5, 9, 13, 17, 24, 27])
def test_tpacf_every_edge_count_class(n1, n2, self_pairs, m):
    say("tpacf edge class", n1, n2, self_pairs, m)
    p1, p2 = sphere(n1, n1 + 3), sphere(n2, n2 + 5)
    e = edges_of(m)
    counts = torch.full((m + 1,), -1, dtype=torch.int64, device=DEV)
    abi.mx_tpacf_f32(dev(p1), dev(p2), dev(e), counts, self_pairs)
    assert np.array_equal(host(counts), O.tpacf(p1, p2, e, self_pairs))


@pytest.mark.parametrize("self_pairs", [False, True])
def test_tpacf_edges_equal_to_pair_dots(self_pairs):
    # edges taken from binary32 dot products of actual pairs: those pairs sit
    # exactly on an edge, which does not count them below it
    n1, n2 = 2000, 1500
    say("tpacf ties", n1, n2, self_pairs)
    p1, p2 = sphere(n1, 41), sphere(n2, 43)
    q = p1 if self_pairs else p2
    rng = np.random.default_rng(5)
    i, j = rng.integers(0, n1, 64), rng.integers(0, q.shape[1], 64)
    d = (p1[0, i] * q[0, j] + p1[1, i] * q[1, j]) + p1[2, i] * q[2, j]
    assert d.dtype == np.float32
    u = np.unique(d)[::-1]  # decreasing edges
    e = u[:: max(1, len(u) // 24)][:24].astype(np.float32)
    counts = torch.full((len(e) + 1,), -1, dtype=torch.int64, device=DEV)
    abi.mx_tpacf_f32(dev(p1), dev(p2), dev(e), counts, self_pairs)
    assert np.array_equal(host(counts), O.tpacf(p1, p2, e, self_pairs))


def test_tpacf_full_size():
    # the bench's launch: 2^15 + 2^15 points, 20 edges.  The full counts hold
    # n (n - 1) / 2 and n^2 pairs; the cross counts of the first 2048 data
    # points against all 2^15 random points (the same two-dimensional grid
    # over set 2) match the oracle bit for bit
    n, m = 1 << 15, 20
    say("tpacf full size", n, m)
    d, r = sphere(n, 101), sphere(n, 102)
    e = edges_of(m)
    dd = torch.empty(m + 1, dtype=torch.int64, device=DEV)
    dr = torch.empty(m + 1, dtype=torch.int64, device=DEV)
    abi.mx_tpacf_f32(dev(d), dev(d), dev(e), dd, True)
    abi.mx_tpacf_f32(dev(d), dev(r), dev(e), dr, False)
    assert host(dd).sum() == n * (n - 1) // 2 and host(dr).sum() == n * n
    assert np.all(host(dd) >= 0) and np.all(host(dr) >= 0)
    part = torch.empty(m + 1, dtype=torch.int64, device=DEV)
    abi.mx_tpacf_f32(dev(d[:, :2048]), dev(r), dev(e), part, False)
    assert np.array_equal(host(part), O.tpacf(d[:, :2048], r, e, False))


def test_tpacf_rejects_too_many_edges():
    p = dev(sphere(4, 0))
    with pytest.raises(abi.MxError) as err:
        abi.mx_tpacf_f32(p, p, dev(edges_of(33)), torch.empty(34, dtype=torch.int64, device=DEV))
    assert err.value.status == abi.MX_ERR_UNSUPPORTED
