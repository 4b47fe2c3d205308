"""The no-allocation entry point (mx_segmented_reduce_noalloc: the split-row
slots in the library's built-in per-device scratch array instead of a caller's
workspace) against the workspace entry point mx_segmented_reduce, through the C
ABI: two calls in a row with the second smaller, bit-identical results and the
oracle's parity bar (tolerance for float32, exact for integers); sizes past the
array's limit are rejected before any device work.
"""
import ctypes

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from parity import check_vector, say

import paper_2211_00621_amd as mx  # noqa: E402

pytestmark = pytest.mark.gpu
abi = mx.abi
DEV = "cuda"


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def test_noalloc_matches_workspace_entry_point_twice():
    abi.mx_init(0)
    # a ragged input with rows split across blocks (their parts go through the
    # array), then a smaller one (the second call reuses the array the first
    # left), then the full nested configuration (row-span schedule)
    for nseg, seed, lmax, empties in ((6000, 2, 30000, 10), (3000, 1, 9000, 40), (65536, 0, 4096, 0)):
        say("noalloc", nseg, seed)
        L, v = W.ragged_f32(nseg, seed, lmax, empty_rows=empties)
        off = O.offsets_from_lengths(L)
        tv, toff = dev(v), dev(off)
        ws = torch.zeros(abi.mx_workspace_bytes(abi.MX_WS_SEGMENTED, v.size), dtype=torch.uint8, device=DEV)
        ref = torch.empty(nseg, device=DEV)
        got = torch.full((nseg,), float("nan"), device=DEV)
        abi.mx_segmented_reduce(abi.MX_ADD, tv, toff, 0.0, ref, ws)
        abi.mx_segmented_reduce_noalloc(abi.MX_ADD, tv, toff, 0.0, got)
        g = host(got)
        assert g.tobytes() == host(ref).tobytes()
        check_vector(g, O.segmented_reduce(O.ADD, 0.0, v, off), O.segmented_reduce(O.ADD, 0.0, np.abs(v), off), L)
        # integers: exact against the oracle as well
        vi = np.random.default_rng(seed).integers(-10 ** 6, 10 ** 6, v.size).astype(np.int64)
        outi = torch.empty(nseg, dtype=torch.int64, device=DEV)
        abi.mx_segmented_reduce_noalloc(abi.MX_MAX, dev(vi), toff, -2 ** 63, outi)
        assert np.array_equal(host(outi), O.segmented_reduce(O.MAX, -2 ** 63, vi, off))


def test_noalloc_rejects_sizes_past_the_array():
    lib = abi._L()
    cap = abi.mx_segmented_noalloc_max_values()
    assert 50_000_000 < cap < 70_000_000
    assert abi.mx_workspace_bytes(abi.MX_WS_SEGMENTED, cap) <= 1 << 20 < abi.mx_workspace_bytes(abi.MX_WS_SEGMENTED,
                                                                                                  cap + 2048)
    fake = ctypes.c_void_p(4096)
    v = ctypes.c_float(0.0)
    st = lib.mx_segmented_reduce_noalloc(0, 0, fake, cap + 2048, fake, 4, ctypes.byref(v), fake, None)
    assert st == abi.MX_ERR_WORKSPACE and "built-in scratch" in lib.mx_last_error().decode()
