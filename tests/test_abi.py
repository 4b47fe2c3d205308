"""The C ABI: the library loads, exports every entry point that include/mx.h
declares, the binding covers them all, and host-side argument checks reject bad
calls before anything reaches a device (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mx.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*(mx_[a-z0-9_]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    from paper_2211_00621_amd import _lib
    return _lib.load()


def test_header_declares_entry_points():
    names = declared_functions()
    assert "mx_map2_reduce" in names and "mx_segmented_reduce" in names
    assert len(names) >= 20


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_header(lib):
    from paper_2211_00621_amd import _lib, abi
    names = declared_functions()
    assert sorted(_lib.SIGNATURES) == names
    for n in names:
        assert callable(getattr(abi, n)), n


def test_exports_are_c_symbols_not_mangled():
    out = os.popen(f"nm -D --defined-only {os.path.join(ROOT, 'paper_2211_00621_amd', 'libmx.so')}").read()
    exported = set(re.findall(r" T (mx_[a-z0-9_]+)$", out, flags=re.M))
    assert set(declared_functions()) <= exported


def test_host_only_calls(lib):
    assert lib.mx_version().decode().startswith("mx ")
    assert lib.mx_workspace_bytes(0, 1 << 20, 0) % 256 == 0
    assert lib.mx_workspace_bytes(1, 65536, 0) >= 256 + 16 * 8
    assert lib.mx_set_debug(1) == 0 and lib.mx_get_debug() == 1
    assert lib.mx_set_debug(0) == 0 and lib.mx_get_debug() == 0


def test_argument_errors_before_any_device_work(lib):
    from paper_2211_00621_amd import abi
    v = ctypes.c_float(0.0)
    # negative sizes, unknown operators, missing workspace, float-only bodies
    assert lib.mx_map(0, 0, None, -1, None, None, None) == abi.MX_ERR_SHAPE
    assert lib.mx_map(99, 0, None, 4, None, None, None) == abi.MX_ERR_INVALID
    assert lib.mx_map(abi.MX_U_EXP, abi.MX_I64, None, 4, None, None, None) == abi.MX_ERR_DTYPE
    assert lib.mx_map2(abi.MX_B_DIV, abi.MX_I32, None, None, 4, None, None) == abi.MX_ERR_DTYPE
    assert lib.mx_map2(0, 7, None, None, 4, None, None) == abi.MX_ERR_DTYPE
    assert lib.mx_reduce(9, 0, None, 4, ctypes.byref(v), None, None, 0, None) == abi.MX_ERR_INVALID
    fake = ctypes.c_void_p(4096)
    assert lib.mx_reduce(0, 0, fake, 4, ctypes.byref(v), fake, fake, 16, None) == abi.MX_ERR_WORKSPACE
    assert lib.mx_segmented_reduce(0, 0, None, 0, None, -1, ctypes.byref(v), None, None, 0, None) == abi.MX_ERR_SHAPE
    assert lib.mx_segmented_reduce(0, 0, fake, -1, fake, 4, ctypes.byref(v), fake, None, 0, None) == abi.MX_ERR_SHAPE
    # more than one 16 KB chunk of values needs the workspace
    assert lib.mx_segmented_reduce(0, 0, fake, 4097, fake, 4, ctypes.byref(v), fake, None, 0,
                                   None) == abi.MX_ERR_WORKSPACE
    assert lib.mx_segmented_reduce(0, 0, fake, 4097, fake, 4, ctypes.byref(v), fake, fake, 64,
                                   None) == abi.MX_ERR_WORKSPACE
    assert lib.mx_map_map_reduce_f32(2, 0, 4, 4, 4, fake, fake, fake, None) == abi.MX_ERR_INVALID
    assert lib.mx_records_to_fields(fake, 4, 17, 4, None, None) == abi.MX_ERR_INVALID
    assert "mx_records_to_fields" in lib.mx_last_error().decode()


def test_segmented_workspace_sizes(lib):
    # one counter and two 16-byte slots per chunk of 2048 elements (the chunk
    # length of 8-byte types; 4-byte types use half as many chunks)
    from paper_2211_00621_amd import abi
    ws = lambda n: lib.mx_workspace_bytes(abi.MX_WS_SEGMENTED, n, 0)  # noqa: E731
    for n in (0, 1, 2048, 2049, 32101627):
        nch = -(-n // 2048)
        need = 256 + (-(-nch * 4 // 256)) * 256 + 2 * (-(-nch * 16 // 256)) * 256
        assert ws(n) == need, n
    assert ws(32101627) < 1 << 20


def test_nbody_workspace_sizes_at_zero_bodies(lib):
    # n = 0 is a valid size (nothing to do): the size queries answer it
    lib.mx_nbody_workspace_bytes.restype = ctypes.c_size_t
    lib.mx_nbody_pair_workspace_bytes.restype = ctypes.c_size_t
    assert lib.mx_nbody_pair_workspace_bytes(ctypes.c_int64(0)) == 256
    assert lib.mx_nbody_workspace_bytes(ctypes.c_int64(0), 20, 5) >= 256
    assert lib.mx_nbody_workspace_bytes(ctypes.c_int64(1), 20, 5) > lib.mx_nbody_workspace_bytes(ctypes.c_int64(0), 20, 5)


def test_histogram_workspace_sizes(lib):
    # the bucketed histogram needs a workspace only past the LDS histogram's
    # 32 768 bins and up to 2^27 bins; it grows with the keys (16 bits each)
    from paper_2211_00621_amd import abi
    ws = lambda n, nbins: lib.mx_workspace_bytes(abi.MX_WS_HISTOGRAM, n, nbins)  # noqa: E731
    assert ws(1 << 24, 4096) == 0 and ws(1 << 24, 32768) == 0
    assert ws(1 << 24, (1 << 27) + 1) == 0 and ws(1 << 24, 0) == 0
    big, small = ws(1 << 24, 1 << 20), ws(1 << 20, 1 << 20)
    assert big % 256 == 0 and small % 256 == 0
    assert big - small >= 2 * ((1 << 24) - (1 << 20))
    assert ws(100, 1 << 27) > 0 and ws(0, 1 << 20) > 0


def test_parboil_argument_errors_before_any_device_work(lib):
    # size, operand and workspace checks of the Parboil-shaped entry points
    # happen on the host, before any launch
    from paper_2211_00621_amd import abi
    fake = ctypes.c_void_p(4096)
    other = ctypes.c_void_p(8192)
    assert lib.mx_histogram_u32(fake, -1, 16, fake, None, 0, None) == abi.MX_ERR_SHAPE
    assert lib.mx_histogram_u32(fake, 16, 0, fake, None, 0, None) == abi.MX_ERR_SHAPE
    assert lib.mx_histogram_u32(fake, 16, 16, None, None, 0, None) == abi.MX_ERR_INVALID
    assert lib.mx_stencil7_f32(fake, fake, 8, 8, 8, ctypes.c_float(0.5), ctypes.c_float(0.1), None) == \
        abi.MX_ERR_INVALID
    assert lib.mx_stencil7_f32(fake, other, 0, 8, 8, ctypes.c_float(0.5), ctypes.c_float(0.1), None) == \
        abi.MX_ERR_SHAPE
    assert lib.mx_mriq_f32(fake, fake, fake, fake, -1, fake, fake, fake, 4, fake, fake, None) == abi.MX_ERR_SHAPE
    assert lib.mx_mriq_f32(fake, fake, fake, fake, 4, None, fake, fake, 4, fake, fake, None) == abi.MX_ERR_INVALID
    assert lib.mx_tpacf_f32(fake, fake, fake, 4, fake, fake, fake, 4, 0, fake, 33, fake, None) == \
        abi.MX_ERR_UNSUPPORTED
    assert lib.mx_tpacf_f32(fake, fake, fake, -1, fake, fake, fake, 4, 0, fake, 20, fake, None) == abi.MX_ERR_SHAPE
    assert lib.mx_tpacf_f32(fake, fake, fake, 4, fake, fake, fake, 4, 0, fake, 20, None, None) == abi.MX_ERR_INVALID
    assert "mx_tpacf_f32" in lib.mx_last_error().decode()


def test_records_layout_on_the_host():
    """mx_records_layout reads host records only: element counts and staging size."""
    import numpy as np
    from paper_2211_00621_amd import abi, api
    schema = [("id", "scalar", np.int64), ("xs", "seq", np.float32), ("k", "scalar", np.int16)]
    rdt = api._record_dtype(schema)
    recs = np.zeros(3, dtype=rdt)
    data = [np.zeros(m, np.float32) for m in (2, 0, 5)]
    for i, a in enumerate(data):
        recs["xs"]["data"][i] = a.ctypes.data if a.size else 0
        recs["xs"]["len"][i] = a.size
    desc = api._field_desc(schema, rdt)
    counts, nbytes = abi.mx_records_layout(recs, desc)
    assert counts.tolist() == [3, 7, 3]
    assert nbytes == 256 + 256 + 256 + 256   # id values, xs values, xs offsets, k values (each 256-aligned)
    recs["xs"]["len"][1] = -1
    with pytest.raises(abi.MxError):
        abi.mx_records_layout(recs, desc)
    recs["xs"]["len"][1] = 4                 # a positive length with null data
    with pytest.raises(abi.MxError):
        abi.mx_records_layout(recs, desc)
