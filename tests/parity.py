"""Parity criteria shared by the GPU tests (FP32 kernel results vs the binary64 oracle).

Integers, indices and labels must be bit-exact.  A floating-point reduction is
one correct bracketing of the fold, so it is compared with a tolerance:

  scalar:  |r - R| <= rtol * max(|R|, S / sqrt(m))

where R is the oracle's binary64 fold, S the binary64 sum of the absolute
values of the m folded terms and rtol = 1e-4.  The S / sqrt(m) floor is the
size of the result a fold of m random-sign terms has, so a sum that cancels to
nearly zero is not held to a relative bound it cannot meet.  Vector outputs
must satisfy the scalar rule elementwise and ||r - R||_2 <= rtol ||R||_2.
"""
import sys

import numpy as np

RTOL = 1e-4


def say(*args):
    """Print a case name before GPU work, flushed (a failing box may keep only stdout)."""
    print(*args, flush=True)
    sys.stdout.flush()


def check_scalar(got, R, S, m, rtol=RTOL, what=""):
    floor = S / np.sqrt(max(m, 1))
    bound = rtol * max(abs(R), floor)
    err = abs(float(got) - float(R))
    assert err <= bound, f"{what}: |{got} - {R}| = {err} > {bound} (S={S}, m={m})"


def check_vector(got, R, S, m, rtol=RTOL, what=""):
    got = np.asarray(got, dtype=np.float64)
    R = np.asarray(R, dtype=np.float64)
    S = np.broadcast_to(np.asarray(S, dtype=np.float64), R.shape)
    m = np.broadcast_to(np.asarray(m, dtype=np.float64), R.shape)
    floor = S / np.sqrt(np.maximum(m, 1))
    bound = rtol * np.maximum(np.abs(R), floor)
    err = np.abs(got - R)
    bad = np.nonzero(err > bound)[0] if err.ndim == 1 else np.argwhere(err > bound)
    assert len(bad) == 0, f"{what}: {len(bad)} elements out of tolerance, first {bad[:5]}, " \
                          f"err {err.ravel()[:1]}"
    nR = np.linalg.norm(R)
    if nR > 0:
        assert np.linalg.norm(got - R) <= rtol * nR, f"{what}: normwise error too large"


def ulp_diff_f32(a, b):
    """Distance in units of the last place between float32 arrays."""
    ai = np.asarray(a, dtype=np.float32).view(np.int32).astype(np.int64)
    bi = np.asarray(b, dtype=np.float32).view(np.int32).astype(np.int64)
    ai = np.where(ai < 0, -(ai & 0x7FFFFFFF), ai)
    bi = np.where(bi < 0, -(bi & 0x7FFFFFFF), bi)
    return np.abs(ai - bi)
