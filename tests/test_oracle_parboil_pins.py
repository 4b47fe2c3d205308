"""Pins for the oracle's Parboil-shaped kernels (histogram, 7-point stencil,
mri-q): library routines on the same data (numpy.bincount, scipy.ndimage
convolution, a numpy matrix formulation of mri-q), closed forms on constant
and affine grids, and symmetry invariants."""
import numpy as np
import pytest
from scipy import ndimage

import oracle as O

RNG = np.random.default_rng(23)


@pytest.mark.parametrize("nbins", [1, 7, 4096])
def test_histogram_is_bincount(nbins):
    keys = RNG.integers(0, nbins + 5, 20000).astype(np.uint32)   # some keys past the last bin
    got = O.histogram(keys, nbins)
    ref = np.bincount(keys[keys < nbins], minlength=nbins)
    assert np.array_equal(got, ref)
    assert got.sum() == int((keys < nbins).sum())
    assert np.array_equal(O.histogram(keys[:0], nbins), np.zeros(nbins, np.int64))


def test_stencil_constant_and_affine_grids_and_boundary():
    c0, c1 = 0.5, 0.25
    g = np.full((5, 6, 7), 3.0)
    out = O.stencil7(g, c0, c1)
    assert np.all(out[1:-1, 1:-1, 1:-1] == (6 * c1 - c0) * 3.0)
    z, y, x = np.meshgrid(np.arange(5.0), np.arange(6.0), np.arange(7.0), indexing="ij")
    f = 2 * x - 3 * y + 5 * z + 1
    out = O.stencil7(f, c0, c1)
    assert np.array_equal(out[1:-1, 1:-1, 1:-1], ((6 * c1 - c0) * f)[1:-1, 1:-1, 1:-1])
    for sl in (np.s_[0], np.s_[-1], np.s_[:, 0], np.s_[:, -1], np.s_[:, :, 0], np.s_[:, :, -1]):
        assert np.array_equal(out[sl], f[sl])


def test_stencil_is_a_convolution():
    g = RNG.uniform(-1, 1, (6, 9, 11))
    c0, c1 = 0.7, 0.15
    kern = np.zeros((3, 3, 3))
    kern[1, 1, 1] = -c0
    for d in ((0, 1, 1), (2, 1, 1), (1, 0, 1), (1, 2, 1), (1, 1, 0), (1, 1, 2)):
        kern[d] = c1
    ref = ndimage.convolve(g, kern, mode="constant")
    out = O.stencil7(g, c0, c1)
    assert np.allclose(out[1:-1, 1:-1, 1:-1], ref[1:-1, 1:-1, 1:-1], rtol=1e-14, atol=1e-14)


def test_mriq_matches_matrix_form_and_symmetries():
    nk, nx = 64, 50
    kx, ky, kz = (RNG.uniform(-0.5, 0.5, nk) for _ in range(3))
    phi = RNG.uniform(0, 1, nk)
    x, y, z = (RNG.uniform(-1, 1, nx) for _ in range(3))
    qr, qi = O.mriq(kx, ky, kz, phi, x, y, z)
    arg = 2 * np.pi * (np.outer(x, kx) + np.outer(y, ky) + np.outer(z, kz))
    assert np.allclose(qr, np.cos(arg) @ phi, rtol=1e-12, atol=1e-12)
    assert np.allclose(qi, np.sin(arg) @ phi, rtol=1e-12, atol=1e-12)
    qr2, qi2 = O.mriq(kx, ky, kz, phi, -x, -y, -z)
    assert np.allclose(qr2, qr, rtol=1e-12, atol=1e-12) and np.allclose(qi2, -qi, rtol=1e-12, atol=1e-12)
    qr0, qi0 = O.mriq(np.zeros(nk), np.zeros(nk), np.zeros(nk), phi, x, y, z)
    assert np.allclose(qr0, phi.sum(), rtol=1e-14) and np.all(qi0 == 0)



def _sphere(n, seed):
    r = np.random.default_rng(seed)
    v = r.normal(size=(3, n))
    return (v / np.linalg.norm(v, axis=0)).astype(np.float32)


def test_tpacf_is_binary32_dot_and_searchsorted():
    p1, p2 = _sphere(120, 1), _sphere(90, 2)
    edges = np.cos(np.radians(np.logspace(-1, 2, 12))).astype(np.float32)   # decreasing cosines
    d = (p1[0][:, None] * p2[0][None, :]).astype(np.float32)                # numpy float32: each op rounded
    d = (d + (p1[1][:, None] * p2[1][None, :]).astype(np.float32)).astype(np.float32)
    d = (d + (p1[2][:, None] * p2[2][None, :]).astype(np.float32)).astype(np.float32)
    bins = np.searchsorted(-edges, -d.ravel(), side="left")    # #{b : -e_b < -d} = #{b : d < e_b}
    ref = np.bincount(bins, minlength=edges.size + 1)
    assert np.array_equal(O.tpacf(p1, p2, edges, False), ref)
    got_self = O.tpacf(p1, None, edges, True)
    assert got_self.sum() == 120 * 119 // 2
    full = O.tpacf(p1, p1, edges, False)                       # all ordered pairs incl. i == j
    diag = O.tpacf(p1[:, :1], p1[:, :1], edges, False)         # a single self pair lands in bin 0 or 1
    assert full.sum() == 120 * 120 and diag.sum() == 1


def test_tpacf_pair_on_an_edge_is_not_below_it():
    # edges equal to binary32 dot products of actual pairs: d < e_b is strict,
    # so such a pair counts in the bin after the edge, not before it
    p1, p2 = _sphere(40, 5), _sphere(30, 6)
    d = (p1[0][:, None] * p2[0][None, :]).astype(np.float32)
    d = (d + (p1[1][:, None] * p2[1][None, :]).astype(np.float32)).astype(np.float32)
    d = (d + (p1[2][:, None] * p2[2][None, :]).astype(np.float32)).astype(np.float32)
    edges = np.unique(d.ravel())[::-1][::97][:12].astype(np.float32)   # decreasing, every one a pair's d
    strict = np.bincount(np.searchsorted(-edges, -d.ravel(), side="left"), minlength=edges.size + 1)
    loose = np.bincount(np.searchsorted(-edges, -d.ravel(), side="right"), minlength=edges.size + 1)
    got = O.tpacf(p1, p2, edges, False)
    assert np.array_equal(got, strict) and not np.array_equal(got, loose)
    # edges one ulp above pairs' dot products: those pairs are below them, so
    # a dot product rounded differently (a fused multiply-add, another order)
    # moves a pair across an edge in one of the two cases
    for e in (np.unique(d.ravel())[::-1][::37][:32],
              np.unique(np.nextafter(d.ravel(), np.float32(np.inf)))[::-1][::37][:32]):
        e = e.astype(np.float32)
        ref = np.bincount(np.searchsorted(-e, -d.ravel(), side="left"), minlength=e.size + 1)
        assert np.array_equal(O.tpacf(p1, p2, e, False), ref)

