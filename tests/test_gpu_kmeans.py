"""GPU parity of the k-means step (map (argmin-reduce) + reduce-by-key) and of
the within-cluster SSE and its gradient, against the oracle.

Lockstep protocol: every iteration starts the GPU and the oracle from the same
float32 centroids (the GPU's previous output); labels and counts must be
bit-exact, new centroids within the reduction tolerance.
"""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from parity import check_vector, say

import paper_2211_00621_amd as mx  # noqa: E402

pytestmark = pytest.mark.gpu
abi, api = mx.abi, mx.api
DEV = "cuda"


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def check_centroids(C_gpu, X, labels, counts, C_ref, C_in):
    """|C' - R| <= 1e-4 max(|R|, S / sqrt(m)) with S the mean |x| of the cluster."""
    k, d = C_ref.shape
    absmean = np.zeros((k, d))
    np.add.at(absmean, labels, np.abs(X.astype(np.float64)))
    m = np.maximum(counts, 1)[:, None]
    absmean = absmean / m
    empty = counts == 0
    assert np.array_equal(C_gpu[empty], C_in[empty].astype(np.float32))
    check_vector(C_gpu[~empty].ravel(), C_ref[~empty].ravel(), (absmean * np.sqrt(m))[~empty].ravel(),
                 np.broadcast_to(m, (k, d))[~empty].ravel(), what="centroids")


def lockstep(X, C0, iters, plain=False):
    Xt = dev(X)
    C = C0.astype(np.float32)
    for it in range(iters):
        say("  iteration", it)
        lab, cnt, Cn = api.kmeans_step(Xt, dev(C), plain=plain)
        lab, cnt, Cn = host(lab), host(cnt), host(Cn)
        ref_lab = O.kmeans_assign(X, C)
        assert np.array_equal(lab, ref_lab), f"labels differ at iteration {it}: {(lab != ref_lab).sum()}"
        ref_cnt, _, ref_C = O.kmeans_update(X, ref_lab, C)
        assert np.array_equal(cnt, ref_cnt)
        check_centroids(Cn, X, lab, cnt, ref_C, C)
        C = Cn
    return C


def test_kmeans_config_lockstep():
    """2^20 points in d = 32 from 64 Gaussian blobs, k = 64: two lockstep iterations."""
    say("kmeans config")
    X, _, _ = W.kmeans_blobs(1 << 20, 32, 64, seed=0)
    lockstep(X, X[:64], 2)


@pytest.mark.parametrize("plain", [False, True])
def test_kmeans_ten_iterations_lockstep(plain):
    say("kmeans 10 iterations plain", plain)
    X, _, _ = W.kmeans_blobs(1 << 16, 32, 64, seed=1)
    lockstep(X, X[:64], 10, plain=plain)


@pytest.mark.parametrize("n,d,k", [(1, 32, 64), (1000, 32, 64), (4097, 5, 3), (3001, 64, 32), (2500, 16, 100),
                                   (5000, 8, 192), (777, 1, 1),
                                   (2000, 17, 240), (1500, 64, 64), (3000, 16, 256)])
def test_kmeans_shapes(n, d, k):
    say("kmeans shape", n, d, k)
    X, _, _ = W.kmeans_blobs(n, d, max(k // 2, 1), seed=n + d)
    C0 = X[np.random.default_rng(k).choice(n, k, replace=n < k)].copy()
    lockstep(X, C0, 1)


def test_kmeans_ties_and_near_ties_take_the_oracle_label():
    say("kmeans ties")
    rng = np.random.default_rng(7)
    d, k = 32, 64
    C = rng.uniform(-10, 10, (k, d)).astype(np.float32)
    C[5] = C[3]                                  # exact duplicate: lowest index wins
    X = np.repeat(C[:8], 64, axis=0).copy()      # points on centroids (distance 0)
    mid = (0.5 * (C[10].astype(np.float64) + C[11])).astype(np.float32)
    X = np.vstack([X, np.repeat(mid[None], 300, axis=0)])  # equidistant up to rounding
    X = np.vstack([X, mid + rng.normal(scale=1e-6, size=(300, d)).astype(np.float32)])
    lab, cnt, _ = api.kmeans_step(dev(X), dev(C))
    assert np.array_equal(host(lab), O.kmeans_assign(X, C))
    lab_p, _, _ = api.kmeans_step(dev(X), dev(C), plain=True)
    assert np.array_equal(host(lab_p), O.kmeans_assign(X, C))
    assert not np.any(host(lab) == 5)


@pytest.mark.parametrize("scale", [1e-25, 1e-15, 1e17, 1e18])
def test_kmeans_extreme_scales_take_the_oracle_label(scale):
    """Points and centroids scaled so the products fall below the normal range
    (1e-25: every certification is refused and binary64 decides; 1e-15: below
    the matrix stage's 2^-40 floor) or near the top of it (1e17; at 1e18 |x|^2
    and |c|^2 overflow in FP32 and binary64 decides): labels and
    counts bit-exact, centroids within the reduction tolerance."""
    say("kmeans scale", scale)
    X, _, _ = W.kmeans_blobs(3000, 16, 8, seed=11)
    X = (X.astype(np.float64) * scale).astype(np.float32)
    C0 = X[np.random.default_rng(5).choice(len(X), 12, replace=False)].copy()
    lockstep(X, C0, 1)


def test_kmeans_empty_cluster_and_determinism():
    say("kmeans empty")
    X, _, _ = W.kmeans_blobs(20000, 32, 8, seed=3)
    C = np.vstack([X[:8], np.full((8, 32), 1e4, dtype=np.float32)])
    Xt, Ct = dev(X), dev(C)
    lab1, cnt1, C1 = api.kmeans_step(Xt, Ct)
    lab2, cnt2, C2 = api.kmeans_step(Xt, Ct)
    assert np.all(host(cnt1)[8:] == 0)
    assert np.array_equal(host(C1)[8:], C[8:])
    assert host(C1).tobytes() == host(C2).tobytes() and host(lab1).tobytes() == host(lab2).tobytes()


def test_sse_and_gradient_vs_oracle():
    say("kmeans sse")
    X, _, _ = W.kmeans_blobs(50000, 32, 16, seed=4)
    C = X[:16].copy()
    lab = O.kmeans_assign(X, C)
    Xt = dev(X).requires_grad_()
    sse = api.kmeans_sse(Xt, dev(C), dev(lab))
    ref = O.kmeans_sse(X, C, lab)
    assert abs(float(host(sse.detach())) - ref) <= 1e-4 * ref
    (0.75 * sse).backward()
    G = host(Xt.grad)
    G_ref = O.kmeans_sse_grad(X, C, lab, 0.75)
    # 2 g (x - c): a subtraction and two products of binary32 values
    assert np.allclose(G, G_ref, rtol=4e-7, atol=4e-7 * np.abs(G_ref).max())


def test_kmeans_graph_replay_ten_iterations():
    say("kmeans graph")
    n, d, k = 1 << 17, 32, 64
    X, _, _ = W.kmeans_blobs(n, d, k, seed=5)
    Xt = dev(X)
    Cs = [dev(X[:k])] + [torch.empty((k, d), device=DEV) for _ in range(10)]
    labels = torch.empty(n, dtype=torch.int32, device=DEV)
    counts = torch.empty(k, dtype=torch.int64, device=DEV)
    ws = torch.zeros(abi.mx_kmeans_workspace_bytes(n, d, k), dtype=torch.uint8, device=DEV)
    for it in range(10):
        abi.mx_kmeans_step_f32(Xt, Cs[it], labels, counts, Cs[it + 1], ws)
    eager = host(Cs[10]).copy()
    eager_lab = host(labels).copy()
    side = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(side):
        abi.mx_graph_begin(side)
        for it in range(10):
            abi.mx_kmeans_step_f32(Xt, Cs[it], labels, counts, Cs[it + 1], ws, stream=side)
        graph = abi.mx_graph_end(side)
    for rep in range(3):
        Cs[10].zero_()
        labels.zero_()
        torch.cuda.synchronize()
        graph.launch(side)
        side.synchronize()
        assert host(Cs[10]).tobytes() == eager.tobytes(), rep
        assert host(labels).tobytes() == eager_lab.tobytes(), rep
        _ = api.kmeans_step(Xt, Cs[0])
        torch.cuda.synchronize()
    abi.mx_graph_destroy(graph)


def test_kmeans_unsupported_sizes():
    X = torch.zeros((10, 65), device=DEV)
    with pytest.raises(abi.MxError) as e:
        api.kmeans_step(X, torch.zeros((4, 65), device=DEV))
    assert e.value.status == abi.MX_ERR_UNSUPPORTED
    X = torch.zeros((10, 64), device=DEV)
    with pytest.raises(abi.MxError) as e:  # k * d = 4160 > 4096
        api.kmeans_step(X, torch.zeros((65, 64), device=DEV))
    assert e.value.status == abi.MX_ERR_UNSUPPORTED
    X = torch.zeros((10, 1), device=DEV)
    with pytest.raises(abi.MxError) as e:  # k > 256
        api.kmeans_step(X, torch.zeros((257, 1), device=DEV))
    assert e.value.status == abi.MX_ERR_UNSUPPORTED
