"""GPU parity of the N-body loop (forward Euler around a pairwise map(reduce))
and its checkpointed adjoint against the oracle, through the C ABI.

The full loop is chaotic at the configured size (close pairs at ~eps): a
1-ulp binary32 perturbation of the initial positions changes the binary64
gradient by ~5e-3 at N = 1024 and ~2e-1 at N = 2048 (test_nbody_conditioning
in test_nbody_host.py).  End-to-end loop parity is therefore checked where the
problem is well conditioned (N = 256).  At the full size N = 16384 the first,
middle and last forward steps and reverse steps are checked against the
oracle from the GPU's own states on 2048 sampled bodies, and the checkpointed
gradient entry point is shown equal, bit for bit, to that chain of steps;
checkpointed and full-tape reverses are bit-identical at N = 4096.
"""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from parity import say

import paper_2211_00621_amd as mx  # noqa: E402

pytestmark = pytest.mark.gpu
abi, api = mx.abi, mx.api
DEV = "cuda"
EPS2, G, DT, T, K = 1e-6, 1.0, 1e-4, 20, 5


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def to4(pos, mass):
    p = np.zeros((len(mass), 4), dtype=np.float32)
    p[:, :3] = pos
    p[:, 3] = mass
    return p


def v4(v):
    out = np.zeros((len(v), 4), dtype=np.float32)
    out[:, :3] = v
    return out


def accel_magnitude(x, m, eps2, rows=None, chunk=256):
    """S[i, c] = sum_j G m_j |d_ij,c| phi_ij: the size of the terms each fold adds."""
    x = x.astype(np.float64)
    m = m.astype(np.float64)
    rows = np.arange(len(m)) if rows is None else rows
    out = np.empty((len(rows), 3))
    for a in range(0, len(rows), chunk):
        r = rows[a:a + chunk]
        d = x[None, :, :] - x[r][:, None, :]
        s = (d * d).sum(-1) + eps2
        phi = s ** -1.5
        out[a:a + chunk] = G * ((m[None, :] * phi)[..., None] * np.abs(d)).sum(1)
    return out


def vjp_magnitude(x, m, abar, eps2, rows=None, chunk=256):
    x = x.astype(np.float64)
    m = m.astype(np.float64)
    ab = abar.astype(np.float64)
    rows = np.arange(len(m)) if rows is None else rows
    out = np.empty((len(rows), 3))
    for a in range(0, len(rows), chunk):
        r = rows[a:a + chunk]
        d = x[None, :, :] - x[r][:, None, :]
        s = (d * d).sum(-1) + eps2
        phi = s ** -1.5
        psi = 3 * phi / s
        w = m[r][:, None, None] * ab[None, :, :] - m[None, :, None] * ab[r][:, None, :]
        dw = np.abs((d * w).sum(-1))
        out[a:a + chunk] = G * (phi[..., None] * np.abs(w) + (psi * dw)[..., None] * np.abs(d)).sum(1)
    return out


def check_bodies(got, ref, S, n, rtol=1e-4, what=""):
    """Per component |g - r| <= rtol max(|r|, S / sqrt(n)), and normwise."""
    got = np.asarray(got, dtype=np.float64)
    bound = rtol * np.maximum(np.abs(ref), S / np.sqrt(n))
    bad = np.argwhere(np.abs(got - ref) > bound)
    assert len(bad) == 0, f"{what}: {len(bad)} components out of tolerance, first {bad[:3].tolist()}"
    assert np.linalg.norm(got - ref) <= rtol * np.linalg.norm(ref), f"{what}: normwise"


@pytest.mark.parametrize("n", [1, 2, 255, 256, 257, 1000, 4097])
def test_accel_vs_oracle(n):
    say("nbody accel", n)
    pos, m, _ = W.nbody(n, seed=n)
    a = host(api.nbody_accel(dev(to4(pos, m)), EPS2, G))
    ref = O.nbody_accel(pos, m, EPS2, G)
    assert np.all(a[:, 3] == 0)
    if n == 1:
        assert np.all(a[:, :3] == 0)
        return
    check_bodies(a[:, :3], ref, accel_magnitude(pos, m, EPS2), n, what=f"a n={n}")


SAMPLE = np.sort(np.random.default_rng(123).choice(16384, 2048, replace=False))


def test_accel_config_16384():
    """All 16384 accelerations from the oracle; 2048 sampled bodies compared."""
    n = 16384
    say("nbody accel 16384")
    pos, m, _ = W.nbody(n, seed=0)
    a = host(api.nbody_accel(dev(to4(pos, m)), EPS2, G))
    ref = O.nbody_accel(pos, m, EPS2, G)
    check_bodies(a[SAMPLE, :3], ref[SAMPLE], accel_magnitude(pos, m, EPS2, rows=SAMPLE), n, what="a 16384")


@pytest.mark.parametrize("plain", [False, True])
def test_step_vs_oracle(plain):
    n = 3000
    say("nbody step plain", plain)
    pos, m, _ = W.nbody(n, seed=1)
    vel = np.random.default_rng(1).normal(scale=0.1, size=(n, 3)).astype(np.float32)
    xo, vo = api.nbody_step(dev(to4(pos, m)), dev(v4(vel)), EPS2, G, DT, plain=plain)
    xo, vo = host(xo), host(vo)
    x_ref, v_ref = O.nbody_step(pos, vel, m, EPS2, G, DT)
    assert np.array_equal(xo[:, 3], m)
    # x' = x + dt v: one FMA or two roundings of binary32
    assert np.allclose(xo[:, :3], x_ref, rtol=2e-7, atol=1e-9)
    S = DT * accel_magnitude(pos, m, EPS2) + np.abs(vel)
    check_bodies(vo[:, :3], v_ref, S, n, what="v'")


@pytest.mark.parametrize("n", [300, 4097])
def test_vjp_and_adjoint_step_vs_oracle(n):
    say("nbody vjp", n)
    pos, m, _ = W.nbody(n, seed=2)
    rng = np.random.default_rng(n)
    abar = rng.normal(size=(n, 3)).astype(np.float32)
    xbar = rng.normal(size=(n, 3)).astype(np.float32)
    out = host(api.nbody_accel_vjp(dev(to4(pos, m)), dev(v4(abar)), EPS2, G))
    ref = O.nbody_accel_vjp(pos, m, abar, EPS2, G)
    S = vjp_magnitude(pos, m, abar, EPS2)
    check_bodies(out[:, :3], ref, S, n, what="vjp")
    # one reverse step
    xbo = torch.empty((n, 4), device=DEV)
    vbo = torch.empty((n, 4), device=DEV)
    ws = api.bytes_workspace(abi.mx_nbody_pair_workspace_bytes(n), "nbody_pair")
    abi.mx_nbody_adjoint_step_f32(dev(to4(pos, m)), dev(v4(xbar)), dev(v4(abar)), EPS2, G, DT, xbo, vbo, ws)
    xb_ref = xbar.astype(np.float64) + DT * ref
    vb_ref = abar.astype(np.float64) + DT * xbar.astype(np.float64)
    check_bodies(host(xbo)[:, :3], xb_ref, DT * S + np.abs(xbar), n, what="xbar_t")
    assert np.allclose(host(vbo)[:, :3], vb_ref, rtol=2e-7, atol=1e-9)


def test_loop_gradient_vs_oracle_small():
    """N = 256 (well conditioned): KE, dKE/dx0 and dKE/dv0 of the 20-step loop."""
    n = 256
    say("nbody loop grad 256")
    pos, m, vel = W.nbody(n, seed=0)
    ke, gx, gv = api.nbody_ke_grad(dev(to4(pos, m)), dev(v4(vel)), EPS2, G, DT, T, K)
    ke_ref, gx_ref, gv_ref = O.nbody_ke_grad(pos, vel, m, EPS2, G, DT, T, ckpt_every=K)
    assert abs(float(host(ke)) - ke_ref) <= 1e-3 * abs(ke_ref)
    for got, ref, what in ((host(gx)[:, :3], gx_ref, "gx"), (host(gv)[:, :3], gv_ref, "gv")):
        rms = np.sqrt(np.mean(ref ** 2))
        assert np.linalg.norm(got - ref) <= 1e-3 * np.linalg.norm(ref), what
        assert np.all(np.abs(got - ref) <= 1e-3 * np.maximum(np.abs(ref), 1e-2 * rms)), what


@pytest.mark.parametrize("k", [1, 3, 5, 7, 20])
def test_checkpointed_reverse_equals_full_tape(k):
    """Recomputation reproduces the forward bit for bit, so every checkpoint
    interval gives the identical gradient (k = 1 stores every state)."""
    n = 4096
    say("nbody ckpt", k)
    pos, m, vel = W.nbody(n, seed=3)
    p4, vv = dev(to4(pos, m)), dev(v4(vel))
    ke1, gx1, gv1 = [host(t) for t in api.nbody_ke_grad(p4, vv, EPS2, G, DT, T, 1)]
    kek, gxk, gvk = [host(t) for t in api.nbody_ke_grad(p4, vv, EPS2, G, DT, T, k)]
    assert ke1.tobytes() == kek.tobytes()
    assert gx1.tobytes() == gxk.tobytes() and gv1.tobytes() == gvk.tobytes()


def test_loop_graph_replay_matches_eager():
    n = 2048
    say("nbody graph")
    pos, m, vel = W.nbody(n, seed=4)
    p4, vv = dev(to4(pos, m)), dev(v4(vel))
    ke = torch.empty((), device=DEV)
    gx = torch.empty((n, 4), device=DEV)
    gv = torch.empty((n, 4), device=DEV)
    ws = torch.zeros(abi.mx_nbody_workspace_bytes(n, T, K), dtype=torch.uint8, device=DEV)
    abi.mx_nbody_ke_grad_f32(p4, vv, EPS2, G, DT, T, K, ke, gx, gv, ws)
    eager = [host(ke).copy(), host(gx).copy(), host(gv).copy()]
    side = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(side):
        abi.mx_graph_begin(side)
        abi.mx_nbody_ke_grad_f32(p4, vv, EPS2, G, DT, T, K, ke, gx, gv, ws, stream=side)
        graph = abi.mx_graph_end(side)
    for rep in range(3):
        ke.fill_(-1.0)
        gx.zero_()
        torch.cuda.synchronize()
        graph.launch(side)
        side.synchronize()
        got = [host(ke), host(gx), host(gv)]
        for a, b in zip(got, eager):
            assert a.tobytes() == b.tobytes(), f"replay {rep}"
        _ = api.nbody_accel(p4, EPS2, G)  # eager work between replays
        torch.cuda.synchronize()
    abi.mx_graph_destroy(graph)


def test_config_16384_steps_vs_oracle_sampled():
    """Full size, the launches the benchmark times.  The GPU's own forward loop
    (mx_nbody_step_f32), its reverse sweep by mx_nbody_adjoint_step_f32 from
    the GPU's own states and adjoints, and mx_nbody_ke_grad_f32:

    * forward steps t = 0, 10, 19: positions and velocities of the sampled
      bodies against the oracle's step from the same state;
    * reverse steps t = 19, 10, 0: xbar_t and vbar_t of the sampled bodies
      against the oracle's adjoint step from the same (x_t, xbar_{t+1},
      vbar_{t+1});
    * mx_nbody_ke_grad_f32 (checkpoints every 5 steps, recomputed segments)
      equals that chain of checked steps bit for bit, and its KE the final
      state's kinetic energy."""
    n = 16384
    say("nbody 16384 steps")
    pos, m, vel = W.nbody(n, seed=0)
    p4, vv = dev(to4(pos, m)), dev(v4(vel))
    states = [(p4, vv)]
    for t in range(T):
        states.append(api.nbody_step(*states[-1], EPS2, G, DT))
    for t in (0, T // 2, T - 1):
        x_t = host(states[t][0])
        v_t = host(states[t][1])
        x_next, v_next = host(states[t + 1][0]), host(states[t + 1][1])
        ref_x, ref_v = O.nbody_step(x_t[:, :3], v_t[:, :3], x_t[:, 3], EPS2, G, DT)
        assert np.array_equal(x_next[:, 3], m), t
        # x' = x + dt v: one FMA or two roundings of binary32 (and dt itself
        # rounded to binary32), so within 2^-22 of the operands' magnitudes
        xs, vs = x_t[SAMPLE, :3].astype(np.float64), v_t[SAMPLE, :3].astype(np.float64)
        assert np.all(np.abs(x_next[SAMPLE, :3] - ref_x[SAMPLE]) <= 2.0 ** -22 * (np.abs(xs) + DT * np.abs(vs))), \
            f"x_{t + 1}"
        S = DT * accel_magnitude(x_t[:, :3], x_t[:, 3], EPS2, rows=SAMPLE) + np.abs(v_t[SAMPLE, :3])
        check_bodies(v_next[SAMPLE, :3], ref_v[SAMPLE], S, n, what=f"v_{t + 1}")
    # reverse sweep: vbar_T = m v_T (binary32 products, as the library forms them), xbar_T = 0
    vT = host(states[T][1])
    xb = dev(np.zeros((n, 4), dtype=np.float32))
    vb = dev(v4(m[:, None] * vT[:, :3]))
    ws = api.bytes_workspace(abi.mx_nbody_pair_workspace_bytes(n), "nbody_pair")
    for t in range(T - 1, -1, -1):
        xbo = torch.empty((n, 4), device=DEV)
        vbo = torch.empty((n, 4), device=DEV)
        abi.mx_nbody_adjoint_step_f32(states[t][0], xb, vb, EPS2, G, DT, xbo, vbo, ws)
        if t in (T - 1, T // 2, 0):
            x_t = host(states[t][0])
            xb_in, vb_in = host(xb)[:, :3], host(vb)[:, :3]
            vjp = O.nbody_accel_vjp(x_t[:, :3], x_t[:, 3], vb_in, EPS2, G)
            xb_ref = xb_in.astype(np.float64) + DT * vjp
            vb_ref = vb_in.astype(np.float64) + DT * xb_in.astype(np.float64)
            S = DT * vjp_magnitude(x_t[:, :3], x_t[:, 3], vb_in, EPS2, rows=SAMPLE) + np.abs(xb_in[SAMPLE])
            check_bodies(host(xbo)[SAMPLE, :3], xb_ref[SAMPLE], S, n, what=f"xbar_{t}")
            # vbar_t = vbar_{t+1} + dt xbar_{t+1}: the same two-operand bound;
            # the terms can cancel, so it is relative to the operands, not the sum
            bnd = 2.0 ** -22 * (np.abs(vb_in[SAMPLE]).astype(np.float64) + DT * np.abs(xb_in[SAMPLE]))
            assert np.all(np.abs(host(vbo)[SAMPLE, :3] - vb_ref[SAMPLE]) <= bnd), f"vbar_{t}"
        xb, vb = xbo, vbo
    ke, gx, gv = api.nbody_ke_grad(p4, vv, EPS2, G, DT, T, K)
    assert host(gx).tobytes() == host(xb).tobytes() and host(gv).tobytes() == host(vb).tobytes()
    kin = torch.empty((), device=DEV)
    abi.mx_nbody_kinetic_f32(states[T][0], states[T][1], kin)
    assert host(ke).tobytes() == host(kin).tobytes()
    ke_ref = O.nbody_kinetic(vT[:, :3], m)
    assert abs(float(host(ke)) - ke_ref) <= 1e-4 * ke_ref


def test_ke_forward_and_vjp_split_equals_fused_grad():
    """mx_nbody_ke_f32 + mx_nbody_ke_vjp_f32 (no gscale) give mx_nbody_ke_grad_f32
    bit for bit; a device gscale g scales the seed: g = 2 exactly doubles the
    gradients (every rounding is scaled by a power of two), g = 0.3 agrees
    with 0.3 times them within binary32 rounding of the seed."""
    n = 1500
    say("nbody ke split")
    pos, m, vel = W.nbody(n, seed=6)
    vel = np.random.default_rng(6).normal(scale=0.1, size=(n, 3)).astype(np.float32)
    p4, vv = dev(to4(pos, m)), dev(v4(vel))
    ke0, gx0, gv0 = [host(t) for t in api.nbody_ke_grad(p4, vv, EPS2, G, DT, T, K)]
    ws = torch.zeros(abi.mx_nbody_workspace_bytes(n, T, K), dtype=torch.uint8, device=DEV)
    ke = torch.empty((), device=DEV)
    abi.mx_nbody_ke_f32(p4, vv, EPS2, G, DT, T, K, ke, ws)
    assert host(ke).tobytes() == ke0.tobytes()
    for g in (None, 2.0, 0.3):
        gx, gv = torch.empty((n, 4), device=DEV), torch.empty((n, 4), device=DEV)
        gs = None if g is None else torch.tensor([g], dtype=torch.float32, device=DEV)
        abi.mx_nbody_ke_vjp_f32(p4, vv, EPS2, G, DT, T, K, gs, gx, gv, ws)
        gx, gv = host(gx), host(gv)
        if g is None:
            assert gx.tobytes() == gx0.tobytes() and gv.tobytes() == gv0.tobytes()
        elif g == 2.0:
            assert np.array_equal(gx, 2 * gx0) and np.array_equal(gv, 2 * gv0)
        else:
            for a, b in ((gx, gx0), (gv, gv0)):
                ref = np.float64(np.float32(g)) * b.astype(np.float64)
                assert np.linalg.norm(a - ref) <= 1e-5 * np.linalg.norm(ref)
    # n = 0: KE = 0, nothing else written
    e = torch.zeros((0, 4), device=DEV)
    k0 = torch.full((), 5.0, device=DEV)
    abi.mx_nbody_ke_f32(e, e, EPS2, G, DT, T, K, k0, torch.zeros(256, dtype=torch.uint8, device=DEV))
    assert float(host(k0)) == 0.0


def test_autograd_wrapper_matches_entry_point():
    n = 512
    say("nbody autograd")
    pos, m, vel = W.nbody(n, seed=5)
    tp = dev(pos).requires_grad_()
    tv = dev(vel).requires_grad_()
    ke = api.nbody_kinetic_energy(tp, tv, dev(m), EPS2, G, DT, T, K)
    (2.0 * ke).backward()
    ke2, gx, gv = api.nbody_ke_grad(dev(to4(pos, m)), dev(v4(vel)), EPS2, G, DT, T, K)
    assert float(host(ke.detach())) == float(host(ke2))
    assert np.array_equal(host(tp.grad), 2.0 * host(gx)[:, :3])
    assert np.array_equal(host(tv.grad), 2.0 * host(gv)[:, :3])
    # kinetic energy entry point alone
    k = torch.empty((), device=DEV)
    abi.mx_nbody_kinetic_f32(dev(to4(pos, m)), dev(v4(vel)), k)
    assert float(host(k)) == 0.0


def test_nbody_errors():
    p = torch.zeros((8, 4), device=DEV)
    with pytest.raises(abi.MxError):
        abi.mx_nbody_step_f32(p, p, EPS2, G, DT, p, p, torch.zeros(256, dtype=torch.uint8, device=DEV))
    with pytest.raises(abi.MxError):
        api.nbody_ke_grad(p, p, EPS2, G, DT, T, 65)
    with pytest.raises(abi.MxError):
        api.nbody_accel(p, 0.0, G)
