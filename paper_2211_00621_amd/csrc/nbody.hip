// Sequential loop around a pairwise map (reduce): gravitational N-body with
// Plummer softening and explicit Euler steps (the ODE-solver pattern of the
// CUDA-backend evaluation, Table 2), its adjoint, and the checkpointed reverse
// sweep of the loop.
//
//   a_i = G sum_j m_j d_ij (|d_ij|^2 + eps2)^(-3/2),   d_ij = x_j - x_i
//   x_{t+1} = x_t + dt v_t,   v_{t+1} = v_t + dt a(x_t)
//   (J_a^T abar)_k = G sum_j [phi I - 3 phi/s d d^T] (m_k abar_j - m_j abar_k),
//     d = x_j - x_k, s = |d|^2 + eps2, phi = s^(-3/2)
//
// Layout: bodies as float4 records (x, y, z, m); velocities and adjoints as
// float4 (x, y, z, 0).
//
// Pair kernels: a block of 256 threads owns a tile of 256 bodies i and one of
// S slices of the bodies j; j bodies are staged through LDS 256 at a time and
// read as LDS broadcasts.  With S > 1 each block writes its partial sums for
// its slice and a second, elementwise kernel adds the S partials in slice
// order and applies the update (the kernel boundary orders the two, with no
// per-block cache flushes); with S = 1 the pair kernel applies the update
// itself.  Results therefore do not depend on block scheduling, and a
// recomputation reproduces the forward bit for bit.
#include "mx_internal.h"

namespace mx {
namespace {

constexpr int NT = 256;
constexpr int kMaxSlices = 64;

enum Mode { ACCEL = 0, STEP = 1, VJP = 2, ADJSTEP = 3 };

struct PairArgs {
    const float4 *pos;   // x_t (with masses)
    const float4 *aux;   // STEP: v_t; VJP/ADJSTEP: abar (= vbar_{t+1})
    const float4 *aux2;  // ADJSTEP: xbar_{t+1}
    float4 *out0;        // ACCEL: a; STEP: x_{t+1}; VJP: J^T abar; ADJSTEP: xbar_t
    float4 *out1;        // STEP: v_{t+1}; ADJSTEP: vbar_t
    float4 *partial;     // [S][N]
    int64_t n;
    int slices;
    int64_t slice_len;   // multiple of NT
    float eps2, G, dt;
};

__device__ __forceinline__ void pair_accel(const float4 xi, const float4 xj, float eps2, float &ax,
                                           float &ay, float &az) {
    const float dx = xj.x - xi.x, dy = xj.y - xi.y, dz = xj.z - xi.z;
    const float s = fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, eps2)));  // eps2 folded into the first FMA
    const float inv = __frsqrt_rn(s);
    const float w = xj.w * (inv * inv * inv);
    ax += w * dx;
    ay += w * dy;
    az += w * dz;
}

__device__ __forceinline__ void pair_vjp(const float4 xk, const float4 ak, const float4 xj,
                                         const float4 aj, float eps2, float &ox, float &oy,
                                         float &oz) {
    const float dx = xj.x - xk.x, dy = xj.y - xk.y, dz = xj.z - xk.z;
    const float s = fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, eps2)));
    const float inv = __frsqrt_rn(s);
    const float inv2 = inv * inv;
    const float phi = inv2 * inv;
    const float psi = 3.0f * phi * inv2;
    // both products rounded before the subtraction (never fused into an FMA),
    // so the self term j = k, where phi = eps^-3 is huge, is exactly zero
    const float wx = sub_rn(mul_rn(xk.w, aj.x), mul_rn(xj.w, ak.x));
    const float wy = sub_rn(mul_rn(xk.w, aj.y), mul_rn(xj.w, ak.y));
    const float wz = sub_rn(mul_rn(xk.w, aj.z), mul_rn(xj.w, ak.z));
    const float t = psi * (dx * wx + dy * wy + dz * wz);
    ox += phi * wx - t * dx;
    oy += phi * wy - t * dy;
    oz += phi * wz - t * dz;
}

template <int MODE>
__device__ __forceinline__ void finish(const PairArgs &p, int64_t i, float4 xi, float4 ai, float ox, float oy,
                                       float oz) {
    const float G = p.G, dt = p.dt;
    if constexpr (MODE == ACCEL || MODE == VJP) {
        p.out0[i] = make_float4(G * ox, G * oy, G * oz, 0.f);
    } else if constexpr (MODE == STEP) {
        const float4 v = p.aux[i];
        p.out0[i] = make_float4(xi.x + dt * v.x, xi.y + dt * v.y, xi.z + dt * v.z, xi.w);
        p.out1[i] = make_float4(v.x + dt * (G * ox), v.y + dt * (G * oy), v.z + dt * (G * oz), 0.f);
    } else {  // ADJSTEP: xbar_t = xbar + dt G J^T vbar;  vbar_t = vbar + dt xbar
        const float4 xb = p.aux2[i];
        p.out0[i] = make_float4(xb.x + dt * (G * ox), xb.y + dt * (G * oy), xb.z + dt * (G * oz), 0.f);
        p.out1[i] = make_float4(ai.x + dt * xb.x, ai.y + dt * xb.y, ai.z + dt * xb.z, 0.f);
    }
}

template <int MODE>
__global__ void __launch_bounds__(NT) k_pairs(PairArgs p) {
    constexpr bool ADJ = MODE == VJP || MODE == ADJSTEP;
    __shared__ float4 sx[NT];
    __shared__ float4 sa[ADJ ? NT : 1];
    const int64_t n = p.n;
    const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
    const float4 zero = make_float4(0.f, 0.f, 0.f, 0.f);
    const float4 xi = i < n ? p.pos[i] : zero;
    float4 ai = zero;
    if constexpr (ADJ) ai = i < n ? p.aux[i] : zero;
    float ox = 0.f, oy = 0.f, oz = 0.f;
    const int64_t js = (int64_t)blockIdx.y * p.slice_len;
    int64_t je = js + p.slice_len;
    if (je > n) je = n;
    for (int64_t j0 = js; j0 < je; j0 += NT) {
        const int64_t j = j0 + threadIdx.x;
        sx[threadIdx.x] = j < je ? p.pos[j] : zero;  // zero mass: no contribution
        if constexpr (ADJ) sa[threadIdx.x] = j < je ? p.aux[j] : zero;
        __syncthreads();
#pragma unroll 8
        for (int jj = 0; jj < NT; ++jj) {
            if constexpr (ADJ) pair_vjp(xi, ai, sx[jj], sa[jj], p.eps2, ox, oy, oz);
            else pair_accel(xi, sx[jj], p.eps2, ox, oy, oz);
        }
        __syncthreads();
    }
    if (i >= n) return;
    if (p.slices > 1) {
        p.partial[(int64_t)blockIdx.y * n + i] = make_float4(ox, oy, oz, 0.f);
        return;
    }
    finish<MODE>(p, i, xi, ai, ox, oy, oz);
}

// Adds the S slice partials of body i in slice order and applies the update.
template <int MODE>
__global__ void __launch_bounds__(NT) k_pairs_finish(PairArgs p) {
    const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (i >= p.n) return;
    float ox = 0.f, oy = 0.f, oz = 0.f;
    for (int s = 0; s < p.slices; ++s) {
        const float4 q = p.partial[(int64_t)s * p.n + i];
        ox += q.x;
        oy += q.y;
        oz += q.z;
    }
    const float4 xi = p.pos[i];
    float4 ai = make_float4(0.f, 0.f, 0.f, 0.f);
    if constexpr (MODE == VJP || MODE == ADJSTEP) ai = p.aux[i];
    finish<MODE>(p, i, xi, ai, ox, oy, oz);
}

// ---------------------------------------------------------------- plain forms
__global__ void __launch_bounds__(NT) k_accel_plain(const float4 *__restrict__ pos, int64_t n, float eps2,
                                                    float G, float4 *__restrict__ acc) {
    const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (i >= n) return;
    const float4 xi = pos[i];
    float ax = 0.f, ay = 0.f, az = 0.f;
    for (int64_t j = 0; j < n; ++j) pair_accel(xi, pos[j], eps2, ax, ay, az);
    acc[i] = make_float4(G * ax, G * ay, G * az, 0.f);
}

__global__ void __launch_bounds__(NT) k_euler(const float4 *__restrict__ pos, const float4 *__restrict__ vel,
                                              const float4 *__restrict__ acc, int64_t n, float dt,
                                              float4 *__restrict__ pos_out, float4 *__restrict__ vel_out) {
    const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (i >= n) return;
    const float4 x = pos[i], v = vel[i], a = acc[i];
    pos_out[i] = make_float4(x.x + dt * v.x, x.y + dt * v.y, x.z + dt * v.z, x.w);
    vel_out[i] = make_float4(v.x + dt * a.x, v.y + dt * a.y, v.z + dt * a.z, 0.f);
}

// ---------------------------------------------------------------- kinetic energy
// KE = 1/2 sum_i m_i |v_i|^2 folded by one block (fixed bracketing), and the
// start of the reverse sweep: vbar = m v, xbar = 0 (either may be null).
__global__ void __launch_bounds__(NT) k_kinetic(const float4 *__restrict__ pos, const float4 *__restrict__ vel,
                                                int64_t n, float *__restrict__ ke, float4 *vbar, float4 *xbar) {
    __shared__ float smem[NT / kWave];
    using R = Red<MX_ADD, float>;
    float acc = 0.f;
    for (int64_t i = threadIdx.x; i < n; i += NT) {
        const float4 v = vel[i];
        const float m = pos[i].w;
        acc += 0.5f * m * (v.x * v.x + v.y * v.y + v.z * v.z);
        if (vbar) vbar[i] = make_float4(m * v.x, m * v.y, m * v.z, 0.f);
        if (xbar) xbar[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    acc = block_reduce<R, NT>(acc, smem);
    if (threadIdx.x == 0) ke[0] = acc;
}

// Start of the reverse sweep for an upstream gradient g of KE (a device
// scalar; null means 1): vbar = g m v, xbar = 0.  With g = 1 the products
// equal k_kinetic's m v bit for bit.
__global__ void __launch_bounds__(NT) k_adjoint_seed(const float4 *__restrict__ pos, const float4 *__restrict__ vel,
                                                     int64_t n, const float *__restrict__ gscale,
                                                     float4 *__restrict__ vbar, float4 *__restrict__ xbar) {
    const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (i >= n) return;
    const float g = gscale ? gscale[0] : 1.f;
    const float4 v = vel[i];
    const float m = pos[i].w;
    vbar[i] = make_float4(m * v.x * g, m * v.y * g, m * v.z * g, 0.f);
    xbar[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}

// ---------------------------------------------------------------- launch helpers
// The j range is cut into S slices so that about kTargetBlocks blocks run
// (8 per CU on 256 CUs); S depends only on n, so results are the same on
// every device.
constexpr int64_t kTargetBlocks = 2048;

int slices_for(int64_t n) {
    if (n <= 0) return 1;  // no bodies: one (empty) slice
    const int64_t tiles = ceil_div(n, NT);
    int64_t s = ceil_div(kTargetBlocks, tiles > 0 ? tiles : 1);
    if (s > tiles) s = tiles;
    if (s > kMaxSlices) s = kMaxSlices;
    if (s < 1) s = 1;
    // snap to whole LDS tiles per slice
    const int64_t len = ceil_div(ceil_div(n, s), NT) * NT;
    return (int)ceil_div(n, len);
}

size_t pair_ws_bytes(int64_t n) {
    const int sl = slices_for(n);
    return kCounterBytes + (sl > 1 ? align256((size_t)sl * (size_t)n * 16) : 0);
}

template <int MODE>
mx_status launch_pairs(PairArgs p, void *ws, hipStream_t s) {
    const int64_t tiles = ceil_div(p.n, NT);
    MX_REQUIRE(tiles < (1LL << 31), MX_ERR_SHAPE, "nbody: too many bodies");
    p.slices = slices_for(p.n);
    p.slice_len = ceil_div(ceil_div(p.n, p.slices), NT) * NT;
    p.partial = (float4 *)((char *)ws + kCounterBytes);
    hipLaunchKernelGGL((k_pairs<MODE>), dim3((unsigned)tiles, (unsigned)p.slices), dim3(NT), 0, s, p);
    if (p.slices > 1) hipLaunchKernelGGL((k_pairs_finish<MODE>), dim3((unsigned)tiles), dim3(NT), 0, s, p);
    return last_launch("nbody pair kernel");
}

inline bool a16(const void *p) { return ((uintptr_t)p & 15) == 0; }

mx_status check_common(const char *who, int64_t n, float eps2, void *ws, size_t ws_bytes, size_t need) {
    MX_REQUIRE(n >= 0, MX_ERR_SHAPE, "%s: n < 0", who);
    MX_REQUIRE(eps2 > 0.f, MX_ERR_INVALID, "%s: eps2 must be positive", who);
    if (n > 0)
        MX_REQUIRE(ws && ws_bytes >= need && ((uintptr_t)ws & 255) == 0, MX_ERR_WORKSPACE,
                   "%s: workspace needs %zu bytes, 256-byte aligned", who, need);
    return MX_OK;
}

mx_status step_impl(const float4 *x, const float4 *v, int64_t n, float eps2, float G, float dt, float4 *xo,
                    float4 *vo, void *pws, hipStream_t s) {
    PairArgs p{};
    p.pos = x; p.aux = v; p.out0 = xo; p.out1 = vo; p.n = n; p.eps2 = eps2; p.G = G; p.dt = dt;
    return launch_pairs<STEP>(p, pws, s);
}

mx_status adjstep_impl(const float4 *x, const float4 *xb, const float4 *vb, int64_t n, float eps2, float G,
                       float dt, float4 *xbo, float4 *vbo, void *pws, hipStream_t s) {
    PairArgs p{};
    p.pos = x; p.aux = vb; p.aux2 = xb; p.out0 = xbo; p.out1 = vbo; p.n = n; p.eps2 = eps2; p.G = G; p.dt = dt;
    return launch_pairs<ADJSTEP>(p, pws, s);
}

mx_status kinetic_impl(const float4 *x, const float4 *v, int64_t n, float *ke, float4 *vbar, float4 *xbar,
                       hipStream_t s) {
    hipLaunchKernelGGL(k_kinetic, dim3(1), dim3(NT), 0, s, x, v, n, ke, vbar, xbar);
    return last_launch("nbody kinetic");
}

// Workspace of mx_nbody_ke_grad_f32: pair partials, then float4 states of n
// bodies -- final state (x, v), two ping-pong states, nck checkpoints (slot 0
// unused: the input is checkpoint 0), a tape of k states, and two adjoint
// ping-pong pairs (xbar, vbar).
struct NbodyWs {
    void *pair;
    float4 *fin_x, *fin_v, *tmp_x[2], *tmp_v[2], *ck_x, *ck_v, *tape_x, *tape_v, *xb[2], *vb[2];
    size_t bytes;
};

NbodyWs nbody_ws_layout(char *base, int64_t n, int nsteps, int k) {
    NbodyWs w{};
    const size_t st = align256((size_t)n * 16);
    const int nck = (nsteps + k - 1) / k;
    size_t off = 0;
    auto take = [&](size_t b) { char *q = base ? base + off : nullptr; off += b; return q; };
    w.pair = take(align256(pair_ws_bytes(n)));
    w.fin_x = (float4 *)take(st);
    w.fin_v = (float4 *)take(st);
    for (int i = 0; i < 2; ++i) { w.tmp_x[i] = (float4 *)take(st); w.tmp_v[i] = (float4 *)take(st); }
    w.ck_x = (float4 *)take(st * (size_t)(nck > 0 ? nck : 1));
    w.ck_v = (float4 *)take(st * (size_t)(nck > 0 ? nck : 1));
    w.tape_x = (float4 *)take(st * (size_t)k);
    w.tape_v = (float4 *)take(st * (size_t)k);
    for (int i = 0; i < 2; ++i) { w.xb[i] = (float4 *)take(st); w.vb[i] = (float4 *)take(st); }
    w.bytes = off;
    return w;
}

constexpr int kMaxCkptEvery = 64;

}  // namespace
}  // namespace mx

using namespace mx;

extern "C" {

size_t mx_nbody_pair_workspace_bytes(int64_t n) { return n < 0 ? 0 : pair_ws_bytes(n); }

size_t mx_nbody_workspace_bytes(int64_t n, int nsteps, int ckpt_every) {
    if (n < 0 || nsteps < 1 || ckpt_every < 1) return 0;
    const int k = ckpt_every < nsteps ? ckpt_every : nsteps;
    return align256(nbody_ws_layout(nullptr, n, nsteps, k).bytes);
}

mx_status mx_nbody_accel_f32(const float *pos4_dev, int64_t n, float eps2, float G, float *acc4_dev, void *ws,
                             size_t ws_bytes, hipStream_t stream) {
    if (mx_status st = check_common("mx_nbody_accel_f32", n, eps2, ws, ws_bytes, pair_ws_bytes(n))) return st;
    if (n == 0) return MX_OK;
    MX_REQUIRE(pos4_dev && acc4_dev && a16(pos4_dev) && a16(acc4_dev), MX_ERR_INVALID,
               "mx_nbody_accel_f32: null or unaligned pointer");
    PairArgs p{};
    p.pos = (const float4 *)pos4_dev; p.out0 = (float4 *)acc4_dev; p.n = n; p.eps2 = eps2; p.G = G;
    return launch_pairs<ACCEL>(p, ws, stream);
}

mx_status mx_nbody_step_f32(const float *pos4_dev, const float *vel4_dev, int64_t n, float eps2, float G,
                            float dt, float *pos4_out_dev, float *vel4_out_dev, void *ws, size_t ws_bytes,
                            hipStream_t stream) {
    if (mx_status st = check_common("mx_nbody_step_f32", n, eps2, ws, ws_bytes, pair_ws_bytes(n))) return st;
    if (n == 0) return MX_OK;
    MX_REQUIRE(pos4_dev && vel4_dev && pos4_out_dev && vel4_out_dev, MX_ERR_INVALID, "mx_nbody_step_f32: null pointer");
    MX_REQUIRE(a16(pos4_dev) && a16(vel4_dev) && a16(pos4_out_dev) && a16(vel4_out_dev), MX_ERR_INVALID,
               "mx_nbody_step_f32: pointers must be 16-byte aligned");
    MX_REQUIRE(pos4_out_dev != pos4_dev && vel4_out_dev != vel4_dev && pos4_out_dev != vel4_dev &&
                   vel4_out_dev != pos4_dev,
               MX_ERR_INVALID, "mx_nbody_step_f32: outputs must not alias inputs");
    return step_impl((const float4 *)pos4_dev, (const float4 *)vel4_dev, n, eps2, G, dt, (float4 *)pos4_out_dev,
                     (float4 *)vel4_out_dev, ws, stream);
}

mx_status mx_nbody_step_plain_f32(const float *pos4_dev, const float *vel4_dev, int64_t n, float eps2,
                                  float G, float dt, float *acc4_dev, float *pos4_out_dev,
                                  float *vel4_out_dev, hipStream_t stream) {
    MX_REQUIRE(n >= 0, MX_ERR_SHAPE, "mx_nbody_step_plain_f32: n < 0");
    MX_REQUIRE(eps2 > 0.f, MX_ERR_INVALID, "mx_nbody_step_plain_f32: eps2 must be positive");
    if (n == 0) return MX_OK;
    MX_REQUIRE(pos4_dev && vel4_dev && acc4_dev && pos4_out_dev && vel4_out_dev, MX_ERR_INVALID,
               "mx_nbody_step_plain_f32: null pointer");
    MX_REQUIRE(a16(pos4_dev) && a16(vel4_dev) && a16(acc4_dev) && a16(pos4_out_dev) && a16(vel4_out_dev),
               MX_ERR_INVALID, "mx_nbody_step_plain_f32: pointers must be 16-byte aligned");
    const int64_t grid = ceil_div(n, NT);
    MX_REQUIRE(grid < (1LL << 31), MX_ERR_SHAPE, "mx_nbody_step_plain_f32: too many bodies");
    hipLaunchKernelGGL(k_accel_plain, dim3((unsigned)grid), dim3(NT), 0, stream, (const float4 *)pos4_dev, n, eps2,
                       G, (float4 *)acc4_dev);
    hipLaunchKernelGGL(k_euler, dim3((unsigned)grid), dim3(NT), 0, stream, (const float4 *)pos4_dev,
                       (const float4 *)vel4_dev, (const float4 *)acc4_dev, n, dt, (float4 *)pos4_out_dev,
                       (float4 *)vel4_out_dev);
    return last_launch("mx_nbody_step_plain_f32");
}

mx_status mx_nbody_accel_vjp_f32(const float *pos4_dev, const float *abar4_dev, int64_t n, float eps2,
                                 float G, float *out4_dev, void *ws, size_t ws_bytes, hipStream_t stream) {
    if (mx_status st = check_common("mx_nbody_accel_vjp_f32", n, eps2, ws, ws_bytes, pair_ws_bytes(n))) return st;
    if (n == 0) return MX_OK;
    MX_REQUIRE(pos4_dev && abar4_dev && out4_dev && a16(pos4_dev) && a16(abar4_dev) && a16(out4_dev),
               MX_ERR_INVALID, "mx_nbody_accel_vjp_f32: null or unaligned pointer");
    PairArgs p{};
    p.pos = (const float4 *)pos4_dev; p.aux = (const float4 *)abar4_dev; p.out0 = (float4 *)out4_dev;
    p.n = n; p.eps2 = eps2; p.G = G;
    return launch_pairs<VJP>(p, ws, stream);
}

mx_status mx_nbody_adjoint_step_f32(const float *pos4_dev, const float *xbar4_dev, const float *vbar4_dev,
                                    int64_t n, float eps2, float G, float dt, float *xbar4_out_dev,
                                    float *vbar4_out_dev, void *ws, size_t ws_bytes, hipStream_t stream) {
    const char *who = "mx_nbody_adjoint_step_f32";
    if (mx_status st = check_common(who, n, eps2, ws, ws_bytes, pair_ws_bytes(n))) return st;
    if (n == 0) return MX_OK;
    MX_REQUIRE(pos4_dev && xbar4_dev && vbar4_dev && xbar4_out_dev && vbar4_out_dev, MX_ERR_INVALID,
               "%s: null pointer", who);
    MX_REQUIRE(a16(pos4_dev) && a16(xbar4_dev) && a16(vbar4_dev) && a16(xbar4_out_dev) && a16(vbar4_out_dev),
               MX_ERR_INVALID, "%s: pointers must be 16-byte aligned", who);
    MX_REQUIRE(xbar4_out_dev != xbar4_dev && vbar4_out_dev != vbar4_dev && vbar4_out_dev != xbar4_dev &&
                   xbar4_out_dev != vbar4_dev,
               MX_ERR_INVALID, "%s: outputs must not alias inputs", who);
    return adjstep_impl((const float4 *)pos4_dev, (const float4 *)xbar4_dev, (const float4 *)vbar4_dev, n, eps2, G,
                        dt, (float4 *)xbar4_out_dev, (float4 *)vbar4_out_dev, ws, stream);
}

mx_status mx_nbody_kinetic_f32(const float *pos4_dev, const float *vel4_dev, int64_t n, float *ke_dev,
                               hipStream_t stream) {
    MX_REQUIRE(n >= 0, MX_ERR_SHAPE, "mx_nbody_kinetic_f32: n < 0");
    MX_REQUIRE(ke_dev && (n == 0 || (pos4_dev && vel4_dev)), MX_ERR_INVALID, "mx_nbody_kinetic_f32: null pointer");
    return kinetic_impl((const float4 *)pos4_dev, (const float4 *)vel4_dev, n, ke_dev, nullptr, nullptr, stream);
}

namespace {
mx_status ke_check(const char *who, const float *pos4_dev, const float *vel4_dev, int64_t n, float eps2,
                   int nsteps, int ckpt_every, void *ws, size_t ws_bytes) {
    MX_REQUIRE(nsteps >= 1 && ckpt_every >= 1 && ckpt_every <= kMaxCkptEvery, MX_ERR_INVALID,
               "%s: need nsteps >= 1 and 1 <= ckpt_every <= %d", who, kMaxCkptEvery);
    if (mx_status st = check_common(who, n, eps2, ws, ws_bytes, mx_nbody_workspace_bytes(n, nsteps, ckpt_every)))
        return st;
    if (n > 0)
        MX_REQUIRE(pos4_dev && vel4_dev && a16(pos4_dev) && a16(vel4_dev), MX_ERR_INVALID,
                   "%s: null or unaligned state pointer", who);
    return MX_OK;
}

// Forward loop: checkpoint c (c >= 1) holds the state at t = c k in the
// workspace (checkpoint 0 is the input itself), the final state goes to
// fin_x / fin_v; then KE of the final state.
mx_status ke_forward(const float4 *x0, const float4 *v0, int64_t n, float eps2, float G, float dt, int nsteps,
                     int k, float *ke_dev, const NbodyWs &w, hipStream_t stream) {
    const int64_t st4 = (int64_t)(align256((size_t)n * 16) / 16);  // float4 stride between states
    const float4 *x = x0, *v = v0;
    for (int t = 0; t < nsteps; ++t) {
        float4 *xo, *vo;
        if (t == nsteps - 1) {
            xo = w.fin_x; vo = w.fin_v;
        } else if ((t + 1) % k == 0) {
            xo = w.ck_x + (int64_t)((t + 1) / k) * st4; vo = w.ck_v + (int64_t)((t + 1) / k) * st4;
        } else {
            xo = w.tmp_x[t & 1]; vo = w.tmp_v[t & 1];
        }
        if (mx_status st = step_impl(x, v, n, eps2, G, dt, xo, vo, w.pair, stream)) return st;
        x = xo;
        v = vo;
    }
    return kinetic_impl(w.fin_x, w.fin_v, n, ke_dev, nullptr, nullptr, stream);
}

// Reverse sweep from the checkpoints ke_forward left: vbar = g m v_T,
// xbar = 0, then segment by segment (last first) the states recomputed
// forward from the segment's checkpoint onto the tape and the adjoint steps
// walked back over them.
mx_status ke_reverse(const float4 *x0, const float4 *v0, int64_t n, float eps2, float G, float dt, int nsteps,
                     int k, const float *gscale, float4 *gx, float4 *gv, const NbodyWs &w, hipStream_t stream) {
    const int64_t st4 = (int64_t)(align256((size_t)n * 16) / 16);
    const int nck = (nsteps + k - 1) / k;
    int cur = 0;
    hipLaunchKernelGGL(k_adjoint_seed, dim3((unsigned)ceil_div(n, NT)), dim3(NT), 0, stream, w.fin_x, w.fin_v, n,
                       gscale, w.vb[0], w.xb[0]);
    if (mx_status st = last_launch("nbody adjoint seed")) return st;
    for (int c = nck - 1; c >= 0; --c) {
        const int t0 = c * k, t1 = (t0 + k < nsteps) ? t0 + k : nsteps;
        // recompute x_t for t0 <= t < t1 from the checkpoint (tape entry 0 is the checkpoint itself)
        const float4 *tape[kMaxCkptEvery];
        const float4 *rx = c == 0 ? x0 : w.ck_x + (int64_t)c * st4;
        const float4 *rv = c == 0 ? v0 : w.ck_v + (int64_t)c * st4;
        tape[0] = rx;
        for (int t = t0; t < t1 - 1; ++t) {
            float4 *xo = w.tape_x + (int64_t)(t - t0 + 1) * st4, *vo = w.tape_v + (int64_t)(t - t0 + 1) * st4;
            if (mx_status st = step_impl(rx, rv, n, eps2, G, dt, xo, vo, w.pair, stream)) return st;
            rx = xo;
            rv = vo;
            tape[t - t0 + 1] = xo;
        }
        for (int t = t1 - 1; t >= t0; --t) {
            float4 *xbo = (t == 0) ? gx : w.xb[cur ^ 1];
            float4 *vbo = (t == 0) ? gv : w.vb[cur ^ 1];
            if (mx_status st = adjstep_impl(tape[t - t0], w.xb[cur], w.vb[cur], n, eps2, G, dt, xbo, vbo, w.pair,
                                            stream))
                return st;
            cur ^= 1;
        }
    }
    return MX_OK;
}
}  // namespace

mx_status mx_nbody_ke_f32(const float *pos4_dev, const float *vel4_dev, int64_t n, float eps2, float G, float dt,
                          int nsteps, int ckpt_every, float *ke_dev, void *ws, size_t ws_bytes,
                          hipStream_t stream) {
    const char *who = "mx_nbody_ke_f32";
    if (mx_status st = ke_check(who, pos4_dev, vel4_dev, n, eps2, nsteps, ckpt_every, ws, ws_bytes)) return st;
    MX_REQUIRE(ke_dev, MX_ERR_INVALID, "%s: null ke pointer", who);
    if (n == 0) return kinetic_impl(nullptr, nullptr, 0, ke_dev, nullptr, nullptr, stream);
    const int k = ckpt_every < nsteps ? ckpt_every : nsteps;
    NbodyWs w = nbody_ws_layout((char *)ws, n, nsteps, k);
    return ke_forward((const float4 *)pos4_dev, (const float4 *)vel4_dev, n, eps2, G, dt, nsteps, k, ke_dev, w,
                      stream);
}

mx_status mx_nbody_ke_vjp_f32(const float *pos4_dev, const float *vel4_dev, int64_t n, float eps2, float G,
                              float dt, int nsteps, int ckpt_every, const float *gscale_dev, float *gx4_dev,
                              float *gv4_dev, void *ws, size_t ws_bytes, hipStream_t stream) {
    const char *who = "mx_nbody_ke_vjp_f32";
    if (mx_status st = ke_check(who, pos4_dev, vel4_dev, n, eps2, nsteps, ckpt_every, ws, ws_bytes)) return st;
    if (n == 0) return MX_OK;
    MX_REQUIRE(gx4_dev && gv4_dev && a16(gx4_dev) && a16(gv4_dev), MX_ERR_INVALID,
               "%s: null or unaligned gradient pointer", who);
    const int k = ckpt_every < nsteps ? ckpt_every : nsteps;
    NbodyWs w = nbody_ws_layout((char *)ws, n, nsteps, k);
    return ke_reverse((const float4 *)pos4_dev, (const float4 *)vel4_dev, n, eps2, G, dt, nsteps, k, gscale_dev,
                      (float4 *)gx4_dev, (float4 *)gv4_dev, w, stream);
}

mx_status mx_nbody_ke_grad_f32(const float *pos4_dev, const float *vel4_dev, int64_t n, float eps2, float G,
                               float dt, int nsteps, int ckpt_every, float *ke_dev, float *gx4_dev,
                               float *gv4_dev, void *ws, size_t ws_bytes, hipStream_t stream) {
    const char *who = "mx_nbody_ke_grad_f32";
    if (mx_status st = ke_check(who, pos4_dev, vel4_dev, n, eps2, nsteps, ckpt_every, ws, ws_bytes)) return st;
    if (n == 0) return MX_OK;
    MX_REQUIRE(ke_dev && gx4_dev && gv4_dev && a16(gx4_dev) && a16(gv4_dev), MX_ERR_INVALID,
               "%s: null or unaligned pointer", who);
    const int k = ckpt_every < nsteps ? ckpt_every : nsteps;
    NbodyWs w = nbody_ws_layout((char *)ws, n, nsteps, k);
    const float4 *x0 = (const float4 *)pos4_dev, *v0 = (const float4 *)vel4_dev;
    if (mx_status st = ke_forward(x0, v0, n, eps2, G, dt, nsteps, k, ke_dev, w, stream)) return st;
    return ke_reverse(x0, v0, n, eps2, G, dt, nsteps, k, nullptr, (float4 *)gx4_dev, (float4 *)gv4_dev, w, stream);
}

}  // extern "C"
