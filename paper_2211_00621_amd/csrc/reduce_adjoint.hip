// Reverse of reduce min / max, flat and per ragged row (derived; the paper
// has no reverse mode).  reduce op ne s is the left fold of op from ne, and
// min / max replace the accumulator only when an element is strictly below
// (above) it, so the result is the element at the lowest index attaining the
// extreme, or ne itself when no element improves on ne.  That element
// receives the upstream gradient; every other element receives 0.
//
// The index is found as the lexicographic best of (value, index) pairs --
// smallest (largest) value first, then lowest index -- with ne standing at
// index -1: an associative and commutative operation, so the tree order of
// the reduction does not change the result: the arg is exact and
// deterministic.  A NaN element never compares below or equal to anything,
// so it is never chosen, as in the fold.
#include "mx_internal.h"

namespace mx {
namespace {

constexpr int NT = 256;
constexpr int kMaxArgBlocks = 2048;  // partial pairs fit MX_WS_REDUCE's 32 KiB
constexpr int64_t kNone = INT64_MAX;

inline bool aligned16(const void *p) { return ((uintptr_t)p & 15) == 0; }

// (v, i) improves on (bv, bi): strictly better value, or the same value at a
// lower index
template <int OP>
__device__ __forceinline__ bool better(float v, int64_t i, float bv, int64_t bi) {
    if (OP == MX_MIN) return v < bv || (v == bv && i < bi);
    return v > bv || (v == bv && i < bi);
}

template <int OP> __device__ __forceinline__ float ident() {
    return OP == MX_MIN ? __builtin_huge_valf() : -__builtin_huge_valf();
}

template <int OP> __device__ __forceinline__ void take(float v, int64_t i, float &bv, int64_t &bi) {
    if (better<OP>(v, i, bv, bi)) {
        bv = v;
        bi = i;
    }
}

template <int OP> __device__ __forceinline__ void wave_argreduce(float &bv, int64_t &bi) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        const float ov = __shfl_xor(bv, off, kWave);
        const int64_t oi = __shfl_xor(bi, off, kWave);
        take<OP>(ov, oi, bv, bi);
    }
}

// all threads of the block; the block's pair in every thread
template <int OP> __device__ __forceinline__ void block_argreduce(float &bv, int64_t &bi) {
    __shared__ float sv[NT / kWave];
    __shared__ int64_t si[NT / kWave];
    wave_argreduce<OP>(bv, bi);
    const int w = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0) {
        sv[w] = bv;
        si[w] = bi;
    }
    __syncthreads();
    bv = sv[0];
    bi = si[0];
#pragma unroll
    for (int k = 1; k < NT / kWave; ++k) take<OP>(sv[k], si[k], bv, bi);
    __syncthreads();
}

// Partial pass: every thread scans a grid-strided set of elements (16-byte
// vectors when x and gx are aligned) for its best pair and writes zeros to
// gx on the way; one pair per block.
template <int OP>
__global__ void __launch_bounds__(NT) k_arg_partial(const float *__restrict__ x, int64_t n, float *__restrict__ gx,
                                                    float *__restrict__ pv, int64_t *__restrict__ pi, int vec) {
    const int64_t tid = (int64_t)blockIdx.x * NT + threadIdx.x, nt = (int64_t)gridDim.x * NT;
    float bv = ident<OP>();
    int64_t bi = kNone;
    int64_t done = 0;
    if (vec) {
        const int64_t nv = n / 4;
        const float4 *xv = reinterpret_cast<const float4 *>(x);
        float4 *gv = reinterpret_cast<float4 *>(gx);
        for (int64_t j = tid; j < nv; j += nt) {
            const float4 q = xv[j];
            take<OP>(q.x, 4 * j, bv, bi);
            take<OP>(q.y, 4 * j + 1, bv, bi);
            take<OP>(q.z, 4 * j + 2, bv, bi);
            take<OP>(q.w, 4 * j + 3, bv, bi);
            gv[j] = make_float4(0.f, 0.f, 0.f, 0.f);
        }
        done = nv * 4;
    }
    for (int64_t i = done + tid; i < n; i += nt) {
        take<OP>(x[i], i, bv, bi);
        gx[i] = 0.f;
    }
    block_argreduce<OP>(bv, bi);
    if (threadIdx.x == 0) {
        pv[blockIdx.x] = bv;
        pi[blockIdx.x] = bi;
    }
}

// Finish (one block): the best of the partials and of (ne, -1); its element
// receives *gout.  Ordered after the partial pass by the kernel boundary, so
// the store lands on the zeros written there.
template <int OP>
__global__ void __launch_bounds__(NT) k_arg_finish(const float *__restrict__ pv, const int64_t *__restrict__ pi,
                                                   int np, float ne, const float *__restrict__ gout,
                                                   float *__restrict__ gx) {
    float bv = ident<OP>();
    int64_t bi = kNone;
    for (int k = threadIdx.x; k < np; k += NT) take<OP>(pv[k], pi[k], bv, bi);
    block_argreduce<OP>(bv, bi);
    if (threadIdx.x == 0) {
        take<OP>(ne, -1, bv, bi);
        // a NaN ne is never improved on by the fold (no comparison with it holds)
        if (bi >= 0 && bi != kNone && ne == ne) gx[bi] = gout[0];
    }
}

// One wave per ragged row (rows grid-strided over the waves): the row's best
// pair, then the row written as g at the arg and 0 elsewhere.
template <int OP>
__global__ void __launch_bounds__(NT) k_seg_arg(const float *__restrict__ values, const int64_t *__restrict__ offsets,
                                                int64_t nseg, float ne, const float *__restrict__ gout,
                                                float *__restrict__ gvalues) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t nw = (int64_t)gridDim.x * (NT / kWave);
    for (int64_t r = (int64_t)blockIdx.x * (NT / kWave) + threadIdx.x / kWave; r < nseg; r += nw) {
        const int64_t s = offsets[r], e = offsets[r + 1];
        float bv = ident<OP>();
        int64_t bi = kNone;
        for (int64_t p = s + lane; p < e; p += kWave) take<OP>(values[p], p, bv, bi);
        wave_argreduce<OP>(bv, bi);
        take<OP>(ne, -1, bv, bi);
        if (ne != ne) bi = -1;  // a NaN ne is never improved on by the fold
        const float g = gout[r];
        for (int64_t p = s + lane; p < e; p += kWave) gvalues[p] = p == bi ? g : 0.f;
    }
}

__global__ void __launch_bounds__(NT) k_fill_from(const float *__restrict__ g, int64_t n, float *__restrict__ out) {
    const float v = g[0];
    const int64_t nt = (int64_t)gridDim.x * NT;
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += nt) out[i] = v;
}

}  // namespace
}  // namespace mx

using namespace mx;

extern "C" {

mx_status mx_reduce_adjoint_f32(mx_redop op, const float *x_dev, int64_t n, const float *ne_host,
                                const float *gout_dev, float *gx_dev, void *ws, size_t ws_bytes, hipStream_t stream) {
    const char *who = "mx_reduce_adjoint_f32";
    MX_REQUIRE(n >= 0, MX_ERR_SHAPE, "%s: n < 0", who);
    MX_REQUIRE(op == MX_ADD || op == MX_MIN || op == MX_MAX,
               op == MX_MUL ? MX_ERR_UNSUPPORTED : MX_ERR_INVALID, "%s: operator %d has no reverse here", who,
               (int)op);
    MX_REQUIRE(ne_host && gout_dev, MX_ERR_INVALID, "%s: null ne or gout", who);
    if (n == 0) return MX_OK;
    MX_REQUIRE(x_dev && gx_dev, MX_ERR_INVALID, "%s: null x or gx", who);
    MX_REQUIRE(gx_dev != x_dev, MX_ERR_INVALID, "%s: gx must not alias x", who);
    const DeviceInfo *d;
    if (mx_status st = device_info(&d)) return st;
    if (op == MX_ADD) {
        int64_t grid = ceil_div(n, NT);
        if (grid > (int64_t)d->num_cus * 8) grid = (int64_t)d->num_cus * 8;
        hipLaunchKernelGGL(k_fill_from, dim3((unsigned)grid), dim3(NT), 0, stream, gout_dev, n, gx_dev);
        return last_launch(who);
    }
    const size_t need = mx_workspace_bytes(MX_WS_REDUCE, n, 0);
    MX_REQUIRE(ws && ws_bytes >= need && ((uintptr_t)ws & 255) == 0, MX_ERR_WORKSPACE,
               "%s: workspace needs %zu bytes, 256-byte aligned", who, need);
    const int vec = aligned16(x_dev) && aligned16(gx_dev);
    const int64_t items = vec ? n / 4 : n;
    int64_t grid = ceil_div(items > 0 ? items : 1, (int64_t)NT * 4);
    int64_t cap = (int64_t)d->num_cus * 8;
    if (cap > kMaxArgBlocks) cap = kMaxArgBlocks;
    if (grid > cap) grid = cap;
    float *pv = (float *)((char *)ws + kCounterBytes);
    int64_t *pi = (int64_t *)((char *)ws + kCounterBytes + kMaxArgBlocks * sizeof(float));
    const float ne = *ne_host;
    if (op == MX_MIN) {
        hipLaunchKernelGGL(k_arg_partial<MX_MIN>, dim3((unsigned)grid), dim3(NT), 0, stream, x_dev, n, gx_dev, pv, pi, vec);
        hipLaunchKernelGGL(k_arg_finish<MX_MIN>, dim3(1), dim3(NT), 0, stream, pv, pi, (int)grid, ne, gout_dev, gx_dev);
    } else {
        hipLaunchKernelGGL(k_arg_partial<MX_MAX>, dim3((unsigned)grid), dim3(NT), 0, stream, x_dev, n, gx_dev, pv, pi, vec);
        hipLaunchKernelGGL(k_arg_finish<MX_MAX>, dim3(1), dim3(NT), 0, stream, pv, pi, (int)grid, ne, gout_dev, gx_dev);
    }
    return last_launch(who);
}

mx_status mx_segmented_reduce_adjoint_f32(mx_redop op, const float *values_dev, int64_t nvalues,
                                          const int64_t *offsets_dev, int64_t nseg, const float *ne_host,
                                          const float *gout_dev, float *gvalues_dev, hipStream_t stream) {
    const char *who = "mx_segmented_reduce_adjoint_f32";
    MX_REQUIRE(nseg >= 0 && nvalues >= 0, MX_ERR_SHAPE, "%s: nseg < 0 or nvalues < 0", who);
    MX_REQUIRE(op == MX_ADD || op == MX_MIN || op == MX_MAX,
               op == MX_MUL ? MX_ERR_UNSUPPORTED : MX_ERR_INVALID, "%s: operator %d has no reverse here", who,
               (int)op);
    MX_REQUIRE(ne_host, MX_ERR_INVALID, "%s: null ne", who);
    if (nseg == 0) return MX_OK;
    MX_REQUIRE(offsets_dev && gout_dev && (gvalues_dev || nvalues == 0), MX_ERR_INVALID, "%s: null pointer", who);
    if (op == MX_ADD) return mx_segmented_sum_adjoint_f32(gout_dev, offsets_dev, nseg, gvalues_dev, nvalues, stream);
    MX_REQUIRE(values_dev, MX_ERR_INVALID, "%s: null values", who);
    MX_REQUIRE(gvalues_dev != values_dev, MX_ERR_INVALID, "%s: gvalues must not alias values", who);
    if (mx_status st = check_offsets_debug(who, offsets_dev, nseg, stream)) return st;
    const DeviceInfo *d;
    if (mx_status st = device_info(&d)) return st;
    int64_t grid = ceil_div(nseg, NT / kWave);
    if (grid > (int64_t)d->num_cus * 16) grid = (int64_t)d->num_cus * 16;
    const float ne = *ne_host;
    if (op == MX_MIN)
        hipLaunchKernelGGL(k_seg_arg<MX_MIN>, dim3((unsigned)grid), dim3(NT), 0, stream, values_dev, offsets_dev, nseg,
                           ne, gout_dev, gvalues_dev);
    else
        hipLaunchKernelGGL(k_seg_arg<MX_MAX>, dim3((unsigned)grid), dim3(NT), 0, stream, values_dev, offsets_dev, nseg,
                           ne, gout_dev, gvalues_dev);
    return last_launch(who);
}

}  // extern "C"
