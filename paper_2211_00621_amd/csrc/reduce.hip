// reduce op ne s and the fused reduce op ne (map2 f a b) (Appendix A).
//
// Two launches.  Partial pass: every thread folds a grid-strided set of 16-byte
// vectors (U per operand in flight) into one accumulator per vector lane, the
// block combines its values with the wave64 DPP tree and writes one partial.
// Finish pass (one block): folds the partials in block order and applies ne.
// The kernel boundary orders the two passes, so no block pays for a
// device-wide fence.  The bracketing depends only on n and the grid, so
// results are bit-identical from run to run.
#include "mx_internal.h"

namespace mx {
namespace {

constexpr int NT = 256;
constexpr int U = 4;
constexpr int kMaxBlocks = 4096;

inline bool aligned16(const void *p) { return ((uintptr_t)p & 15) == 0; }

// F < 0: plain reduce of a; otherwise element = Bin<F>(a[i], b[i]).
template <mx_dtype D, int OP, int F> struct Elem {
    using Acc = typename DT<D>::Acc;
    using In = typename DT<D>::In;
    static __device__ __forceinline__ Acc at(In x, In y) {
        if constexpr (F < 0) return Acc(x);
        else return Bin<F, Acc>::ap(Acc(x), Acc(y));
    }
};

template <mx_dtype D, int OP, int F>
__global__ void __launch_bounds__(NT) k_reduce(const typename DT<D>::In *__restrict__ a,
                                               const typename DT<D>::In *__restrict__ b, int64_t n,
                                               typename DT<D>::Acc *__restrict__ partials, int vec) {
    using In = typename DT<D>::In;
    using Acc = typename DT<D>::Acc;
    using Vec = typename DT<D>::Vec;
    using R = Red<OP, Acc>;
    using E = Elem<D, OP, F>;
    constexpr int V = DT<D>::kVec;
    constexpr bool TWO = F >= 0;
    __shared__ Acc smem[NT / kWave];

    Acc acc[V];
#pragma unroll
    for (int j = 0; j < V; ++j) acc[j] = R::id();
    const int64_t gtid = (int64_t)blockIdx.x * NT + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * NT;
    if (vec) {
        const int64_t nv = n / V;
        const Vec *av = reinterpret_cast<const Vec *>(a);
        const Vec *bv = reinterpret_cast<const Vec *>(b);
        int64_t i = gtid;
        for (; i + (U - 1) * stride < nv; i += U * stride) {
            Vec va[U], vb[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                va[u] = av[i + u * stride];
                if constexpr (TWO) vb[u] = bv[i + u * stride];
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int j = 0; j < V; ++j)
                    acc[j] = R::ap(acc[j], E::at(vget<Vec, In>(va[u], j), TWO ? vget<Vec, In>(vb[u], j) : In(0)));
        }
        for (; i < nv; i += stride) {
            Vec va = av[i];
            Vec vb;
            if constexpr (TWO) vb = bv[i];
#pragma unroll
            for (int j = 0; j < V; ++j)
                acc[j] = R::ap(acc[j], E::at(vget<Vec, In>(va, j), TWO ? vget<Vec, In>(vb, j) : In(0)));
        }
        if (gtid < n - nv * V) acc[0] = R::ap(acc[0], E::at(a[nv * V + gtid], TWO ? b[nv * V + gtid] : In(0)));
    } else {
        for (int64_t i = gtid; i < n; i += stride) acc[0] = R::ap(acc[0], E::at(a[i], TWO ? b[i] : In(0)));
    }
    Acc t = acc[0];
#pragma unroll
    for (int j = 1; j < V; ++j) t = R::ap(t, acc[j]);
    t = block_reduce<R, NT>(t, smem);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

// one block: out = ne (op) (partial_0 (op) ... (op) partial_{nb-1}), strided
// per thread then the DPP tree
template <mx_dtype D, int OP>
__global__ void __launch_bounds__(NT) k_reduce_finish(const typename DT<D>::Acc *__restrict__ partials, int nb,
                                                      typename DT<D>::Acc ne, typename DT<D>::Acc *out) {
    using Acc = typename DT<D>::Acc;
    using R = Red<OP, Acc>;
    __shared__ Acc smem[NT / kWave];
    Acc v = R::id();
    for (int i = threadIdx.x; i < nb; i += NT) v = R::ap(v, partials[i]);
    v = block_reduce<R, NT>(v, smem);
    if (threadIdx.x == 0) out[0] = R::ap(ne, v);
}

template <mx_dtype D, int OP, int F>
mx_status launch(const void *a, const void *b, int64_t n, const void *ne_host, void *out, void *ws,
                 hipStream_t s, const DeviceInfo *dev) {
    using In = typename DT<D>::In;
    using Acc = typename DT<D>::Acc;
    Acc ne;
    __builtin_memcpy(&ne, ne_host, sizeof(Acc));
    const int vec = aligned16(a) && (F < 0 || aligned16(b));
    const int64_t items = vec ? n / DT<D>::kVec : n;
    int64_t grid = ceil_div(items > 0 ? items : 1, (int64_t)NT * U);
    int64_t cap = (int64_t)dev->num_cus * 8;
    if (cap > kMaxBlocks) cap = kMaxBlocks;
    if (grid > cap) grid = cap;
    Acc *partials = (Acc *)((char *)ws + kCounterBytes);
    hipLaunchKernelGGL((k_reduce<D, OP, F>), dim3((unsigned)grid), dim3(NT), 0, s, (const In *)a,
                       (const In *)b, n, partials, vec);
    if (mx_status st = last_launch("reduce")) return st;
    hipLaunchKernelGGL((k_reduce_finish<D, OP>), dim3(1), dim3(NT), 0, s, (const Acc *)partials, (int)grid, ne,
                       (Acc *)out);
    return last_launch("reduce finish");
}

template <mx_dtype D, int F>
mx_status by_op(int op, const void *a, const void *b, int64_t n, const void *ne, void *out, void *ws,
                hipStream_t s, const DeviceInfo *dev) {
    switch (op) {
    case MX_ADD: return launch<D, MX_ADD, F>(a, b, n, ne, out, ws, s, dev);
    case MX_MUL: return launch<D, MX_MUL, F>(a, b, n, ne, out, ws, s, dev);
    case MX_MIN: return launch<D, MX_MIN, F>(a, b, n, ne, out, ws, s, dev);
    case MX_MAX: return launch<D, MX_MAX, F>(a, b, n, ne, out, ws, s, dev);
    }
    return set_error(MX_ERR_INVALID, "unknown reduce operator %d", op);
}

template <mx_dtype D>
mx_status by_f(int f, int op, const void *a, const void *b, int64_t n, const void *ne, void *out,
               void *ws, hipStream_t s, const DeviceInfo *dev) {
    switch (f) {
    case -1: return by_op<D, -1>(op, a, b, n, ne, out, ws, s, dev);
    case MX_B_ADD: return by_op<D, MX_B_ADD>(op, a, b, n, ne, out, ws, s, dev);
    case MX_B_SUB: return by_op<D, MX_B_SUB>(op, a, b, n, ne, out, ws, s, dev);
    case MX_B_MUL: return by_op<D, MX_B_MUL>(op, a, b, n, ne, out, ws, s, dev);
    case MX_B_MIN: return by_op<D, MX_B_MIN>(op, a, b, n, ne, out, ws, s, dev);
    case MX_B_MAX: return by_op<D, MX_B_MAX>(op, a, b, n, ne, out, ws, s, dev);
    case MX_B_DIV:
        if constexpr (D == MX_F32 || D == MX_F64) return by_op<D, MX_B_DIV>(op, a, b, n, ne, out, ws, s, dev);
        else return set_error(MX_ERR_DTYPE, "division needs a floating-point type");
    }
    return set_error(MX_ERR_INVALID, "unknown map2 body %d", f);
}

mx_status run(const char *who, int f, int op, mx_dtype dtype, const void *a, const void *b,
              int64_t n, const void *ne, void *out, void *ws, size_t ws_bytes, hipStream_t s) {
    MX_REQUIRE(n >= 0, MX_ERR_SHAPE, "%s: n < 0", who);
    MX_REQUIRE(dtype_valid(dtype), MX_ERR_DTYPE, "%s: bad dtype %d", who, (int)dtype);
    MX_REQUIRE(op >= MX_ADD && op <= MX_MAX, MX_ERR_INVALID, "%s: unknown operator %d", who, op);
    MX_REQUIRE(f >= -1 && f <= MX_B_MAX, MX_ERR_INVALID, "%s: unknown map2 body %d", who, f);
    MX_REQUIRE(ne && out, MX_ERR_INVALID, "%s: null ne or out", who);
    MX_REQUIRE(n == 0 || (a && (f < 0 || b)), MX_ERR_INVALID, "%s: null input", who);
    MX_REQUIRE(ws && ws_bytes >= mx_workspace_bytes(MX_WS_REDUCE, n, 0), MX_ERR_WORKSPACE,
               "%s: workspace needs %zu bytes", who, mx_workspace_bytes(MX_WS_REDUCE, n, 0));
    MX_REQUIRE(((uintptr_t)ws & 255) == 0, MX_ERR_INVALID, "%s: workspace must be 256-byte aligned", who);
    const DeviceInfo *d;
    if (mx_status st = device_info(&d)) return st;
    switch (dtype) {
    case MX_F32: return by_f<MX_F32>(f, op, a, b, n, ne, out, ws, s, d);
    case MX_F64: return by_f<MX_F64>(f, op, a, b, n, ne, out, ws, s, d);
    case MX_I32: return by_f<MX_I32>(f, op, a, b, n, ne, out, ws, s, d);
    case MX_I64: return by_f<MX_I64>(f, op, a, b, n, ne, out, ws, s, d);
    }
    return MX_ERR_DTYPE;
}

}  // namespace
}  // namespace mx

using namespace mx;

extern "C" {

mx_status mx_reduce(mx_redop op, mx_dtype dtype, const void *x_dev, int64_t n, const void *ne_host,
                    void *out_dev, void *ws, size_t ws_bytes, hipStream_t stream) {
    return run("mx_reduce", -1, op, dtype, x_dev, nullptr, n, ne_host, out_dev, ws, ws_bytes, stream);
}

mx_status mx_map2_reduce(mx_binop f, mx_redop op, mx_dtype dtype, const void *a_dev,
                         const void *b_dev, int64_t n, const void *ne_host, void *out_dev, void *ws,
                         size_t ws_bytes, hipStream_t stream) {
    MX_REQUIRE((int)f >= 0, MX_ERR_INVALID, "mx_map2_reduce: unknown map2 body %d", (int)f);
    return run("mx_map2_reduce", (int)f, op, dtype, a_dev, b_dev, n, ne_host, out_dev, ws, ws_bytes,
               stream);
}

}  // extern "C"
