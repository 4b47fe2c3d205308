// map / map2 (Appendix A) and the elementwise adjoint of the fused dot product.
// Streaming kernels: 16-byte vector loads and stores in a grid-stride loop
// when every pointer is 16-byte aligned, scalar otherwise.
#include "mx_internal.h"

namespace mx {
namespace {

constexpr int NT = 256;

inline bool aligned16(const void *p) { return ((uintptr_t)p & 15) == 0; }

int grid_for(int64_t work_items, const DeviceInfo *d) {
    int64_t g = ceil_div(work_items > 0 ? work_items : 1, NT);
    int64_t cap = (int64_t)d->num_cus * 16;
    return (int)(g < cap ? g : cap);
}

// ---------------------------------------------------------------- map
template <mx_dtype D, int F>
__global__ void __launch_bounds__(NT) k_map(const typename DT<D>::In *__restrict__ x,
                                            typename DT<D>::Acc *__restrict__ out, int64_t n,
                                            typename DT<D>::Acc p0, typename DT<D>::Acc p1,
                                            int vec) {
    using In = typename DT<D>::In;
    using Acc = typename DT<D>::Acc;
    constexpr int V = DT<D>::kVec;
    const int64_t stride = (int64_t)gridDim.x * NT;
    int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (vec) {
        const int64_t nv = n / V;
        const auto *xv = reinterpret_cast<const typename DT<D>::Vec *>(x);
        for (; i < nv; i += stride) {
            auto v = xv[i];
            Acc r[V];
#pragma unroll
            for (int j = 0; j < V; ++j) r[j] = Un<F, Acc>::ap(Acc(vget<decltype(v), In>(v, j)), p0, p1);
            if constexpr (sizeof(Acc) * V == 16) {
                typename DT<D>::Vec o;
                __builtin_memcpy(&o, r, 16);
                if constexpr (std::is_same_v<In, Acc>) reinterpret_cast<typename DT<D>::Vec *>(out)[i] = o;
            }
            if constexpr (!std::is_same_v<In, Acc>) {
                // I32 -> I64: two 16-byte stores
                longlong2 *o2 = reinterpret_cast<longlong2 *>(out) + 2 * i;
                o2[0] = make_longlong2(r[0], r[1]);
                o2[1] = make_longlong2(r[2], r[3]);
            }
        }
        const int64_t t = (int64_t)blockIdx.x * NT + threadIdx.x;
        if (t < n - nv * V) out[nv * V + t] = Un<F, Acc>::ap(Acc(x[nv * V + t]), p0, p1);
    } else {
        for (; i < n; i += stride) out[i] = Un<F, Acc>::ap(Acc(x[i]), p0, p1);
    }
}

// ---------------------------------------------------------------- map2
template <mx_dtype D, int F>
__global__ void __launch_bounds__(NT) k_map2(const typename DT<D>::In *__restrict__ a,
                                             const typename DT<D>::In *__restrict__ b,
                                             typename DT<D>::Acc *out, int64_t n, int vec) {
    using In = typename DT<D>::In;
    using Acc = typename DT<D>::Acc;
    constexpr int V = DT<D>::kVec;
    const int64_t stride = (int64_t)gridDim.x * NT;
    int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (vec) {
        const int64_t nv = n / V;
        const auto *av = reinterpret_cast<const typename DT<D>::Vec *>(a);
        const auto *bv = reinterpret_cast<const typename DT<D>::Vec *>(b);
        for (; i < nv; i += stride) {
            auto va = av[i];
            auto vb = bv[i];
            Acc r[V];
#pragma unroll
            for (int j = 0; j < V; ++j)
                r[j] = Bin<F, Acc>::ap(Acc(vget<decltype(va), In>(va, j)), Acc(vget<decltype(vb), In>(vb, j)));
            if constexpr (std::is_same_v<In, Acc>) {
                typename DT<D>::Vec o;
                __builtin_memcpy(&o, r, 16);
                reinterpret_cast<typename DT<D>::Vec *>(out)[i] = o;
            } else {
                longlong2 *o2 = reinterpret_cast<longlong2 *>(out) + 2 * i;
                o2[0] = make_longlong2(r[0], r[1]);
                o2[1] = make_longlong2(r[2], r[3]);
            }
        }
        const int64_t t = (int64_t)blockIdx.x * NT + threadIdx.x;
        if (t < n - nv * V) out[nv * V + t] = Bin<F, Acc>::ap(Acc(a[nv * V + t]), Acc(b[nv * V + t]));
    } else {
        for (; i < n; i += stride) out[i] = Bin<F, Acc>::ap(Acc(a[i]), Acc(b[i]));
    }
}

// ---------------------------------------------------------------- dot adjoint
__global__ void __launch_bounds__(NT) k_dot_adjoint(const float *__restrict__ a,
                                                    const float *__restrict__ b, int64_t n,
                                                    const float *__restrict__ gout,
                                                    float *__restrict__ ga,
                                                    float *__restrict__ gb, int vec) {
    const float g = gout[0];
    const int64_t stride = (int64_t)gridDim.x * NT;
    int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (vec) {
        const int64_t nv = n / 4;
        for (; i < nv; i += stride) {
            if (ga) {
                float4 v = reinterpret_cast<const float4 *>(b)[i];
                reinterpret_cast<float4 *>(ga)[i] = make_float4(g * v.x, g * v.y, g * v.z, g * v.w);
            }
            if (gb) {
                float4 v = reinterpret_cast<const float4 *>(a)[i];
                reinterpret_cast<float4 *>(gb)[i] = make_float4(g * v.x, g * v.y, g * v.z, g * v.w);
            }
        }
        const int64_t t = (int64_t)blockIdx.x * NT + threadIdx.x;
        if (t < n - nv * 4) {
            if (ga) ga[nv * 4 + t] = g * b[nv * 4 + t];
            if (gb) gb[nv * 4 + t] = g * a[nv * 4 + t];
        }
    } else {
        for (; i < n; i += stride) {
            if (ga) ga[i] = g * b[i];
            if (gb) gb[i] = g * a[i];
        }
    }
}

// ---------------------------------------------------------------- dispatch
template <mx_dtype D>
mx_status launch_map(int f, const void *x, int64_t n, const void *params, void *out, hipStream_t s,
                     const DeviceInfo *dev) {
    using In = typename DT<D>::In;
    using Acc = typename DT<D>::Acc;
    Acc p0 = Acc(0), p1 = Acc(0);
    if (params) {
        __builtin_memcpy(&p0, params, sizeof(Acc));
        __builtin_memcpy(&p1, (const char *)params + sizeof(Acc), sizeof(Acc));
    }
    const int vec = aligned16(x) && aligned16(out);
    const int grid = grid_for(vec ? n / DT<D>::kVec : n, dev);
    const In *xi = (const In *)x;
    Acc *o = (Acc *)out;
#define MX_MAPCASE(F)                                                                       \
    case F:                                                                                 \
        hipLaunchKernelGGL((k_map<D, F>), dim3(grid), dim3(NT), 0, s, xi, o, n, p0, p1, vec); \
        break;
    switch (f) {
        MX_MAPCASE(MX_U_ID)
        MX_MAPCASE(MX_U_NEG)
        MX_MAPCASE(MX_U_ABS)
        MX_MAPCASE(MX_U_SQ)
        MX_MAPCASE(MX_U_AFFINE)
    default:
        if constexpr (D == MX_F32 || D == MX_F64) {
            switch (f) {
                MX_MAPCASE(MX_U_EXP)
                MX_MAPCASE(MX_U_LOG)
                MX_MAPCASE(MX_U_SQRT)
                MX_MAPCASE(MX_U_RSQRT)
            default:
                return set_error(MX_ERR_INVALID, "mx_map: unknown map body %d", f);
            }
        } else {
            return set_error(MX_ERR_DTYPE, "mx_map: body %d needs a floating-point type", f);
        }
    }
#undef MX_MAPCASE
    return last_launch("mx_map");
}

template <mx_dtype D>
mx_status launch_map2(int f, const void *a, const void *b, int64_t n, void *out, hipStream_t s,
                      const DeviceInfo *dev) {
    using In = typename DT<D>::In;
    using Acc = typename DT<D>::Acc;
    const int vec = aligned16(a) && aligned16(b) && aligned16(out);
    const int grid = grid_for(vec ? n / DT<D>::kVec : n, dev);
    const In *ai = (const In *)a, *bi = (const In *)b;
    Acc *o = (Acc *)out;
#define MX_MAP2CASE(F)                                                                   \
    case F:                                                                              \
        hipLaunchKernelGGL((k_map2<D, F>), dim3(grid), dim3(NT), 0, s, ai, bi, o, n, vec); \
        break;
    switch (f) {
        MX_MAP2CASE(MX_B_ADD)
        MX_MAP2CASE(MX_B_SUB)
        MX_MAP2CASE(MX_B_MUL)
        MX_MAP2CASE(MX_B_MIN)
        MX_MAP2CASE(MX_B_MAX)
    case MX_B_DIV:
        if constexpr (D == MX_F32 || D == MX_F64) {
            hipLaunchKernelGGL((k_map2<D, MX_B_DIV>), dim3(grid), dim3(NT), 0, s, ai, bi, o, n, vec);
            break;
        } else {
            return set_error(MX_ERR_DTYPE, "mx_map2: division needs a floating-point type");
        }
    default:
        return set_error(MX_ERR_INVALID, "mx_map2: unknown map2 body %d", f);
    }
#undef MX_MAP2CASE
    return last_launch("mx_map2");
}

}  // namespace
}  // namespace mx

using namespace mx;

extern "C" {

mx_status mx_map(mx_unop f, mx_dtype dtype, const void *x_dev, int64_t n, const void *params_host,
                 void *out_dev, hipStream_t stream) {
    MX_REQUIRE(n >= 0, MX_ERR_SHAPE, "mx_map: n < 0");
    MX_REQUIRE(dtype_valid(dtype), MX_ERR_DTYPE, "mx_map: bad dtype %d", (int)dtype);
    MX_REQUIRE((int)f >= 0 && (int)f <= MX_U_RSQRT, MX_ERR_INVALID, "mx_map: unknown body %d", (int)f);
    MX_REQUIRE(f != MX_U_AFFINE || params_host, MX_ERR_INVALID, "mx_map: AFFINE needs params");
    if (!is_float(dtype) && f >= MX_U_EXP)
        return set_error(MX_ERR_DTYPE, "mx_map: body %d needs a floating-point type", (int)f);
    if (n == 0) return MX_OK;
    MX_REQUIRE(x_dev && out_dev, MX_ERR_INVALID, "mx_map: null pointer");
    const DeviceInfo *d;
    if (mx_status st = device_info(&d)) return st;
    switch (dtype) {
    case MX_F32: return launch_map<MX_F32>(f, x_dev, n, params_host, out_dev, stream, d);
    case MX_F64: return launch_map<MX_F64>(f, x_dev, n, params_host, out_dev, stream, d);
    case MX_I32: return launch_map<MX_I32>(f, x_dev, n, params_host, out_dev, stream, d);
    case MX_I64: return launch_map<MX_I64>(f, x_dev, n, params_host, out_dev, stream, d);
    }
    return MX_ERR_DTYPE;
}

mx_status mx_map2(mx_binop f, mx_dtype dtype, const void *a_dev, const void *b_dev, int64_t n,
                  void *out_dev, hipStream_t stream) {
    MX_REQUIRE(n >= 0, MX_ERR_SHAPE, "mx_map2: n < 0");
    MX_REQUIRE(dtype_valid(dtype), MX_ERR_DTYPE, "mx_map2: bad dtype %d", (int)dtype);
    MX_REQUIRE((int)f >= 0 && (int)f <= MX_B_MAX, MX_ERR_INVALID, "mx_map2: unknown body %d", (int)f);
    if (!is_float(dtype) && f == MX_B_DIV)
        return set_error(MX_ERR_DTYPE, "mx_map2: division needs a floating-point type");
    if (n == 0) return MX_OK;
    MX_REQUIRE(a_dev && b_dev && out_dev, MX_ERR_INVALID, "mx_map2: null pointer");
    const DeviceInfo *d;
    if (mx_status st = device_info(&d)) return st;
    switch (dtype) {
    case MX_F32: return launch_map2<MX_F32>(f, a_dev, b_dev, n, out_dev, stream, d);
    case MX_F64: return launch_map2<MX_F64>(f, a_dev, b_dev, n, out_dev, stream, d);
    case MX_I32: return launch_map2<MX_I32>(f, a_dev, b_dev, n, out_dev, stream, d);
    case MX_I64: return launch_map2<MX_I64>(f, a_dev, b_dev, n, out_dev, stream, d);
    }
    return MX_ERR_DTYPE;
}

mx_status mx_dot_adjoint_f32(const float *a_dev, const float *b_dev, int64_t n,
                             const float *gout_dev, float *ga_dev, float *gb_dev,
                             hipStream_t stream) {
    MX_REQUIRE(n >= 0, MX_ERR_SHAPE, "mx_dot_adjoint_f32: n < 0");
    if (n == 0) return MX_OK;
    MX_REQUIRE(gout_dev, MX_ERR_INVALID, "mx_dot_adjoint_f32: null gout");
    MX_REQUIRE(!ga_dev || b_dev, MX_ERR_INVALID, "mx_dot_adjoint_f32: ga needs b");
    MX_REQUIRE(!gb_dev || a_dev, MX_ERR_INVALID, "mx_dot_adjoint_f32: gb needs a");
    if (!ga_dev && !gb_dev) return MX_OK;
    const DeviceInfo *d;
    if (mx_status st = device_info(&d)) return st;
    const int vec = (!ga_dev || (aligned16(ga_dev) && aligned16(b_dev))) &&
                    (!gb_dev || (aligned16(gb_dev) && aligned16(a_dev)));
    const int grid = grid_for(vec ? n / 4 : n, d);
    hipLaunchKernelGGL(k_dot_adjoint, dim3(grid), dim3(NT), 0, stream, a_dev, b_dev, n, gout_dev,
                       ga_dev, gb_dev, vec);
    return last_launch("mx_dot_adjoint_f32");
}

}  // extern "C"
