// Internal helpers shared by the library's translation units (never by the
// oracle): error reporting, device properties, element-type traits, operator
// functors and wave64 / block reductions for gfx950.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <limits>
#include <string>
#include <type_traits>

#include "mx.h"

namespace mx {

// ---------------------------------------------------------------- errors
mx_status set_error(mx_status s, const char *fmt, ...);
mx_status hip_error(hipError_t e, const char *what);
mx_status last_launch(const char *what);  // hipGetLastError after a launch

#define MX_TRY_HIP(call)                                         \
    do {                                                         \
        hipError_t _e = (call);                                  \
        if (_e != hipSuccess) return ::mx::hip_error(_e, #call); \
    } while (0)

#define MX_REQUIRE(cond, status, ...)                      \
    do {                                                   \
        if (!(cond)) return ::mx::set_error(status, __VA_ARGS__); \
    } while (0)

// ---------------------------------------------------------------- device info
struct DeviceInfo {
    int device = -1;
    int num_cus = 256;
    int lds_bytes = 160 * 1024;
    int warp = 64;
};
mx_status device_info(const DeviceInfo **out);  // current device, cached
bool debug_mode();
// block-span segmented reduce: rows per block; check of offsets (debug mode only, else MX_OK)
int segmented_rows_per_block(int64_t nseg, const DeviceInfo *d);
mx_status check_offsets_debug(const char *who, const int64_t *off, int64_t nseg, hipStream_t s);
// bytes of the chunked segmented reduce's workspace for nval values (any dtype)
size_t segmented_ws_bytes(int64_t nval);
// device address of the no-allocation variant's scratch array (per device)
mx_status segmented_scratch(void **out);
// exclusive scan of int64 lengths into nseg + 1 offsets (workspace kind MX_WS_SCAN)
mx_status lengths_to_offsets(const int64_t *len, int64_t nseg, int64_t *off, void *ws, size_t ws_bytes,
                             hipStream_t s);
// bytes of the bucketed histogram's workspace (0: the call takes none)
size_t histogram_ws_bytes(int64_t n, int64_t nbins);
// hipRTC: compiles HIP source for the current device and loads it; modules
// are cached per (device, source) for the life of the process
mx_status rtc_module(const std::string &src, const char *name, hipModule_t *out);

constexpr int kWave = 64;

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// ---------------------------------------------------------------- workspace layout
// Every workspace starts with a 256-byte block of counters that the kernels
// leave at zero; partial results follow.
constexpr size_t kCounterBytes = 256;

// ---------------------------------------------------------------- type traits
template <mx_dtype D> struct DT;
template <> struct DT<MX_F32> { using In = float; using Acc = float; using Vec = float4; static constexpr int kVec = 4; };
template <> struct DT<MX_F64> { using In = double; using Acc = double; using Vec = double2; static constexpr int kVec = 2; };
template <> struct DT<MX_I32> { using In = int32_t; using Acc = int64_t; using Vec = int4; static constexpr int kVec = 4; };
template <> struct DT<MX_I64> { using In = int64_t; using Acc = int64_t; using Vec = longlong2; static constexpr int kVec = 2; };

inline size_t dtype_size(mx_dtype d) { return (d == MX_F32 || d == MX_I32) ? 4 : 8; }
inline size_t acc_size(mx_dtype d) { return d == MX_F32 ? 4 : 8; }
inline bool dtype_valid(int d) { return d >= MX_F32 && d <= MX_I64; }
inline bool is_float(mx_dtype d) { return d == MX_F32 || d == MX_F64; }

// element i of a 16-byte vector
template <class V, class T> __device__ __forceinline__ T vget(const V &v, int i) {
    return reinterpret_cast<const T *>(&v)[i];
}

// ---------------------------------------------------------------- integer wrap helpers
template <class T> __host__ __device__ __forceinline__ T wadd(T a, T b) {
    if constexpr (std::is_integral_v<T>) {
        using U = std::make_unsigned_t<T>;
        return T(U(a) + U(b));
    } else {
        return a + b;
    }
}
template <class T> __host__ __device__ __forceinline__ T wsub(T a, T b) {
    if constexpr (std::is_integral_v<T>) {
        using U = std::make_unsigned_t<T>;
        return T(U(a) - U(b));
    } else {
        return a - b;
    }
}
template <class T> __host__ __device__ __forceinline__ T wmul(T a, T b) {
    if constexpr (std::is_integral_v<T>) {
        using U = std::make_unsigned_t<T>;
        return T(U(a) * U(b));
    } else {
        return a * b;
    }
}

// ---------------------------------------------------------------- reduce operators
template <int OP, class T> struct Red;
template <class T> struct Red<MX_ADD, T> {
    static __host__ __device__ __forceinline__ T id() { return T(0); }
    static __host__ __device__ __forceinline__ T ap(T a, T b) { return wadd(a, b); }
};
template <class T> struct Red<MX_MUL, T> {
    static __host__ __device__ __forceinline__ T id() { return T(1); }
    static __host__ __device__ __forceinline__ T ap(T a, T b) { return wmul(a, b); }
};
template <class T> struct Red<MX_MIN, T> {
    static __host__ __device__ __forceinline__ T id() {
        if constexpr (std::is_integral_v<T>) return std::numeric_limits<T>::max();
        else return std::numeric_limits<T>::infinity();
    }
    static __host__ __device__ __forceinline__ T ap(T a, T b) { return b < a ? b : a; }
};
template <class T> struct Red<MX_MAX, T> {
    static __host__ __device__ __forceinline__ T id() {
        if constexpr (std::is_integral_v<T>) return std::numeric_limits<T>::lowest();
        else return -std::numeric_limits<T>::infinity();
    }
    static __host__ __device__ __forceinline__ T ap(T a, T b) { return b > a ? b : a; }
};

// ---------------------------------------------------------------- uncontracted arithmetic
// hipcc fuses a multiply and a dependent add into one FMA by default, and the
// __fmul_rn family are plain operators in HIP, so they are fused as well.
// These helpers carry no contraction permission: every result is rounded on
// its own, as in the binary64 / binary32 definition of the operation.
template <class T> __device__ __forceinline__ T mul_rn(T a, T b) {
#pragma clang fp contract(off)
    return a * b;
}
template <class T> __device__ __forceinline__ T add_rn(T a, T b) {
#pragma clang fp contract(off)
    return a + b;
}
template <class T> __device__ __forceinline__ T sub_rn(T a, T b) {
#pragma clang fp contract(off)
    return a - b;
}

// ---------------------------------------------------------------- map bodies
template <int F, class T> struct Un;
template <class T> struct Un<MX_U_ID, T> { static __device__ __forceinline__ T ap(T x, T, T) { return x; } };
template <class T> struct Un<MX_U_NEG, T> { static __device__ __forceinline__ T ap(T x, T, T) { return wsub(T(0), x); } };
template <class T> struct Un<MX_U_ABS, T> { static __device__ __forceinline__ T ap(T x, T, T) { return x < T(0) ? wsub(T(0), x) : x; } };
template <class T> struct Un<MX_U_SQ, T> { static __device__ __forceinline__ T ap(T x, T, T) { return wmul(x, x); } };
template <class T> struct Un<MX_U_AFFINE, T> {
    // two roundings (multiply, then add), never contracted into an FMA
    static __device__ __forceinline__ T ap(T x, T p0, T p1) {
        if constexpr (std::is_floating_point_v<T>) return add_rn(mul_rn(p0, x), p1);
        else return wadd(wmul(p0, x), p1);
    }
};
template <class T> struct Un<MX_U_EXP, T> { static __device__ __forceinline__ T ap(T x, T, T) { return exp(x); } };
template <class T> struct Un<MX_U_LOG, T> { static __device__ __forceinline__ T ap(T x, T, T) { return log(x); } };
template <class T> struct Un<MX_U_SQRT, T> { static __device__ __forceinline__ T ap(T x, T, T) { return sqrt(x); } };
template <class T> struct Un<MX_U_RSQRT, T> { static __device__ __forceinline__ T ap(T x, T, T) { return T(1) / sqrt(x); } };

template <int F, class T> struct Bin;
template <class T> struct Bin<MX_B_ADD, T> { static __device__ __forceinline__ T ap(T a, T b) { return wadd(a, b); } };
template <class T> struct Bin<MX_B_SUB, T> { static __device__ __forceinline__ T ap(T a, T b) { return wsub(a, b); } };
template <class T> struct Bin<MX_B_MUL, T> { static __device__ __forceinline__ T ap(T a, T b) { return wmul(a, b); } };
template <class T> struct Bin<MX_B_DIV, T> { static __device__ __forceinline__ T ap(T a, T b) { return a / b; } };
template <class T> struct Bin<MX_B_MIN, T> { static __device__ __forceinline__ T ap(T a, T b) { return b < a ? b : a; } };
template <class T> struct Bin<MX_B_MAX, T> { static __device__ __forceinline__ T ap(T a, T b) { return b > a ? b : a; } };

// ---------------------------------------------------------------- wave64 DPP reduction
// Cross-lane data movement with DPP (data-parallel primitives of the VALU):
// quad permutations, row mirrors and the GFX9 row broadcasts.  Lanes that a
// row mask disables receive `ident`.
template <int CTRL, int ROW_MASK, class T>
__device__ __forceinline__ T dpp_move(T v, T ident) {
    static_assert(sizeof(T) == 4 || sizeof(T) == 8, "32- or 64-bit values only");
    if constexpr (sizeof(T) == 4) {
        int vi, ii;
        __builtin_memcpy(&vi, &v, 4);
        __builtin_memcpy(&ii, &ident, 4);
        int r = __builtin_amdgcn_update_dpp(ii, vi, CTRL, ROW_MASK, 0xF, false);
        T out;
        __builtin_memcpy(&out, &r, 4);
        return out;
    } else {
        int vi[2], ii[2], r[2];
        __builtin_memcpy(vi, &v, 8);
        __builtin_memcpy(ii, &ident, 8);
        r[0] = __builtin_amdgcn_update_dpp(ii[0], vi[0], CTRL, ROW_MASK, 0xF, false);
        r[1] = __builtin_amdgcn_update_dpp(ii[1], vi[1], CTRL, ROW_MASK, 0xF, false);
        T out;
        __builtin_memcpy(&out, r, 8);
        return out;
    }
}

template <class T> __device__ __forceinline__ T read_lane(T v, int lane) {
    if constexpr (sizeof(T) == 4) {
        int vi;
        __builtin_memcpy(&vi, &v, 4);
        int r = __builtin_amdgcn_readlane(vi, lane);
        T out;
        __builtin_memcpy(&out, &r, 4);
        return out;
    } else {
        int vi[2], r[2];
        __builtin_memcpy(vi, &v, 8);
        r[0] = __builtin_amdgcn_readlane(vi[0], lane);
        r[1] = __builtin_amdgcn_readlane(vi[1], lane);
        T out;
        __builtin_memcpy(&out, r, 8);
        return out;
    }
}

// Reduction of one value per lane over the full wave64 with a fixed tree:
// pairs, quads, half rows, rows (16 lanes), then rows 0+1 and 2+3 through the
// row broadcasts; the total ends in lane 63 and is broadcast to all lanes.
// Must be called with all 64 lanes active.
template <class Op, class T> __device__ __forceinline__ T wave_reduce(T v) {
    const T id = Op::id();
    v = Op::ap(v, dpp_move<0xB1, 0xF>(v, id));   // quad_perm [1,0,3,2]
    v = Op::ap(v, dpp_move<0x4E, 0xF>(v, id));   // quad_perm [2,3,0,1]
    v = Op::ap(v, dpp_move<0x141, 0xF>(v, id));  // row_half_mirror
    v = Op::ap(v, dpp_move<0x140, 0xF>(v, id));  // row_mirror
    v = Op::ap(v, dpp_move<0x142, 0xA>(v, id));  // row_bcast:15 into rows 1, 3
    v = Op::ap(v, dpp_move<0x143, 0xC>(v, id));  // row_bcast:31 into rows 2, 3
    return read_lane(v, 63);
}

// Block reduction for NT threads (a multiple of 64); result valid in every
// thread.  smem must hold NT/64 values.
template <class Op, int NT, class T> __device__ __forceinline__ T block_reduce(T v, T *smem) {
    constexpr int NW = NT / kWave;
    T w = wave_reduce<Op>(v);
    const int wave = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0) smem[wave] = w;
    __syncthreads();
    T r = smem[0];
#pragma unroll
    for (int i = 1; i < NW; ++i) r = Op::ap(r, smem[i]);
    __syncthreads();
    return r;
}

}  // namespace mx
