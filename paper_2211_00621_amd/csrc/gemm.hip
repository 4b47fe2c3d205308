// Dense nested map (map (reduce (+) 0 (map2 (*) row col))): FP32 matrix
// product on the CDNA matrix cores (v_mfma_f32_16x16x4_f32), FP32 accumulate.
//
// Block tile 128 x 128, K-slice 32, 256 threads = 4 waves in a 2 x 2 grid,
// each wave owning a 64 x 64 sub-tile as 4 x 4 MFMA blocks of 16 x 16 (64
// accumulator registers per lane).  Both operand tiles live in LDS with k
// contiguous ([row][k], row stride 36 floats), double-buffered with one
// barrier per K-slice; the next slice's global loads are issued before the
// current slice's MFMAs.
//
// The reduction over k is associative, so the k values of a slice may be
// dealt to the MFMA steps in any order as long as A and B agree: lane group
// g = lane / 16 takes k = 8g .. 8g+7 for steps 0 .. 7, which makes each lane's
// eight A (and B) values contiguous in LDS and readable with two 16-byte loads.
#include "mx_internal.h"

namespace mx {
namespace {

constexpr int BM = 128, BN = 128, BK = 32, NT = 256;
constexpr int LDK = BK + 4;  // LDS row stride in floats ([row][k] tiles)
constexpr int kGroupM = 4;   // tile rows per scheduling group

typedef float v4f __attribute__((ext_vector_type(4)));

// Element (r, c) of a row-major R x C matrix with leading dimension ld, as
// a float4 of columns c .. c+3, zero outside the matrix.
__device__ __forceinline__ float4 ld4(const float *__restrict__ p, int64_t ld, int64_t r, int64_t c,
                                      int64_t R, int64_t C, bool fast) {
    if (fast) return *reinterpret_cast<const float4 *>(p + r * ld + c);
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (r < R) {
        const float *q = p + r * ld;
        if (c + 0 < C) v.x = q[c + 0];
        if (c + 1 < C) v.y = q[c + 1];
        if (c + 2 < C) v.z = q[c + 2];
        if (c + 3 < C) v.w = q[c + 3];
    }
    return v;
}

// Loads one K-slice of an operand into 4 float4 registers per thread.
// ROWK: the operand is stored [row][k] (k contiguous) -- A with ta = 0, B with
// tb = 1; otherwise it is stored [k][row] (row contiguous).
template <bool ROWK>
__device__ __forceinline__ void load_slice(float4 (&r)[4], const float *__restrict__ p, int64_t ld,
                                           int64_t row0, int64_t k0, int64_t rows, int64_t K,
                                           bool fast) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int idx = threadIdx.x + NT * i;
        if constexpr (ROWK) {
            const int row = idx >> 3, kq = idx & 7;  // 128 rows x 8 quads of k
            r[i] = ld4(p, ld, row0 + row, k0 + 4 * kq, rows, K, fast);
        } else {
            const int k = idx >> 5, rq = idx & 31;  // 32 k x 32 quads of rows
            r[i] = ld4(p, ld, k0 + k, row0 + 4 * rq, K, rows, fast);
        }
    }
}

template <bool ROWK>
__device__ __forceinline__ void store_slice(float *__restrict__ s, const float4 (&r)[4]) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int idx = threadIdx.x + NT * i;
        if constexpr (ROWK) {
            const int row = idx >> 3, kq = idx & 7;
            *reinterpret_cast<float4 *>(s + row * LDK + 4 * kq) = r[i];
        } else {
            const int k = idx >> 5, rq = idx & 31;
            s[(4 * rq + 0) * LDK + k] = r[i].x;
            s[(4 * rq + 1) * LDK + k] = r[i].y;
            s[(4 * rq + 2) * LDK + k] = r[i].z;
            s[(4 * rq + 3) * LDK + k] = r[i].w;
        }
    }
}

// Tile scheduling: consecutive blocks land on different XCDs (round robin over
// 8), so blocks b, b+8, b+16, ... share an L2.  Give each XCD a contiguous
// range of logical tiles, and walk logical tiles in groups of kGroupM tile rows
// so that neighbouring tiles reuse the same A row panels and B column panels.
__device__ __forceinline__ void tile_of(int b, int tiles_m, int tiles_n, int &tm, int &tn) {
    const int nt = tiles_m * tiles_n;
    int L = b;
    if ((nt & 7) == 0) L = (b & 7) * (nt >> 3) + (b >> 3);
    const int per_group = kGroupM * tiles_n;
    const int g = L / per_group;
    const int first_m = g * kGroupM;
    const int gm = min(tiles_m - first_m, kGroupM);
    const int in = L - g * per_group;
    tm = first_m + in % gm;
    tn = in / gm;
}

template <int TA, int TB>
__global__ void __launch_bounds__(NT) k_gemm_mfma(const float *__restrict__ A,
                                                  const float *__restrict__ B, float *__restrict__ C,
                                                  int64_t M, int64_t N, int64_t K, int tiles_m,
                                                  int tiles_n, int vec_ok) {
    __shared__ __attribute__((aligned(16))) float As[2][BM * LDK];
    __shared__ __attribute__((aligned(16))) float Bs[2][BN * LDK];

    int tm, tn;
    tile_of(blockIdx.x, tiles_m, tiles_n, tm, tn);
    const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int l16 = lane & 15, g = lane >> 4;

    const int64_t lda = TA ? M : K;
    const int64_t ldb = TB ? K : N;
    const bool interior = vec_ok && (m0 + BM <= M) && (n0 + BN <= N);
    const int nk = (int)((K + BK - 1) / BK);

    v4f acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};

    float4 ra[4], rb[4];
    {
        const bool fast = interior && (BK <= K);
        load_slice<!TA>(ra, A, lda, m0, 0, M, K, fast);
        load_slice<(bool)TB>(rb, B, ldb, n0, 0, N, K, fast);
        store_slice<!TA>(As[0], ra);
        store_slice<(bool)TB>(Bs[0], rb);
    }
    __syncthreads();

    for (int kt = 0; kt < nk; ++kt) {
        const int buf = kt & 1;
        const bool more = kt + 1 < nk;
        if (more) {
            const int64_t k0 = (int64_t)(kt + 1) * BK;
            const bool fast = interior && (k0 + BK <= K);
            load_slice<!TA>(ra, A, lda, m0, k0, M, K, fast);
            load_slice<(bool)TB>(rb, B, ldb, n0, k0, N, K, fast);
        }
        const float *as = As[buf] + (wm * 64 + l16) * LDK + 8 * g;
        const float *bs = Bs[buf] + (wn * 64 + l16) * LDK + 8 * g;
        float4 a0[4], a1[4], b0[4], b1[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            a0[i] = *reinterpret_cast<const float4 *>(as + i * 16 * LDK);
            a1[i] = *reinterpret_cast<const float4 *>(as + i * 16 * LDK + 4);
            b0[i] = *reinterpret_cast<const float4 *>(bs + i * 16 * LDK);
            b1[i] = *reinterpret_cast<const float4 *>(bs + i * 16 * LDK + 4);
        }
#pragma unroll
        for (int kk = 0; kk < 8; ++kk) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float av = kk < 4 ? vget<float4, float>(a0[i], kk) : vget<float4, float>(a1[i], kk - 4);
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const float bv = kk < 4 ? vget<float4, float>(b0[j], kk) : vget<float4, float>(b1[j], kk - 4);
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc[i][j], 0, 0, 0);
                }
            }
        }
        if (more) {
            store_slice<!TA>(As[buf ^ 1], ra);
            store_slice<(bool)TB>(Bs[buf ^ 1], rb);
        }
        __syncthreads();
    }

    // D block (i, j): lane holds rows 4g .. 4g+3 of column l16
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t col = n0 + wn * 64 + j * 16 + l16;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = m0 + wm * 64 + i * 16 + 4 * g + r;
                if (interior || (row < M && col < N)) C[row * N + col] = acc[i][j][r];
            }
        }
    }
}

// Plain form: one thread per output element, k loop over global memory.
template <int TA, int TB>
__global__ void __launch_bounds__(256) k_gemm_plain(const float *__restrict__ A,
                                                    const float *__restrict__ B,
                                                    float *__restrict__ C, int64_t M, int64_t N,
                                                    int64_t K) {
    const int64_t j = (int64_t)blockIdx.x * 16 + (threadIdx.x & 15);
    const int64_t i = (int64_t)blockIdx.y * 16 + (threadIdx.x >> 4);
    if (i >= M || j >= N) return;
    float acc = 0.f;
    for (int64_t k = 0; k < K; ++k) {
        const float a = TA ? A[k * M + i] : A[i * K + k];
        const float b = TB ? B[j * K + k] : B[k * N + j];
        acc += a * b;
    }
    C[i * N + j] = acc;
}

mx_status check(const char *who, int ta, int tb, int64_t M, int64_t N, int64_t K, const float *A,
                const float *B, float *C) {
    MX_REQUIRE((ta == 0 || ta == 1) && (tb == 0 || tb == 1), MX_ERR_INVALID, "%s: ta, tb must be 0 or 1", who);
    MX_REQUIRE(M >= 0 && N >= 0 && K >= 0, MX_ERR_SHAPE, "%s: negative size", who);
    MX_REQUIRE(M == 0 || N == 0 || C, MX_ERR_INVALID, "%s: null C", who);
    MX_REQUIRE(M == 0 || N == 0 || K == 0 || (A && B), MX_ERR_INVALID, "%s: null A or B", who);
    MX_REQUIRE(M < (1LL << 31) && N < (1LL << 31), MX_ERR_SHAPE, "%s: M, N must be below 2^31", who);
    return MX_OK;
}

}  // namespace
}  // namespace mx

using namespace mx;

extern "C" {

mx_status mx_map_map_reduce_f32(int ta, int tb, int64_t M, int64_t N, int64_t K, const float *A_dev,
                                const float *B_dev, float *C_dev, hipStream_t stream) {
    if (mx_status st = check("mx_map_map_reduce_f32", ta, tb, M, N, K, A_dev, B_dev, C_dev)) return st;
    if (M == 0 || N == 0) return MX_OK;
    const DeviceInfo *d;
    if (mx_status st = device_info(&d)) return st;
    const int64_t tiles_m = ceil_div(M, BM), tiles_n = ceil_div(N, BN);
    MX_REQUIRE(tiles_m * tiles_n < (1LL << 31), MX_ERR_SHAPE, "mx_map_map_reduce_f32: too many tiles");
    const int64_t lda = ta ? M : K, ldb = tb ? K : N;
    const int vec_ok = ((uintptr_t)A_dev % 16 == 0) && ((uintptr_t)B_dev % 16 == 0) && (lda % 4 == 0) &&
                       (ldb % 4 == 0);
    const dim3 grid((unsigned)(tiles_m * tiles_n));
#define MX_GEMM(TA, TB)                                                                              \
    hipLaunchKernelGGL((k_gemm_mfma<TA, TB>), grid, dim3(NT), 0, stream, A_dev, B_dev, C_dev, M, N, \
                       K, (int)tiles_m, (int)tiles_n, vec_ok)
    if (!ta && !tb) MX_GEMM(0, 0);
    else if (!ta && tb) MX_GEMM(0, 1);
    else if (ta && !tb) MX_GEMM(1, 0);
    else MX_GEMM(1, 1);
#undef MX_GEMM
    return last_launch("mx_map_map_reduce_f32");
}

mx_status mx_map_map_reduce_plain_f32(int ta, int tb, int64_t M, int64_t N, int64_t K,
                                      const float *A_dev, const float *B_dev, float *C_dev,
                                      hipStream_t stream) {
    if (mx_status st = check("mx_map_map_reduce_plain_f32", ta, tb, M, N, K, A_dev, B_dev, C_dev)) return st;
    if (M == 0 || N == 0) return MX_OK;
    MX_REQUIRE(ceil_div(M, 16) < 65536, MX_ERR_SHAPE, "mx_map_map_reduce_plain_f32: M too large");
    const dim3 grid((unsigned)ceil_div(N, 16), (unsigned)ceil_div(M, 16));
#define MX_GEMMP(TA, TB) \
    hipLaunchKernelGGL((k_gemm_plain<TA, TB>), grid, dim3(256), 0, stream, A_dev, B_dev, C_dev, M, N, K)
    if (!ta && !tb) MX_GEMMP(0, 0);
    else if (!ta && tb) MX_GEMMP(0, 1);
    else if (ta && !tb) MX_GEMMP(1, 0);
    else MX_GEMMP(1, 1);
#undef MX_GEMMP
    return last_launch("mx_map_map_reduce_plain_f32");
}

}  // extern "C"
