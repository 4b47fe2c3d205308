// Dense nested map (map (reduce (+) 0 (map2 (*) row col))): FP32 matrix
// product on the CDNA matrix cores (v_mfma_f32_16x16x4_f32), FP32 accumulate.
//
// A block owns a BM x BN tile of C and walks K in slices of 32; its waves form
// a WM x WN grid, each owning a (BM/WM) x (BN/WN) sub-tile of 16 x 16 MFMA
// blocks.  Each operand slice is staged in LDS in the orientation it has in
// memory -- [row][k] (32-float rows, 16-byte quads swizzled by row) when k is
// contiguous, [k][row] (row stride BM + 4) when rows are contiguous -- so
// every global load is a 16-byte vector and every LDS store a 16-byte store.  Two LDS buffers, one
// barrier per slice; the next slice's global loads are issued before the
// current slice's MFMAs.
//
// Fragments.  MFMA step s of a slice takes k = 8g + s in lane group
// g = lane / 16 (the reduction over k is associative, so any fixed dealing of
// the 32 k values over steps and lane groups is valid), and every operand is
// read from LDS in vectors:
//  * [row][k] operand: lane (g, l16) needs the 8 consecutive k values 8g..8g+7
//    of one row per 16-row block -- two 16-byte reads per block per slice;
//  * [k][row] operand with R 16-row blocks per wave: at step s the lane reads
//    rows R*l16 .. R*l16 + R-1 of LDS row k = 8g + s in one 8- or 16-byte
//    read, and value c feeds the MFMA of block c.  Block c thus covers the
//    interleaved rows R*rho + c of the wave's tile (rho = 0..15), which the
//    epilogue maps back; for C's columns this makes each lane's R outputs
//    contiguous, so they are stored as one vector.
#include <cstdlib>
#include <cstring>

#include "mx_internal.h"

namespace mx {
namespace {

constexpr int BK = 32;
// [row][k] slices: rows of BK = 32 floats (eight 16-byte quads) with the quad
// position swizzled by the row, quad q of row r at q ^ ((r >> 1) & 7): the
// 16-byte stores of two consecutive rows and the reads of quads 2g, 2g + 1 by
// 16 consecutive rows then fall on distinct banks.
__device__ __forceinline__ int swz(int row, int quad) { return row * BK + 4 * (quad ^ ((row >> 1) & 7)); }
constexpr int kGroupM = 4;   // tile rows per scheduling group

typedef float v4f __attribute__((ext_vector_type(4)));

// Element (r, c..c+3) of a row-major R x C matrix with leading dimension ld
// as a float4, zero outside the matrix.
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

template <int ROWS, bool ROWK> struct Operand {
    static constexpr int LD = ROWK ? BK : ROWS;  // LDS stride in floats
    static constexpr int FLOATS = ROWS * BK;
};

// [k][row] slices: k rows of ROWS floats, unpadded, the 16-byte group q of
// row k at q ^ (8 (k >> 3 & 1)), so the k rows 8 apart that lane groups g and
// g + 1 read in one pass land 32 banks apart.  (Rows padded to ROWS + 4
// floats did the same for the reads; with this layout A^T dC, whose operands
// are both [k][row], runs as fast as the other transposes, 134 against 139 us
// at 2048^3.)
template <int ROWS> __device__ __forceinline__ int kswz(int k, int row) {
    static_assert(ROWS >= 64, "the swizzle moves groups by 8 of at least 16 per row");
    return k * ROWS + 4 * ((row >> 2) ^ (((k >> 3) & 1) << 3)) + (row & 3);
}

// One K-slice of an operand (ROWS rows) into registers, NT threads.
template <int ROWS, bool ROWK, int NT>
__device__ __forceinline__ void load_slice(float4 (&r)[ROWS * BK / 4 / NT], const float *__restrict__ p,
                                           int64_t ld, int64_t row0, int64_t k0, int64_t rows, int64_t K,
                                           bool fast) {
#pragma unroll
    for (int i = 0; i < ROWS * BK / 4 / NT; ++i) {
        const int idx = threadIdx.x + NT * i;
        if constexpr (ROWK) {
            const int row = idx >> 3, kq = idx & 7;  // rows x 8 quads of k
            r[i] = ld4(p, ld, row0 + row, k0 + 4 * kq, rows, K, fast);
        } else {
            constexpr int Q = ROWS / 4;  // quads of rows per k
            const int k = idx / Q, rq = idx % Q;
            r[i] = ld4(p, ld, k0 + k, row0 + 4 * rq, K, rows, fast);
        }
    }
}

template <int ROWS, bool ROWK, int NT>
__device__ __forceinline__ void store_slice(float *__restrict__ s, const float4 (&r)[ROWS * BK / 4 / NT]) {
#pragma unroll
    for (int i = 0; i < ROWS * BK / 4 / NT; ++i) {
        const int idx = threadIdx.x + NT * i;
        if constexpr (ROWK) {
            const int row = idx >> 3, kq = idx & 7;
            *reinterpret_cast<float4 *>(s + swz(row, kq)) = r[i];
        } else {
            constexpr int Q = ROWS / 4;
            const int k = idx / Q, rq = idx % Q;
            *reinterpret_cast<float4 *>(s + kswz<ROWS>(k, 4 * rq)) = r[i];
        }
    }
}

template <int R> struct VecOf;
template <> struct VecOf<1> { using T = float; };
template <> struct VecOf<2> { using T = float2; };
template <> struct VecOf<4> { using T = float4; };

// R consecutive floats from LDS (16-byte aligned for R = 4, 8-byte for R = 2)
template <int R> __device__ __forceinline__ void lds_read(float (&v)[R], const float *p) {
    const typename VecOf<R>::T t = *reinterpret_cast<const typename VecOf<R>::T *>(p);
    __builtin_memcpy(v, &t, sizeof t);
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
    const int gi = L / per_group;
    const int first_m = gi * kGroupM;
    const int gm = min(tiles_m - first_m, kGroupM);
    const int in = L - gi * per_group;
    tm = first_m + in % gm;
    tn = in / gm;
}

// The wave's operand fragments of one K slice held in LDS: fa[s][i] is the
// value lane (g, l16) feeds MFMA step s of row block i, fb[s][j] that of column
// block j.
template <int BM, int BN, int WM, int WN, bool RA, bool RB>
__device__ __forceinline__ void read_frags(float (&fa)[8][BM / WM / 16], float (&fb)[8][BN / WN / 16],
                                           const float *__restrict__ as, const float *__restrict__ bs, int wrow0,
                                           int wcol0, int l16, int g) {
    constexpr int MI = BM / WM / 16, NI = BN / WN / 16;
    if constexpr (RA) {
#pragma unroll
        for (int i = 0; i < MI; ++i) {
            const int row = wrow0 + 16 * i + l16;
            const float4 lo = *reinterpret_cast<const float4 *>(as + swz(row, 2 * g));
            const float4 hi = *reinterpret_cast<const float4 *>(as + swz(row, 2 * g + 1));
            fa[0][i] = lo.x; fa[1][i] = lo.y; fa[2][i] = lo.z; fa[3][i] = lo.w;
            fa[4][i] = hi.x; fa[5][i] = hi.y; fa[6][i] = hi.z; fa[7][i] = hi.w;
        }
    } else {
#pragma unroll
        for (int s = 0; s < 8; ++s) lds_read<MI>(fa[s], as + kswz<BM>(8 * g + s, wrow0 + MI * l16));
    }
    if constexpr (RB) {
#pragma unroll
        for (int j = 0; j < NI; ++j) {
            const int row = wcol0 + 16 * j + l16;
            const float4 lo = *reinterpret_cast<const float4 *>(bs + swz(row, 2 * g));
            const float4 hi = *reinterpret_cast<const float4 *>(bs + swz(row, 2 * g + 1));
            fb[0][j] = lo.x; fb[1][j] = lo.y; fb[2][j] = lo.z; fb[3][j] = lo.w;
            fb[4][j] = hi.x; fb[5][j] = hi.y; fb[6][j] = hi.z; fb[7][j] = hi.w;
        }
    } else {
#pragma unroll
        for (int s = 0; s < 8; ++s) lds_read<NI>(fb[s], bs + kswz<BN>(8 * g + s, wcol0 + NI * l16));
    }
}

// MFMA work of one K slice from its fragments: the wave's MI x NI blocks of 16 x 16
template <int MI, int NI>
__device__ __forceinline__ void mma_frags(v4f (&acc)[MI][NI], const float (&fa)[8][MI], const float (&fb)[8][NI]) {
#pragma unroll
    for (int step = 0; step < 8; ++step)
#pragma unroll
        for (int i = 0; i < MI; ++i)
#pragma unroll
            for (int j = 0; j < NI; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[step][i], fb[step][j], acc[i][j], 0, 0, 0);
}

template <int BM, int BN, int WM, int WN, bool RA, bool RB>
__device__ __forceinline__ void mma_slice(v4f (&acc)[BM / WM / 16][BN / WN / 16], const float *__restrict__ as,
                                          const float *__restrict__ bs, int wrow0, int wcol0, int l16, int g) {
    float fa[8][BM / WM / 16], fb[8][BN / WN / 16];
    read_frags<BM, BN, WM, WN, RA, RB>(fa, fb, as, bs, wrow0, wcol0, l16, g);
    mma_frags(acc, fa, fb);
}

template <int BM, int BN, int WM, int WN, int TA, int TB>
__global__ void __launch_bounds__(64 * WM * WN) k_gemm_mfma(const float *__restrict__ A, const float *__restrict__ B,
                                                            float *__restrict__ C, int64_t M, int64_t N, int64_t K,
                                                            int tiles_m, int tiles_n, int vec_ok, int cvec) {
    constexpr int NT = 64 * WM * WN;
    static_assert((BM * BK / 4) % NT == 0 && (BN * BK / 4) % NT == 0, "slice loads must split evenly");
    static_assert(BM % (16 * WM) == 0 && BN % (16 * WN) == 0, "wave tiles are whole 16 x 16 blocks");
    constexpr bool RA = !TA, RB = TB;  // [row][k] in memory
    constexpr int MI = BM / WM / 16, NI = BN / WN / 16;
    static_assert(RA || MI == 1 || MI == 2 || MI == 4, "[k][row] A: reads of 1, 2 or 4 rows");
    static_assert(RB || NI == 1 || NI == 2 || NI == 4, "[k][row] B: reads of 1, 2 or 4 columns");
    using OA = Operand<BM, RA>;
    using OB = Operand<BN, RB>;
    __shared__ __attribute__((aligned(16))) float As0[OA::FLOATS], As1[OA::FLOATS];
    __shared__ __attribute__((aligned(16))) float Bs0[OB::FLOATS], Bs1[OB::FLOATS];
    auto As = [&](int i) { return i ? As1 : As0; };
    auto Bs = [&](int i) { return i ? Bs1 : Bs0; };

    int tm, tn;
    tile_of(blockIdx.x, tiles_m, tiles_n, tm, tn);
    const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave / WN, wn = wave % WN;
    const int l16 = lane & 15, g = lane >> 4;
    const int64_t lda = TA ? M : K;
    const int64_t ldb = TB ? K : N;
    const bool interior = vec_ok && (m0 + BM <= M) && (n0 + BN <= N);
    const int nk = (int)((K + BK - 1) / BK);

    v4f acc[MI][NI];
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < NI; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};

    const int wrow0 = wm * (BM / WM), wcol0 = wn * (BN / WN);
    constexpr int NA = BM * BK / 4 / NT, NB = BN * BK / 4 / NT;
    if (interior && K % (2 * BK) == 0 && nk >= 4) {
        // Interior tile, an even number (at least four) of whole slices.
        // Iteration kt multiplies slice kt from fragments already in registers
        // while the fragments of slice kt + 1 are read from LDS, then stores
        // slice kt + 2 (loaded two iterations earlier) into the buffer slice kt
        // occupied and issues the global loads of slice kt + 4; one barrier.
        // The fragment reads are in flight across the MFMAs and the barrier,
        // so no wave waits on LDS latency between slices.  The last four
        // iterations are peeled: nothing is loaded past the end of K.
        float4 ga[NA], gb[NB], ha[NA], hb[NB];  // staging of two slices in flight
        float fa0[8][MI], fb0[8][NI], fa1[8][MI], fb1[8][NI];
        load_slice<BM, RA, NT>(ga, A, lda, m0, 0, M, K, true);
        load_slice<BN, RB, NT>(gb, B, ldb, n0, 0, N, K, true);
        load_slice<BM, RA, NT>(ha, A, lda, m0, BK, M, K, true);
        load_slice<BN, RB, NT>(hb, B, ldb, n0, BK, N, K, true);
        store_slice<BM, RA, NT>(As(0), ga);
        store_slice<BN, RB, NT>(Bs(0), gb);
        load_slice<BM, RA, NT>(ga, A, lda, m0, 2 * BK, M, K, true);
        load_slice<BN, RB, NT>(gb, B, ldb, n0, 2 * BK, N, K, true);
        __syncthreads();
        read_frags<BM, BN, WM, WN, RA, RB>(fa0, fb0, As(0), Bs(0), wrow0, wcol0, l16, g);
        store_slice<BM, RA, NT>(As(1), ha);
        store_slice<BN, RB, NT>(Bs(1), hb);
        load_slice<BM, RA, NT>(ha, A, lda, m0, 3 * BK, M, K, true);
        load_slice<BN, RB, NT>(hb, B, ldb, n0, 3 * BK, N, K, true);
        __syncthreads();
        // one iteration; buffer (kt + 1) & 1 holds slice kt + 1, buffer kt & 1
        // is free once slice kt's fragments are in registers
#define MX_GEMM_ITER(KT, FA, FB, NFA, NFB, SA, SB, DO_R, DO_S, DO_L)                                      \
        {                                                                                                 \
            const int b1 = ((KT) + 1) & 1, b0 = (KT) & 1;                                                 \
            if (DO_R) read_frags<BM, BN, WM, WN, RA, RB>(NFA, NFB, As(b1), Bs(b1), wrow0, wcol0, l16, g); \
            __builtin_amdgcn_sched_barrier(0);                                                            \
            mma_frags(acc, FA, FB);                                                                       \
            __builtin_amdgcn_sched_barrier(0);                                                            \
            if (DO_S) {                                                                                   \
                store_slice<BM, RA, NT>(As(b0), SA);                                                      \
                store_slice<BN, RB, NT>(Bs(b0), SB);                                                      \
            }                                                                                             \
            if (DO_L) {                                                                                   \
                const int64_t kl = (int64_t)((KT) + 4) * BK;                                              \
                load_slice<BM, RA, NT>(SA, A, lda, m0, kl, M, K, true);                                   \
                load_slice<BN, RB, NT>(SB, B, ldb, n0, kl, N, K, true);                                   \
            }                                                                                             \
            if (DO_S) __syncthreads();                                                                    \
        }
        int kt = 0;
        for (; kt + 4 < nk; kt += 2) {
            MX_GEMM_ITER(kt, fa0, fb0, fa1, fb1, ga, gb, true, true, true)
            MX_GEMM_ITER(kt + 1, fa1, fb1, fa0, fb0, ha, hb, true, true, true)
        }
        MX_GEMM_ITER(kt, fa0, fb0, fa1, fb1, ga, gb, true, true, false)
        MX_GEMM_ITER(kt + 1, fa1, fb1, fa0, fb0, ha, hb, true, true, false)
        MX_GEMM_ITER(kt + 2, fa0, fb0, fa1, fb1, ga, gb, true, false, false)
        MX_GEMM_ITER(kt + 3, fa1, fb1, fa0, fb0, ha, hb, false, false, false)
#undef MX_GEMM_ITER
    } else {
        // edge tiles and ragged K: bounds-checked loads, one slice ahead
        float4 ra[NA], rb[NB];
        {
            const bool fast = interior && (BK <= K);
            load_slice<BM, RA, NT>(ra, A, lda, m0, 0, M, K, fast);
            load_slice<BN, RB, NT>(rb, B, ldb, n0, 0, N, K, fast);
            store_slice<BM, RA, NT>(As(0), ra);
            store_slice<BN, RB, NT>(Bs(0), rb);
        }
        __syncthreads();
        for (int kt = 0; kt < nk; ++kt) {
            const int buf = kt & 1;
            const bool more = kt + 1 < nk;
            if (more) {
                const int64_t k0 = (int64_t)(kt + 1) * BK;
                const bool fast = interior && (k0 + BK <= K);
                load_slice<BM, RA, NT>(ra, A, lda, m0, k0, M, K, fast);
                load_slice<BN, RB, NT>(rb, B, ldb, n0, k0, N, K, fast);
            }
            mma_slice<BM, BN, WM, WN, RA, RB>(acc, As(buf), Bs(buf), wrow0, wcol0, l16, g);
            if (more) {
                store_slice<BM, RA, NT>(As(buf ^ 1), ra);
                store_slice<BN, RB, NT>(Bs(buf ^ 1), rb);
            }
            __syncthreads();
        }
    }

    // D block (i, j): lane holds block rows rho = 4g .. 4g+3 of block column
    // l16; blocked or interleaved as the operand layout dealt them
#pragma unroll
    for (int i = 0; i < MI; ++i) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int rho = 4 * g + r;
            const int64_t row = m0 + wrow0 + (RA ? 16 * i + rho : MI * rho + i);
            if constexpr (!RB) {
                // the lane's NI columns NI*l16 .. NI*l16 + NI-1 are contiguous
                const int64_t col = n0 + wcol0 + NI * l16;
                if (interior && cvec) {
                    float v[NI];
#pragma unroll
                    for (int j = 0; j < NI; ++j) v[j] = acc[i][j][r];
                    typename VecOf<NI>::T t;
                    __builtin_memcpy(&t, v, sizeof t);
                    *reinterpret_cast<typename VecOf<NI>::T *>(C + row * N + col) = t;
                } else {
#pragma unroll
                    for (int j = 0; j < NI; ++j)
                        if (row < M && col + j < N) C[row * N + col + j] = acc[i][j][r];
                }
            } else {
#pragma unroll
                for (int j = 0; j < NI; ++j) {
                    const int64_t col = n0 + wcol0 + 16 * j + l16;
                    if (interior || (row < M && col < N)) C[row * N + col] = acc[i][j][r];
                }
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

// Tile shapes: 128 x 128 with 16 waves (2 x 2 blocks of 16 x 16 per wave, four
// waves per SIMD) when there are enough tiles for every CU, else 128 x 64 with
// 8 waves (2 x 2 per wave); more waves per SIMD hide each other's barrier and
// LDS waits (at 2048^3 the 16-wave tile measured 2-4 % faster than 8 waves
// with 2 x 4 blocks each).  MX_GEMM_TILE in the environment forces one of the
// configurations below (for tuning and for testing every tile at small
// shapes).
template <int BM, int BN, int WM, int WN>
mx_status launch_gemm(int ta, int tb, int64_t M, int64_t N, int64_t K, const float *A, const float *B, float *C,
                      int vec_ok, hipStream_t s) {
    const int cvec = ((uintptr_t)C % 16 == 0) && (N % 4 == 0);
    const int64_t tiles_m = ceil_div(M, BM), tiles_n = ceil_div(N, BN);
    MX_REQUIRE(tiles_m * tiles_n < (1LL << 31), MX_ERR_SHAPE, "mx_map_map_reduce_f32: too many tiles");
    const dim3 grid((unsigned)(tiles_m * tiles_n)), block(64 * WM * WN);
#define MX_GEMM(TA, TB)                                                                                    \
    hipLaunchKernelGGL((k_gemm_mfma<BM, BN, WM, WN, TA, TB>), grid, block, 0, s, A, B, C, M, N, K, (int)tiles_m, \
                       (int)tiles_n, vec_ok, cvec)
    if (!ta && !tb) MX_GEMM(0, 0);
    else if (!ta && tb) MX_GEMM(0, 1);
    else if (ta && !tb) MX_GEMM(1, 0);
    else MX_GEMM(1, 1);
#undef MX_GEMM
    return last_launch("mx_map_map_reduce_f32");
}

// Tile configurations: BM x BN block tile, WM x WN waves.
enum GemmTile { kT128x64 = 1, kT128x128, kT128x64w8, kT128x128w8, kT64x64, kT128x128w8b, kT128x128w16 };

int gemm_tile_choice(int ta, int tb, int64_t M, int64_t N, const DeviceInfo *d) {
    // read on every call (a getenv is cheap next to a launch), so one process
    // can run every configuration
    if (const char *e = getenv("MX_GEMM_TILE")) {
        static const struct { const char *name; int tile; } names[] = {
            {"128x64", kT128x64}, {"128x128", kT128x128}, {"128x64w8", kT128x64w8},
            {"128x128w8", kT128x128w8}, {"64x64", kT64x64}, {"128x128w8b", kT128x128w8b},
            {"128x128w16", kT128x128w16}};
        for (const auto &n : names)
            if (!strcmp(e, n.name)) return n.tile;
    }
    // 128 x 128 when it still gives every CU a tile
    const int64_t big = ceil_div(M, 128) * ceil_div(N, 128);
    if (big >= d->num_cus) return kT128x128w16;
    return kT128x64w8;
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
    const int64_t lda = ta ? M : K, ldb = tb ? K : N;
    const int vec_ok = ((uintptr_t)A_dev % 16 == 0) && ((uintptr_t)B_dev % 16 == 0) && (lda % 4 == 0) &&
                       (ldb % 4 == 0);
    switch (gemm_tile_choice(ta, tb, M, N, d)) {
    case kT128x64: return launch_gemm<128, 64, 2, 2>(ta, tb, M, N, K, A_dev, B_dev, C_dev, vec_ok, stream);
    case kT128x64w8: return launch_gemm<128, 64, 4, 2>(ta, tb, M, N, K, A_dev, B_dev, C_dev, vec_ok, stream);
    case kT128x128w8: return launch_gemm<128, 128, 4, 2>(ta, tb, M, N, K, A_dev, B_dev, C_dev, vec_ok, stream);
    case kT64x64: return launch_gemm<64, 64, 2, 2>(ta, tb, M, N, K, A_dev, B_dev, C_dev, vec_ok, stream);
    case kT128x128w8b: return launch_gemm<128, 128, 2, 4>(ta, tb, M, N, K, A_dev, B_dev, C_dev, vec_ok, stream);
    case kT128x128w16: return launch_gemm<128, 128, 4, 4>(ta, tb, M, N, K, A_dev, B_dev, C_dev, vec_ok, stream);
    default: return launch_gemm<128, 128, 2, 2>(ta, tb, M, N, K, A_dev, B_dev, C_dev, vec_ok, stream);
    }
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
