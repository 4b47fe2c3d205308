// Many uneven accelerated expressions in one persistent launch.
//
// The paper notes that expression acceleration pays off when work is
// concentrated in few `accelerate` uses and that small problems leave the GPU
// idle (Section 5.2).  A batch runs thousands of independent small
// expressions -- dot products reduce (+) 0 (map2 (*) a b) and matrix-vector
// products map (reduce (+) 0 . map2 (*) x) over rows -- as one launch.
//
// Plan (host, once): every task is cut into tiles of equal bytes -- element
// ranges of `tile_elems` for a dot (two streamed operands), whole-row ranges
// of about 2 * `tile_elems` elements for a matvec (one) -- and the tiles are
// ordered longest first.  Forward: a persistent grid pulls tiles
// with an atomic ticket; a single-tile task writes its result, a multi-tile dot
// writes one partial per tile.  A combine launch adds each task's partials in
// tile order (deterministic for a given plan) and resets the ticket.  Backward
// (dot: ga = g b, gb = g a; matvec y = A x: gA = g x^T, gx = A^T g) has the same
// structure, with per-tile partial column sums for gx.  No float atomics, no
// cross-block fences.  The autotuner times candidate (tile_elems,
// blocks_per_cu) pairs on the caller's buffers and caches the choice per task
// table and device in a JSON file.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "mx_internal.h"

namespace mx {
namespace {

constexpr int NT = 256;
constexpr int kDot = 0, kMatvec = 1;
constexpr int kMinTile = 4096;
constexpr int kXLds = 2048;  // matvec x staged in LDS up to this many columns

inline bool aligned16(const void *p) { return ((uintptr_t)p & 15) == 0; }

struct TaskDev {
    int32_t kind, pad;
    int64_t rows, cols, a_off, b_off, out_off;
    int64_t fwd_part, fwd_ntiles, bwd_part, bwd_ntiles;
};

// One tile, carrying the task fields its kernels need so that taking a tile
// costs one descriptor load.
struct TileDev {
    int32_t task, kind;
    int64_t begin, end;  // dot: elements; matvec: rows
    int64_t part;        // partial slot (float offset) or -1 to write the result directly
    int64_t cols, a_off, b_off, out_off;
};

// sum over the 16 lanes of a DPP row, result in every lane of the row
__device__ __forceinline__ float row16_sum(float v) {
    using R = Red<MX_ADD, float>;
    v = R::ap(v, dpp_move<0xB1, 0xF>(v, 0.f));
    v = R::ap(v, dpp_move<0x4E, 0xF>(v, 0.f));
    v = R::ap(v, dpp_move<0x141, 0xF>(v, 0.f));
    v = R::ap(v, dpp_move<0x140, 0xF>(v, 0.f));
    return v;
}

// Tile loop of the persistent kernels: thread 0 takes a ticket, the block
// reads it after a barrier and loads the tile descriptor.  (Taking the next
// ticket while the current tile streams was measured slower: a busy block
// then holds a tile an idle block could already be working on.)
#define MX_TILE_LOOP_BEGIN                                                         \
    __shared__ int64_t slot;                                                     \
    for (;;) {                                                                   \
        __syncthreads();                                                         \
        if (threadIdx.x == 0) slot = (int64_t)atomicAdd(ticket, 1u);             \
        __syncthreads();                                                         \
        const int64_t t = slot;                                                  \
        if (t >= ntiles) break;                                                  \
        const TileDev tl = tiles[t];                                             \
        const TileDev &tk = tl;

#define MX_TILE_LOOP_END }

__global__ void __launch_bounds__(NT) k_batch_fwd(const TaskDev *__restrict__ tasks, const TileDev *__restrict__ tiles,
                                                  int64_t ntiles, const float *__restrict__ A,
                                                  const float *__restrict__ B, float *__restrict__ out,
                                                  float *__restrict__ part, unsigned *ticket, int vec) {
    __shared__ float red[NT / kWave];
    __shared__ float xs[kXLds];
    using R = Red<MX_ADD, float>;
    MX_TILE_LOOP_BEGIN
        if (tk.kind == kDot) {
            const float *a = A + tk.a_off, *b = B + tk.b_off;
            float ac[4] = {0.f, 0.f, 0.f, 0.f};
            if (vec && ((tk.a_off | tk.b_off | tl.begin) & 3) == 0) {
                // 16-byte vectors, four per operand in flight, scalar tail
                const float4 *a4 = reinterpret_cast<const float4 *>(a), *b4 = reinterpret_cast<const float4 *>(b);
                const int64_t ve = tl.end >> 2;
                int64_t i = (tl.begin >> 2) + threadIdx.x;
                for (; i + 3 * NT < ve; i += 4 * NT) {
                    float4 x[4], y[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        x[u] = a4[i + u * NT];
                        y[u] = b4[i + u * NT];
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u) ac[u] += x[u].x * y[u].x + x[u].y * y[u].y + x[u].z * y[u].z + x[u].w * y[u].w;
                }
                for (; i < ve; i += NT) {
                    const float4 x = a4[i], y = b4[i];
                    ac[0] += x.x * y.x + x.y * y.y + x.z * y.z + x.w * y.w;
                }
                for (int64_t e = 4 * ve + threadIdx.x; e < tl.end; e += NT) ac[1] += a[e] * b[e];
            } else {
                int64_t e = tl.begin + threadIdx.x;
                for (; e + 3 * NT < tl.end; e += 4 * NT) {
                    float av[4], bv[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        av[u] = a[e + u * NT];
                        bv[u] = b[e + u * NT];
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u) ac[u] += av[u] * bv[u];
                }
                for (; e < tl.end; e += NT) ac[0] += a[e] * b[e];
            }
            float acc = block_reduce<R, NT>((ac[0] + ac[1]) + (ac[2] + ac[3]), red);
            if (threadIdx.x == 0) {
                if (tl.part >= 0) part[tl.part] = acc;
                else out[tk.out_off] = acc;
            }
        } else {
            // 16 lanes per row, 16 rows at a time.  x is staged in LDS once
            // per tile (when it fits), so every row can be read with 16-byte
            // loads whatever its alignment: a scalar head up to the next
            // 16-byte boundary of A, the vector body (eight loads per lane in
            // flight), a scalar tail; x values come from LDS.
            const int grp = threadIdx.x >> 4, l = threadIdx.x & 15;
            const int64_t c = tk.cols;
            const float *x = B + tk.b_off;
            const bool stage = vec && c <= kXLds;
            if (stage) {
                for (int64_t q = threadIdx.x; q < c; q += NT) xs[q] = x[q];
                __syncthreads();
            }
            for (int64_t r0 = tl.begin; r0 < tl.end; r0 += NT / 16) {
                const int64_t r = r0 + grp;
                float ac[4] = {0.f, 0.f, 0.f, 0.f};
                if (r < tl.end) {
                    const int64_t e0 = tk.a_off + r * c;  // row start in A
                    const float *row = A + e0;
                    if (stage) {
                        const int64_t head = ((4 - (e0 & 3)) & 3) < c ? ((4 - (e0 & 3)) & 3) : c;
                        const int64_t nb4 = (c - head) >> 2;
                        const float4 *row4 = reinterpret_cast<const float4 *>(row + head);
                        if (l < head) ac[1] += row[l] * xs[l];
                        // eight loads per lane in flight, the last round
                        // predicated (a row's remainder is not a latency chain)
                        for (int64_t v = l; v < nb4; v += 128) {
                            float4 av[8];
#pragma unroll
                            for (int u = 0; u < 8; ++u)
                                av[u] = v + 16 * u < nb4 ? row4[v + 16 * u] : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
                            for (int u = 0; u < 8; ++u) {
                                if (v + 16 * u < nb4) {
                                    const float *xq = xs + head + 4 * (v + 16 * u);
                                    ac[u & 3] += av[u].x * xq[0] + av[u].y * xq[1] + av[u].z * xq[2] + av[u].w * xq[3];
                                }
                            }
                        }
                        const int64_t t0 = head + 4 * nb4;
                        if (t0 + l < c) ac[2] += row[t0 + l] * xs[t0 + l];
                    } else {
                        int64_t j = l;
                        for (; j + 48 < c; j += 64) {
                            float av[4], xv[4];
#pragma unroll
                            for (int u = 0; u < 4; ++u) {
                                av[u] = row[j + 16 * u];
                                xv[u] = x[j + 16 * u];
                            }
#pragma unroll
                            for (int u = 0; u < 4; ++u) ac[u] += av[u] * xv[u];
                        }
                        for (; j < c; j += 16) ac[0] += row[j] * x[j];
                    }
                }
                const float acc = row16_sum((ac[0] + ac[1]) + (ac[2] + ac[3]));
                if (l == 0 && r < tl.end) out[tk.out_off + r] = acc;
            }
        }
    MX_TILE_LOOP_END
}

// Column group j of a matvec tile's adjoint, V = float4 (4 columns, rows
// 16-byte aligned) or float (1 column): gA rows r = r0, r0 + step, ... below
// r1 get g[r] x, and the function returns the sum over those rows of
// g[r] A[r][cols of j] in row order, U rows per round in flight.
template <class V> struct Lanes;
template <> struct Lanes<float> {
    static __device__ __forceinline__ float scale(float v, float s) { return v * s; }
    static __device__ __forceinline__ void fma(float &acc, float a, float s) { acc += a * s; }
};
template <> struct Lanes<float4> {
    static __device__ __forceinline__ float4 scale(float4 v, float s) { return make_float4(v.x * s, v.y * s, v.z * s, v.w * s); }
    static __device__ __forceinline__ void fma(float4 &acc, float4 a, float s) {
        acc.x += a.x * s;
        acc.y += a.y * s;
        acc.z += a.z * s;
        acc.w += a.w * s;
    }
};

template <class V, int U>
__device__ __forceinline__ V matvec_adj_cols(const V *__restrict__ a, const V *__restrict__ x,
                                             const float *__restrict__ g, V *__restrict__ ga, int64_t cv,
                                             int64_t j, int64_t r0, int64_t r1, int step) {
    using Ln = Lanes<V>;
    const V xj = x[j];
    V acc;
    __builtin_memset(&acc, 0, sizeof acc);
    int64_t r = r0;
    for (; r + (U - 1) * step < r1; r += U * step) {
        V av[U];
        float gv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            av[u] = a[(r + u * step) * cv + j];
            gv[u] = g[r + u * step];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            Ln::fma(acc, av[u], gv[u]);
            ga[(r + u * step) * cv + j] = Ln::scale(xj, gv[u]);
        }
    }
    for (; r < r1; r += step) {
        const float gr = g[r];
        Ln::fma(acc, a[r * cv + j], gr);
        ga[r * cv + j] = Ln::scale(xj, gr);
    }
    return acc;
}

// One matvec tile's backward with column groups of V: one thread per column
// group; when there are fewer groups than threads the threads split the rows
// into P phases (rows ph, ph + P, ...) and the phase partials are added in
// phase order through LDS.  dst: the tile's partial column sums or gB.
template <class V, int U>
__device__ __forceinline__ void matvec_adj_tile(const V *__restrict__ a, const V *__restrict__ x,
                                                const float *__restrict__ g, V *__restrict__ ga, int64_t cv,
                                                int64_t rb, int64_t re, float *__restrict__ dst, V *red) {
    constexpr int W = sizeof(V) / sizeof(float);
    const int P = cv >= NT ? 1 : (int)(NT / cv);
    if (P == 1) {
        for (int64_t j = threadIdx.x; j < cv; j += NT) {
            const V s = matvec_adj_cols<V, U>(a, x, g, ga, cv, j, rb, re, 1);
            __builtin_memcpy(dst + W * j, &s, sizeof s);
        }
    } else {
        const int j = (int)(threadIdx.x % cv), ph = (int)(threadIdx.x / cv);
        V s;
        __builtin_memset(&s, 0, sizeof s);
        if (ph < P) s = matvec_adj_cols<V, U>(a, x, g, ga, cv, j, rb + ph, re, P);
        red[threadIdx.x] = s;
        __syncthreads();
        if (threadIdx.x < cv) {
            float t[W];
            __builtin_memcpy(t, &red[threadIdx.x], sizeof t);
            for (int q = 1; q < P; ++q) {
                float u[W];
                __builtin_memcpy(u, &red[q * cv + threadIdx.x], sizeof u);
#pragma unroll
                for (int e = 0; e < W; ++e) t[e] += u[e];
            }
            __builtin_memcpy(dst + W * threadIdx.x, t, sizeof t);
        }
    }
}

__global__ void __launch_bounds__(NT) k_batch_bwd(const TaskDev *__restrict__ tasks, const TileDev *__restrict__ tiles,
                                                  int64_t ntiles, const float *__restrict__ A,
                                                  const float *__restrict__ B, const float *__restrict__ gout,
                                                  float *__restrict__ gA, float *__restrict__ gB,
                                                  float *__restrict__ part, unsigned *ticket, int vec) {
    __shared__ float4 red4[NT];
    __shared__ float red1[NT];
    MX_TILE_LOOP_BEGIN
        if (tk.kind == kDot) {
            const float g = gout[tk.out_off];
            const float *a = A + tk.a_off, *b = B + tk.b_off;
            float *ga = gA + tk.a_off, *gb = gB + tk.b_off;
            int64_t e = tl.begin + threadIdx.x;
            if (vec && ((tk.a_off | tk.b_off | tl.begin) & 3) == 0) {
                const float4 *a4 = reinterpret_cast<const float4 *>(a), *b4 = reinterpret_cast<const float4 *>(b);
                float4 *ga4 = reinterpret_cast<float4 *>(ga), *gb4 = reinterpret_cast<float4 *>(gb);
                const int64_t ve = tl.end >> 2;
                int64_t i = (tl.begin >> 2) + threadIdx.x;
                for (; i + 3 * NT < ve; i += 4 * NT) {
                    float4 x[4], y[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        x[u] = a4[i + u * NT];
                        y[u] = b4[i + u * NT];
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        ga4[i + u * NT] = make_float4(g * y[u].x, g * y[u].y, g * y[u].z, g * y[u].w);
                        gb4[i + u * NT] = make_float4(g * x[u].x, g * x[u].y, g * x[u].z, g * x[u].w);
                    }
                }
                for (; i < ve; i += NT) {
                    const float4 x = a4[i], y = b4[i];
                    ga4[i] = make_float4(g * y.x, g * y.y, g * y.z, g * y.w);
                    gb4[i] = make_float4(g * x.x, g * x.y, g * x.z, g * x.w);
                }
                e = 4 * ve + threadIdx.x;
            } else {
                for (; e + 3 * NT < tl.end; e += 4 * NT) {
                    float av[4], bv[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        av[u] = a[e + u * NT];
                        bv[u] = b[e + u * NT];
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        ga[e + u * NT] = g * bv[u];
                        gb[e + u * NT] = g * av[u];
                    }
                }
            }
            for (; e < tl.end; e += NT) {
                ga[e] = g * b[e];
                gb[e] = g * a[e];
            }
        } else {
            const int64_t c = tk.cols;
            const float *x = B + tk.b_off, *g = gout + tk.out_off;
            const float *a = A + tk.a_off;
            float *ga = gA + tk.a_off;
            float *dst = tl.part >= 0 ? part + tl.part : gB + tk.b_off;
            if (vec && ((tk.a_off | tk.b_off | c) & 3) == 0)
                matvec_adj_tile<float4, 8>(reinterpret_cast<const float4 *>(a), reinterpret_cast<const float4 *>(x),
                                           g, reinterpret_cast<float4 *>(ga), c >> 2, tl.begin, tl.end, dst, red4);
            else
                matvec_adj_tile<float, 16>(a, x, g, ga, c, tl.begin, tl.end, dst, red1);
        }
    MX_TILE_LOOP_END
}

// sum of q = 0 .. nq-1 of p[q * stride], in q order, eight loads in flight
__device__ __forceinline__ float sum_strided(const float *__restrict__ p, int64_t nq, int64_t stride) {
    float s = 0.f;
    int64_t q = 0;
    for (; q + 8 <= nq; q += 8) {
        float v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = p[(q + u) * stride];
#pragma unroll
        for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; q < nq; ++q) s += p[q * stride];
    return s;
}

// Adds the tile partials of each multi-tile task in tile order; resets the ticket.
__global__ void __launch_bounds__(NT) k_batch_combine_fwd(const TaskDev *__restrict__ tasks,
                                                          const int32_t *__restrict__ list, int64_t nlist,
                                                          const float *__restrict__ part, float *__restrict__ out,
                                                          unsigned *ticket) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *ticket = 0u;
    const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (i >= nlist) return;
    const TaskDev tk = tasks[list[i]];
    out[tk.out_off] = sum_strided(part + tk.fwd_part, tk.fwd_ntiles, 1);
}

// grid (tasks in the list, column chunks of NT): column j of task gets the sum
// of its per-tile partial column sums in tile order
__global__ void __launch_bounds__(NT) k_batch_combine_bwd(const TaskDev *__restrict__ tasks,
                                                          const int32_t *__restrict__ list, int64_t nlist,
                                                          const float *__restrict__ part, float *__restrict__ gB,
                                                          unsigned *ticket) {
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) *ticket = 0u;
    if ((int64_t)blockIdx.x >= nlist) return;
    const TaskDev tk = tasks[list[blockIdx.x]];
    const int64_t c = tk.cols;
    for (int64_t j = (int64_t)blockIdx.y * NT + threadIdx.x; j < c; j += (int64_t)gridDim.y * NT)
        gB[tk.b_off + j] = sum_strided(part + tk.bwd_part + j, tk.bwd_ntiles, c);
}

// ---------------------------------------------------------------- plain: one launch per task
__global__ void __launch_bounds__(NT) k_dot_plain(const float *__restrict__ a, const float *__restrict__ b, int64_t n,
                                                  float *__restrict__ out) {
    __shared__ float red[NT / kWave];
    float acc = 0.f;
    for (int64_t e = threadIdx.x; e < n; e += NT) acc += a[e] * b[e];
    acc = block_reduce<Red<MX_ADD, float>, NT>(acc, red);
    if (threadIdx.x == 0) out[0] = acc;
}

__global__ void __launch_bounds__(NT) k_matvec_plain(const float *__restrict__ A, const float *__restrict__ x,
                                                     int64_t rows, int64_t cols, float *__restrict__ y) {
    const int64_t r = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (r >= rows) return;
    float acc = 0.f;
    for (int64_t j = 0; j < cols; ++j) acc += A[r * cols + j] * x[j];
    y[r] = acc;
}

__global__ void __launch_bounds__(NT) k_dot_adj_plain(const float *__restrict__ a, const float *__restrict__ b,
                                                      int64_t n, const float *__restrict__ g, float *__restrict__ ga,
                                                      float *__restrict__ gb) {
    const int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (e >= n) return;
    ga[e] = g[0] * b[e];
    gb[e] = g[0] * a[e];
}

__global__ void __launch_bounds__(NT) k_matvec_adj_plain(const float *__restrict__ A, const float *__restrict__ x,
                                                         int64_t rows, int64_t cols, const float *__restrict__ g,
                                                         float *__restrict__ gA, float *__restrict__ gx) {
    const int64_t j = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (j >= cols) return;
    float acc = 0.f;
    for (int64_t r = 0; r < rows; ++r) {
        acc += A[r * cols + j] * g[r];
        gA[r * cols + j] = g[r] * x[j];
    }
    gx[j] = acc;
}

}  // namespace
}  // namespace mx

using namespace mx;

struct mx_batch_plan {
    int device = 0;
    int num_cus = 256;
    std::vector<int64_t> table;  // [ntasks][6]
    int64_t ntasks = 0;
    int64_t a_len = 0, b_len = 0, out_len = 0;
    mx_batch_config cfg{};
    TaskDev *d_tasks = nullptr;
    TileDev *d_fwd = nullptr, *d_bwd = nullptr;
    int32_t *d_fwd_list = nullptr, *d_bwd_list = nullptr;
    int64_t n_fwd = 0, n_bwd = 0, n_fwd_list = 0, n_bwd_list = 0;
    int64_t bwd_list_max_cols = 1;
    int64_t fwd_part_floats = 0, bwd_part_floats = 0;
    size_t ws_need = 0;
};

namespace {

void free_device(mx_batch_plan *p) {
    (void)hipFree(p->d_tasks);
    (void)hipFree(p->d_fwd);
    (void)hipFree(p->d_bwd);
    (void)hipFree(p->d_fwd_list);
    (void)hipFree(p->d_bwd_list);
    p->d_tasks = nullptr;
    p->d_fwd = p->d_bwd = nullptr;
    p->d_fwd_list = p->d_bwd_list = nullptr;
}

// Partial-storage requirement at the smallest tile size (covers every candidate).
void partial_floats(const std::vector<int64_t> &tb, int64_t ntasks, int64_t tile, int64_t *fwd, int64_t *bwd) {
    *fwd = 0;
    *bwd = 0;
    for (int64_t t = 0; t < ntasks; ++t) {
        const int64_t kind = tb[6 * t], rows = tb[6 * t + 1], cols = tb[6 * t + 2];
        if (kind == kDot) {
            const int64_t nt = ceil_div(cols > 0 ? cols : 1, tile);
            if (nt > 1) *fwd += nt;
        } else {
            const int64_t rpt = std::max<int64_t>(1, 2 * tile / std::max<int64_t>(cols, 1));
            const int64_t nt = ceil_div(rows > 0 ? rows : 1, rpt);
            if (nt > 1) *bwd += nt * cols;
        }
    }
}

TileDev make_tile(int64_t t, const TaskDev &tk, int64_t begin, int64_t end, int64_t part) {
    return TileDev{(int32_t)t, tk.kind, begin, end, part, tk.cols, tk.a_off, tk.b_off, tk.out_off};
}

mx_status build_tiles(mx_batch_plan *p) {
    const int64_t T = p->cfg.tile_elems;
    std::vector<TaskDev> tasks((size_t)p->ntasks);
    std::vector<TileDev> fwd, bwd;
    std::vector<int32_t> fwd_list, bwd_list;
    int64_t fpart = 0, bpart = 0, max_cols = 1;
    for (int64_t t = 0; t < p->ntasks; ++t) {
        const int64_t *r = &p->table[(size_t)(6 * t)];
        TaskDev &tk = tasks[(size_t)t];
        tk.kind = (int32_t)r[0];
        tk.rows = r[1];
        tk.cols = r[2];
        tk.a_off = r[3];
        tk.b_off = r[4];
        tk.out_off = r[5];
        if (tk.kind == kDot) {
            const int64_t n = tk.cols;
            const int64_t nt = std::max<int64_t>(1, ceil_div(n, T));
            tk.fwd_ntiles = nt;
            tk.fwd_part = nt > 1 ? fpart : -1;
            for (int64_t q = 0; q < nt; ++q)
                fwd.push_back(make_tile(t, tk, q * T, std::min(n, (q + 1) * T), nt > 1 ? fpart + q : -1));
            if (nt > 1) {
                fwd_list.push_back((int32_t)t);
                fpart += nt;
            }
            for (int64_t q = 0; q < nt; ++q)
                bwd.push_back(make_tile(t, tk, q * T, std::min(n, (q + 1) * T), -1));
            tk.bwd_ntiles = nt;
            tk.bwd_part = -1;
        } else {
            const int64_t c = std::max<int64_t>(tk.cols, 1);
            // a matvec streams one operand (4 bytes per element) where a dot
            // streams two: twice the elements give tiles of equal bytes
            const int64_t rpt = std::max<int64_t>(1, 2 * T / c);
            const int64_t nt = std::max<int64_t>(1, ceil_div(tk.rows, rpt));
            tk.fwd_ntiles = nt;
            tk.fwd_part = -1;
            tk.bwd_ntiles = nt;
            tk.bwd_part = nt > 1 ? bpart : -1;
            for (int64_t q = 0; q < nt; ++q) {
                const int64_t b = q * rpt, e = std::min(tk.rows, (q + 1) * rpt);
                fwd.push_back(make_tile(t, tk, b, e, -1));
                bwd.push_back(make_tile(t, tk, b, e, nt > 1 ? bpart + q * tk.cols : -1));
            }
            if (nt > 1) {
                bwd_list.push_back((int32_t)t);
                bpart += nt * tk.cols;
                max_cols = std::max(max_cols, tk.cols);
            }
        }
    }
    // longest first (stable: ties keep task order, so plans are reproducible)
    auto cost = [&](const TileDev &x) {
        const TaskDev &tk = tasks[(size_t)x.task];
        return tk.kind == kDot ? (x.end - x.begin) : (x.end - x.begin) * tk.cols;
    };
    std::stable_sort(fwd.begin(), fwd.end(), [&](const TileDev &x, const TileDev &y) { return cost(x) > cost(y); });
    std::stable_sort(bwd.begin(), bwd.end(), [&](const TileDev &x, const TileDev &y) { return cost(x) > cost(y); });
    MX_REQUIRE((int64_t)fwd.size() < (1LL << 31) && (int64_t)bwd.size() < (1LL << 31), MX_ERR_SHAPE,
               "mx_batch_plan: too many tiles");
    free_device(p);
    auto up = [](auto **dst, const auto &v) -> mx_status {
        using E = typename std::decay_t<decltype(v)>::value_type;
        const size_t bytes = std::max<size_t>(v.size() * sizeof(E), 16);
        MX_TRY_HIP(hipMalloc((void **)dst, bytes));
        if (!v.empty()) MX_TRY_HIP(hipMemcpy(*dst, v.data(), v.size() * sizeof(E), hipMemcpyHostToDevice));
        return MX_OK;
    };
    if (mx_status st = up(&p->d_tasks, tasks)) return st;
    if (mx_status st = up(&p->d_fwd, fwd)) return st;
    if (mx_status st = up(&p->d_bwd, bwd)) return st;
    if (mx_status st = up(&p->d_fwd_list, fwd_list)) return st;
    if (mx_status st = up(&p->d_bwd_list, bwd_list)) return st;
    p->n_fwd = (int64_t)fwd.size();
    p->n_bwd = (int64_t)bwd.size();
    p->n_fwd_list = (int64_t)fwd_list.size();
    p->n_bwd_list = (int64_t)bwd_list.size();
    p->bwd_list_max_cols = max_cols;
    p->fwd_part_floats = fpart;
    p->bwd_part_floats = bpart;
    return MX_OK;
}

size_t plan_ws_bytes(const mx_batch_plan *p) {
    int64_t f, b;
    partial_floats(p->table, p->ntasks, kMinTile, &f, &b);
    return kCounterBytes + align256((size_t)f * 4) + align256((size_t)b * 4);
}

mx_status check_ws(const char *who, const mx_batch_plan *p, void *ws, size_t ws_bytes) {
    MX_REQUIRE(p, MX_ERR_INVALID, "%s: null plan", who);
    MX_REQUIRE(ws && ws_bytes >= p->ws_need && ((uintptr_t)ws & 255) == 0, MX_ERR_WORKSPACE,
               "%s: workspace needs %zu bytes, 256-byte aligned", who, p->ws_need);
    return MX_OK;
}

float *fwd_part_ptr(const mx_batch_plan *p, void *ws) { return (float *)((char *)ws + kCounterBytes); }
float *bwd_part_ptr(const mx_batch_plan *p, void *ws) {
    int64_t f, b;
    partial_floats(p->table, p->ntasks, kMinTile, &f, &b);
    return (float *)((char *)ws + kCounterBytes + align256((size_t)f * 4));
}

int grid_of(const mx_batch_plan *p, int64_t ntiles) {
    int64_t g = (int64_t)p->num_cus * p->cfg.blocks_per_cu;
    if (g > ntiles) g = ntiles;
    return (int)std::max<int64_t>(g, 1);
}

mx_status fwd_impl(const mx_batch_plan *p, const float *A, const float *B, float *out, void *ws, hipStream_t s) {
    unsigned *ticket = (unsigned *)ws;
    float *part = fwd_part_ptr(p, ws);
    const int vec = aligned16(A) && aligned16(B);
    hipLaunchKernelGGL(k_batch_fwd, dim3(grid_of(p, p->n_fwd)), dim3(NT), 0, s, p->d_tasks, p->d_fwd, p->n_fwd, A, B,
                       out, part, ticket, vec);
    hipLaunchKernelGGL(k_batch_combine_fwd, dim3((unsigned)std::max<int64_t>(1, ceil_div(p->n_fwd_list, NT))),
                       dim3(NT), 0, s, p->d_tasks, p->d_fwd_list, p->n_fwd_list, part, out, ticket);
    return last_launch("mx_batch_forward");
}

mx_status bwd_impl(const mx_batch_plan *p, const float *A, const float *B, const float *gout, float *gA, float *gB,
                   void *ws, hipStream_t s) {
    unsigned *ticket = (unsigned *)ws + 1;
    float *part = bwd_part_ptr(p, ws);
    const int vec = aligned16(A) && aligned16(B) && aligned16(gA) && aligned16(gB);
    hipLaunchKernelGGL(k_batch_bwd, dim3(grid_of(p, p->n_bwd)), dim3(NT), 0, s, p->d_tasks, p->d_bwd, p->n_bwd, A, B,
                       gout, gA, gB, part, ticket, vec);
    const dim3 cgrid((unsigned)std::max<int64_t>(1, p->n_bwd_list),
                     (unsigned)std::min<int64_t>(1024, ceil_div(p->bwd_list_max_cols, NT)));
    hipLaunchKernelGGL(k_batch_combine_bwd, cgrid, dim3(NT), 0, s,
                       p->d_tasks, p->d_bwd_list, p->n_bwd_list, part, gB, ticket);
    return last_launch("mx_batch_backward");
}

uint64_t fnv1a(const void *data, size_t n, uint64_t h = 1469598103934665603ull) {
    const unsigned char *c = (const unsigned char *)data;
    for (size_t i = 0; i < n; ++i) {
        h ^= c[i];
        h *= 1099511628211ull;
    }
    return h;
}

std::string cache_key(const mx_batch_plan *p) {
    // sizes and kinds only: offsets do not change the work
    std::vector<int64_t> shape;
    shape.reserve((size_t)p->ntasks * 3);
    for (int64_t t = 0; t < p->ntasks; ++t)
        for (int c = 0; c < 3; ++c) shape.push_back(p->table[(size_t)(6 * t + c)]);
    hipDeviceProp_t prop;
    char name[300] = "unknown";
    if (hipGetDeviceProperties(&prop, p->device) == hipSuccess) snprintf(name, sizeof name, "%s", prop.gcnArchName);
    char buf[128];
    snprintf(buf, sizeof buf, "%016llx-%s", (unsigned long long)fnv1a(shape.data(), shape.size() * 8), name);
    return buf;
}

bool cache_lookup(const char *path, const std::string &key, mx_batch_config *cfg) {
    std::ifstream f(path);
    if (!f) return false;
    std::string line;
    bool found = false;
    while (std::getline(f, line)) {
        // one JSON object per line: {"key": "...", "tile_elems": N, "blocks_per_cu": M, "us": X}
        if (line.find("\"" + key + "\"") == std::string::npos) continue;
        int te = 0, bpc = 0;
        const size_t a = line.find("\"tile_elems\":"), b = line.find("\"blocks_per_cu\":");
        if (a == std::string::npos || b == std::string::npos) continue;
        te = std::atoi(line.c_str() + a + 13);
        bpc = std::atoi(line.c_str() + b + 16);
        if (te >= kMinTile && bpc >= 1 && bpc <= 32) {
            cfg->tile_elems = te;
            cfg->blocks_per_cu = bpc;
            found = true;  // the last matching line wins
        }
    }
    return found;
}

}  // namespace

extern "C" {

mx_status mx_batch_plan_create(const int64_t *table_host, int64_t ntasks, const mx_batch_config *cfg,
                               mx_batch_plan **plan) {
    MX_REQUIRE(plan, MX_ERR_INVALID, "mx_batch_plan_create: null output");
    *plan = nullptr;
    MX_REQUIRE(ntasks >= 0 && ntasks < (1LL << 31), MX_ERR_SHAPE, "mx_batch_plan_create: bad ntasks");
    MX_REQUIRE(ntasks == 0 || table_host, MX_ERR_INVALID, "mx_batch_plan_create: null table");
    const DeviceInfo *d;
    if (mx_status st = device_info(&d)) return st;
    auto *p = new mx_batch_plan();
    p->device = d->device;
    p->num_cus = d->num_cus;
    p->ntasks = ntasks;
    p->table.assign(table_host, table_host + 6 * ntasks);
    for (int64_t t = 0; t < ntasks; ++t) {
        const int64_t *r = table_host + 6 * t;
        if (!((r[0] == kDot && r[1] == 1) || r[0] == kMatvec) || r[1] < 0 || r[2] < 0 || r[3] < 0 || r[4] < 0 ||
            r[5] < 0) {
            delete p;
            return set_error(MX_ERR_SHAPE, "mx_batch_plan_create: bad task %lld", (long long)t);
        }
        p->a_len = std::max(p->a_len, r[3] + r[1] * r[2]);
        p->b_len = std::max(p->b_len, r[4] + r[2]);
        p->out_len = std::max(p->out_len, r[5] + (r[0] == kDot ? 1 : r[1]));
    }
    p->cfg.tile_elems = cfg ? cfg->tile_elems : 16384;
    p->cfg.blocks_per_cu = cfg ? cfg->blocks_per_cu : 8;
    if (p->cfg.tile_elems < kMinTile || p->cfg.blocks_per_cu < 1 || p->cfg.blocks_per_cu > 32) {
        delete p;
        return set_error(MX_ERR_INVALID, "mx_batch_plan_create: need tile_elems >= %d and 1 <= blocks_per_cu <= 32",
                         kMinTile);
    }
    p->ws_need = plan_ws_bytes(p);
    if (mx_status st = build_tiles(p)) {
        free_device(p);
        delete p;
        return st;
    }
    *plan = p;
    return MX_OK;
}

mx_status mx_batch_plan_destroy(mx_batch_plan *plan) {
    if (!plan) return MX_OK;
    free_device(plan);
    delete plan;
    return MX_OK;
}

size_t mx_batch_workspace_bytes(const mx_batch_plan *plan) { return plan ? plan->ws_need : 0; }

mx_status mx_batch_get_config(const mx_batch_plan *plan, mx_batch_config *cfg) {
    MX_REQUIRE(plan && cfg, MX_ERR_INVALID, "mx_batch_get_config: null pointer");
    *cfg = plan->cfg;
    return MX_OK;
}

mx_status mx_batch_set_config(mx_batch_plan *plan, const mx_batch_config *cfg) {
    MX_REQUIRE(plan && cfg, MX_ERR_INVALID, "mx_batch_set_config: null pointer");
    MX_REQUIRE(cfg->tile_elems >= kMinTile && cfg->blocks_per_cu >= 1 && cfg->blocks_per_cu <= 32, MX_ERR_INVALID,
               "mx_batch_set_config: need tile_elems >= %d and 1 <= blocks_per_cu <= 32", kMinTile);
    plan->cfg.tile_elems = cfg->tile_elems;
    plan->cfg.blocks_per_cu = cfg->blocks_per_cu;
    return build_tiles(plan);
}

mx_status mx_batch_forward(const mx_batch_plan *plan, const float *A_dev, const float *B_dev, float *out_dev,
                           void *ws, size_t ws_bytes, hipStream_t stream) {
    if (mx_status st = check_ws("mx_batch_forward", plan, ws, ws_bytes)) return st;
    if (plan->ntasks == 0) return MX_OK;
    MX_REQUIRE(A_dev && B_dev && out_dev, MX_ERR_INVALID, "mx_batch_forward: null pointer");
    return fwd_impl(plan, A_dev, B_dev, out_dev, ws, stream);
}

mx_status mx_batch_backward(const mx_batch_plan *plan, const float *A_dev, const float *B_dev, const float *gout_dev,
                            float *gA_dev, float *gB_dev, void *ws, size_t ws_bytes, hipStream_t stream) {
    if (mx_status st = check_ws("mx_batch_backward", plan, ws, ws_bytes)) return st;
    if (plan->ntasks == 0) return MX_OK;
    MX_REQUIRE(A_dev && B_dev && gout_dev && gA_dev && gB_dev, MX_ERR_INVALID, "mx_batch_backward: null pointer");
    return bwd_impl(plan, A_dev, B_dev, gout_dev, gA_dev, gB_dev, ws, stream);
}

mx_status mx_batch_forward_plain(const mx_batch_plan *plan, const float *A_dev, const float *B_dev, float *out_dev,
                                 hipStream_t stream) {
    MX_REQUIRE(plan, MX_ERR_INVALID, "mx_batch_forward_plain: null plan");
    if (plan->ntasks == 0) return MX_OK;
    MX_REQUIRE(A_dev && B_dev && out_dev, MX_ERR_INVALID, "mx_batch_forward_plain: null pointer");
    for (int64_t t = 0; t < plan->ntasks; ++t) {
        const int64_t *r = &plan->table[(size_t)(6 * t)];
        if (r[0] == kDot)
            hipLaunchKernelGGL(k_dot_plain, dim3(1), dim3(NT), 0, stream, A_dev + r[3], B_dev + r[4], r[2],
                               out_dev + r[5]);
        else if (r[1] > 0)
            hipLaunchKernelGGL(k_matvec_plain, dim3((unsigned)ceil_div(r[1], NT)), dim3(NT), 0, stream, A_dev + r[3],
                               B_dev + r[4], r[1], r[2], out_dev + r[5]);
    }
    return last_launch("mx_batch_forward_plain");
}

mx_status mx_batch_backward_plain(const mx_batch_plan *plan, const float *A_dev, const float *B_dev,
                                  const float *gout_dev, float *gA_dev, float *gB_dev, hipStream_t stream) {
    MX_REQUIRE(plan, MX_ERR_INVALID, "mx_batch_backward_plain: null plan");
    if (plan->ntasks == 0) return MX_OK;
    MX_REQUIRE(A_dev && B_dev && gout_dev && gA_dev && gB_dev, MX_ERR_INVALID, "mx_batch_backward_plain: null pointer");
    for (int64_t t = 0; t < plan->ntasks; ++t) {
        const int64_t *r = &plan->table[(size_t)(6 * t)];
        if (r[0] == kDot) {
            if (r[2] > 0)
                hipLaunchKernelGGL(k_dot_adj_plain, dim3((unsigned)ceil_div(r[2], NT)), dim3(NT), 0, stream,
                                   A_dev + r[3], B_dev + r[4], r[2], gout_dev + r[5], gA_dev + r[3], gB_dev + r[4]);
        } else if (r[2] > 0) {
            hipLaunchKernelGGL(k_matvec_adj_plain, dim3((unsigned)ceil_div(r[2], NT)), dim3(NT), 0, stream,
                               A_dev + r[3], B_dev + r[4], r[1], r[2], gout_dev + r[5], gA_dev + r[3], gB_dev + r[4]);
        }
    }
    return last_launch("mx_batch_backward_plain");
}

mx_status mx_batch_autotune(mx_batch_plan *plan, const float *A_dev, const float *B_dev, float *out_dev,
                            const float *gout_dev, float *gA_dev, float *gB_dev, void *ws, size_t ws_bytes,
                            const char *cache_path, hipStream_t stream, mx_batch_config *chosen) {
    const char *who = "mx_batch_autotune";
    if (mx_status st = check_ws(who, plan, ws, ws_bytes)) return st;
    MX_REQUIRE(A_dev && B_dev && out_dev && gout_dev && gA_dev && gB_dev, MX_ERR_INVALID, "%s: null pointer", who);
    const std::string key = cache_key(plan);
    mx_batch_config best = plan->cfg;
    if (cache_path && cache_lookup(cache_path, key, &best)) {
        if (mx_status st = mx_batch_set_config(plan, &best)) return st;
        if (chosen) *chosen = plan->cfg;
        return MX_OK;
    }
    static const int tiles[] = {4096, 8192, 16384, 32768, 65536};
    static const int bpcs[] = {2, 4, 8, 16};
    hipEvent_t e0, e1;
    MX_TRY_HIP(hipEventCreate(&e0));
    MX_TRY_HIP(hipEventCreate(&e1));
    float best_us = 1e30f;
    mx_status rc = MX_OK;
    for (int te : tiles) {
        for (int bpc : bpcs) {
            mx_batch_config c{te, bpc, {0, 0}};
            if ((rc = mx_batch_set_config(plan, &c))) goto done;
            // one warm pass, then the minimum of three timed passes of forward + backward
            if ((rc = fwd_impl(plan, A_dev, B_dev, out_dev, ws, stream))) goto done;
            if ((rc = bwd_impl(plan, A_dev, B_dev, gout_dev, gA_dev, gB_dev, ws, stream))) goto done;
            float tmin = 1e30f;
            for (int rep = 0; rep < 3; ++rep) {
                if (hipEventRecord(e0, stream) != hipSuccess) { rc = hip_error(hipGetLastError(), "hipEventRecord"); goto done; }
                if ((rc = fwd_impl(plan, A_dev, B_dev, out_dev, ws, stream))) goto done;
                if ((rc = bwd_impl(plan, A_dev, B_dev, gout_dev, gA_dev, gB_dev, ws, stream))) goto done;
                if (hipEventRecord(e1, stream) != hipSuccess) { rc = hip_error(hipGetLastError(), "hipEventRecord"); goto done; }
                if (hipEventSynchronize(e1) != hipSuccess) { rc = hip_error(hipGetLastError(), "hipEventSynchronize"); goto done; }
                float ms = 0.f;
                (void)hipEventElapsedTime(&ms, e0, e1);
                tmin = std::min(tmin, ms * 1000.f);
            }
            if (tmin < best_us) {
                best_us = tmin;
                best = c;
            }
        }
    }
    if ((rc = mx_batch_set_config(plan, &best))) goto done;
    if (cache_path) {
        FILE *f = fopen(cache_path, "a");
        if (f) {
            fprintf(f, "{\"key\": \"%s\", \"tile_elems\": %d, \"blocks_per_cu\": %d, \"us\": %.1f}\n", key.c_str(),
                    best.tile_elems, best.blocks_per_cu, best_us);
            fclose(f);
        }
    }
    if (chosen) *chosen = plan->cfg;
done:
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}

}  // extern "C"
