// Kernels of the shapes in the paper's Parboil comparison (Table 1): the
// histogram reduce-by-key (histo), the neighbour-access map of a 7-point
// stencil sweep (stencil), the trigonometric per-output reduction over
// samples (mri-q) and the pairwise angular histogram (tpacf).  The paper's Futhark programs for these are compiled
// whole; here each is one gfx950 kernel family behind the C ABI.
#include <algorithm>
#include <cmath>

#include "mx_internal.h"

namespace mx {
namespace {

constexpr int NT = 256;
constexpr int64_t kHistLdsBins = 32768;  // 128 KiB of LDS counters per block

__global__ void __launch_bounds__(NT) k_zero32(uint32_t *__restrict__ p, int64_t m) {
    const int64_t stride = (int64_t)gridDim.x * NT;
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < m; i += stride) p[i] = 0u;
}

// ---------------------------------------------------------------- histo
// Few bins: each block counts its keys into private LDS histograms (LDS
// integer atomics), then adds its non-zero bins to the global counts.  With
// `copies` > 1 lane l counts into copy l % copies (copies nbins + 1 words
// apart, so equal bins of different copies sit in different banks): lanes of
// one instruction that hit the same bin wait for each other `copies` times
// less.  Blocks of 1024 threads: the copies fill 64 KiB at 4096 bins, so two
// blocks fit a CU, and 32 waves keep the key loads and atomics in flight.
// Integer additions commute, so the counts do not depend on the order.
constexpr int NTH = 1024;
__global__ void __launch_bounds__(NTH) k_hist_lds(const uint32_t *__restrict__ keys, int64_t n, int nbins,
                                                 int copies, uint32_t *__restrict__ counts, int vec) {
    extern __shared__ uint32_t hist_all[];
    const int stride = nbins + 1;
    for (int b = threadIdx.x; b < stride * copies; b += NTH) hist_all[b] = 0u;
    __syncthreads();
    uint32_t *hist = hist_all + (threadIdx.x % copies) * stride;
    const int64_t tid = (int64_t)blockIdx.x * NTH + threadIdx.x, nt = (int64_t)gridDim.x * NTH;
    const uint32_t nb = (uint32_t)nbins;
    int64_t done = 0;
    if (vec) {
        const int64_t nv = n / 4;
        const uint4 *kv = reinterpret_cast<const uint4 *>(keys);
        // four 16-byte loads in flight before their atomics (keys past the
        // end read as ~0, which no bin takes)
        for (int64_t j = tid; j < nv; j += 4 * nt) {
            uint4 k[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) k[u] = j + u * nt < nv ? kv[j + u * nt] : make_uint4(~0u, ~0u, ~0u, ~0u);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (k[u].x < nb) atomicAdd(&hist[k[u].x], 1u);
                if (k[u].y < nb) atomicAdd(&hist[k[u].y], 1u);
                if (k[u].z < nb) atomicAdd(&hist[k[u].z], 1u);
                if (k[u].w < nb) atomicAdd(&hist[k[u].w], 1u);
            }
        }
        done = nv * 4;
    }
    for (int64_t i = done + tid; i < n; i += nt) {
        const uint32_t k = keys[i];
        if (k < nb) atomicAdd(&hist[k], 1u);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < nbins; b += NTH) {
        uint32_t c = 0u;
        for (int q = 0; q < copies; ++q) c += hist_all[q * stride + b];
        if (c) atomicAdd(&counts[b], c);
    }
}

// Many bins: integer atomics on the global counts.
__global__ void __launch_bounds__(NT) k_hist_global(const uint32_t *__restrict__ keys, int64_t n, int64_t nbins,
                                                    uint32_t *__restrict__ counts, int vec) {
    const int64_t tid = (int64_t)blockIdx.x * NT + threadIdx.x, nt = (int64_t)gridDim.x * NT;
    int64_t done = 0;
    if (vec) {
        const int64_t nv = n / 4;
        const uint4 *kv = reinterpret_cast<const uint4 *>(keys);
        for (int64_t j = tid; j < nv; j += nt) {
            const uint4 k = kv[j];
            if ((int64_t)k.x < nbins) atomicAdd(&counts[k.x], 1u);
            if ((int64_t)k.y < nbins) atomicAdd(&counts[k.y], 1u);
            if ((int64_t)k.z < nbins) atomicAdd(&counts[k.z], 1u);
            if ((int64_t)k.w < nbins) atomicAdd(&counts[k.w], 1u);
        }
        done = nv * 4;
    }
    for (int64_t i = done + tid; i < n; i += nt) {
        const uint32_t k = keys[i];
        if ((int64_t)k < nbins) atomicAdd(&counts[k], 1u);
    }
}

// Many bins with a workspace: bucket the keys first.  Bucket b holds the
// bins [b 2^w, (b + 1) 2^w), at most 4096 buckets of 2048..32768 bins.
// (1) every block counts its chunk of keys per bucket in LDS and writes one
// column of the bucket-major count matrix; (2) an exclusive scan of the
// matrix gives every (bucket, block) its place; (3) every block re-reads its
// chunk and writes each key's bin-within-bucket (16 bits) to its bucket's
// range, places taken with LDS atomics; (4) one block per bucket counts its
// range in an LDS histogram and writes the bucket's bins.  Every bin is
// written once, by one block: no global atomics and no zero-fill of the
// counts.  Global atomics on 2^20 counters cost a 32-byte memory-side write
// each on this GPU; the four passes move about 12 bytes per key.
constexpr int64_t kHbChunk = 16384;   // keys per block in passes 1 and 3 (at least)
constexpr int64_t kHbMaxBlocks = 2048;
constexpr int64_t kHbMaxBuckets = 4096;
constexpr int kHbMinShift = 11, kHbMaxShift = 15;
constexpr int NTB = 1024;  // threads per bucket block in pass 4

struct HbPlan {
    bool ok;            // the bucketed passes apply
    int w;              // log2 of the bins per bucket
    int64_t nb, g;      // buckets, blocks of passes 1 and 3
    int64_t chunk;      // keys per block (a multiple of 4)
    size_t scan_bytes, cnt_off, off_off, sorted_off, bytes;
};

HbPlan hb_plan(int64_t n, int64_t nbins) {
    HbPlan p{};
    int w = kHbMinShift;
    while (w < kHbMaxShift && ((int64_t)512 << w) < nbins) ++w;  // about 512 buckets where possible
    p.w = w;
    p.nb = ceil_div(nbins, (int64_t)1 << w);
    p.ok = nbins > kHistLdsBins && p.nb <= kHbMaxBuckets;
    p.g = std::min<int64_t>(kHbMaxBlocks, std::max<int64_t>(1, ceil_div(n, kHbChunk)));
    p.chunk = ceil_div(ceil_div(std::max<int64_t>(n, 1), p.g), (int64_t)4) * 4;
    const int64_t m = p.g * p.nb;
    p.scan_bytes = mx_workspace_bytes(MX_WS_SCAN, m, 0);
    p.cnt_off = align256(p.scan_bytes);
    p.off_off = p.cnt_off + align256((size_t)m * 8);
    p.sorted_off = p.off_off + align256((size_t)(m + 1) * 8);
    p.bytes = p.sorted_off + align256((size_t)std::max<int64_t>(n, 1) * 2);
    return p;
}

// Passes 1 and 3 walk their block's keys in pieces of kHbPiece, every thread
// loading its kHbPiece / NTS keys of the piece before it uses any (all loads
// in flight at once; keys past the end read as ~0, which no bin takes).
constexpr int kHbPiece = 16384;
constexpr int NTS = 1024;  // threads per block of passes 1 and 3
constexpr int kHbKpt = kHbPiece / NTS;

__device__ __forceinline__ void hb_load_piece(const uint32_t *__restrict__ keys, int64_t p0, int cnt,
                                              uint32_t (&kk)[kHbKpt]) {
#pragma unroll
    for (int u = 0; u < kHbKpt; ++u) {
        const int i = (int)threadIdx.x + u * NTS;
        kk[u] = i < cnt ? keys[p0 + i] : ~0u;
    }
}

__global__ void __launch_bounds__(NTS) k_hb_count(const uint32_t *__restrict__ keys, int64_t n, int64_t nbins,
                                                  int64_t chunk, int w, int nb, int64_t g,
                                                  int64_t *__restrict__ cnt) {
    extern __shared__ uint32_t bc[];
    for (int b = threadIdx.x; b < nb; b += NTS) bc[b] = 0u;
    __syncthreads();
    const int64_t lo = (int64_t)blockIdx.x * chunk, hi = lo + chunk < n ? lo + chunk : n;
    for (int64_t p0 = lo; p0 < hi; p0 += kHbPiece) {
        uint32_t kk[kHbKpt];
        hb_load_piece(keys, p0, (int)(hi - p0 < kHbPiece ? hi - p0 : kHbPiece), kk);
#pragma unroll
        for (int u = 0; u < kHbKpt; ++u)
            if ((int64_t)kk[u] < nbins) atomicAdd(&bc[kk[u] >> w], 1u);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < nb; b += NTS) cnt[(int64_t)b * g + blockIdx.x] = bc[b];
}

// In-place exclusive scan of a[0..m) in LDS by the whole block of BS
// threads; returns the total.  Thread t owns the entries [t per, (t + 1) per).
template <int BS> __device__ __forceinline__ uint32_t hb_block_scan(uint32_t *a, int m) {
    __shared__ uint32_t wsum[BS / 64];
    const int per = (m + BS - 1) / BS;
    const int b0 = threadIdx.x * per, b1 = b0 + per < m ? b0 + per : m;
    uint32_t s = 0u;
    for (int i = b0; i < b1; ++i) s += a[i];
    uint32_t x = s;  // inclusive scan over the wave
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) wsum[threadIdx.x >> 6] = x;
    __syncthreads();
    uint32_t base = 0u, total = 0u;
#pragma unroll
    for (int q = 0; q < BS / 64; ++q) {
        if (q < (int)(threadIdx.x >> 6)) base += wsum[q];
        total += wsum[q];
    }
    uint32_t run = base + x - s;
    for (int i = b0; i < b1; ++i) {
        const uint32_t v = a[i];
        a[i] = run;
        run += v;
    }
    __syncthreads();
    return total;
}

// Pass 3, per piece: rank each key within its bucket (LDS atomics, ranks kept
// in registers), scan the piece's bucket counts, stage the keys in LDS in
// bucket order, then write each bucket's run to its place: consecutive lanes
// write consecutive 16-bit entries.  LDS: 2 nb words + 2 kHbPiece half-words.
__global__ void __launch_bounds__(NTS) k_hb_scatter(const uint32_t *__restrict__ keys, int64_t n, int64_t nbins,
                                                    int64_t chunk, int w, int nb, int64_t g,
                                                    const int64_t *__restrict__ off,
                                                    uint16_t *__restrict__ sorted) {
    extern __shared__ uint32_t sm[];
    uint32_t *lc = sm, *cur = sm + nb;
    uint16_t *sbin = reinterpret_cast<uint16_t *>(sm + 2 * nb), *sbkt = sbin + kHbPiece;
    for (int b = threadIdx.x; b < nb; b += NTS) cur[b] = (uint32_t)off[(int64_t)b * g + blockIdx.x];
    const int64_t lo = (int64_t)blockIdx.x * chunk, hi = lo + chunk < n ? lo + chunk : n;
    const uint32_t mask = (1u << w) - 1u;
    for (int64_t p0 = lo; p0 < hi; p0 += kHbPiece) {
        uint32_t kk[kHbKpt], rk[kHbKpt];
        hb_load_piece(keys, p0, (int)(hi - p0 < kHbPiece ? hi - p0 : kHbPiece), kk);
        for (int b = threadIdx.x; b < nb; b += NTS) lc[b] = 0u;
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kHbKpt; ++u) rk[u] = (int64_t)kk[u] < nbins ? atomicAdd(&lc[kk[u] >> w], 1u) : 0u;
        __syncthreads();
        const uint32_t tot = hb_block_scan<NTS>(lc, nb);
#pragma unroll
        for (int u = 0; u < kHbKpt; ++u) {
            if ((int64_t)kk[u] < nbins) {
                const uint32_t pos = lc[kk[u] >> w] + rk[u];
                sbin[pos] = (uint16_t)(kk[u] & mask);
                sbkt[pos] = (uint16_t)(kk[u] >> w);
            }
        }
        __syncthreads();
        for (int i = threadIdx.x; i < (int)tot; i += NTS) {
            const int b = sbkt[i];
            sorted[cur[b] + ((uint32_t)i - lc[b])] = sbin[i];
        }
        __syncthreads();
        for (int b = threadIdx.x; b < nb; b += NTS) cur[b] += (b + 1 < nb ? lc[b + 1] : tot) - lc[b];
        __syncthreads();
    }
}

// Pass 4: one block per bucket; 16-byte loads of eight entries, four in
// flight per thread, between an unaligned head and tail.
__global__ void __launch_bounds__(NTB) k_hb_bins(const uint16_t *__restrict__ sorted, const int64_t *__restrict__ off,
                                                 int64_t g, int w, int64_t nbins, uint32_t *__restrict__ counts) {
    extern __shared__ uint32_t h[];
    const int nbb = 1 << w;
    for (int i = threadIdx.x; i < nbb; i += NTB) h[i] = 0u;
    __syncthreads();
    const int64_t b = blockIdx.x;
    const int64_t s = off[b * g], e = off[(b + 1) * g];
    int64_t a0 = (s + 7) & ~(int64_t)7;
    if (a0 > e) a0 = e;
    for (int64_t i = s + threadIdx.x; i < a0; i += NTB) atomicAdd(&h[sorted[i]], 1u);
    const int64_t nv = (e - a0) / 8, a1 = a0 + nv * 8;
    const uint4 *v = reinterpret_cast<const uint4 *>(sorted + a0);
    auto count8 = [&](uint4 q) {
        atomicAdd(&h[q.x & 0xffffu], 1u);
        atomicAdd(&h[q.x >> 16], 1u);
        atomicAdd(&h[q.y & 0xffffu], 1u);
        atomicAdd(&h[q.y >> 16], 1u);
        atomicAdd(&h[q.z & 0xffffu], 1u);
        atomicAdd(&h[q.z >> 16], 1u);
        atomicAdd(&h[q.w & 0xffffu], 1u);
        atomicAdd(&h[q.w >> 16], 1u);
    };
    int64_t j = threadIdx.x;
    for (; j + 3 * NTB < nv; j += 4 * NTB) {
        const uint4 q0 = v[j], q1 = v[j + NTB], q2 = v[j + 2 * NTB], q3 = v[j + 3 * NTB];
        count8(q0);
        count8(q1);
        count8(q2);
        count8(q3);
    }
    for (; j < nv; j += NTB) count8(v[j]);
    for (int64_t i = a1 + threadIdx.x; i < e; i += NTB) atomicAdd(&h[sorted[i]], 1u);
    __syncthreads();
    const int64_t base = b << w;
    const int64_t m = nbins - base < nbb ? nbins - base : nbb;
    for (int64_t i = threadIdx.x; i < m; i += NTB) counts[base + i] = h[i];
}

// ---------------------------------------------------------------- stencil
// One Jacobi sweep of the 7-point stencil.  A thread owns one (x, y) column
// and marches up a slab of kSlab planes keeping the z - 1, z and z + 1 values
// in registers, so each input value is read from HBM about once; the four
// in-plane neighbours are cache hits of the neighbouring lanes' loads.  The
// six neighbours are added x-, x+, y-, y+, z-, z+ and every operation is
// rounded on its own.  Boundary points are copied.
constexpr int kSlab = 16;

// Blocks are dealt to the 8 XCDs in turn, each XCD with its own L2; the
// column tiles are renumbered so that XCD k takes one contiguous band of
// rows, and the rows above and below a tile are mostly in the same L2.
__global__ void __launch_bounds__(NT) k_stencil7(const float *__restrict__ in, float *__restrict__ out, int64_t nx,
                                                 int64_t ny, int64_t nz, float c0, float c1) {
#pragma clang fp contract(off)
    const int64_t ntiles = gridDim.x, per = ntiles / 8;
    int64_t tile = blockIdx.x;
    if (tile < per * 8) tile = (tile % 8) * per + tile / 8;
    const int64_t col = tile * NT + threadIdx.x;
    if (col >= nx * ny) return;
    const int64_t y = col / nx, x = col - y * nx;
    const int64_t z0 = (int64_t)blockIdx.y * kSlab;
    const int64_t z1 = z0 + kSlab < nz ? z0 + kSlab : nz;
    const int64_t plane = nx * ny;
    const bool edge = x == 0 || y == 0 || x == nx - 1 || y == ny - 1;
    const float *p = in + col;
    float below = z0 > 0 ? p[(z0 - 1) * plane] : 0.f;
    float cur = p[z0 * plane];
    for (int64_t z = z0; z < z1; ++z) {
        const float above = z + 1 < nz ? p[(z + 1) * plane] : 0.f;
        const int64_t i = z * plane + col;
        float r;
        if (edge || z == 0 || z == nz - 1) {
            r = cur;
        } else {
            float s = in[i - 1];
            s = s + in[i + 1];
            s = s + in[i - nx];
            s = s + in[i + nx];
            s = s + below;
            s = s + above;
            r = c1 * s - c0 * cur;
        }
        out[i] = r;
        below = cur;
        cur = above;
    }
}

// ---------------------------------------------------------------- mri-q
// Qr_i = sum_k phi_k cos(2 pi t_ik), Qi_i = sum_k phi_k sin(2 pi t_ik) with
// t_ik = kx_k x_i + ky_k y_i + kz_k z_i.  The samples go through LDS in tiles
// (every lane reads the same sample: a broadcast); each thread owns two
// voxels.  sin and cos of 2 pi t come from the hardware sine and cosine,
// whose argument is in revolutions, so the angle is never multiplied by pi
// in floating point: t is first reduced to r = t - rint(t) in [-1/2, 1/2]
// (exact for every float) and v_sin / v_cos take r.  Their absolute error,
// measured against binary64 over 2^24 arguments in [-24, 24], is at most
// 1.26e-7 (2.1 units of 2^-24), against 5.1e-8 for the library sincospi,
// which costs about 30 more instructions per pair.
constexpr int kMriTile = 1024;

__global__ void __launch_bounds__(NT) k_mriq(const float *__restrict__ kx, const float *__restrict__ ky,
                                             const float *__restrict__ kz, const float *__restrict__ phi,
                                             int64_t nk, const float *__restrict__ x, const float *__restrict__ y,
                                             const float *__restrict__ z, int64_t nv, float *__restrict__ qr,
                                             float *__restrict__ qi) {
    __shared__ float4 ks[kMriTile];
    const int64_t v0 = (int64_t)blockIdx.x * NT * 2 + threadIdx.x, v1 = v0 + NT;
    const bool h0 = v0 < nv, h1 = v1 < nv;
    const float x0 = h0 ? x[v0] : 0.f, y0 = h0 ? y[v0] : 0.f, z0 = h0 ? z[v0] : 0.f;
    const float x1 = h1 ? x[v1] : 0.f, y1 = h1 ? y[v1] : 0.f, z1 = h1 ? z[v1] : 0.f;
    float r0 = 0.f, i0 = 0.f, r1 = 0.f, i1 = 0.f;
    for (int64_t k0 = 0; k0 < nk; k0 += kMriTile) {
        const int cnt = (int)(nk - k0 < kMriTile ? nk - k0 : kMriTile);
        __syncthreads();
        for (int j = threadIdx.x; j < cnt; j += NT)
            ks[j] = make_float4(kx[k0 + j], ky[k0 + j], kz[k0 + j], phi[k0 + j]);
        __syncthreads();
        for (int j = 0; j < cnt; ++j) {
            const float4 s = ks[j];
            const float t0 = s.x * x0 + s.y * y0 + s.z * z0;
            const float t1 = s.x * x1 + s.y * y1 + s.z * z1;
            const float u0 = t0 - rintf(t0), u1 = t1 - rintf(t1);
            const float sn0 = __builtin_amdgcn_sinf(u0), cs0 = __builtin_amdgcn_cosf(u0);
            const float sn1 = __builtin_amdgcn_sinf(u1), cs1 = __builtin_amdgcn_cosf(u1);
            r0 += s.w * cs0;
            i0 += s.w * sn0;
            r1 += s.w * cs1;
            i1 += s.w * sn1;
        }
    }
    if (h0) { qr[v0] = r0; qi[v0] = i0; }
    if (h1) { qr[v1] = r1; qi[v1] = i1; }
}

// ---------------------------------------------------------------- tpacf
// Angular pair counts: a thread owns one point of set 1 and walks set 2 in
// LDS tiles (broadcast reads); per pair the binary32 dot product (three
// products, two additions, each rounded) and its bin k = #{b : d < e_b}.  The
// edges decrease, so {b : d < e_b} is a prefix and k is found by a binary
// search over a table of TB = 32 (or 64, for 32 edges) edges padded with -inf
// (d < -inf never holds, so the search never passes the m real edges), each
// probe one float compare of d with an edge as the definition has it; the
// first two levels' three pivots sit in registers, the rest are LDS reads
// (a chain of dependent reads: four pairs are searched side by side, and the
// counters take only m + 1 bins of LDS so more blocks share a CU).  Each thread then
// adds one to its own counter of bin k: counter (k, t) sits at word
// k * NT + t, so the 64 lanes of a wave always hit 64 different banks and the
// add needs no ordering.  The grid is two-dimensional: blockIdx.x picks 256
// points of set 1, blockIdx.y a chunk of set 2, so a few thousand blocks fill
// the chip even when set 1 is small.  The block's counters are summed per bin
// (wave trees, then one LDS atomic per wave) and each bin goes to the global
// int64 counts with one atomic add; integer sums, so the result does not
// depend on the order.
constexpr int kTpTile = 256;
constexpr int kTpMaxEdges = 32;
constexpr int kTpBins = kTpMaxEdges + 1;

template <int TB>  // probe table size: edges, then -inf
__global__ void __launch_bounds__(NT) k_tpacf(const float *__restrict__ x1, const float *__restrict__ y1,
                                              const float *__restrict__ z1, int64_t n1,
                                              const float *__restrict__ x2, const float *__restrict__ y2,
                                              const float *__restrict__ z2, int64_t n2, int64_t chunk,
                                              int self, const float *__restrict__ edges, int m,
                                              unsigned long long *__restrict__ counts) {
#pragma clang fp contract(off)
    __shared__ float4 tile[kTpTile];
    __shared__ float et[TB];
    __shared__ unsigned long long red[kTpBins];
    extern __shared__ uint32_t cnt[];  // [m + 1][NT]
    const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
    // this block's part of set 2; self pairs need only j > i, and the block's
    // smallest i bounds the part it needs (whole-block exit, before any barrier)
    const int64_t c0 = (int64_t)blockIdx.y * chunk;
    const int64_t jend = c0 + chunk < n2 ? c0 + chunk : n2;
    const int64_t jstart = self && (int64_t)blockIdx.x * NT + 1 > c0 ? (int64_t)blockIdx.x * NT + 1 : c0;
    if (jstart >= jend) return;
    for (int b = threadIdx.x; b < TB; b += NT) et[b] = b < m ? edges[b] : -INFINITY;
    for (int b = threadIdx.x; b < (m + 1) * NT; b += NT) cnt[b] = 0u;
    if (threadIdx.x < kTpBins) red[threadIdx.x] = 0ull;
    const bool has = i < n1;
    const float xi = has ? x1[i] : 0.f, yi = has ? y1[i] : 0.f, zi = has ? z1[i] : 0.f;
    uint32_t *mine = cnt + threadIdx.x;  // bin k of this thread at mine[k * NT]
    for (int64_t t0 = jstart; t0 < jend; t0 += kTpTile) {
        const int ct = (int)(jend - t0 < kTpTile ? jend - t0 : kTpTile);
        __syncthreads();
        for (int j = threadIdx.x; j < ct; j += NT) tile[j] = make_float4(x2[t0 + j], y2[t0 + j], z2[t0 + j], 0.f);
        __syncthreads();
        if (!has) continue;
        const float p1 = et[TB / 2 - 1], p2lo = et[TB / 4 - 1], p2hi = et[3 * TB / 4 - 1];
        const int jlo = self ? (int)(i + 1 - t0 > 0 ? (i + 1 - t0 < ct ? i + 1 - t0 : ct) : 0) : 0;
        // four pairs at a time: their searches interleave (the counter adds,
        // LDS writes, come after all four); byte offsets k4 = 4 k into the
        // table, so each probe is one LDS read at k4 plus a constant
        const char *etb = reinterpret_cast<const char *>(et);
        char *mb = reinterpret_cast<char *>(mine);
        int j = jlo;
        for (; j + 4 <= ct; j += 4) {
            float d[4];
            uint32_t k4[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const float4 q = tile[j + u];
                d[u] = xi * q.x;
                d[u] = d[u] + yi * q.y;
                d[u] = d[u] + zi * q.z;
                k4[u] = d[u] < p1 ? 4u * (TB / 2) : 0u;
                k4[u] += d[u] < (k4[u] ? p2hi : p2lo) ? 4u * (TB / 4) : 0u;
            }
#pragma unroll
            for (int s = TB / 8; s >= 1; s >>= 1)
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    k4[u] += d[u] < *reinterpret_cast<const float *>(etb + k4[u] + 4 * (s - 1)) ? 4u * s : 0u;
#pragma unroll
            for (int u = 0; u < 4; ++u)  // this thread's own counters: no other lane adds to them
                atomicAdd(reinterpret_cast<uint32_t *>(mb + (size_t)k4[u] * NT), 1u);
        }
        for (; j < ct; ++j) {
            const float4 q = tile[j];
            float d = xi * q.x;
            d = d + yi * q.y;
            d = d + zi * q.z;
            int k = d < p1 ? TB / 2 : 0;
            k += d < (k ? p2hi : p2lo) ? TB / 4 : 0;
#pragma unroll
            for (int s = TB / 8; s >= 1; s >>= 1) k += d < et[k + s - 1] ? s : 0;
            atomicAdd(&mine[k * NT], 1u);
        }
    }
    // per bin: the block's 256 counters, a wave tree each, one LDS atomic per
    // wave, one global atomic per bin
    __syncthreads();
    for (int k = 0; k <= m; ++k) {
        unsigned long long c = cnt[k * NT + threadIdx.x];
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) c += __shfl_xor(c, o, 64);
        if ((threadIdx.x & 63) == 0 && c) atomicAdd(&red[k], c);
    }
    __syncthreads();
    if ((int)threadIdx.x <= m && red[threadIdx.x]) atomicAdd(&counts[threadIdx.x], red[threadIdx.x]);
}

__global__ void __launch_bounds__(NT) k_zero64(unsigned long long *__restrict__ p, int m) {
    if ((int)threadIdx.x < m) p[threadIdx.x] = 0ull;
}

}  // namespace

size_t histogram_ws_bytes(int64_t n, int64_t nbins) {
    if (n < 0 || nbins < 1) return 0;
    const HbPlan p = hb_plan(n, nbins);
    return p.ok ? p.bytes : 0;
}

}  // namespace mx

using namespace mx;

extern "C" {

mx_status mx_histogram_u32(const uint32_t *keys_dev, int64_t n, int64_t nbins, uint32_t *counts_dev, void *ws,
                           size_t ws_bytes, hipStream_t stream) {
    const char *who = "mx_histogram_u32";
    MX_REQUIRE(n >= 0 && n < (int64_t)0xffffffff, MX_ERR_SHAPE, "%s: need 0 <= n < 2^32 - 1", who);
    MX_REQUIRE(nbins >= 1 && nbins <= ((int64_t)1 << 32), MX_ERR_SHAPE, "%s: need 1 <= nbins <= 2^32", who);
    MX_REQUIRE(counts_dev && (keys_dev || n == 0), MX_ERR_INVALID, "%s: null pointer", who);
    const DeviceInfo *d;
    if (mx_status st = device_info(&d)) return st;
    const int vec = ((uintptr_t)keys_dev & 15) == 0;
    const HbPlan p = hb_plan(n, nbins);
    if (ws && p.ok && n > 0) {
        MX_REQUIRE(ws_bytes >= p.bytes, MX_ERR_WORKSPACE, "%s: workspace needs %zu bytes", who, p.bytes);
        MX_REQUIRE(((uintptr_t)ws & 255) == 0, MX_ERR_INVALID, "%s: workspace must be 256-byte aligned", who);
        MX_REQUIRE(((int64_t)4 << p.w) <= (int64_t)d->lds_bytes, MX_ERR_UNSUPPORTED, "%s: LDS too small", who);
        char *base = (char *)ws;
        int64_t *cnt = (int64_t *)(base + p.cnt_off), *off = (int64_t *)(base + p.off_off);
        uint16_t *sorted = (uint16_t *)(base + p.sorted_off);
        const size_t lds_nb = (size_t)p.nb * 4;
        hipLaunchKernelGGL(k_hb_count, dim3((unsigned)p.g), dim3(NTS), lds_nb, stream, keys_dev, n, nbins, p.chunk,
                           p.w, (int)p.nb, p.g, cnt);
        if (mx_status st = last_launch(who)) return st;
        if (mx_status st = lengths_to_offsets(cnt, p.g * p.nb, off, ws, p.scan_bytes, stream)) return st;
        hipLaunchKernelGGL(k_hb_scatter, dim3((unsigned)p.g), dim3(NTS), 2 * lds_nb + 2 * kHbPiece * 2, stream,
                           keys_dev, n, nbins, p.chunk, p.w, (int)p.nb, p.g, (const int64_t *)off, sorted);
        if (mx_status st = last_launch(who)) return st;
        hipLaunchKernelGGL(k_hb_bins, dim3((unsigned)p.nb), dim3(NTB), (size_t)4 << p.w, stream,
                           (const uint16_t *)sorted, (const int64_t *)off, p.g, p.w, nbins, counts_dev);
        return last_launch(who);
    }
    const int64_t zb = ceil_div(nbins, NT);
    hipLaunchKernelGGL(k_zero32, dim3((unsigned)(zb < d->num_cus * 8 ? zb : d->num_cus * 8)), dim3(NT), 0, stream,
                       counts_dev, nbins);
    if (mx_status st = last_launch(who)) return st;
    if (n == 0) return MX_OK;
    if (nbins <= kHistLdsBins && (size_t)(nbins + 1) * 4 <= (size_t)d->lds_bytes) {
        // as many blocks as fit the CUs' LDS (at most eight per CU); each
        // block's flush adds at most nbins global atomics
        // up to four copies within 64 KiB; as many blocks as fit the CUs'
        // LDS (at most eight per CU); each block's flush adds at most nbins
        // global atomics
        const int copies = (int)std::max<int64_t>(1, std::min<int64_t>(4, 16383 / (nbins + 1)));
        const size_t lds = (size_t)(nbins + 1) * copies * 4;
        const int64_t per_cu = std::min<int64_t>(8, std::max<int64_t>(1, (int64_t)d->lds_bytes / (int64_t)lds));
        int64_t grid = ceil_div(n, (int64_t)NTH * 64);
        if (grid > d->num_cus * per_cu) grid = d->num_cus * per_cu;
        hipLaunchKernelGGL(k_hist_lds, dim3((unsigned)grid), dim3(NTH), lds, stream, keys_dev, n, (int)nbins, copies,
                           counts_dev, vec);
    } else {
        int64_t grid = ceil_div(n, (int64_t)NT * 16);
        if (grid > d->num_cus * 8) grid = d->num_cus * 8;
        hipLaunchKernelGGL(k_hist_global, dim3((unsigned)grid), dim3(NT), 0, stream, keys_dev, n, nbins,
                           counts_dev, vec);
    }
    return last_launch(who);
}

mx_status mx_stencil7_f32(const float *in_dev, float *out_dev, int64_t nx, int64_t ny, int64_t nz, float c0,
                          float c1, hipStream_t stream) {
    const char *who = "mx_stencil7_f32";
    MX_REQUIRE(nx >= 1 && ny >= 1 && nz >= 1, MX_ERR_SHAPE, "%s: empty grid", who);
    MX_REQUIRE(nx * ny <= ((int64_t)0x7fffffff) * NT, MX_ERR_SHAPE, "%s: plane too large", who);
    MX_REQUIRE(in_dev && out_dev && in_dev != out_dev, MX_ERR_INVALID, "%s: null or aliased grids", who);
    const int64_t gx = ceil_div(nx * ny, NT), gz = ceil_div(nz, kSlab);
    MX_REQUIRE(gz <= 65535, MX_ERR_SHAPE, "%s: nz too large", who);
    hipLaunchKernelGGL(k_stencil7, dim3((unsigned)gx, (unsigned)gz), dim3(NT), 0, stream, in_dev, out_dev, nx, ny,
                       nz, c0, c1);
    return last_launch(who);
}

mx_status mx_tpacf_f32(const float *x1_dev, const float *y1_dev, const float *z1_dev, int64_t n1,
                       const float *x2_dev, const float *y2_dev, const float *z2_dev, int64_t n2, int self_pairs,
                       const float *edges_dev, int nedges, int64_t *counts_dev, hipStream_t stream) {
    const char *who = "mx_tpacf_f32";
    MX_REQUIRE(n1 >= 0 && n2 >= 0, MX_ERR_SHAPE, "%s: negative size", who);
    MX_REQUIRE(nedges >= 0 && nedges <= kTpMaxEdges, MX_ERR_UNSUPPORTED, "%s: at most %d edges", who, kTpMaxEdges);
    MX_REQUIRE(counts_dev && (nedges == 0 || edges_dev), MX_ERR_INVALID, "%s: null counts or edges", who);
    if (self_pairs) {
        x2_dev = x1_dev;
        y2_dev = y1_dev;
        z2_dev = z1_dev;
        n2 = n1;
    }
    MX_REQUIRE((n1 == 0 || (x1_dev && y1_dev && z1_dev)) && (n2 == 0 || (x2_dev && y2_dev && z2_dev)),
               MX_ERR_INVALID, "%s: null point array", who);
    hipLaunchKernelGGL(k_zero64, dim3(1), dim3(64), 0, stream, (unsigned long long *)counts_dev, nedges + 1);
    if (mx_status st = last_launch(who)) return st;
    if (n1 == 0 || n2 == 0) return MX_OK;
    const DeviceInfo *d;
    if (mx_status st = device_info(&d)) return st;
    const int64_t gx = ceil_div(n1, (int64_t)NT);
    MX_REQUIRE(gx <= 0x7fffffff, MX_ERR_SHAPE, "%s: too many points", who);
    // split set 2 into whole tiles so that about 32 blocks per CU exist
    // (several rounds of resident blocks, a short tail; self pairs skip the
    // blocks below the diagonal)
    const int64_t tiles = ceil_div(n2, (int64_t)kTpTile);
    int64_t gy = ceil_div((int64_t)d->num_cus * 32, gx);
    if (gy > tiles) gy = tiles;
    if (gy > 65535) gy = 65535;
    if (gy < 1) gy = 1;
    int64_t chunk = ceil_div(tiles, gy) * kTpTile;
    if (chunk > ((int64_t)1 << 31)) chunk = (int64_t)1 << 31;  // per-thread counts stay below 2^32
    gy = ceil_div(n2, chunk);
    MX_REQUIRE(gy <= 65535, MX_ERR_SHAPE, "%s: set 2 too large", who);
const size_t lds = (size_t)(nedges + 1) * NT * 4;
    if (nedges < 32)
        hipLaunchKernelGGL(k_tpacf<32>, dim3((unsigned)gx, (unsigned)gy), dim3(NT), lds, stream, x1_dev, y1_dev,
                           z1_dev, n1, x2_dev, y2_dev, z2_dev, n2, chunk, self_pairs ? 1 : 0, edges_dev, nedges,
                           (unsigned long long *)counts_dev);
    else
        hipLaunchKernelGGL(k_tpacf<64>, dim3((unsigned)gx, (unsigned)gy), dim3(NT), lds, stream, x1_dev, y1_dev,
                           z1_dev, n1, x2_dev, y2_dev, z2_dev, n2, chunk, self_pairs ? 1 : 0, edges_dev, nedges,
                           (unsigned long long *)counts_dev);
    return last_launch(who);
}

mx_status mx_mriq_f32(const float *kx_dev, const float *ky_dev, const float *kz_dev, const float *phi_dev,
                      int64_t nk, const float *x_dev, const float *y_dev, const float *z_dev, int64_t nv,
                      float *qr_dev, float *qi_dev, hipStream_t stream) {
    const char *who = "mx_mriq_f32";
    MX_REQUIRE(nk >= 0 && nv >= 0, MX_ERR_SHAPE, "%s: negative size", who);
    if (nv == 0) return MX_OK;
    MX_REQUIRE(x_dev && y_dev && z_dev && qr_dev && qi_dev, MX_ERR_INVALID, "%s: null voxel array", who);
    MX_REQUIRE(nk == 0 || (kx_dev && ky_dev && kz_dev && phi_dev), MX_ERR_INVALID, "%s: null sample array", who);
    const int64_t grid = ceil_div(nv, (int64_t)NT * 2);
    MX_REQUIRE(grid <= 0x7fffffff, MX_ERR_SHAPE, "%s: too many voxels", who);
    hipLaunchKernelGGL(k_mriq, dim3((unsigned)grid), dim3(NT), 0, stream, kx_dev, ky_dev, kz_dev, phi_dev, nk, x_dev,
                       y_dev, z_dev, nv, qr_dev, qi_dev);
    return last_launch(who);
}

}  // extern "C"
