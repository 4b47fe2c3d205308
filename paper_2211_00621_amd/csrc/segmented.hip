// Ragged sequences in the flat marshalled layout (values + int64 offsets):
// nested map (reduce) over rows, its reverse (broadcast), the lengths ->
// offsets scan of marshaling, offset composition for `map flatten`, and the
// debug-mode validation of offsets (Appendix "Dynamic Assumptions").
#include <mutex>

#include "mx_internal.h"

namespace mx {
namespace {

constexpr int NT = 256;

inline bool aligned16(const void *p) { return ((uintptr_t)p & 15) == 0; }

// ---------------------------------------------------------------- debug validation
// flag bit 0: offsets[0] != 0; bit 1: a decreasing pair; bit 2: negative length
__global__ void __launch_bounds__(NT) k_check_offsets(const int64_t *__restrict__ off, int64_t nseg,
                                                      unsigned *flag) {
    const int64_t stride = (int64_t)gridDim.x * NT;
    for (int64_t r = (int64_t)blockIdx.x * NT + threadIdx.x; r < nseg; r += stride)
        if (off[r + 1] < off[r]) atomicOr(flag, 2u);
    if (blockIdx.x == 0 && threadIdx.x == 0 && off[0] != 0) atomicOr(flag, 1u);
}

__global__ void __launch_bounds__(NT) k_check_lengths(const int64_t *__restrict__ len, int64_t n,
                                                      unsigned *flag) {
    const int64_t stride = (int64_t)gridDim.x * NT;
    for (int64_t r = (int64_t)blockIdx.x * NT + threadIdx.x; r < n; r += stride)
        if (len[r] < 0) atomicOr(flag, 4u);
}

std::mutex g_flag_mu;
unsigned *g_flag[64] = {};

// Debug mode only: runs a validation kernel and waits for it.
mx_status debug_flag(int dev, unsigned **out) {
    std::lock_guard<std::mutex> lk(g_flag_mu);
    if (!g_flag[dev]) MX_TRY_HIP(hipMalloc(&g_flag[dev], sizeof(unsigned)));
    *out = g_flag[dev];
    return MX_OK;
}

mx_status validate_offsets(const char *who, const int64_t *off, int64_t nseg, hipStream_t s,
                           const DeviceInfo *d) {
    unsigned *flag;
    if (mx_status st = debug_flag(d->device, &flag)) return st;
    MX_TRY_HIP(hipMemsetAsync(flag, 0, sizeof(unsigned), s));
    int grid = (int)ceil_div(nseg > 0 ? nseg : 1, NT);
    if (grid > d->num_cus * 4) grid = d->num_cus * 4;
    hipLaunchKernelGGL(k_check_offsets, dim3(grid), dim3(NT), 0, s, off, nseg, flag);
    if (mx_status st = last_launch(who)) return st;
    unsigned h = 0;
    MX_TRY_HIP(hipMemcpyAsync(&h, flag, sizeof h, hipMemcpyDeviceToHost, s));
    MX_TRY_HIP(hipStreamSynchronize(s));
    if (h & 1u) return set_error(MX_ERR_SHAPE, "%s: offsets[0] != 0", who);
    if (h & 2u) return set_error(MX_ERR_SHAPE, "%s: offsets are not non-decreasing", who);
    return MX_OK;
}

mx_status validate_lengths(const char *who, const int64_t *len, int64_t n, hipStream_t s,
                           const DeviceInfo *d) {
    unsigned *flag;
    if (mx_status st = debug_flag(d->device, &flag)) return st;
    MX_TRY_HIP(hipMemsetAsync(flag, 0, sizeof(unsigned), s));
    int grid = (int)ceil_div(n > 0 ? n : 1, NT);
    if (grid > d->num_cus * 4) grid = d->num_cus * 4;
    hipLaunchKernelGGL(k_check_lengths, dim3(grid), dim3(NT), 0, s, len, n, flag);
    if (mx_status st = last_launch(who)) return st;
    unsigned h = 0;
    MX_TRY_HIP(hipMemcpyAsync(&h, flag, sizeof h, hipMemcpyDeviceToHost, s));
    MX_TRY_HIP(hipStreamSynchronize(s));
    if (h & 4u) return set_error(MX_ERR_SHAPE, "%s: negative row length", who);
    return MX_OK;
}

// ---------------------------------------------------------------- block-span reduce
// A block takes `rb` consecutive rows, whose values form one contiguous span
// [offsets[r0], offsets[r0 + rb]).  The span's 16-byte vectors are cut into
// four contiguous quarters, one per wave; inside its quarter a wave's lanes
// interleave (coalesced), eight vectors per lane in flight.  So a block keeps
// up to 32 KB of loads in flight whatever the row lengths, and the offsets
// cost one round trip per rb rows instead of one per row.
//
// Row attribution: the positions a thread visits increase, so the row they
// fall in never decreases.  A thread keeps one accumulator for its current
// row; on crossing a row end it parks that value in its own LDS slot
// (row, thread) and starts afresh.  A wave finds the row of its quarter's
// first position with one ballot, so a lane crosses only the row ends inside
// its quarter.  Afterwards each row's NT slots are folded in a fixed order
// (four per lane, then the DPP wave tree), so the result depends only on the
// offsets, never on timing.
constexpr int kMaxRowsPerBlock = 16;

// LDS: rb + 1 offsets (padded to 16 bytes), then rb x NT accumulator slots
__host__ __device__ constexpr size_t span_off_bytes(int rb) { return ((size_t)(rb + 1) * 8 + 15) & ~(size_t)15; }
template <mx_dtype D> constexpr size_t span_lds_bytes(int rb) {
    return span_off_bytes(rb) + (size_t)rb * NT * sizeof(typename DT<D>::Acc);
}

// row (0-based within the block) holding position p: the number of row ends
// soff[1..nrows] at or before p, counted by one ballot (nrows < 64)
__device__ __forceinline__ int row_of(const int64_t *soff, int nrows, int64_t p) {
    const int lane = threadIdx.x & (kWave - 1);
    const bool past = lane < nrows && soff[lane + 1] <= p;
    return __popcll(__ballot(past));
}

template <mx_dtype D, int OP>
__global__ void __launch_bounds__(NT) k_seg_span(const typename DT<D>::In *__restrict__ values,
                                                 const int64_t *__restrict__ offsets, int64_t nseg, int rb,
                                                 typename DT<D>::Acc ne, typename DT<D>::Acc *__restrict__ out,
                                                 int vec) {
    using In = typename DT<D>::In;
    using Acc = typename DT<D>::Acc;
    using Vec = typename DT<D>::Vec;
    using R = Red<OP, Acc>;
    constexpr int V = DT<D>::kVec;
    constexpr int U = 8;
    constexpr int NW = NT / kWave;
    extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
    int64_t *soff = reinterpret_cast<int64_t *>(lds);
    Acc *slot = reinterpret_cast<Acc *>(lds + span_off_bytes(rb));
    const int t = threadIdx.x, lane = t & (kWave - 1), w = t / kWave;
    const int64_t r0 = (int64_t)blockIdx.x * rb;
    const int nrows = (int)(nseg - r0 < rb ? nseg - r0 : rb);  // >= 1: the grid covers nseg exactly
    if (t <= nrows) soff[t] = offsets[r0 + t];
    for (int k = 0; k < nrows; ++k) slot[k * NT + t] = R::id();
    __syncthreads();

    const int64_t S = soff[0], E = soff[nrows];
    int cur = 0;
    int64_t end = soff[1];
    Acc a = R::id();
    // fold element x at position p into its row
    auto take = [&](int64_t p, Acc x) {
        while (p >= end) {
            slot[cur * NT + t] = a;
            a = R::id();
            ++cur;
            end = soff[cur + 1];
        }
        a = R::ap(a, x);
    };
    if (vec) {
        const int64_t vs = (S + V - 1) / V, ve = E / V > vs ? E / V : vs;  // whole vectors inside [S, E)
        const int64_t head_end = vs * V < E ? vs * V : E;
        const int64_t q = (ve - vs + NW - 1) / NW;                          // vectors per wave
        const int64_t cs = vs + w * q < ve ? vs + w * q : ve;
        const int64_t ce = cs + q < ve ? cs + q : ve;
        if (w == 0) {
            if (S + lane < head_end) take(S + lane, Acc(values[S + lane]));
        } else if (cs < ce) {
            cur = row_of(soff, nrows, cs * V);
            end = soff[cur + 1];
        }
        const Vec *vv = reinterpret_cast<const Vec *>(values);
        for (int64_t i = cs + lane; i < ce; i += U * kWave) {
            Vec x[U];
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (i + u * kWave < ce) x[u] = vv[i + u * kWave];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (i + u * kWave < ce) {
                    const int64_t p0 = (i + u * kWave) * V;
                    if (p0 + V - 1 < end) {
#pragma unroll
                        for (int j = 0; j < V; ++j) a = R::ap(a, Acc(vget<Vec, In>(x[u], j)));
                    } else {
#pragma unroll
                        for (int j = 0; j < V; ++j) take(p0 + j, Acc(vget<Vec, In>(x[u], j)));
                    }
                }
            }
        }
        if (w == NW - 1) {
            const int64_t tail_start = ve * V > head_end ? ve * V : head_end;
            if (cs >= ce && tail_start < E) {  // wave-uniform: no vectors, only the tail
                cur = row_of(soff, nrows, tail_start);
                end = soff[cur + 1];
            }
            if (tail_start + lane < E) take(tail_start + lane, Acc(values[tail_start + lane]));
        }
    } else {
        for (int64_t i = S + t; i < E; i += NT) take(i, Acc(values[i]));
    }
    slot[cur * NT + t] = a;
    __syncthreads();

    for (int k = w; k < nrows; k += NW) {
        Acc v = slot[k * NT + lane];
#pragma unroll
        for (int qq = 1; qq < NW; ++qq) v = R::ap(v, slot[k * NT + qq * kWave + lane]);
        v = wave_reduce<R>(v);
        if (lane == 0) out[r0 + k] = R::ap(ne, v);
    }
}

// rows per block: enough blocks for eight per CU, at most kMaxRowsPerBlock rows each
int rows_per_block(int64_t nseg, const DeviceInfo *d) {
    const int64_t target = (int64_t)d->num_cus * 8;
    int64_t rb = ceil_div(nseg, target);
    return (int)(rb < 1 ? 1 : rb > kMaxRowsPerBlock ? kMaxRowsPerBlock : rb);
}

// Plain: one thread folds one row left to right.
template <mx_dtype D, int OP>
__global__ void __launch_bounds__(NT) k_seg_thread(const typename DT<D>::In *__restrict__ values,
                                                   const int64_t *__restrict__ offsets,
                                                   int64_t nseg, typename DT<D>::Acc ne,
                                                   typename DT<D>::Acc *__restrict__ out) {
    using Acc = typename DT<D>::Acc;
    using R = Red<OP, Acc>;
    const int64_t row = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (row >= nseg) return;
    Acc acc = ne;
    for (int64_t i = offsets[row]; i < offsets[row + 1]; ++i) acc = R::ap(acc, Acc(values[i]));
    out[row] = acc;
}

// Reverse of the row sums: gval[p] = gout[row of p].  Same block-span walk as
// the reduce: a block loads the offsets and gradients of its rb rows once and
// writes its whole span in 16-byte stores.
__global__ void __launch_bounds__(NT) k_seg_broadcast(const float *__restrict__ gout,
                                                      const int64_t *__restrict__ offsets, int64_t nseg, int rb,
                                                      float *__restrict__ gval, int vec) {
    __shared__ int64_t soff[kMaxRowsPerBlock + 1];
    __shared__ float sg[kMaxRowsPerBlock];
    const int t = threadIdx.x;
    const int64_t r0 = (int64_t)blockIdx.x * rb;
    const int nrows = (int)(nseg - r0 < rb ? nseg - r0 : rb);
    if (t <= nrows) soff[t] = offsets[r0 + t];
    if (t < nrows) sg[t] = gout[r0 + t];
    __syncthreads();
    const int64_t S = soff[0], E = soff[nrows];
    int cur = 0;
    int64_t end = soff[1];
    float g = sg[0];
    auto at = [&](int64_t p) {
        while (p >= end) {
            ++cur;
            end = soff[cur + 1];
            g = sg[cur];
        }
        return g;
    };
    if (vec) {
        const int64_t vs = (S + 3) / 4, ve = E / 4;
        const int64_t head_end = vs * 4 < E ? vs * 4 : E;
        if (S + t < head_end) gval[S + t] = at(S + t);
        float4 *gv = reinterpret_cast<float4 *>(gval);
        for (int64_t i = vs + t; i < ve; i += NT) {
            const int64_t p0 = i * 4;
            float4 y;
            if (p0 + 3 < end) {
                y = make_float4(g, g, g, g);
            } else {
                y.x = at(p0);
                y.y = at(p0 + 1);
                y.z = at(p0 + 2);
                y.w = at(p0 + 3);
            }
            gv[i] = y;
        }
        const int64_t tail_start = ve * 4 > head_end ? ve * 4 : head_end;
        if (tail_start + t < E) gval[tail_start + t] = at(tail_start + t);
    } else {
        for (int64_t i = S + t; i < E; i += NT) gval[i] = at(i);
    }
}

// ---------------------------------------------------------------- lengths -> offsets
// Tiles of 4096 rows (16 per thread), scanned in LDS (padded against bank
// conflicts).  One tile: one block.  More: a single pass with decoupled
// look-back -- blocks claim tiles in order from a counter, publish their
// tile's total, then walk back over earlier tiles' published totals until one
// carries its inclusive prefix, and publish their own.  A status word packs
// the flag (2 bits) with the value (62 bits), so one relaxed device-scope
// atomic carries both; tile i waits only on tiles claimed before it, whose
// blocks are running, so the wait always ends.  The last block to finish
// clears the status words and counters for the next call.
constexpr int kScanPer = 16;
constexpr int kScanTile = NT * kScanPer;
constexpr uint64_t kStatAgg = 1ull << 62, kStatPre = 2ull << 62, kStatVal = (1ull << 62) - 1;
// one pad slot per 16 entries keeps the per-thread runs of 16 on distinct banks
__device__ __forceinline__ int spad(int i) { return i + (i >> 4); }

__device__ __forceinline__ int64_t block_excl_scan(int64_t v, int64_t *wsum, int64_t *total) {
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    int64_t incl = v;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        int64_t o = __shfl_up(incl, d, kWave);
        if (lane >= d) incl += o;
    }
    if (lane == kWave - 1) wsum[wave] = incl;
    __syncthreads();
    int64_t before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < NT / kWave; ++w) {
        if (w < wave) before += wsum[w];
        all += wsum[w];
    }
    __syncthreads();
    *total = all;
    return before + incl - v;
}

__device__ __forceinline__ uint64_t status_load(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void status_store(uint64_t *p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// counters[0]: next tile to claim; counters[1]: blocks finished.  LOOKBACK
// false: a single block scans the single tile.
template <bool LOOKBACK>
__global__ void __launch_bounds__(NT) k_scan_tiles(const int64_t *__restrict__ len, int64_t n,
                                                   int64_t *__restrict__ off, unsigned *counters,
                                                   uint64_t *status, int ntiles) {
    __shared__ int64_t tile[kScanTile + kScanTile / 16];
    __shared__ int64_t wsum[NT / kWave];
    __shared__ int64_t sh_prefix;
    __shared__ int sh_tile, sh_last;
    if (LOOKBACK) {
        if (threadIdx.x == 0) sh_tile = (int)atomicAdd(&counters[0], 1u);
        __syncthreads();
    }
    const int t = LOOKBACK ? sh_tile : 0;
    const int64_t base = (int64_t)t * kScanTile;
    // coalesced load into LDS
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) {
        int64_t i = base + j * NT + threadIdx.x;
        tile[spad(j * NT + threadIdx.x)] = i < n ? len[i] : 0;
    }
    __syncthreads();
    int64_t mine[kScanPer];
    int64_t s = 0;
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) {
        mine[j] = tile[spad(threadIdx.x * kScanPer + j)];
        s += mine[j];
    }
    int64_t total;
    const int64_t ex = block_excl_scan(s, wsum, &total);
    if (LOOKBACK) {
        if (threadIdx.x == 0)
            status_store(&status[t], (t == 0 ? kStatPre : kStatAgg) | ((uint64_t)total & kStatVal));
        if (threadIdx.x < kWave) {
            // wave 0 looks back over 64 predecessors at a time: once every one of
            // them has published, add the totals down to the nearest published
            // inclusive prefix (positions before tile 0 count as a prefix of 0)
            const int lane = threadIdx.x;
            int64_t prefix = 0;
            for (int hi = t - 1; hi >= 0; hi -= kWave) {
                const int p = hi - lane;
                uint64_t w;
                for (;;) {
                    w = p >= 0 ? status_load(&status[p]) : kStatPre;
                    if (__ballot((w >> 62) == 0) == 0) break;
                    __builtin_amdgcn_s_sleep(1);
                }
                const uint64_t pre = __ballot((w >> 62) == 2);
                const int stop = pre ? __builtin_ctzll(pre) : kWave;  // nearest prefix in this window
                const int64_t v = lane <= stop ? (int64_t)(w & kStatVal) : 0;
                prefix += wave_reduce<Red<MX_ADD, int64_t>>(v);
                if (pre) break;
            }
            if (lane == 0) {
                if (t > 0) status_store(&status[t], kStatPre | ((uint64_t)(prefix + total) & kStatVal));
                sh_prefix = prefix;
            }
        }
    } else if (threadIdx.x == 0) {
        sh_prefix = 0;
    }
    __syncthreads();
    const int64_t prefix = sh_prefix;
    int64_t run = prefix + ex;
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) {
        tile[spad(threadIdx.x * kScanPer + j)] = run;
        run += mine[j];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) {
        int64_t i = base + j * NT + threadIdx.x;
        if (i < n) off[i] = tile[spad(j * NT + threadIdx.x)];
    }
    if (base + kScanTile >= n && threadIdx.x == 0) off[n] = prefix + total;
    if (LOOKBACK) {
        // every other block has finished its look-back when the last one arrives
        if (threadIdx.x == 0) sh_last = atomicAdd(&counters[1], 1u) == (unsigned)ntiles - 1;
        __syncthreads();
        if (sh_last) {
            for (int i = threadIdx.x; i < ntiles; i += NT) status_store(&status[i], 0);
            if (threadIdx.x == 0) {
                __hip_atomic_store(&counters[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&counters[1], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
}

__global__ void __launch_bounds__(NT) k_compose(const int64_t *__restrict__ outer, int64_t nouter,
                                                const int64_t *__restrict__ inner,
                                                int64_t *__restrict__ out) {
    const int64_t stride = (int64_t)gridDim.x * NT;
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i <= nouter; i += stride)
        out[i] = inner[outer[i]];
}

// ---------------------------------------------------------------- dispatch
template <mx_dtype D, int OP>
mx_status launch_seg(bool plain, const void *values, const int64_t *off, int64_t nseg,
                     const void *ne_host, void *out, hipStream_t s) {
    using In = typename DT<D>::In;
    using Acc = typename DT<D>::Acc;
    Acc ne;
    __builtin_memcpy(&ne, ne_host, sizeof(Acc));
    if (plain) {
        int grid = (int)ceil_div(nseg, NT);
        hipLaunchKernelGGL((k_seg_thread<D, OP>), dim3(grid), dim3(NT), 0, s, (const In *)values, off,
                           nseg, ne, (Acc *)out);
    } else {
        const DeviceInfo *d;
        if (mx_status st = device_info(&d)) return st;
        const int rb = rows_per_block(nseg, d);
        const int64_t grid = ceil_div(nseg, rb);
        MX_REQUIRE(grid <= 0x7fffffff, MX_ERR_SHAPE, "mx_segmented_reduce: too many rows");
        hipLaunchKernelGGL((k_seg_span<D, OP>), dim3((unsigned)grid), dim3(NT), span_lds_bytes<D>(rb), s,
                           (const In *)values, off, nseg, rb, ne, (Acc *)out, (int)aligned16(values));
    }
    return last_launch("mx_segmented_reduce");
}

template <mx_dtype D>
mx_status seg_by_op(bool plain, int op, const void *v, const int64_t *off, int64_t nseg,
                    const void *ne, void *out, hipStream_t s) {
    switch (op) {
    case MX_ADD: return launch_seg<D, MX_ADD>(plain, v, off, nseg, ne, out, s);
    case MX_MUL: return launch_seg<D, MX_MUL>(plain, v, off, nseg, ne, out, s);
    case MX_MIN: return launch_seg<D, MX_MIN>(plain, v, off, nseg, ne, out, s);
    case MX_MAX: return launch_seg<D, MX_MAX>(plain, v, off, nseg, ne, out, s);
    }
    return set_error(MX_ERR_INVALID, "mx_segmented_reduce: unknown operator %d", op);
}

mx_status segmented(const char *who, bool plain, int op, mx_dtype dtype, const void *values,
                    const int64_t *off, int64_t nseg, const void *ne, void *out, hipStream_t s) {
    MX_REQUIRE(nseg >= 0, MX_ERR_SHAPE, "%s: nseg < 0", who);
    MX_REQUIRE(dtype_valid(dtype), MX_ERR_DTYPE, "%s: bad dtype %d", who, (int)dtype);
    MX_REQUIRE(op >= MX_ADD && op <= MX_MAX, MX_ERR_INVALID, "%s: unknown operator %d", who, op);
    MX_REQUIRE(ne, MX_ERR_INVALID, "%s: null ne", who);
    if (nseg == 0) return MX_OK;
    MX_REQUIRE(off && out, MX_ERR_INVALID, "%s: null offsets or out", who);
    const DeviceInfo *d;
    if (mx_status st = device_info(&d)) return st;
    if (debug_mode())
        if (mx_status st = validate_offsets(who, off, nseg, s, d)) return st;
    switch (dtype) {
    case MX_F32: return seg_by_op<MX_F32>(plain, op, values, off, nseg, ne, out, s);
    case MX_F64: return seg_by_op<MX_F64>(plain, op, values, off, nseg, ne, out, s);
    case MX_I32: return seg_by_op<MX_I32>(plain, op, values, off, nseg, ne, out, s);
    case MX_I64: return seg_by_op<MX_I64>(plain, op, values, off, nseg, ne, out, s);
    }
    return MX_ERR_DTYPE;
}

}  // namespace

// Shared with the generated map-body kernels: rows per block of a block-span
// reduce, and the debug-mode check of an offsets array.
int segmented_rows_per_block(int64_t nseg, const DeviceInfo *d) { return rows_per_block(nseg, d); }

mx_status check_offsets_debug(const char *who, const int64_t *off, int64_t nseg, hipStream_t s) {
    const DeviceInfo *d;
    if (mx_status st = device_info(&d)) return st;
    return validate_offsets(who, off, nseg, s, d);
}

// Also used by marshaling.
mx_status lengths_to_offsets(const int64_t *len, int64_t nseg, int64_t *off, void *ws,
                             size_t ws_bytes, hipStream_t s) {
    MX_REQUIRE(nseg >= 0, MX_ERR_SHAPE, "mx_lengths_to_offsets: nseg < 0");
    MX_REQUIRE(off, MX_ERR_INVALID, "mx_lengths_to_offsets: null offsets");
    MX_REQUIRE(nseg == 0 || len, MX_ERR_INVALID, "mx_lengths_to_offsets: null lengths");
    const DeviceInfo *d;
    if (mx_status st = device_info(&d)) return st;
    if (nseg > 0 && debug_mode())
        if (mx_status st = validate_lengths("mx_lengths_to_offsets", len, nseg, s, d)) return st;
    const int64_t ntiles = ceil_div(nseg, kScanTile);
    MX_REQUIRE(ntiles <= 0x7fffffff, MX_ERR_SHAPE, "mx_lengths_to_offsets: too many rows");
    if (ntiles <= 1) {
        hipLaunchKernelGGL(k_scan_tiles<false>, dim3(1), dim3(NT), 0, s, len, nseg, off, (unsigned *)nullptr,
                           (uint64_t *)nullptr, 1);
        return last_launch("mx_lengths_to_offsets");
    }
    size_t need = mx_workspace_bytes(MX_WS_SCAN, nseg, 0);
    MX_REQUIRE(ws && ws_bytes >= need, MX_ERR_WORKSPACE, "mx_lengths_to_offsets: workspace needs %zu bytes", need);
    MX_REQUIRE(((uintptr_t)ws & 255) == 0, MX_ERR_INVALID, "mx_lengths_to_offsets: workspace must be 256-byte aligned");
    unsigned *counters = (unsigned *)ws;
    uint64_t *status = (uint64_t *)((char *)ws + kCounterBytes);
    hipLaunchKernelGGL(k_scan_tiles<true>, dim3((unsigned)ntiles), dim3(NT), 0, s, len, nseg, off, counters, status,
                       (int)ntiles);
    return last_launch("mx_lengths_to_offsets");
}

}  // namespace mx

using namespace mx;

extern "C" {

mx_status mx_segmented_reduce(mx_redop op, mx_dtype dtype, const void *values_dev,
                              const int64_t *offsets_dev, int64_t nseg, const void *ne_host,
                              void *out_dev, hipStream_t stream) {
    return segmented("mx_segmented_reduce", false, op, dtype, values_dev, offsets_dev, nseg, ne_host,
                     out_dev, stream);
}

mx_status mx_segmented_reduce_plain(mx_redop op, mx_dtype dtype, const void *values_dev,
                                    const int64_t *offsets_dev, int64_t nseg, const void *ne_host,
                                    void *out_dev, hipStream_t stream) {
    return segmented("mx_segmented_reduce_plain", true, op, dtype, values_dev, offsets_dev, nseg,
                     ne_host, out_dev, stream);
}

mx_status mx_segmented_sum_adjoint_f32(const float *gout_dev, const int64_t *offsets_dev,
                                       int64_t nseg, float *gvalues_dev, hipStream_t stream) {
    MX_REQUIRE(nseg >= 0, MX_ERR_SHAPE, "mx_segmented_sum_adjoint_f32: nseg < 0");
    if (nseg == 0) return MX_OK;
    MX_REQUIRE(gout_dev && offsets_dev && gvalues_dev, MX_ERR_INVALID,
               "mx_segmented_sum_adjoint_f32: null pointer");
    const DeviceInfo *d;
    if (mx_status st = device_info(&d)) return st;
    if (debug_mode())
        if (mx_status st = validate_offsets("mx_segmented_sum_adjoint_f32", offsets_dev, nseg, stream, d))
            return st;
    const int rb = rows_per_block(nseg, d);
    const int64_t grid = ceil_div(nseg, rb);
    MX_REQUIRE(grid <= 0x7fffffff, MX_ERR_SHAPE, "mx_segmented_sum_adjoint_f32: too many rows");
    hipLaunchKernelGGL(k_seg_broadcast, dim3((unsigned)grid), dim3(NT), 0, stream, gout_dev,
                       offsets_dev, nseg, rb, gvalues_dev, (int)aligned16(gvalues_dev));
    return last_launch("mx_segmented_sum_adjoint_f32");
}

mx_status mx_lengths_to_offsets(const int64_t *lengths_dev, int64_t nseg, int64_t *offsets_dev,
                                void *ws, size_t ws_bytes, hipStream_t stream) {
    return lengths_to_offsets(lengths_dev, nseg, offsets_dev, ws, ws_bytes, stream);
}

mx_status mx_compose_offsets(const int64_t *outer_dev, int64_t nouter, const int64_t *inner_dev,
                             int64_t *out_dev, hipStream_t stream) {
    MX_REQUIRE(nouter >= 0, MX_ERR_SHAPE, "mx_compose_offsets: nouter < 0");
    MX_REQUIRE(outer_dev && inner_dev && out_dev, MX_ERR_INVALID, "mx_compose_offsets: null pointer");
    const DeviceInfo *d;
    if (mx_status st = device_info(&d)) return st;
    int grid = (int)ceil_div(nouter + 1, NT);
    if (grid > d->num_cus * 8) grid = d->num_cus * 8;
    hipLaunchKernelGGL(k_compose, dim3(grid), dim3(NT), 0, stream, outer_dev, nouter, inner_dev, out_dev);
    return last_launch("mx_compose_offsets");
}

}  // extern "C"
