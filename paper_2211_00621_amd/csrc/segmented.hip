// Ragged sequences in the flat marshalled layout (values + int64 offsets):
// nested map (reduce) over rows, its reverse (broadcast), the lengths ->
// offsets scan of marshaling, offset composition for `map flatten`, and the
// debug-mode validation of offsets (Appendix "Dynamic Assumptions").
#include <algorithm>
#include <mutex>

#include "mx_internal.h"

namespace mx {
namespace {

constexpr int NT = 256;

inline bool aligned16(const void *p) { return ((uintptr_t)p & 15) == 0; }

// ---------------------------------------------------------------- debug validation
// flag bit 0: offsets[0] != 0; bit 1: a decreasing pair; bit 2: negative
// length; bit 3: offsets[nseg] differs from the value count (nval >= 0 only)
__global__ void __launch_bounds__(NT) k_check_offsets(const int64_t *__restrict__ off, int64_t nseg,
                                                      int64_t nval, unsigned *flag) {
    const int64_t stride = (int64_t)gridDim.x * NT;
    for (int64_t r = (int64_t)blockIdx.x * NT + threadIdx.x; r < nseg; r += stride)
        if (off[r + 1] < off[r]) atomicOr(flag, 2u);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (off[0] != 0) atomicOr(flag, 1u);
        if (nval >= 0 && off[nseg] != nval) atomicOr(flag, 8u);
    }
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

// nval >= 0: also require offsets[nseg] == nval
mx_status validate_offsets(const char *who, const int64_t *off, int64_t nseg, int64_t nval, hipStream_t s,
                           const DeviceInfo *d) {
    unsigned *flag;
    if (mx_status st = debug_flag(d->device, &flag)) return st;
    MX_TRY_HIP(hipMemsetAsync(flag, 0, sizeof(unsigned), s));
    int grid = (int)ceil_div(nseg > 0 ? nseg : 1, NT);
    if (grid > d->num_cus * 4) grid = d->num_cus * 4;
    hipLaunchKernelGGL(k_check_offsets, dim3(grid), dim3(NT), 0, s, off, nseg, nval, flag);
    if (mx_status st = last_launch(who)) return st;
    unsigned h = 0;
    MX_TRY_HIP(hipMemcpyAsync(&h, flag, sizeof h, hipMemcpyDeviceToHost, s));
    MX_TRY_HIP(hipStreamSynchronize(s));
    if (h & 1u) return set_error(MX_ERR_SHAPE, "%s: offsets[0] != 0", who);
    if (h & 2u) return set_error(MX_ERR_SHAPE, "%s: offsets are not non-decreasing", who);
    if (h & 8u) return set_error(MX_ERR_SHAPE, "%s: offsets[nseg] differs from the number of values", who);
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

// ---------------------------------------------------------------- chunked ragged kernels
// The flat value array is cut into chunks of kChunkBytes: chunk c holds the
// positions [c S, (c + 1) S) of the array (S = kChunkBytes / element size), and
// one block takes one chunk, so every block streams the same number of bytes
// whatever the row lengths.  A block issues its chunk's loads first (their
// addresses depend only on c) and, while they are in flight, two waves find
// by search in the offsets the first and last rows that touch the chunk.  The
// chunk is staged in LDS; each row's segment in the chunk is then folded by
// one lane (at most kShortSeg values, sequentially) or by a whole wave (lanes
// interleaved, then the wave tree).  The fold structure depends only on the
// offsets and S, never on timing.
//
// Row ownership: a row belongs to the chunk that holds its last element; an
// empty row to the chunk that holds its position (the last chunk for rows at
// the very end).  A row split across chunks b0 < ... < b1 is finished by
// whichever of its chunks arrives last: chunk b0 publishes the fold of its
// part (tail slot T[b0]), every later chunk the fold of its part (head slot
// H[b]), each then adds one to the counter of b0; the block that brings the
// count to b1 - b0 + 1 folds T[b0], H[b0+1], ..., H[b1] in that order and
// writes the row.  Nobody waits for a block that may not have started: a
// slot is read only after its writer has counted itself in, and the slot's
// own tag shows when its (already issued) store has landed.  Slots are tagged
// 64-bit words written and read with device-scope atomics, so no cache
// flushes are needed; the finishing block clears the slots and the counter.
constexpr int kChunkBytes = 16384;
constexpr int kShortSeg = 32;                        // longer segments take a whole wave
constexpr int kMaxLong = kChunkBytes / 4 / (kShortSeg + 1) + 1;  // long segments in one chunk, at most

template <mx_dtype D> constexpr int chunk_len() { return kChunkBytes / (int)sizeof(typename DT<D>::In); }

int64_t chunks_of(int64_t nval, int S) { return (nval + S - 1) / S; }

struct LongSeg {
    int64_t row;
    int s, e;  // its segment in the chunk, chunk-relative [s, e)
};

// Upper bound over the sorted offsets: the first index i in [0, n] with
// off[i] > x (n + 1 when there is none), found by one wave in rounds of 64
// probes -- a 65 537-entry array takes three rounds.  All 64 lanes must call.
__device__ int64_t wave_upper_bound(const int64_t *__restrict__ off, int64_t n, int64_t x) {
    const int lane = threadIdx.x & (kWave - 1);
    int64_t lo = 0, hi = n + 1;  // the answer lies in [lo, hi]
    while (lo < hi) {
        const int64_t step = (hi - lo + kWave - 1) / kWave;
        const int64_t idx = lo + (int64_t)(lane + 1) * step - 1;
        // indices at or past hi are past the answer: no load needed
        const bool gt = idx >= hi || off[idx] > x;
        const uint64_t m = __ballot(gt);
        const int f = m ? __builtin_ctzll(m) : kWave;
        const int64_t nlo = lo + (int64_t)f * step;
        const int64_t nhi = f < kWave ? lo + (int64_t)(f + 1) * step - 1 : hi;
        lo = nlo < hi ? nlo : hi;
        hi = nhi < hi ? nhi : hi;
    }
    return lo;
}

// Upper bound by interpolation, returning the same index as
// wave_upper_bound: the first round reads 64 entries spaced kGuessStep apart
// around the entry the answer would be if every row had the same length
// (x n / total); when the answer falls between two of them -- for lengths
// drawn independently it almost always does -- the second round reads the
// 128 consecutive entries from the one below, which hold the answer and the
// offsets of the rows that follow it: lane l keeps entries base + l and
// base + 64 + l in win[0], win[1].  Otherwise the plain search takes over and
// *base is set to -1 (no window).
constexpr int64_t kGuessStep = 64;
__device__ int64_t wave_upper_bound_guess(const int64_t *__restrict__ off, int64_t n, int64_t total, int64_t x,
                                          int64_t *base, int64_t (&win)[2]) {
    const int lane = threadIdx.x & (kWave - 1);
    int64_t g = (int64_t)((double)x / (double)total * (double)n);
    g = g < 0 ? 0 : g > n ? n : g;
    int64_t first = g - 32 * kGuessStep;
    first = first < 0 ? 0 : first;
    const int64_t idx = first + lane * kGuessStep;
    const bool gt = idx > n || off[idx] > x;  // past n: as if +infinity
    const uint64_t m = __ballot(gt);
    const int f = m ? __builtin_ctzll(m) : kWave;
    if (f == 0 && first > 0) {  // the answer is below the window
        *base = -1;
        return wave_upper_bound(off, first, x);  // off[first] > x, so the answer is at most first
    }
    if (f == kWave) {  // above the window: search the rest
        *base = -1;
        const int64_t last = first + (kWave - 1) * kGuessStep;
        // answer in [last + 1, n + 1]: offsets from last + 1 on, shifted
        return last + 1 + wave_upper_bound(off + last + 1, n - last - 1, x);
    }
    // the answer lies in (first + (f-1) step, first + f step] (f = 0: it is 0)
    const int64_t b0 = f == 0 ? 0 : first + (int64_t)(f - 1) * kGuessStep + 1;
    *base = b0;
    win[0] = b0 + lane <= n ? off[b0 + lane] : INT64_MAX;
    win[1] = b0 + kWave + lane <= n ? off[b0 + kWave + lane] : INT64_MAX;
    const uint64_t m2 = __ballot(win[0] > x);
    // kGuessStep <= 64, so the answer is within the first 64 entries
    return b0 + (m2 ? __builtin_ctzll(m2) : kWave);
}

// Rows [lo, hi) touch chunk c = [P0, P1): the row holding P0 - 1 when it runs
// past P0 (its head part is here), up to the row holding P1 - 1 (its tail may
// run on).  Empty rows at P0 are included, those at P1 belong to chunk c + 1.
// Wave 0 finds lo and leaves the offsets from lo on in s_off (when the
// interpolation round found them: s_off_n entries, else 0), wave 1 finds hi
// and the bounds of row hi - 1.
struct ChunkRows {
    int64_t lo, hi;
    int64_t head_s, head_e;  // bounds of row lo
    int64_t tail_s, tail_e;  // bounds of row hi - 1
    int n_off;               // s_off holds offsets[lo .. lo + n_off)
};
constexpr int kOffWin = 2 * kWave;

__device__ void chunk_rows(const int64_t *__restrict__ off, int64_t nseg, int64_t nval, int64_t c, int64_t nchunks,
                           int64_t P0, int64_t P1, ChunkRows *cr, int64_t *s_off) {
    const int w = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
    if (w == 0) {
        int64_t lo = 0, base = 0, win[2];
        if (c > 0) {
            // row u - 1 holds P0 - 1 (u <= nseg when offsets[nseg] = nval)
            int64_t u = wave_upper_bound_guess(off, nseg, nval, P0 - 1, &base, win);
            u = u < nseg ? u : nseg;
            lo = off[u] > P0 ? u - 1 : u;
            lo = lo < 0 ? 0 : lo;
        } else {
            win[0] = lane <= nseg ? off[lane] : INT64_MAX;
            win[1] = kWave + lane <= nseg ? off[kWave + lane] : INT64_MAX;
        }
        // offsets[lo ..] from the window: entries lo - base .. kOffWin - 1
        int nwin = 0;
        if (base >= 0 && lo >= base && lo - base < kOffWin) {
            const int sh = (int)(lo - base);
            nwin = kOffWin - sh;
            const int64_t avail = nseg + 1 - lo;
            nwin = avail < nwin ? (int)avail : nwin;
            if (lane >= sh) s_off[lane - sh] = win[0];
            if (kWave + lane >= sh) s_off[kWave + lane - sh] = win[1];
        }
        if (lane == 0) {
            cr->lo = lo;
            cr->n_off = nwin;
            cr->head_s = off[lo];
            cr->head_e = lo < nseg ? off[lo + 1] : off[lo];
        }
    } else if (w == 1) {
        int64_t hi = nseg, base, win[2];
        if (c + 1 < nchunks) {
            hi = wave_upper_bound_guess(off, nseg, nval, P1 - 1, &base, win);
            hi = hi < nseg ? hi : nseg;
        }
        if (lane == 0) {
            cr->hi = hi;
            cr->tail_s = hi > 0 ? off[hi - 1] : 0;
            cr->tail_e = off[hi];
        }
    }
}

// ---- tagged slots: one 64-bit word per 32 bits of value, the high half a tag
template <class Acc> __device__ __forceinline__ void slot_put(uint64_t *slot, Acc v) {
    uint64_t b = 0;
    __builtin_memcpy(&b, &v, sizeof(Acc));
    __hip_atomic_store(slot, (1ull << 32) | (b & 0xffffffffull), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if constexpr (sizeof(Acc) == 8)
        __hip_atomic_store(slot + 1, (1ull << 32) | (b >> 32), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t tagged_load(uint64_t *p) {
    uint64_t w;
    // the writer counted itself in after issuing this store, so it is on its
    // way; the poll count is bounded all the same (offsets that break the
    // contract then give a wrong row, not a kernel that never ends)
    for (int k = 0; k < (1 << 22); ++k) {
        w = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (w >> 32) break;
        __builtin_amdgcn_s_sleep(1);
    }
    return w;
}
template <class Acc> __device__ __forceinline__ Acc slot_get(uint64_t *slot) {
    uint64_t b = tagged_load(slot) & 0xffffffffull;
    if constexpr (sizeof(Acc) == 8) b |= (tagged_load(slot + 1) & 0xffffffffull) << 32;
    Acc v;
    __builtin_memcpy(&v, &b, sizeof(Acc));
    return v;
}
template <class Acc> __device__ __forceinline__ void slot_clear(uint64_t *slot) {
    __hip_atomic_store(slot, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if constexpr (sizeof(Acc) == 8) __hip_atomic_store(slot + 1, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// workspace of the chunked reduce: counters (256 B), then per chunk a 32-bit
// counter, a head slot and a tail slot (two words each)
struct SegWs {
    unsigned *cnt;
    uint64_t *head, *tail;
};
constexpr int64_t kMinChunk = kChunkBytes / 8;  // the chunk length of 8-byte elements
size_t seg_ws_bytes(int64_t nval) {
    const int64_t nch = chunks_of(nval < 0 ? 0 : nval, (int)kMinChunk);
    return kCounterBytes + align256((size_t)nch * 4) + 2 * align256((size_t)nch * 16);
}
SegWs seg_ws(void *ws, int64_t nval) {
    const int64_t nch = chunks_of(nval, (int)kMinChunk);
    char *p = (char *)ws + kCounterBytes;
    SegWs w;
    w.cnt = (unsigned *)p;
    p += align256((size_t)nch * 4);
    w.head = (uint64_t *)p;
    p += align256((size_t)nch * 16);
    w.tail = (uint64_t *)p;
    return w;
}

// Stages chunk [P0, P0 + n) of `values` in LDS: 16-byte loads (vec) or one
// element per lane, issued before the row search and stored after it.
template <class In, class Vec, int V, int S, bool VEC>
struct ChunkLoad;
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));  // 16 raw bytes
template <class In, class Vec, int V, int S>
struct ChunkLoad<In, Vec, V, S, true> {
    static constexpr int PER = S / V / NT;  // vectors per thread
    u32x4 x[PER];
    __device__ __forceinline__ void issue(const In *__restrict__ values, int64_t P0, int n) {
        const u32x4 *vv = reinterpret_cast<const u32x4 *>(values + P0);
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int q = threadIdx.x + NT * u;
            if (q * V + V <= n) x[u] = __builtin_nontemporal_load(vv + q);
        }
    }
    __device__ __forceinline__ void store(In *sv, const In *__restrict__ values, int64_t P0, int n) {
        u32x4 *sv4 = reinterpret_cast<u32x4 *>(sv);
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int q = threadIdx.x + NT * u;
            if (q * V + V <= n) {
                sv4[q] = x[u];
            } else if (q * V < n) {  // the chunk's last, partial vector
                for (int j = q * V; j < n; ++j) sv[j] = values[P0 + j];
            }
        }
    }
};
template <class In, class Vec, int V, int S>
struct ChunkLoad<In, Vec, V, S, false> {
    static constexpr int PER = S / NT;  // elements per thread
    In x[PER];
    __device__ __forceinline__ void issue(const In *__restrict__ values, int64_t P0, int n) {
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int k = threadIdx.x + NT * j;
            if (k < n) x[j] = values[P0 + k];
        }
    }
    __device__ __forceinline__ void store(In *sv, const In *__restrict__ values, int64_t P0, int n) {
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int k = threadIdx.x + NT * j;
            if (k < n) sv[k] = x[j];
        }
    }
};
// Segmented reduce over chunk blockIdx.x.  nchunks = ceil(nval / S) > 0.
template <mx_dtype D, int OP, bool VEC>
__global__ void __launch_bounds__(NT) k_seg_chunk(const typename DT<D>::In *__restrict__ values,
                                                  const int64_t *__restrict__ offsets, int64_t nseg, int64_t nval,
                                                  int64_t nchunks, typename DT<D>::Acc ne,
                                                  typename DT<D>::Acc *__restrict__ out, SegWs ws) {
    using In = typename DT<D>::In;
    using Acc = typename DT<D>::Acc;
    using R = Red<OP, Acc>;
    constexpr int S = chunk_len<D>();
    constexpr int NW = NT / kWave;
    __shared__ __attribute__((aligned(16))) In sv[S];
    __shared__ LongSeg slong[kMaxLong];
    __shared__ int64_t s_off[kOffWin];
    __shared__ ChunkRows cr;
    __shared__ int s_nlong;
    // parts of split rows: [0] the head part (row lo began in an earlier
    // chunk), [1] the tail part (row hi - 1 runs on into later chunks)
    __shared__ Acc s_cval[2];
    __shared__ unsigned s_arrived[2];

    const int t = threadIdx.x, w = t / kWave, lane = t & (kWave - 1);
    const int64_t c = blockIdx.x;
    const int64_t P0 = c * S;
    const int n = (int)(nval - P0 < S ? nval - P0 : S);
    const int64_t P1 = P0 + n;

    ChunkLoad<In, typename DT<D>::Vec, DT<D>::kVec, S, VEC> ld;
    ld.issue(values, P0, n);
    if (t == 0) s_nlong = 0;
    chunk_rows(offsets, nseg, nval, c, nchunks, P0, P1, &cr, s_off);
    // the split rows' counters are bumped now, so that the round trip runs
    // while the chunk is folded; the parts' values follow at the end
    // (lane 0 of wave 0 / 1 wrote the cr fields it reads here)
    if (w == 0 && lane == 0 && c > 0 && cr.head_s < P0) {
        const int64_t b0 = cr.head_s / S;
        s_arrived[0] = atomicAdd(&ws.cnt[b0 < 0 ? 0 : b0], 1u);
    }
    if (w == 1 && lane == 0 && cr.tail_e > P1 && cr.tail_s >= P0) s_arrived[1] = atomicAdd(&ws.cnt[c], 1u);
    ld.store(sv, values, P0, n);
    __syncthreads();
    const int64_t lo = cr.lo, hi = cr.hi;
    const int n_off = cr.n_off;
    const bool has_head = c > 0 && cr.head_s < P0;
    const bool has_tail = cr.tail_e > P1 && cr.tail_s >= P0;

    // a finished segment: write the row, or keep the chunk's part of a split
    // row (row lo when it began in an earlier chunk, row hi - 1 when it runs on)
    auto finish = [&](int64_t r, bool empty, Acc v) {
        if (r == lo && has_head) s_cval[0] = v;
        else if (r == hi - 1 && has_tail) s_cval[1] = v;
        else out[r] = empty ? ne : R::ap(ne, v);
    };

    for (int64_t base = lo; base < hi; base += NT) {
        const int64_t r = base + t;
        if (r < hi) {
            const int64_t k = r - lo;
            const int64_t sa = k < n_off ? s_off[k] : offsets[r];
            const int64_t ea = k + 1 < n_off ? s_off[k + 1] : offsets[r + 1];
            // clamped to the chunk (they are inside it whenever the offsets are valid)
            const int s = (int)(sa >= P1 ? n : sa > P0 ? sa - P0 : 0);
            const int e = (int)(ea <= P0 ? s : ea < P1 ? (ea - P0 > s ? ea - P0 : s) : n);
            if (e - s <= kShortSeg) {
                Acc a = R::id();
                int p = s;
                for (; p + 8 <= e; p += 8) {
                    In x[8];
#pragma unroll
                    for (int j = 0; j < 8; ++j) x[j] = sv[p + j];
#pragma unroll
                    for (int j = 0; j < 8; ++j) a = R::ap(a, Acc(x[j]));
                }
                for (; p < e; ++p) a = R::ap(a, Acc(sv[p]));
                finish(r, sa == ea, a);
            } else {
                const int kk = atomicAdd(&s_nlong, 1);
                if (kk < kMaxLong) slong[kk] = LongSeg{r, s, e};
            }
        }
        __syncthreads();
        const int nlong = s_nlong < kMaxLong ? s_nlong : kMaxLong;
        for (int k = w; k < nlong; k += NW) {
            const LongSeg g = slong[k];
            Acc a = R::id();
            int p = g.s + lane;
            for (; p + 3 * kWave < g.e; p += 4 * kWave) {
                const In x0 = sv[p], x1 = sv[p + kWave], x2 = sv[p + 2 * kWave], x3 = sv[p + 3 * kWave];
                a = R::ap(R::ap(R::ap(R::ap(a, Acc(x0)), Acc(x1)), Acc(x2)), Acc(x3));
            }
            for (; p < g.e; p += kWave) a = R::ap(a, Acc(sv[p]));
            a = wave_reduce<R>(a);
            if (lane == 0) finish(g.row, false, a);
        }
        __syncthreads();
        if (t == 0) s_nlong = 0;
        __syncthreads();
    }

    // split rows: wave 0 publishes the head part, wave 1 the tail part; the
    // part that arrived last at the row's counter folds them all
    if (w < 2) {
        const bool has = w == 0 ? has_head : has_tail;
        if (has) {
            const int64_t r = w == 0 ? lo : hi - 1;
            const int64_t sa = w == 0 ? cr.head_s : cr.tail_s, ea = w == 0 ? cr.head_e : cr.tail_e;
            int64_t b0 = sa / S, b1 = (ea - 1) / S;
            b0 = b0 < 0 ? 0 : b0;
            b1 = b1 < nchunks ? b1 : nchunks - 1;
            if (lane == 0) slot_put((w == 0 ? ws.head : ws.tail) + 2 * c, s_cval[w]);
            if (s_arrived[w] == (unsigned)(b1 - b0)) {  // the last of the row's b1 - b0 + 1 parts
                Acc a = R::id();
                if (lane == 0) a = slot_get<Acc>(ws.tail + 2 * b0);
                for (int64_t b = b0 + 1; b <= b1; b += kWave) {
                    const int m = (int)(b1 - b + 1 < kWave ? b1 - b + 1 : kWave);
                    Acc h = R::id();
                    if (lane < m) h = slot_get<Acc>(ws.head + 2 * (b + lane));
                    for (int j = 0; j < m; ++j) a = R::ap(a, __shfl(h, j));  // lane 0's a: parts in order
                    if (lane < m) slot_clear<Acc>(ws.head + 2 * (b + lane));
                }
                if (lane == 0) {
                    out[r] = R::ap(ne, a);
                    slot_clear<Acc>(ws.tail + 2 * b0);
                    __hip_atomic_store(&ws.cnt[b0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
            }
        }
    }
}

// ---- the no-allocation variant's scratch: the split-row slots of
// mx_segmented_reduce_noalloc live in this fixed array (one copy per device,
// zero at load).  Host code never passes the array's name to a kernel: it
// takes the device address from hipGetSymbolAddress once per device.
constexpr size_t kScratchBytes = (size_t)1 << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

// Zero-fills n 32-bit words (a kernel rather than a memset node, so that the
// call can sit in a captured graph).
__global__ void __launch_bounds__(NT) k_zero_words(uint32_t *__restrict__ p, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * NT;
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += stride) p[i] = 0u;
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

// Every row empty (no values): out[r] = ne.
template <class Acc>
__global__ void __launch_bounds__(NT) k_fill(Acc *__restrict__ out, int64_t n, Acc v) {
    const int64_t stride = (int64_t)gridDim.x * NT;
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += stride) out[i] = v;
}

// Reverse of the row sums: gval[p] = gout[row of p], over the same chunks.
// The rows touching the chunk fill its LDS copy (short segments one lane
// each, long ones a wave each); the chunk then leaves in 16-byte stores.
__global__ void __launch_bounds__(NT) k_seg_broadcast(const float *__restrict__ gout,
                                                      const int64_t *__restrict__ offsets, int64_t nseg,
                                                      int64_t nval, int64_t nchunks, float *__restrict__ gval,
                                                      int vec) {
    constexpr int S = kChunkBytes / 4;
    constexpr int NW = NT / kWave;
    struct Fill {
        int s, e;  // chunk-relative [s, e)
        float g;
    };
    __shared__ __attribute__((aligned(16))) float sv[S];
    __shared__ Fill slong[kMaxLong];
    __shared__ int64_t s_off[kOffWin];
    __shared__ ChunkRows cr;
    __shared__ int s_nlong;
    const int t = threadIdx.x, w = t / kWave, lane = t & (kWave - 1);
    const int64_t c = blockIdx.x;
    const int64_t P0 = c * S;
    const int n = (int)(nval - P0 < S ? nval - P0 : S);
    const int64_t P1 = P0 + n;
    if (t == 0) s_nlong = 0;
    chunk_rows(offsets, nseg, nval, c, nchunks, P0, P1, &cr, s_off);
    __syncthreads();
    const int64_t lo = cr.lo, hi = cr.hi;
    const int n_off = cr.n_off;
    for (int64_t base = lo; base < hi; base += NT) {
        const int64_t r = base + t;
        if (r < hi) {
            const int64_t k = r - lo;
            const int64_t sa = k < n_off ? s_off[k] : offsets[r];
            const int64_t ea = k + 1 < n_off ? s_off[k + 1] : offsets[r + 1];
            // clamped to the chunk (they are inside it whenever the offsets are valid)
            const int s = (int)(sa >= P1 ? n : sa > P0 ? sa - P0 : 0);
            const int e = (int)(ea <= P0 ? s : ea < P1 ? (ea - P0 > s ? ea - P0 : s) : n);
            const float g = s < e ? gout[r] : 0.0f;
            if (e - s <= kShortSeg) {
                for (int p = s; p < e; ++p) sv[p] = g;
            } else {
                const int k = atomicAdd(&s_nlong, 1);
                if (k < kMaxLong) slong[k] = Fill{s, e, g};
            }
        }
        __syncthreads();
        const int nlong = s_nlong < kMaxLong ? s_nlong : kMaxLong;
        for (int k = w; k < nlong; k += NW) {
            const Fill f = slong[k];
            for (int p = f.s + lane; p < f.e; p += kWave) sv[p] = f.g;
        }
        __syncthreads();
        if (t == 0) s_nlong = 0;
        __syncthreads();
    }
    if (vec) {
        u32x4 *dst = reinterpret_cast<u32x4 *>(gval + P0);
        const u32x4 *src = reinterpret_cast<const u32x4 *>(sv);
#pragma unroll
        for (int u = 0; u < S / 4 / NT; ++u) {
            const int q = t + NT * u;
            if (q * 4 + 4 <= n) {
                __builtin_nontemporal_store(src[q], dst + q);
            } else if (q * 4 < n) {
                for (int j = q * 4; j < n; ++j) gval[P0 + j] = sv[j];
            }
        }
    } else {
        for (int k = t; k < n; k += NT) gval[P0 + k] = sv[k];
    }
}

// Rows per block of the row-chunked schedule the generated map-body kernels
// use: enough blocks for eight per CU, at most 16 rows each.
constexpr int kMaxRowsPerBlock = 16;
int rows_per_block(int64_t nseg, const DeviceInfo *d) {
    const int64_t target = (int64_t)d->num_cus * 8;
    int64_t rb = ceil_div(nseg, target);
    return (int)(rb < 1 ? 1 : rb > kMaxRowsPerBlock ? kMaxRowsPerBlock : rb);
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
mx_status launch_seg(bool plain, const void *values, int64_t nval, const int64_t *off, int64_t nseg,
                     const void *ne_host, void *out, void *ws, size_t ws_bytes, hipStream_t s) {
    using In = typename DT<D>::In;
    using Acc = typename DT<D>::Acc;
    Acc ne;
    __builtin_memcpy(&ne, ne_host, sizeof(Acc));
    if (plain) {
        int grid = (int)ceil_div(nseg, NT);
        hipLaunchKernelGGL((k_seg_thread<D, OP>), dim3(grid), dim3(NT), 0, s, (const In *)values, off,
                           nseg, ne, (Acc *)out);
    } else if (nval == 0) {
        const DeviceInfo *d;
        if (mx_status st = device_info(&d)) return st;
        const int64_t grid = std::min<int64_t>(ceil_div(nseg, NT), (int64_t)d->num_cus * 8);
        hipLaunchKernelGGL((k_fill<Acc>), dim3((unsigned)grid), dim3(NT), 0, s, (Acc *)out, nseg, ne);
    } else {
        const int64_t nch = chunks_of(nval, chunk_len<D>());
        MX_REQUIRE(nch <= 0x7fffffff, MX_ERR_SHAPE, "mx_segmented_reduce: too many values");
        SegWs w{};
        if (nch > 1) {
            const size_t need = seg_ws_bytes(nval);
            MX_REQUIRE(ws && ws_bytes >= need, MX_ERR_WORKSPACE, "mx_segmented_reduce: workspace needs %zu bytes",
                       need);
            MX_REQUIRE(((uintptr_t)ws & 255) == 0, MX_ERR_INVALID,
                       "mx_segmented_reduce: workspace must be 256-byte aligned");
            w = seg_ws(ws, nval);
        }
        if (aligned16(values))
            hipLaunchKernelGGL((k_seg_chunk<D, OP, true>), dim3((unsigned)nch), dim3(NT), 0, s, (const In *)values,
                               off, nseg, nval, nch, ne, (Acc *)out, w);
        else
            hipLaunchKernelGGL((k_seg_chunk<D, OP, false>), dim3((unsigned)nch), dim3(NT), 0, s, (const In *)values,
                               off, nseg, nval, nch, ne, (Acc *)out, w);
    }
    return last_launch("mx_segmented_reduce");
}

template <mx_dtype D>
mx_status seg_by_op(bool plain, int op, const void *v, int64_t nval, const int64_t *off, int64_t nseg,
                    const void *ne, void *out, void *ws, size_t wsb, hipStream_t s) {
    switch (op) {
    case MX_ADD: return launch_seg<D, MX_ADD>(plain, v, nval, off, nseg, ne, out, ws, wsb, s);
    case MX_MUL: return launch_seg<D, MX_MUL>(plain, v, nval, off, nseg, ne, out, ws, wsb, s);
    case MX_MIN: return launch_seg<D, MX_MIN>(plain, v, nval, off, nseg, ne, out, ws, wsb, s);
    case MX_MAX: return launch_seg<D, MX_MAX>(plain, v, nval, off, nseg, ne, out, ws, wsb, s);
    }
    return set_error(MX_ERR_INVALID, "mx_segmented_reduce: unknown operator %d", op);
}

mx_status segmented(const char *who, bool plain, int op, mx_dtype dtype, const void *values, int64_t nval,
                    const int64_t *off, int64_t nseg, const void *ne, void *out, void *ws, size_t wsb,
                    hipStream_t s) {
    MX_REQUIRE(nseg >= 0, MX_ERR_SHAPE, "%s: nseg < 0", who);
    MX_REQUIRE(nval >= 0, MX_ERR_SHAPE, "%s: nvalues < 0", who);
    MX_REQUIRE(dtype_valid(dtype), MX_ERR_DTYPE, "%s: bad dtype %d", who, (int)dtype);
    MX_REQUIRE(op >= MX_ADD && op <= MX_MAX, MX_ERR_INVALID, "%s: unknown operator %d", who, op);
    MX_REQUIRE(ne, MX_ERR_INVALID, "%s: null ne", who);
    if (nseg == 0) return MX_OK;
    MX_REQUIRE(off && out, MX_ERR_INVALID, "%s: null offsets or out", who);
    MX_REQUIRE(nval == 0 || values, MX_ERR_INVALID, "%s: null values", who);
    if (debug_mode()) {
        const DeviceInfo *d;
        if (mx_status st = device_info(&d)) return st;
        if (mx_status st = validate_offsets(who, off, nseg, nval, s, d)) return st;
    }
    switch (dtype) {
    case MX_F32: return seg_by_op<MX_F32>(plain, op, values, nval, off, nseg, ne, out, ws, wsb, s);
    case MX_F64: return seg_by_op<MX_F64>(plain, op, values, nval, off, nseg, ne, out, ws, wsb, s);
    case MX_I32: return seg_by_op<MX_I32>(plain, op, values, nval, off, nseg, ne, out, ws, wsb, s);
    case MX_I64: return seg_by_op<MX_I64>(plain, op, values, nval, off, nseg, ne, out, ws, wsb, s);
    }
    return MX_ERR_DTYPE;
}

std::mutex g_scratch_mu;
void *g_scratch_addr[64] = {};

}  // namespace

// Device address of this device's scratch array (looked up once per device,
// with that device current).
mx_status segmented_scratch(void **out) {
    int dev = 0;
    MX_TRY_HIP(hipGetDevice(&dev));
    MX_REQUIRE(dev >= 0 && dev < 64, MX_ERR_INVALID, "device ordinal %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void *p = nullptr;
        MX_TRY_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        MX_REQUIRE(p != nullptr, MX_ERR_HIP, "hipGetSymbolAddress returned no address for the scratch array");
        g_scratch_addr[dev] = p;
    }
    *out = g_scratch_addr[dev];
    return MX_OK;
}

// Shared with the generated map-body kernels: rows per block of a block-span
// reduce, and the debug-mode check of an offsets array.
int segmented_rows_per_block(int64_t nseg, const DeviceInfo *d) { return rows_per_block(nseg, d); }

mx_status check_offsets_debug(const char *who, const int64_t *off, int64_t nseg, hipStream_t s) {
    if (!debug_mode()) return MX_OK;
    const DeviceInfo *d;
    if (mx_status st = device_info(&d)) return st;
    return validate_offsets(who, off, nseg, -1, s, d);
}

size_t segmented_ws_bytes(int64_t nval) { return seg_ws_bytes(nval); }

// The reverse of the row sums over the chunks of gvalues (the caller checks
// pointers and shapes).
mx_status segmented_broadcast(const float *gout, const int64_t *off, int64_t nseg, float *gval, int64_t nval,
                              hipStream_t s) {
    if (nval == 0) return MX_OK;
    const int64_t nch = chunks_of(nval, kChunkBytes / 4);
    MX_REQUIRE(nch <= 0x7fffffff, MX_ERR_SHAPE, "mx_segmented_sum_adjoint_f32: too many values");
    hipLaunchKernelGGL(k_seg_broadcast, dim3((unsigned)nch), dim3(NT), 0, s, gout, off, nseg, nval, nch, gval,
                       (int)aligned16(gval));
    return last_launch("mx_segmented_sum_adjoint_f32");
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

mx_status mx_segmented_reduce(mx_redop op, mx_dtype dtype, const void *values_dev, int64_t nvalues,
                              const int64_t *offsets_dev, int64_t nseg, const void *ne_host, void *out_dev,
                              void *ws, size_t ws_bytes, hipStream_t stream) {
    return segmented("mx_segmented_reduce", false, op, dtype, values_dev, nvalues, offsets_dev, nseg, ne_host,
                     out_dev, ws, ws_bytes, stream);
}

mx_status mx_segmented_reduce_noalloc(mx_redop op, mx_dtype dtype, const void *values_dev, int64_t nvalues,
                                      const int64_t *offsets_dev, int64_t nseg, const void *ne_host, void *out_dev,
                                      hipStream_t stream) {
    const char *who = "mx_segmented_reduce_noalloc";
    MX_REQUIRE(nvalues >= 0, MX_ERR_SHAPE, "%s: nvalues < 0", who);
    const size_t need = seg_ws_bytes(nvalues);
    MX_REQUIRE(need <= kScratchBytes, MX_ERR_WORKSPACE,
               "%s: %lld values need %zu bytes of split-row slots, more than the %zu-byte built-in scratch "
               "(at most %lld values); use mx_segmented_reduce with a workspace",
               who, (long long)nvalues, need, kScratchBytes, (long long)mx_segmented_noalloc_max_values());
    void *ws = nullptr;
    if (mx_status st = segmented_scratch(&ws)) return st;
    if (nseg > 0 && nvalues > 0) {
        // the kernels leave the slots zero; clear the part this call uses all
        // the same, in case an earlier call on this device did not finish
        const int64_t words = (int64_t)(need / 4);
        hipLaunchKernelGGL(k_zero_words, dim3((unsigned)std::min<int64_t>(ceil_div(words, NT), 1024)), dim3(NT), 0,
                           stream, (uint32_t *)ws, words);
        if (mx_status st = last_launch(who)) return st;
    }
    return segmented(who, false, op, dtype, values_dev, nvalues, offsets_dev, nseg, ne_host, out_dev, ws,
                     kScratchBytes, stream);
}

int64_t mx_segmented_noalloc_max_values(void) {
    // the largest n with seg_ws_bytes(n) <= kScratchBytes (whole 2048-element chunks)
    int64_t lo = 0, hi = (int64_t)kScratchBytes * 2048;
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo + 1) / 2;
        if (seg_ws_bytes(mid) <= kScratchBytes) lo = mid; else hi = mid - 1;
    }
    return lo;
}

mx_status mx_segmented_reduce_plain(mx_redop op, mx_dtype dtype, const void *values_dev, int64_t nvalues,
                                    const int64_t *offsets_dev, int64_t nseg, const void *ne_host,
                                    void *out_dev, hipStream_t stream) {
    return segmented("mx_segmented_reduce_plain", true, op, dtype, values_dev, nvalues, offsets_dev, nseg,
                     ne_host, out_dev, nullptr, 0, stream);
}

mx_status mx_segmented_sum_adjoint_f32(const float *gout_dev, const int64_t *offsets_dev, int64_t nseg,
                                       float *gvalues_dev, int64_t nvalues, hipStream_t stream) {
    const char *who = "mx_segmented_sum_adjoint_f32";
    MX_REQUIRE(nseg >= 0 && nvalues >= 0, MX_ERR_SHAPE, "%s: nseg < 0 or nvalues < 0", who);
    if (nseg == 0) return MX_OK;
    MX_REQUIRE(gout_dev && offsets_dev && (gvalues_dev || nvalues == 0), MX_ERR_INVALID, "%s: null pointer", who);
    const DeviceInfo *d;
    if (mx_status st = device_info(&d)) return st;
    if (debug_mode())
        if (mx_status st = validate_offsets(who, offsets_dev, nseg, nvalues, stream, d)) return st;
    return segmented_broadcast(gout_dev, offsets_dev, nseg, gvalues_dev, nvalues, stream);
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
