// Ragged sequences in the flat marshalled layout (values + int64 offsets):
// nested map (reduce) over rows, its reverse (broadcast), the lengths ->
// offsets scan of marshaling, offset composition for `map flatten`, and the
// debug-mode validation of offsets (Appendix "Dynamic Assumptions").
#include <algorithm>
#include <mutex>
#include <vector>

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
// The path for long rows (see seg_span_path below).  The flat value array is cut
// into chunks of kChunkBytes (S elements), and a
// block streams q consecutive chunks, the value range [PS, PE) with
// PS = B q S, so every block reads about the same number of bytes whatever the
// row lengths (q is chosen so that the grid is as many blocks as the device
// holds at once).  A block issues its first chunk's loads at once (their
// addresses depend only on B) and, while they are in flight, two waves find by
// search in the offsets the rows that touch its range.  Each chunk is staged
// in LDS, the next chunk's loads go out, and each row's segment in the chunk
// is folded by a whole wave (lanes interleaved, then the wave tree) or, where
// a chunk holds many short rows, by one lane.  The fold structure depends only
// on the offsets and S, never on timing, so results repeat bit for bit.
//
// Row ownership: a row belongs to the block whose range holds its start (an
// empty row: its position; rows at the very end: the last block).  The owner
// folds its last row to the row's end, reading up to S values past PE, so a
// row shorter than S never needs a second block.  A row that runs more than S
// past the end of its owner's range ("long") is split at the block edges
// instead: its blocks b0 < ... < b1 each fold their part, and the part that
// arrives last combines them in order.  Each part counts itself in at the
// counter of b0 when its block starts; block b0 then publishes its part in
// the tail slot T[b0], every later block in its head slot H[b]; the block
// whose count is b1 - b0 folds T[b0], H[b0+1], ..., H[b1] and writes the row.
// Nobody waits for a block that may not have started: a slot is read only
// after its writer has counted itself in, every block publishes its parts
// before it reads any, and the slot's own tag shows when its store has
// landed.  Slots are tagged 64-bit words written and read with device-scope
// atomics, so no cache flushes are needed; the finishing block clears the
// slots and the counter.
constexpr int kChunkBytes = 16384;
// a chunk with more rows than this folds its short segments one lane each
constexpr int kWaveRows = 32;
constexpr int kShortSeg = 32;  // longest segment one lane folds
constexpr int kMaxChunks = 48;  // chunks one block streams, at most (q + 1 <= kMaxChunks)

template <mx_dtype D> constexpr int chunk_len() { return kChunkBytes / (int)sizeof(typename DT<D>::In); }

int64_t chunks_of(int64_t nval, int S) { return (nval + S - 1) / S; }

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
        // a scalar base per round and one lane offset: one address register
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const u32x4 *vu = reinterpret_cast<const u32x4 *>(values + P0 + (int64_t)NT * V * u);
            if ((int)(threadIdx.x + NT * u) * V + V <= n) x[u] = __builtin_nontemporal_load(vu + threadIdx.x);
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
// ---- the block's rows
//
// Block B's range [PS, PE) is touched by rows [lo, hi): lo the row holding
// PS - 1 when it runs past PS (else the first row starting at PS or later;
// row 0 for B = 0), hi the first row starting at PE or later (nseg for the
// last block).  They are found in two dependent rounds of loads: wave 0
// reads 64 offsets kGuessStep apart around the entry the answer would be if
// every row had the same length, which brackets the first row starting at PS
// or later within kGuessStep entries; then every thread reads one entry of
// the window of offsets that starts just below the bracket.  The window holds
// lo and, for rows of ordinary length, hi and the bounds of every row between
// them.  Plain searches take over where the bracket misses or the rows run
// past the window.
//
// The window keeps positions relative to PS as 32-bit integers, clamped to
// +-2^30 (every comparison the kernels make is with positions within a few
// chunks of the block, so the clamp never changes one), so the row
// bookkeeping runs on the scalar unit.

constexpr int64_t kGuessStep = 64;
constexpr int32_t kRelMax = 1 << 30;

__device__ __forceinline__ int32_t rel_of(int64_t x, int64_t PS) {
    const int64_t d = x - PS;
    return (int32_t)(d < -kRelMax ? -kRelMax : d > kRelMax ? kRelMax : d);
}

// Values every lane of the block holds alike (read from LDS) moved to scalar
// registers.
__device__ __forceinline__ int64_t uniform(int64_t v) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
template <class T> __device__ __forceinline__ T uniform_val(T v) {
    if constexpr (sizeof(T) == 4) {
        int b;
        __builtin_memcpy(&b, &v, 4);
        b = __builtin_amdgcn_readfirstlane(b);
        __builtin_memcpy(&v, &b, 4);
    } else {
        int64_t b;
        __builtin_memcpy(&b, &v, 8);
        b = uniform(b);
        __builtin_memcpy(&v, &b, 8);
    }
    return v;
}

// A global load that stays one: with a plain load, the compiler may merge
// "LDS window entry, else global memory" into one generic-address load, whose
// wait also waits for the next chunk's loads in flight.  A relaxed atomic
// load is never merged with a plain one.
template <class T> __device__ __forceinline__ T gload(const T *p) {
    return __hip_atomic_load(const_cast<T *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int64_t blk_end(int64_t b, int64_t NB, int64_t nval) {
    return (b + 1) * NB < nval ? (b + 1) * NB : nval;
}

struct BlockRows {
    int64_t lo, hi;
    int64_t wb;              // the window holds offsets[wb .. wb + nwin), relative to PS
    int nwin;
    int32_t head_s, head_e;  // bounds of row lo
    int32_t tail_e;          // end of row hi - 1
};

// Round 1, wave 0 only: the base of the window (s_sh[0]); s_sh[1], s_sh[2]
// (the first rows starting at PS and at PE or later) are set to -1.
__device__ void rows_bracket(const int64_t *__restrict__ off, int64_t nseg, int64_t nval, int64_t B, int64_t PS,
                             int64_t *s_sh) {
    const int lane = threadIdx.x & (kWave - 1);
    int64_t wb = 0;
    if (B > 0) {
        const int64_t x = PS - 1;
        int64_t g = (int64_t)((double)x / (double)nval * (double)nseg);
        g = g < 0 ? 0 : g > nseg ? nseg : g;
        int64_t first = g - 32 * kGuessStep;
        first = first < 0 ? 0 : first;
        const int64_t idx = first + lane * kGuessStep;
        const bool gt = idx > nseg || off[idx] > x;  // past nseg: as if +infinity
        const uint64_t m = __ballot(gt);
        const int f = m ? __builtin_ctzll(m) : kWave;
        int64_t u;  // the first index with off[u] > x lies in (u - kGuessStep, u]
        if ((f == 0 && first > 0) || f == kWave) u = wave_upper_bound(off, nseg, x);
        else u = f == 0 ? 0 : first + (int64_t)(f - 1) * kGuessStep + 1;
        wb = u - 1;  // the row before the answer may be lo
        wb = wb < 0 ? 0 : wb > nseg ? nseg : wb;
    }
    if (lane == 0) {
        s_sh[0] = wb;
        s_sh[1] = -1;
        s_sh[2] = -1;
    }
}

// Round 2, all threads: the window, relative to PS (and, for the broadcast,
// the gradients of its rows).  WIN + 1 <= NT entries.
template <int WIN>
__device__ __forceinline__ int window_count(int64_t nseg, int64_t wb) {
    const int64_t avail = nseg + 1 - wb;
    return (int)(avail < WIN + 1 ? avail : WIN + 1);
}
template <int WIN>
__device__ __forceinline__ void rows_window(const int64_t *__restrict__ off, int64_t nseg, int64_t PS,
                                            const int64_t *s_sh, int32_t *s_w, const float *__restrict__ gsrc,
                                            float *s_g) {
    const int t = threadIdx.x;
    const int64_t wb = uniform(s_sh[0]);
    const int cnt = window_count<WIN>(nseg, wb);
    if (t < cnt) {
        s_w[t] = rel_of(off[wb + t], PS);
        if (gsrc && t < cnt - 1) s_g[t] = gsrc[wb + t];
    }
}

// After the window is in (a barrier between each step): the answers in the
// window, then wave 0 fills *br, searching where the window falls short.
template <int WIN>
__device__ __forceinline__ void rows_find(int64_t nseg, int64_t B, int64_t nblk, int32_t PEr, const int32_t *s_w,
                                          int64_t *s_sh) {
    const int t = threadIdx.x;
    const int64_t wb = uniform(s_sh[0]);
    const int cnt = window_count<WIN>(nseg, wb);
    if (t < cnt) {
        const int32_t v = s_w[t], pv = t > 0 ? s_w[t - 1] : INT32_MIN;
        if (B > 0 && v >= 0 && pv < 0) s_sh[1] = wb + t;
        if (B + 1 < nblk && v >= PEr && pv < PEr) s_sh[2] = wb + t;
    }
}
template <int WIN>
__device__ void rows_finish(const int64_t *__restrict__ off, int64_t nseg, int64_t B, int64_t nblk, int64_t PS,
                            int64_t PE, const int32_t *s_w, const int64_t *s_sh, BlockRows *br) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t wb = uniform(s_sh[0]);
    const int cnt = window_count<WIN>(nseg, wb);
    auto relv = [&](int64_t i) { return i >= wb && i - wb < cnt ? s_w[i - wb] : rel_of(gload(off + i), PS); };
    int64_t u = uniform(s_sh[1]), hi = uniform(s_sh[2]);
    // the window missed (offsets outside the contract, or rows past it)
    if (B > 0 && u < 0) u = wave_upper_bound(off, nseg, PS - 1);
    if (B + 1 >= nblk) hi = nseg;
    else if (hi < 0) hi = wave_upper_bound(off, nseg, PE - 1);
    u = u < 0 ? 0 : u > nseg ? nseg : u;
    hi = hi > nseg ? nseg : hi;
    int64_t lo = 0;
    if (B > 0) lo = (u > 0 && relv(u) > 0) ? u - 1 : u;
    hi = hi < lo ? lo : hi;
    if (lane == 0) {
        br->lo = lo;
        br->hi = hi;
        br->wb = wb;
        br->nwin = cnt;
        br->head_s = relv(lo);
        br->head_e = lo < nseg ? relv(lo + 1) : br->head_s;
        br->tail_e = relv(hi);
    }
}

// Row bounds relative to PS as a block folds them, a long row's part clipped
// to [0, PEr); i is a row's index in the window.  The folds read the window
// alone (a global load there, even on a branch not taken, makes the compiler
// wait for every load in flight, the next chunk's included); the window moves
// on when a chunk's rows run past it.
struct RowBounds {
    const int32_t *win;
    int lo_i, last_i;  // window indices of rows lo and hi - 1 (-1: not in the window)
    int32_t PEr;
    bool has_head, has_tail;
    __device__ __forceinline__ int32_t s(int i) const { return i == lo_i && has_head ? 0 : win[i]; }
    __device__ __forceinline__ int32_t e(int i) const {
        if (i == lo_i && has_head) {
            const int32_t v = win[i + 1];
            return v < PEr ? v : PEr;
        }
        return i == last_i && has_tail ? PEr : win[i + 1];
    }
};
// Rows clipped to the block's range (the broadcast).
struct FillBounds {
    const int32_t *win;
    int32_t PEr;
    __device__ __forceinline__ int32_t s(int i) const { return win[i] > 0 ? win[i] : 0; }
    __device__ __forceinline__ int32_t e(int i) const { return win[i + 1] < PEr ? win[i + 1] : PEr; }
};
__device__ __forceinline__ int win_index(int64_t r, int64_t wb) {
    const int64_t d = r - wb;
    return (int)(d < -1 ? -1 : d > INT32_MAX ? INT32_MAX : d);
}

// The rows of each chunk [k S, k S + S) (relative to PS) of a block: [ra, rb),
// ra the first row that ends past the chunk's start or starts at it or later,
// rb the first row starting at the chunk's end or later (the last chunk:
// every row left).  From the window, in one pass: thread t takes row lo + t
// and marks the chunks whose first later-starting row it is; then ra(k) is
// rb(k - 1), or the row before it when that row runs past the chunk's start.
// All threads call; three barriers inside.
template <int S, class RB>
__device__ __forceinline__ void chunk_ranges(const RB &rw, int64_t lo, int64_t hi, int64_t wb, int nchunk,
                                             int64_t *s_ra, int64_t *s_rb) {
    const int t = threadIdx.x;
    if (t < nchunk) s_rb[t] = hi;
    __syncthreads();
    const int i0 = (int)(lo - wb);
    if (t < hi - lo) {
        const int i = i0 + t;
        auto cidx = [&](int32_t p) {
            const int32_t c = p < 0 ? 0 : p / S;
            return c > nchunk - 1 ? nchunk - 1 : (int)c;
        };
        const int cs = cidx(rw.s(i)), cp = t == 0 ? 0 : cidx(rw.s(i - 1));
        for (int k = cp; k < cs; ++k) s_rb[k] = lo + t;
    }
    __syncthreads();
    if (t < nchunk) {
        int64_t ra = lo;
        if (t > 0) {
            const int64_t rbp = s_rb[t - 1];
            ra = (rbp > lo && rw.e((int)(rbp - 1 - wb)) > t * S) ? rbp - 1 : rbp;
        }
        s_ra[t] = ra;
    }
    __syncthreads();
}

// The same where the window does not hold all the block's rows: one thread
// per chunk, binary search with bounds from global memory past the window.
template <bool CLIP_PART>
__device__ void chunk_ranges_search(const int64_t *__restrict__ off, const int32_t *s_w, int64_t wb, int nwin,
                                    int64_t PS, int32_t PEr, int64_t lo, int64_t hi, bool has_head, bool has_tail,
                                    int S, int32_t ver, int nchunk, int64_t *s_ra, int64_t *s_rb) {
    const int t = threadIdx.x;
    if (t < nchunk) {
        auto offr = [&](int64_t i) { return i - wb < nwin ? s_w[i - wb] : rel_of(gload(off + i), PS); };
        auto rs = [&](int64_t r) -> int32_t {
            if (CLIP_PART) return r == lo && has_head ? 0 : offr(r);
            const int32_t v = offr(r);
            return v > 0 ? v : 0;
        };
        auto re = [&](int64_t r) -> int32_t {
            const int32_t v = offr(r + 1);
            if (CLIP_PART) {
                if (r == lo && has_head) return v < PEr ? v : PEr;
                return r == hi - 1 && has_tail ? PEr : v;
            }
            return v < PEr ? v : PEr;
        };
        const int32_t C0 = t * S, C1 = C0 + S < ver ? C0 + S : ver;
        int64_t a = lo, b = hi;
        while (a < b) {
            const int64_t m = (a + b) / 2;
            if (re(m) > C0 || rs(m) >= C0) b = m;
            else a = m + 1;
        }
        s_ra[t] = a;
        if (t + 1 == nchunk) {
            s_rb[t] = hi;
        } else {
            b = hi;
            while (a < b) {
                const int64_t m = (a + b) / 2;
                if (rs(m) >= C1) b = m;
                else a = m + 1;
            }
            s_rb[t] = a;
        }
    }
    __syncthreads();
}

// Folds chunk-relative [s, e) of the LDS chunk, lanes interleaved, then the
// wave tree (s, e alike in every lane; the result is in every lane).  Four
// loads per lane go out together; in the last, partial round, lanes past e
// read element s and drop it.
template <class R, class Acc, class In>
__device__ __forceinline__ Acc wave_fold(const In *sv, int s, int e) {
    const int lane = threadIdx.x & (kWave - 1);
    Acc a = R::id();
    int base = s;
    for (; base + 4 * kWave <= e; base += 4 * kWave) {
        const In *p = sv + base + lane;
        const In x0 = p[0], x1 = p[kWave], x2 = p[2 * kWave], x3 = p[3 * kWave];
        a = R::ap(R::ap(R::ap(R::ap(a, Acc(x0)), Acc(x1)), Acc(x2)), Acc(x3));
    }
    if (base < e) {
        const int p = base + lane;
        In x[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) x[j] = sv[p + j * kWave < e ? p + j * kWave : s];
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (p + j * kWave < e) a = R::ap(a, Acc(x[j]));
    }
    return wave_reduce<R>(a);
}
// One lane folds [s, e) left to right.
template <class R, class Acc, class In>
__device__ __forceinline__ Acc lane_fold(const In *sv, int s, int e) {
    Acc a = R::id();
    int p = s;
    for (; p + 4 <= e; p += 4) {
        In x[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) x[j] = sv[p + j];
#pragma unroll
        for (int j = 0; j < 4; ++j) a = R::ap(a, Acc(x[j]));
    }
    for (; p < e; ++p) a = R::ap(a, Acc(sv[p]));
    return a;
}

// A row's segment [sa, ea) clipped to the chunk [C0, C0 + n), chunk-relative
// (clamped, so that offsets breaking their contract cannot index out of LDS).
__device__ __forceinline__ void seg_in_chunk(int32_t sa, int32_t ea, int32_t C0, int n, int *s, int *e) {
    const int32_t a = sa - C0, b = ea - C0;
    const int ss = a < 0 ? 0 : a > n ? n : a;
    *s = ss;
    *e = b < ss ? ss : b > n ? n : b;
}

// Rows in the window of a block of the reduce: 255 for 4-byte results, fewer
// for 8-byte ones (their result buffer is twice the size), so that eight
// blocks fit in one CU's LDS.
template <class Acc> constexpr int win_rows() { return sizeof(Acc) == 4 ? 255 : 159; }

// ---- the reduce
//
// Ownership: row lo is another block's unless it is long (its part is folded
// here); the last row may run past PE, to its end, unless it is long.  A row
// that starts in block b0 < B is long if it starts before PS - NB (it spans a
// whole block) or ends more than S past PS; one that starts here is long if
// it ends more than S past PE.
template <mx_dtype D, int OP, bool VEC>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(8, 8)))
k_seg_blocks(const typename DT<D>::In *__restrict__ values, const int64_t *__restrict__ offsets, int64_t nseg,
             int64_t nval, int64_t q, int64_t nblk, typename DT<D>::Acc ne, typename DT<D>::Acc *__restrict__ out,
             SegWs ws) {
    using In = typename DT<D>::In;
    using Acc = typename DT<D>::Acc;
    using R = Red<OP, Acc>;
    constexpr int S = chunk_len<D>();
    constexpr int NW = NT / kWave;
    constexpr int WIN = win_rows<Acc>();
    __shared__ __attribute__((aligned(16))) In sv[S];
    __shared__ int32_t s_w[WIN + 1];
    __shared__ int64_t s_ra[kMaxChunks], s_rb[kMaxChunks];
    __shared__ int64_t s_sh[3];
    __shared__ int64_t s_long[3];  // the blocks of the long rows' parts: [hb0, hb1] and [B, tb1]
    __shared__ BlockRows br;
    __shared__ Acc s_res[WIN];     // finished rows of the window, written out when it moves
    __shared__ Acc s_carry[2];     // partial fold of the row running into the next chunk, by chunk parity
    __shared__ Acc s_part[2];      // the long rows' parts: [0] row lo, [1] row hi - 1
    __shared__ unsigned s_arrived[2];

    const int t = threadIdx.x, lane = t & (kWave - 1);
    const int w = __builtin_amdgcn_readfirstlane(t / kWave);
    const int64_t B = blockIdx.x, NB = q * S;
    const int64_t PS = B * NB, PE = blk_end(B, NB, nval);
    const int32_t PEr = (int32_t)(PE - PS);

    // chunk 0 streams in during round 1, chunk 1 during round 2
    ChunkLoad<In, typename DT<D>::Vec, DT<D>::kVec, S, VEC> ld;
    const int n0 = (int)(nval - PS < S ? nval - PS : S);
    ld.issue(values, PS, n0);
    if (w == 0) rows_bracket(offsets, nseg, nval, B, PS, s_sh);
    __syncthreads();
    ld.store(sv, values, PS, n0);
    if (PS + S < nval) ld.issue(values, PS + S, (int)(nval - PS - S < S ? nval - PS - S : S));
    rows_window<WIN>(offsets, nseg, PS, s_sh, s_w, nullptr, nullptr);
    __syncthreads();
    rows_find<WIN>(nseg, B, nblk, PEr, s_w, s_sh);
    __syncthreads();
    if (w == 0) rows_finish<WIN>(offsets, nseg, B, nblk, PS, PE, s_w, s_sh, &br);
    __syncthreads();

    // ownership, alike in every thread
    int64_t lo = uniform(br.lo);
    const int64_t hi = uniform(br.hi), wb = uniform(br.wb);
    const int32_t head_s = uniform(br.head_s), head_e = uniform(br.head_e), tail_e = uniform(br.tail_e);
    const int nwin = uniform(br.nwin);
    const bool straddle = B > 0 && head_s < 0;
    const bool has_head = straddle && (head_s < -(int32_t)NB || head_e > S);
    if (straddle && !has_head) lo += 1;  // its owner reads it to its end
    const bool last_starts_here = hi > lo && !(has_head && hi - 1 == lo);
    const bool has_tail = last_starts_here && tail_e - PEr > S;
    int32_t ver = PEr;  // values read: [PS, PS + ver)
    if (last_starts_here && tail_e > PEr && !has_tail) {
        const int64_t left = nval - PS;
        ver = tail_e < left ? tail_e : (int32_t)left;
    }
    const int nchunk = hi > lo ? (ver + S - 1) / S : 0;
    if (t == 0) {
        // the long rows' blocks, from their absolute bounds
        if (has_head) {
            const int64_t hs = offsets[lo], he = offsets[lo + 1];
            int64_t b1 = (he - 1) / NB;
            s_long[0] = hs / NB;
            s_long[1] = b1 < nblk - 1 ? b1 : nblk - 1;
            s_arrived[0] = atomicAdd(&ws.cnt[s_long[0]], 1u);
        }
        if (has_tail) {
            int64_t b1 = (offsets[hi] - 1) / NB;
            s_long[2] = b1 < nblk - 1 ? b1 : nblk - 1;
            s_arrived[1] = atomicAdd(&ws.cnt[B], 1u);
        }
    }
    if (hi + 1 - wb <= nwin) {  // the window holds every row's bounds
        const RowBounds rw{s_w, win_index(lo, wb), win_index(hi - 1, wb), PEr, has_head, has_tail};
        chunk_ranges<S>(rw, lo, hi, wb, nchunk, s_ra, s_rb);
    } else {
        chunk_ranges_search<true>(offsets, s_w, wb, nwin, PS, PEr, lo, hi, has_head, has_tail, S, ver, nchunk, s_ra,
                                  s_rb);
    }

    int64_t cwb = wb;  // the window: offsets[cwb .. cwb + cnwin)
    int cnwin = nwin;
    // rows [from, to) of the window finished: out of LDS into the output (the
    // long rows' parts excepted)
    const int64_t own_lo = has_head ? lo + 1 : lo, own_hi = has_tail ? hi - 1 : hi;
    auto flush = [&](int64_t from, int64_t to) {
        from = from > own_lo ? from : own_lo;
        to = to < own_hi ? to : own_hi;
        for (int64_t r = from + t; r < to; r += NT) out[r] = s_res[r - cwb];
    };
    for (int k = 0; k < nchunk; ++k) {
        const int32_t C0 = k * S;
        const int n = ver - C0 < S ? ver - C0 : S;
        const int32_t C1 = C0 + n;
        if (k > 0) {  // chunk 0 is in LDS already
            ld.store(sv, values, PS + C0, n);
            __syncthreads();
            if (k + 1 < nchunk)  // the next chunk streams in while this one is folded
                ld.issue(values, PS + C1, ver - C1 < S ? ver - C1 : S);
        }
        const Acc carry_in = uniform_val(s_carry[k & 1]);
        const int64_t ra = uniform(s_ra[k]), rb = uniform(s_rb[k]);
        for (int64_t r_lo = ra;;) {
            if (r_lo < rb && (r_lo < cwb || r_lo + 1 >= cwb + cnwin)) {
                // the rows run past the window: the finished ones leave, and
                // the window moves to r_lo
                flush(cwb, r_lo);
                const int cnt = window_count<WIN>(nseg, r_lo);
                for (int j = t; j < cnt; j += NT) s_w[j] = rel_of(offsets[r_lo + j], PS);
                cwb = r_lo;
                cnwin = cnt;
                __syncthreads();
            }
            const RowBounds rw{s_w, win_index(lo, cwb), win_index(hi - 1, cwb), PEr, has_head, has_tail};
            // a row's fold over this chunk joins what came before and goes on:
            // into the next chunk, a long row's part, or the results (rows of
            // the window leave together when it moves: no global store is
            // pending while the next chunk's loads are waited for)
            auto finish = [&](int i, int32_t sa, int32_t ea, Acc v) {
                if (sa < C0) v = R::ap(carry_in, v);
                if (ea > C1) s_carry[(k + 1) & 1] = v;
                else if (i == rw.lo_i && has_head) s_part[0] = v;
                else if (i == rw.last_i && has_tail) s_part[1] = v;
                else s_res[i] = sa == ea ? ne : R::ap(ne, v);
            };
            // rows with both bounds in the window, as window indices [i_lo, i_hi)
            const int64_t r_hi = rb < cwb + cnwin - 1 ? rb : cwb + cnwin - 1;
            const int i_lo = (int)(r_lo - cwb), i_hi = (int)(r_hi - cwb);
            if (i_hi - i_lo <= kWaveRows) {  // a wave per row
                for (int i = i_lo + w; i < i_hi; i += NW) {
                    const int32_t sa = uniform(rw.s(i)), ea = uniform(rw.e(i));
                    int s, e;
                    seg_in_chunk(sa, ea, C0, n, &s, &e);
                    const Acc a = wave_fold<R, Acc>(sv, s, e);
                    if (lane == 0) finish(i, sa, ea, a);
                }
            } else {  // many rows: a lane per short row, a wave per long one
                for (int i0 = i_lo; i0 < i_hi; i0 += NT) {
                    const int i = i0 + lane * NW + w;
                    bool lng = false;
                    if (i < i_hi) {
                        const int32_t sa = rw.s(i), ea = rw.e(i);
                        int s, e;
                        seg_in_chunk(sa, ea, C0, n, &s, &e);
                        if (e - s <= kShortSeg) finish(i, sa, ea, lane_fold<R, Acc>(sv, s, e));
                        else lng = true;
                    }
                    uint64_t m = __ballot(lng);
                    while (m) {
                        const int j = __builtin_ctzll(m);
                        m &= m - 1;
                        const int ij = i0 + j * NW + w;
                        const int32_t sa = uniform(rw.s(ij)), ea = uniform(rw.e(ij));
                        int s, e;
                        seg_in_chunk(sa, ea, C0, n, &s, &e);
                        const Acc a = wave_fold<R, Acc>(sv, s, e);
                        if (lane == 0) finish(ij, sa, ea, a);
                    }
                }
            }
            if (r_hi >= rb) break;
            r_lo = r_hi;
            __syncthreads();  // the window is read no more before it moves
        }
        __syncthreads();
    }
    if (nchunk > 0) flush(cwb, hi);

    // long rows: wave 0 publishes the head part, wave 1 the tail part; the
    // part that counted itself in last folds them all in order
    if (w < 2) {
        const bool has = w == 0 ? has_head : has_tail;
        if (has) {
            const int64_t r = w == 0 ? lo : hi - 1;
            const int64_t b0 = w == 0 ? uniform(s_long[0]) : B;
            const int64_t b1 = w == 0 ? uniform(s_long[1]) : uniform(s_long[2]);
            if (lane == 0) slot_put((w == 0 ? ws.head : ws.tail) + 2 * B, s_part[w]);
            if (s_arrived[w] == (unsigned)(b1 - b0)) {  // the last of the row's b1 - b0 + 1 parts
                Acc a = R::id();
                if (lane == 0) a = slot_get<Acc>(ws.tail + 2 * b0);
                for (int64_t b = b0 + 1; b <= b1; b += kWave) {
                    const int mm = (int)(b1 - b + 1 < kWave ? b1 - b + 1 : kWave);
                    Acc h = R::id();
                    if (lane < mm) h = slot_get<Acc>(ws.head + 2 * (b + lane));
                    for (int j = 0; j < mm; ++j) a = R::ap(a, __shfl(h, j));  // lane 0's a: parts in order
                    if (lane < mm) slot_clear<Acc>(ws.head + 2 * (b + lane));
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

// ---------------------------------------------------------------- row-span reduce
// The path for rows of ordinary length (see seg_span_path below).  A block takes
// `rb` consecutive rows, whose values form one contiguous span
// [offsets[r0], offsets[r0 + rb]).  The span's 16-byte vectors are cut into
// four contiguous quarters, one per wave; inside its quarter a wave's lanes
// interleave (coalesced), four vectors per lane in flight (16 KB per block;
// eight blocks per CU).  The offsets cost one round trip per rb rows.
//
// Row attribution: the positions a thread visits increase, so the row they
// fall in never decreases.  A thread keeps one accumulator for its current
// row; on crossing a row end it parks that value in its own LDS slot
// (row, thread) and starts afresh.  A wave finds the row of its quarter's
// first position with one ballot, so a lane crosses only the row ends inside
// its quarter.  Afterwards each row's NT slots are folded in a fixed order
// (four per lane, then the DPP wave tree), so the result depends only on the
// offsets, never on timing.
constexpr int kSpanRows = 8;  // rows per block, at most

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
    constexpr int U = 4;
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
        // Nontemporal loads: the values are read once, and not allocating
        // them in the last-level cache keeps them from evicting dirty lines
        // that earlier kernels left there (whose write-back would then share
        // HBM with this read: inside the nested step, after the 129 MB
        // broadcast of the previous step, 43.5 us with plain loads against
        // 27.2 us).
        typedef unsigned nt_u32x4 __attribute__((ext_vector_type(4)));
        static_assert(sizeof(Vec) == sizeof(nt_u32x4), "16-byte groups");
        for (int64_t i = cs + lane; i < ce; i += U * kWave) {
            Vec x[U];
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (i + u * kWave < ce)
                    x[u] = __builtin_bit_cast(Vec, __builtin_nontemporal_load(reinterpret_cast<const nt_u32x4 *>(vv + i + u * kWave)));
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

// Reverse of the row sums on the row-span path: gval[p] = gout[row of p].  A
// block loads the offsets and gradients of its rb rows once and writes its
// whole span in 16-byte stores, lanes interleaved.
__global__ void __launch_bounds__(NT) k_seg_broadcast(const float *__restrict__ gout,
                                                      const int64_t *__restrict__ offsets, int64_t nseg, int rb,
                                                      float *__restrict__ gval, int vec) {
    __shared__ int64_t soff[kSpanRows + 1];
    __shared__ float sg[kSpanRows];
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

// Reverse of the row sums over the same block ranges: gval[p] = gout[row of
// p].  Every block writes exactly its own range [PS, PE), so no row needs
// another block.  The rows of a chunk fill its LDS copy (a wave per row, in
// 16-byte writes, or, where a chunk holds many short rows, a lane per short
// row), which then leaves in 16-byte stores while the next chunk is filled.
// The fills read row bounds and gradients from an LDS window alone, as the
// reduce does.
__device__ __forceinline__ void wave_fill(float *sv, int s, int e, float g) {
    const int lane = threadIdx.x & (kWave - 1);
    if (e - s < 8) {
        if (lane < e - s) sv[s + lane] = g;
        return;
    }
    const int a = (s + 3) & ~3, b = e & ~3;  // the 16-byte aligned middle [a, b)
    if (lane < a - s) sv[s + lane] = g;
    if (lane < e - b) sv[b + lane] = g;
    float4 *v4 = reinterpret_cast<float4 *>(sv);
    const float4 gv = make_float4(g, g, g, g);
    for (int p = a / 4 + lane; p < b / 4; p += kWave) v4[p] = gv;
}

__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(8, 8)))
k_bcast_blocks(const float *__restrict__ gout, const int64_t *__restrict__ offsets, int64_t nseg, int64_t nval,
               int64_t q, int64_t nblk, float *__restrict__ gval, int vec) {
    constexpr int S = kChunkBytes / 4;
    constexpr int NW = NT / kWave;
    constexpr int WIN = 255;
    constexpr int kShortFill = 64;  // a fill is cheap per element: one lane takes segments of up to 64
    __shared__ __attribute__((aligned(16))) float sv[S];
    __shared__ int32_t s_w[WIN + 1];
    __shared__ float s_g[WIN];
    __shared__ int64_t s_ra[kMaxChunks], s_rb[kMaxChunks];
    __shared__ int64_t s_sh[3];
    __shared__ BlockRows br;
    const int t = threadIdx.x, lane = t & (kWave - 1);
    const int w = __builtin_amdgcn_readfirstlane(t / kWave);
    const int64_t B = blockIdx.x, NB = q * S;
    const int64_t PS = B * NB, PE = blk_end(B, NB, nval);
    const int32_t PEr = (int32_t)(PE - PS);
    const int nchunk = (PEr + S - 1) / S;
    if (w == 0) rows_bracket(offsets, nseg, nval, B, PS, s_sh);
    __syncthreads();
    rows_window<WIN>(offsets, nseg, PS, s_sh, s_w, gout, s_g);
    __syncthreads();
    rows_find<WIN>(nseg, B, nblk, PEr, s_w, s_sh);
    __syncthreads();
    if (w == 0) rows_finish<WIN>(offsets, nseg, B, nblk, PS, PE, s_w, s_sh, &br);
    __syncthreads();
    const int64_t lo = uniform(br.lo), hi = uniform(br.hi), wb = uniform(br.wb);
    const int nwin = uniform(br.nwin);
    if (hi + 1 - wb <= nwin) {
        const FillBounds rw{s_w, PEr};
        chunk_ranges<S>(rw, lo, hi, wb, nchunk, s_ra, s_rb);
    } else {
        chunk_ranges_search<false>(offsets, s_w, wb, nwin, PS, PEr, lo, hi, false, false, S, PEr, nchunk, s_ra,
                                   s_rb);
    }
    int64_t cwb = wb;  // the window: offsets[cwb .. cwb + cnwin), gradients of its rows
    int cnwin = nwin;
    for (int k = 0; k < nchunk; ++k) {
        const int32_t C0 = k * S;
        const int n = PEr - C0 < S ? PEr - C0 : S;
        const int64_t ra = uniform(s_ra[k]), rb = uniform(s_rb[k]);
        for (int64_t r_lo = ra;;) {
            if (r_lo < rb && (r_lo < cwb || r_lo + 1 >= cwb + cnwin)) {
                // the rows run past the window: move it to r_lo
                const int cnt = window_count<WIN>(nseg, r_lo);
                for (int j = t; j < cnt; j += NT) {
                    s_w[j] = rel_of(offsets[r_lo + j], PS);
                    if (j < cnt - 1) s_g[j] = gout[r_lo + j];
                }
                cwb = r_lo;
                cnwin = cnt;
                __syncthreads();
            }
            const FillBounds rw{s_w, PEr};
            const int64_t r_hi = rb < cwb + cnwin - 1 ? rb : cwb + cnwin - 1;
            const int i_lo = (int)(r_lo - cwb), i_hi = (int)(r_hi - cwb);
            if (i_hi - i_lo <= kWaveRows) {
                for (int i = i_lo + w; i < i_hi; i += NW) {
                    int s, e;
                    seg_in_chunk(uniform(rw.s(i)), uniform(rw.e(i)), C0, n, &s, &e);
                    wave_fill(sv, s, e, uniform_val(s_g[i]));
                }
            } else {
                for (int i0 = i_lo; i0 < i_hi; i0 += NT) {
                    const int i = i0 + lane * NW + w;
                    bool lng = false;
                    if (i < i_hi) {
                        int s, e;
                        seg_in_chunk(rw.s(i), rw.e(i), C0, n, &s, &e);
                        if (e - s <= kShortFill) {
                            const float g = s_g[i];
                            for (int p = s; p < e; ++p) sv[p] = g;
                        } else {
                            lng = true;
                        }
                    }
                    uint64_t m = __ballot(lng);
                    while (m) {
                        const int j = __builtin_ctzll(m);
                        m &= m - 1;
                        const int ij = i0 + j * NW + w;
                        int s, e;
                        seg_in_chunk(uniform(rw.s(ij)), uniform(rw.e(ij)), C0, n, &s, &e);
                        wave_fill(sv, s, e, uniform_val(s_g[ij]));
                    }
                }
            }
            if (r_hi >= rb) break;
            r_lo = r_hi;
            __syncthreads();  // the window is read no more before it moves
        }
        __syncthreads();
        // the chunk leaves; its stores drain while the next chunk is filled
        float *dst0 = gval + PS + C0;
        if (vec) {
            u32x4 *dst = reinterpret_cast<u32x4 *>(dst0);
            const u32x4 *src = reinterpret_cast<const u32x4 *>(sv);
#pragma unroll
            for (int u = 0; u < S / 4 / NT; ++u) {
                const int qv = t + NT * u;
                if (qv * 4 + 4 <= n) {
                    __builtin_nontemporal_store(src[qv], dst + qv);
                } else if (qv * 4 < n) {
                    for (int j = qv * 4; j < n; ++j) dst0[j] = sv[j];
                }
            }
        } else {
            for (int k2 = t; k2 < n; k2 += NT) dst0[k2] = sv[k2];
        }
        __syncthreads();
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
// Tiles of 1024 rows (4 per thread) up to 64 tiles (65 536 rows: 5.5 us back
// to back against 6.7-7.1 us with tiles of 4096), else tiles of 4096 (16 per
// thread), scanned in LDS (one pad slot per 16 entries).  One tile: one block.  More: a single pass with decoupled
// look-back -- blocks claim tiles in order from a counter, publish their
// tile's total, then walk back over earlier tiles' published totals until one
// carries its inclusive prefix, and publish their own.  A status word packs
// the flag (2 bits) with the value (62 bits), so one relaxed device-scope
// atomic carries both; tile i waits only on tiles claimed before it, whose
// blocks are running, so the wait always ends.  The last block to finish
// clears the status words and counters for the next call.
// rows per thread: 4 (tiles of 1024 rows) up to 64 such tiles, where the
// tiles' own loads set the pace; 16 (tiles of 4096) beyond, where the
// look-back over more tiles would (2^20 rows: 16.4 us with tiles of 1024
// against 11.5 us)
constexpr int kScanPerSmall = 4, kScanPerLarge = 16;
constexpr int64_t kScanSmallRows = 64 * NT * kScanPerSmall;
constexpr uint64_t kStatAgg = 1ull << 62, kStatPre = 2ull << 62, kStatVal = (1ull << 62) - 1;
// one pad slot per 16 entries
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
template <bool LOOKBACK, int PER>
__global__ void __launch_bounds__(NT) k_scan_tiles(const int64_t *__restrict__ len, int64_t n,
                                                   int64_t *__restrict__ off, unsigned *counters,
                                                   uint64_t *status, int ntiles) {
    __shared__ int64_t tile[(NT * PER) + (NT * PER) / 16];
    __shared__ int64_t wsum[NT / kWave];
    __shared__ int64_t sh_prefix;
    __shared__ int sh_tile, sh_last;
    if (LOOKBACK) {
        if (threadIdx.x == 0) sh_tile = (int)atomicAdd(&counters[0], 1u);
        __syncthreads();
    }
    const int t = LOOKBACK ? sh_tile : 0;
    const int64_t base = (int64_t)t * (NT * PER);
    // coalesced load into LDS
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        int64_t i = base + j * NT + threadIdx.x;
        tile[spad(j * NT + threadIdx.x)] = i < n ? len[i] : 0;
    }
    __syncthreads();
    int64_t mine[PER];
    int64_t s = 0;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        mine[j] = tile[spad(threadIdx.x * PER + j)];
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
    for (int j = 0; j < PER; ++j) {
        tile[spad(threadIdx.x * PER + j)] = run;
        run += mine[j];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        int64_t i = base + j * NT + threadIdx.x;
        if (i < n) off[i] = tile[spad(j * NT + threadIdx.x)];
    }
    if (base + (NT * PER) >= n && threadIdx.x == 0) off[n] = prefix + total;
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
// Blocks of `kernel` one CU holds at once on the current device (asked of the
// runtime once per kernel and device).
std::mutex g_occ_mu;
std::vector<std::pair<std::pair<int, const void *>, int>> g_occ;
mx_status blocks_per_cu(const void *kernel, const DeviceInfo *d, int *out) {
    std::lock_guard<std::mutex> lk(g_occ_mu);
    for (const auto &e : g_occ)
        if (e.first.first == d->device && e.first.second == kernel) {
            *out = e.second;
            return MX_OK;
        }
    int n = 0;
    MX_TRY_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kernel, NT, 0));
    n = n < 1 ? 1 : n;
    g_occ.push_back({{d->device, kernel}, n});
    *out = n;
    return MX_OK;
}

// Chunks per block and blocks: as many blocks as the device holds at once,
// each streaming q consecutive chunks (q < kMaxChunks: beyond that, more
// blocks than the device holds at once).
mx_status stream_grid(const void *kernel, int64_t nch, const DeviceInfo *d, int64_t *q, int64_t *nblk) {
    int bpc = 1;
    if (mx_status st = blocks_per_cu(kernel, d, &bpc)) return st;
    const int64_t slots = (int64_t)d->num_cus * bpc;
    *q = nch <= slots ? 1 : (nch + slots - 1) / slots;
    *q = *q < kMaxChunks - 1 ? *q : kMaxChunks - 1;
    *nblk = (nch + *q - 1) / *q;
    return MX_OK;
}

// Which kernels take a ragged reduce or broadcast.  The row-span kernels need
// no search and fold in registers; they are the faster ones (measured on
// 65 536 rows of log-uniform length, mean 490: 25 us against 35 us for the
// reduce) while there are enough row groups to fill the device and a block's
// span stays short.  Rows longer on average, or too few of them, go to the
// chunked kernels, which split the values evenly whatever the row lengths.
constexpr int64_t kSpanAvgMax = 16384;  // average row length, at most
bool seg_span_path(int64_t nseg, int64_t nval, const DeviceInfo *d) {
    return nseg >= (int64_t)d->num_cus * 32 && nval <= nseg * kSpanAvgMax;
}
// rows per block of the row-span kernels: 32 blocks per CU, at most kSpanRows rows each
int span_rows(int64_t nseg, const DeviceInfo *d) {
    const int64_t rb = ceil_div(nseg, (int64_t)d->num_cus * 32);
    return (int)(rb < 1 ? 1 : rb > kSpanRows ? kSpanRows : rb);
}

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
        const DeviceInfo *d;
        if (mx_status st = device_info(&d)) return st;
        const bool vec = aligned16(values);
        if (seg_span_path(nseg, nval, d)) {
            const int rb = span_rows(nseg, d);
            const int64_t grid = ceil_div(nseg, rb);
            MX_REQUIRE(grid <= 0x7fffffff, MX_ERR_SHAPE, "mx_segmented_reduce: too many rows");
            hipLaunchKernelGGL((k_seg_span<D, OP>), dim3((unsigned)grid), dim3(NT), span_lds_bytes<D>(rb), s,
                               (const In *)values, off, nseg, rb, ne, (Acc *)out, (int)vec);
            return last_launch("mx_segmented_reduce");
        }
        const void *kern = vec ? reinterpret_cast<const void *>(&k_seg_blocks<D, OP, true>)
                               : reinterpret_cast<const void *>(&k_seg_blocks<D, OP, false>);
        int64_t q, nblk;
        if (mx_status st = stream_grid(kern, nch, d, &q, &nblk)) return st;
        if (vec)
            hipLaunchKernelGGL((k_seg_blocks<D, OP, true>), dim3((unsigned)nblk), dim3(NT), 0, s, (const In *)values,
                               off, nseg, nval, q, nblk, ne, (Acc *)out, w);
        else
            hipLaunchKernelGGL((k_seg_blocks<D, OP, false>), dim3((unsigned)nblk), dim3(NT), 0, s, (const In *)values,
                               off, nseg, nval, q, nblk, ne, (Acc *)out, w);
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
    const DeviceInfo *d;
    if (mx_status st = device_info(&d)) return st;
    if (seg_span_path(nseg, nval, d)) {
        const int rb = span_rows(nseg, d);
        const int64_t grid = ceil_div(nseg, rb);
        MX_REQUIRE(grid <= 0x7fffffff, MX_ERR_SHAPE, "mx_segmented_sum_adjoint_f32: too many rows");
        hipLaunchKernelGGL(k_seg_broadcast, dim3((unsigned)grid), dim3(NT), 0, s, gout, off, nseg, rb, gval,
                           (int)aligned16(gval));
        return last_launch("mx_segmented_sum_adjoint_f32");
    }
    int64_t q, nblk;
    if (mx_status st = stream_grid(reinterpret_cast<const void *>(&k_bcast_blocks), nch, d, &q, &nblk)) return st;
    hipLaunchKernelGGL(k_bcast_blocks, dim3((unsigned)nblk), dim3(NT), 0, s, gout, off, nseg, nval, q, nblk,
                       gval, (int)aligned16(gval));
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
    const bool small = nseg <= kScanSmallRows;
    const int64_t ntiles = ceil_div(nseg, (int64_t)NT * (small ? kScanPerSmall : kScanPerLarge));
    MX_REQUIRE(ntiles <= 0x7fffffff, MX_ERR_SHAPE, "mx_lengths_to_offsets: too many rows");
    if (ntiles <= 1) {
        hipLaunchKernelGGL((k_scan_tiles<false, kScanPerSmall>), dim3(1), dim3(NT), 0, s, len, nseg, off,
                           (unsigned *)nullptr, (uint64_t *)nullptr, 1);
        return last_launch("mx_lengths_to_offsets");
    }
    size_t need = mx_workspace_bytes(MX_WS_SCAN, nseg, 0);
    MX_REQUIRE(ws && ws_bytes >= need, MX_ERR_WORKSPACE, "mx_lengths_to_offsets: workspace needs %zu bytes", need);
    MX_REQUIRE(((uintptr_t)ws & 255) == 0, MX_ERR_INVALID, "mx_lengths_to_offsets: workspace must be 256-byte aligned");
    unsigned *counters = (unsigned *)ws;
    uint64_t *status = (uint64_t *)((char *)ws + kCounterBytes);
    if (small)
        hipLaunchKernelGGL((k_scan_tiles<true, kScanPerSmall>), dim3((unsigned)ntiles), dim3(NT), 0, s, len, nseg, off,
                           counters, status, (int)ntiles);
    else
        hipLaunchKernelGGL((k_scan_tiles<true, kScanPerLarge>), dim3((unsigned)ntiles), dim3(NT), 0, s, len, nseg, off,
                           counters, status, (int)ntiles);
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
