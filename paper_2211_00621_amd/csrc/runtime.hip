// Runtime: error text, per-device property cache, debug flag, workspace
// sizing and the plain streaming copy kernel.
#include <algorithm>
#include <atomic>
#include <cstdarg>
#include <cstdio>
#include <mutex>

#include "mx_internal.h"

namespace mx {

namespace {
thread_local char g_err[512] = "";
std::atomic<int> g_debug{0};
std::mutex g_dev_mu;
DeviceInfo g_devs[64];
bool g_dev_ok[64] = {};
}  // namespace

mx_status set_error(mx_status s, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return s;
}

mx_status hip_error(hipError_t e, const char *what) {
    return set_error(MX_ERR_HIP, "%s failed: %s", what, hipGetErrorString(e));
}

mx_status last_launch(const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_error(e, what);
    return MX_OK;
}

mx_status device_info(const DeviceInfo **out) {
    int dev = 0;
    MX_TRY_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return set_error(MX_ERR_INVALID, "device ordinal %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_dev_mu);
    if (!g_dev_ok[dev]) {
        hipDeviceProp_t p;
        MX_TRY_HIP(hipGetDeviceProperties(&p, dev));
        DeviceInfo &d = g_devs[dev];
        d.device = dev;
        d.num_cus = p.multiProcessorCount > 0 ? p.multiProcessorCount : 256;
        d.lds_bytes = (int)p.sharedMemPerBlock;
        d.warp = p.warpSize;
        g_dev_ok[dev] = true;
    }
    *out = &g_devs[dev];
    return MX_OK;
}

bool debug_mode() { return g_debug.load(std::memory_order_relaxed) != 0; }

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Streaming copy: grid-stride over 16-byte vectors, two in flight per thread.
__global__ void __launch_bounds__(256) k_copy32(const uint32_t *__restrict__ src,
                                                uint32_t *__restrict__ dst, int64_t n) {
    const int64_t nv = n / 4;
    const u32x4 *s4 = reinterpret_cast<const u32x4 *>(src);
    u32x4 *d4 = reinterpret_cast<u32x4 *>(dst);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + stride < nv; i += 2 * stride) {
        u32x4 a = __builtin_nontemporal_load(s4 + i);
        u32x4 b = __builtin_nontemporal_load(s4 + i + stride);
        __builtin_nontemporal_store(a, d4 + i);
        __builtin_nontemporal_store(b, d4 + i + stride);
    }
    for (; i < nv; i += stride) d4[i] = s4[i];
    if (blockIdx.x == 0 && threadIdx.x < (n & 3)) dst[nv * 4 + threadIdx.x] = src[nv * 4 + threadIdx.x];
}

// Read-only stream: block b reads the contiguous 16 KB chunk b (1024 16-byte
// vectors, four per thread, all in flight together) and folds it by XOR.
constexpr int kReadChunkVec = 1024;
constexpr int kReadSlots = MX_STREAM_READ_SLOTS;
__global__ void __launch_bounds__(256) k_stream_read(const u32x4 *__restrict__ src, int64_t nv,
                                                     const uint32_t *__restrict__ tail, int ntail,
                                                     uint32_t *xor_out) {
    __shared__ uint32_t red[4];
    const int64_t nchunks = (nv + kReadChunkVec - 1) / kReadChunkVec;
    uint32_t a = 0;
    for (int64_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
        const int64_t base = c * kReadChunkVec;
        u32x4 x[kReadChunkVec / 256];
#pragma unroll
        for (int u = 0; u < kReadChunkVec / 256; ++u) {
            const int64_t i = base + threadIdx.x + 256 * u;
            x[u] = i < nv ? __builtin_nontemporal_load(src + i) : u32x4{0, 0, 0, 0};
        }
#pragma unroll
        for (int u = 0; u < kReadChunkVec / 256; ++u) a ^= x[u].x ^ x[u].y ^ x[u].z ^ x[u].w;
    }
    if (blockIdx.x == 0 && (int)threadIdx.x < ntail) a ^= tail[threadIdx.x];
    for (int d = 32; d > 0; d >>= 1) a ^= __shfl_xor(a, d);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x / 64] = a;
    __syncthreads();
    // one word per block: atomics into shared words measured the pass 20 %
    // slower than plain stores
    if (threadIdx.x == 0) xor_out[blockIdx.x] = red[0] ^ red[1] ^ red[2] ^ red[3];
}

}  // namespace mx

using namespace mx;

extern "C" {

mx_status mx_init(int device) {
    MX_TRY_HIP(hipSetDevice(device));
    const DeviceInfo *d;
    if (mx_status st = device_info(&d)) return st;
    void *scr = nullptr;
    return segmented_scratch(&scr);  // the no-allocation entry point's array on this device
}

const char *mx_last_error(void) { return g_err; }

const char *mx_version(void) { return "mx 0.1.0 gfx950"; }

mx_status mx_set_debug(int on) {
    g_debug.store(on ? 1 : 0);
    return MX_OK;
}

int mx_get_debug(void) { return g_debug.load(); }

size_t mx_workspace_bytes(mx_ws_kind kind, int64_t n, int64_t aux) {
    if (n < 0) n = 0;
    switch (kind) {
    case MX_WS_REDUCE:
        // counters + one 8-byte partial per block (at most 4096 blocks)
        return kCounterBytes + align256(8 * 4096);
    case MX_WS_SCAN: {
        // counters + one int64 per scan tile of 1024 rows (+1)
        int64_t tiles = (n + 1023) / 1024 + 1;
        return kCounterBytes + align256((size_t)tiles * 8);
    }
    case MX_WS_HISTOGRAM: return histogram_ws_bytes(n, aux);
    case MX_WS_SEGMENTED: return segmented_ws_bytes(n);
    }
    return 0;
}

struct mx_graph {
    hipGraph_t graph;
    hipGraphExec_t exec;
};

mx_status mx_graph_begin(hipStream_t stream) {
    MX_REQUIRE(stream != nullptr, MX_ERR_INVALID, "mx_graph_begin: the null stream cannot be captured");
    MX_REQUIRE(!debug_mode(), MX_ERR_INVALID, "mx_graph_begin: debug mode synchronises and cannot be captured");
    MX_TRY_HIP(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
    return MX_OK;
}

mx_status mx_graph_end(hipStream_t stream, mx_graph **graph) {
    MX_REQUIRE(graph, MX_ERR_INVALID, "mx_graph_end: null output");
    *graph = nullptr;
    hipGraph_t g = nullptr;
    MX_TRY_HIP(hipStreamEndCapture(stream, &g));
    hipGraphExec_t e = nullptr;
    hipError_t err = hipGraphInstantiate(&e, g, nullptr, nullptr, 0);
    if (err != hipSuccess) {
        (void)hipGraphDestroy(g);
        return hip_error(err, "hipGraphInstantiate");
    }
    *graph = new mx_graph{g, e};
    return MX_OK;
}

mx_status mx_graph_launch(mx_graph *graph, hipStream_t stream) {
    MX_REQUIRE(graph, MX_ERR_INVALID, "mx_graph_launch: null graph");
    MX_TRY_HIP(hipGraphLaunch(graph->exec, stream));
    return MX_OK;
}

mx_status mx_graph_destroy(mx_graph *graph) {
    if (!graph) return MX_OK;
    hipError_t e1 = hipGraphExecDestroy(graph->exec);
    hipError_t e2 = hipGraphDestroy(graph->graph);
    delete graph;
    if (e1 != hipSuccess) return hip_error(e1, "hipGraphExecDestroy");
    if (e2 != hipSuccess) return hip_error(e2, "hipGraphDestroy");
    return MX_OK;
}

mx_status mx_copy32(const void *src_dev, void *dst_dev, int64_t n, hipStream_t stream) {
    MX_REQUIRE(n >= 0, MX_ERR_SHAPE, "mx_copy32: n < 0");
    if (n == 0) return MX_OK;
    MX_REQUIRE(src_dev && dst_dev, MX_ERR_INVALID, "mx_copy32: null pointer");
    MX_REQUIRE(((uintptr_t)src_dev % 16) == 0 && ((uintptr_t)dst_dev % 16) == 0, MX_ERR_INVALID,
               "mx_copy32: pointers must be 16-byte aligned");
    const DeviceInfo *d;
    mx_status st = device_info(&d);
    if (st) return st;
    int64_t nv = n / 4;
    int64_t blocks = ceil_div(nv > 0 ? nv : 1, 256 * 2);
    int64_t cap = (int64_t)d->num_cus * 8;
    if (blocks > cap) blocks = cap;
    hipLaunchKernelGGL(k_copy32, dim3((unsigned)blocks), dim3(256), 0, stream,
                       (const uint32_t *)src_dev, (uint32_t *)dst_dev, n);
    return last_launch("mx_copy32");
}

mx_status mx_stream_read(const void *src_dev, int64_t n, uint32_t *xor_dev, hipStream_t stream) {
    MX_REQUIRE(n >= 0, MX_ERR_SHAPE, "mx_stream_read: n < 0");
    if (n == 0) return MX_OK;
    MX_REQUIRE(src_dev && xor_dev, MX_ERR_INVALID, "mx_stream_read: null pointer");
    MX_REQUIRE(((uintptr_t)src_dev % 16) == 0, MX_ERR_INVALID, "mx_stream_read: src must be 16-byte aligned");
    const int64_t nv = n / 4;
    const int64_t blocks = std::min<int64_t>(kReadSlots, std::max<int64_t>(1, ceil_div(nv, kReadChunkVec)));
    hipLaunchKernelGGL(k_stream_read, dim3((unsigned)blocks), dim3(256), 0, stream, (const u32x4 *)src_dev, nv,
                       (const uint32_t *)src_dev + nv * 4, (int)(n & 3), xor_dev);
    return last_launch("mx_stream_read");
}

}  // extern "C"
