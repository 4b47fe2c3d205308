// Marshaling (Section 4.3): the host language's boxed nested sequences and
// records <-> the flat device layout (values + offsets, one array per field).
//
// Ragged rows: host threads gather the rows, in order, into the caller's
// pinned staging buffer (followed by the lengths), one host-to-device copy moves
// both, and the offsets are computed on the device by the lengths scan.
// Records: an interleaved array of records is split into one array per field
// on the device (and joined back), 16-byte vectors per thread where possible.
#include <algorithm>
#include <thread>
#include <vector>

#include <climits>
#include <mutex>

#include "mx_internal.h"

namespace mx {
namespace {

constexpr int NT = 256;
constexpr int kMaxFields = 16;

struct FieldPtrs {
    void *p[kMaxFields];
};

template <class T>
__global__ void __launch_bounds__(NT) k_aos_to_soa(const T *__restrict__ aos, int64_t n, int f,
                                                   FieldPtrs soa) {
    const int64_t stride = (int64_t)gridDim.x * NT;
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += stride) {
        const T *rec = aos + i * f;
        for (int j = 0; j < f; ++j) reinterpret_cast<T *>(soa.p[j])[i] = rec[j];
    }
}

// Four fields of 4 bytes: one 16-byte load per record.
__global__ void __launch_bounds__(NT) k_aos4_to_soa(const float4 *__restrict__ aos, int64_t n,
                                                    FieldPtrs soa) {
    const int64_t stride = (int64_t)gridDim.x * NT;
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += stride) {
        float4 r = aos[i];
        reinterpret_cast<float *>(soa.p[0])[i] = r.x;
        reinterpret_cast<float *>(soa.p[1])[i] = r.y;
        reinterpret_cast<float *>(soa.p[2])[i] = r.z;
        reinterpret_cast<float *>(soa.p[3])[i] = r.w;
    }
}

template <class T>
__global__ void __launch_bounds__(NT) k_soa_to_aos(FieldPtrs soa, int64_t n, int f, T *__restrict__ aos) {
    const int64_t stride = (int64_t)gridDim.x * NT;
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += stride) {
        T *rec = aos + i * f;
        for (int j = 0; j < f; ++j) rec[j] = reinterpret_cast<const T *>(soa.p[j])[i];
    }
}

__global__ void __launch_bounds__(NT) k_soa_to_aos4(FieldPtrs soa, int64_t n, float4 *__restrict__ aos) {
    const int64_t stride = (int64_t)gridDim.x * NT;
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += stride)
        aos[i] = make_float4(reinterpret_cast<const float *>(soa.p[0])[i], reinterpret_cast<const float *>(soa.p[1])[i],
                             reinterpret_cast<const float *>(soa.p[2])[i], reinterpret_cast<const float *>(soa.p[3])[i]);
}

// smallest and largest row length of an offsets array (integer atomics: the
// result does not depend on the order)
__global__ void __launch_bounds__(NT) k_row_len_range(const int64_t *__restrict__ off, int64_t nseg,
                                                      long long *__restrict__ mm) {
    long long lo = LLONG_MAX, hi = LLONG_MIN;
    const int64_t stride = (int64_t)gridDim.x * NT;
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < nseg; i += stride) {
        const long long len = (long long)(off[i + 1] - off[i]);
        lo = len < lo ? len : lo;
        hi = len > hi ? len : hi;
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        const long long a = __shfl_xor(lo, o, kWave), b = __shfl_xor(hi, o, kWave);
        lo = a < lo ? a : lo;
        hi = b > hi ? b : hi;
    }
    if ((threadIdx.x & (kWave - 1)) == 0) {
        atomicMin(&mm[0], lo);
        atomicMax(&mm[1], hi);
    }
}

__global__ void k_range_init(long long *mm) {
    mm[0] = LLONG_MAX;
    mm[1] = LLONG_MIN;
}

// one two-word device buffer per device for the range, kept for the process
long long *g_range[64] = {};
std::mutex g_range_mu;

int grid_for(int64_t n, const DeviceInfo *d) {
    int64_t g = ceil_div(n > 0 ? n : 1, NT);
    int64_t cap = (int64_t)d->num_cus * 8;
    return (int)(g < cap ? g : cap);
}

// Copies rows into a contiguous host buffer with up to 16 threads, each
// taking a contiguous range of rows of about equal byte count.
void gather_rows(const void *const *rows, const int64_t *lengths, const int64_t *starts, int64_t nseg,
                 size_t eb, char *dst, int64_t total) {
    unsigned hw = std::thread::hardware_concurrency();
    int nth = (int)std::min<int64_t>(std::max(1u, std::min(hw, 16u)), std::max<int64_t>(1, total * (int64_t)eb / (4 << 20)));
    auto work = [&](int64_t r0, int64_t r1) {
        for (int64_t r = r0; r < r1; ++r)
            if (lengths[r] > 0) std::memcpy(dst + starts[r] * eb, rows[r], (size_t)lengths[r] * eb);
    };
    if (nth <= 1) {
        work(0, nseg);
        return;
    }
    std::vector<std::thread> th;
    int64_t r = 0;
    for (int t = 0; t < nth && r < nseg; ++t) {
        const int64_t goal = total * (t + 1) / nth;
        int64_t r1 = r;
        while (r1 < nseg && starts[r1] < goal) ++r1;
        if (t == nth - 1) r1 = nseg;
        th.emplace_back(work, r, r1);
        r = r1;
    }
    for (auto &x : th) x.join();
}

// Field-wise layout of records whose fields are scalars or sequences: where
// each field's values (and a sequence field's lengths / offsets) sit in the
// staging buffer.
struct FieldPlan {
    int64_t count = 0;   // values of the field
    size_t vpos = 0, vbytes = 0, lpos = 0;
};

mx_hseq seq_at(const void *recs, size_t rec_bytes, int64_t r, int64_t offset) {
    mx_hseq h;
    std::memcpy(&h, (const char *)recs + (size_t)r * rec_bytes + (size_t)offset, sizeof h);
    return h;
}

mx_status plan_records(const char *who, const void *recs, int64_t nrec, size_t rec_bytes, const mx_field *fields,
                       int nf, std::vector<FieldPlan> &plan, size_t *staging) {
    MX_REQUIRE(nrec >= 0, MX_ERR_SHAPE, "%s: nrec < 0", who);
    MX_REQUIRE(fields && nf >= 1 && nf <= kMaxFields, MX_ERR_INVALID, "%s: 1..%d fields", who, kMaxFields);
    MX_REQUIRE(nrec == 0 || (recs && rec_bytes > 0), MX_ERR_INVALID, "%s: null records", who);
    plan.assign((size_t)nf, FieldPlan{});
    size_t pos = 0;
    for (int f = 0; f < nf; ++f) {
        const mx_field &fd = fields[f];
        const int eb = fd.elem_bytes;
        MX_REQUIRE(fd.kind == MX_FIELD_SCALAR || fd.kind == MX_FIELD_SEQ, MX_ERR_INVALID, "%s: field %d: bad kind", who, f);
        MX_REQUIRE(eb == 1 || eb == 2 || eb == 4 || eb == 8, MX_ERR_INVALID, "%s: field %d: elem_bytes 1, 2, 4 or 8",
                   who, f);
        const size_t width = fd.kind == MX_FIELD_SCALAR ? (size_t)eb : sizeof(mx_hseq);
        MX_REQUIRE(fd.offset >= 0 && (size_t)fd.offset + width <= rec_bytes, MX_ERR_INVALID,
                   "%s: field %d lies outside the record", who, f);
        FieldPlan &p = plan[(size_t)f];
        if (fd.kind == MX_FIELD_SCALAR) {
            p.count = nrec;
        } else {
            for (int64_t r = 0; r < nrec; ++r) {
                const mx_hseq h = seq_at(recs, rec_bytes, r, fd.offset);
                MX_REQUIRE(h.len >= 0, MX_ERR_SHAPE, "%s: field %d, record %lld: negative length", who, f, (long long)r);
                MX_REQUIRE(h.len == 0 || h.data, MX_ERR_INVALID, "%s: field %d, record %lld: null data", who, f,
                           (long long)r);
                p.count += h.len;
            }
        }
        p.vpos = pos;
        p.vbytes = (size_t)p.count * (size_t)eb;
        pos += align256(p.vbytes);
        if (fd.kind == MX_FIELD_SEQ) {
            p.lpos = pos;
            pos += align256((size_t)(nrec + 1) * 8);
        }
    }
    *staging = pos;
    return MX_OK;
}

// Runs fn(r0, r1) over record ranges on up to 16 host threads (one when the
// work is small).
template <class Fn> void parallel_records(int64_t nrec, int64_t bytes, Fn fn) {
    unsigned hw = std::thread::hardware_concurrency();
    int nth = (int)std::min<int64_t>(std::max(1u, std::min(hw, 16u)), std::max<int64_t>(1, bytes / (4 << 20)));
    if (nth <= 1 || nrec < 2) {
        fn((int64_t)0, nrec);
        return;
    }
    std::vector<std::thread> th;
    for (int t = 0; t < nth; ++t) {
        const int64_t r0 = nrec * t / nth, r1 = nrec * (t + 1) / nth;
        if (r1 > r0) th.emplace_back(fn, r0, r1);
    }
    for (auto &x : th) x.join();
}

}  // namespace
}  // namespace mx

using namespace mx;

extern "C" {

mx_status mx_marshal_rows(const void *const *rows_host, const int64_t *lengths_host, int64_t nseg,
                          size_t elem_bytes, void *staging_host, size_t staging_bytes,
                          void *values_dev, int64_t *lengths_dev, int64_t *offsets_dev, void *ws,
                          size_t ws_bytes, hipStream_t stream) {
    MX_REQUIRE(nseg >= 0, MX_ERR_SHAPE, "mx_marshal_rows: nseg < 0");
    MX_REQUIRE(elem_bytes == 1 || elem_bytes == 2 || elem_bytes == 4 || elem_bytes == 8, MX_ERR_INVALID,
               "mx_marshal_rows: elem_bytes must be 1, 2, 4 or 8");
    MX_REQUIRE(offsets_dev, MX_ERR_INVALID, "mx_marshal_rows: null offsets");
    MX_REQUIRE(nseg == 0 || (rows_host && lengths_host && lengths_dev && staging_host), MX_ERR_INVALID,
               "mx_marshal_rows: null pointer");
    std::vector<int64_t> starts((size_t)nseg + 1, 0);
    for (int64_t r = 0; r < nseg; ++r) {
        MX_REQUIRE(lengths_host[r] >= 0, MX_ERR_SHAPE, "mx_marshal_rows: negative length at row %lld", (long long)r);
        MX_REQUIRE(lengths_host[r] == 0 || rows_host[r], MX_ERR_INVALID, "mx_marshal_rows: null row %lld", (long long)r);
        starts[r + 1] = starts[r] + lengths_host[r];
    }
    const int64_t total = starts[nseg];
    const size_t vbytes = (size_t)total * elem_bytes;
    const size_t lpos = align256(vbytes);
    const size_t need = lpos + (size_t)nseg * 8;
    MX_REQUIRE(staging_bytes >= need, MX_ERR_INVALID, "mx_marshal_rows: staging needs %zu bytes", need);
    MX_REQUIRE(total == 0 || values_dev, MX_ERR_INVALID, "mx_marshal_rows: null values");
    if (nseg > 0) {
        // the previous use of the staging buffer on this stream must be finished
        MX_TRY_HIP(hipStreamSynchronize(stream));
        char *st = (char *)staging_host;
        gather_rows(rows_host, lengths_host, starts.data(), nseg, elem_bytes, st, total);
        std::memcpy(st + lpos, lengths_host, (size_t)nseg * 8);
        if (vbytes) MX_TRY_HIP(hipMemcpyAsync(values_dev, st, vbytes, hipMemcpyHostToDevice, stream));
        MX_TRY_HIP(hipMemcpyAsync(lengths_dev, st + lpos, (size_t)nseg * 8, hipMemcpyHostToDevice, stream));
    }
    return lengths_to_offsets(lengths_dev, nseg, offsets_dev, ws, ws_bytes, stream);
}

mx_status mx_unmarshal_rows(const void *values_dev, const int64_t *offsets_host, int64_t nseg,
                            size_t elem_bytes, void *staging_host, size_t staging_bytes,
                            void *const *rows_host, hipStream_t stream) {
    MX_REQUIRE(nseg >= 0, MX_ERR_SHAPE, "mx_unmarshal_rows: nseg < 0");
    MX_REQUIRE(elem_bytes == 1 || elem_bytes == 2 || elem_bytes == 4 || elem_bytes == 8, MX_ERR_INVALID,
               "mx_unmarshal_rows: elem_bytes must be 1, 2, 4 or 8");
    if (nseg == 0) return MX_OK;
    MX_REQUIRE(offsets_host && rows_host && staging_host, MX_ERR_INVALID, "mx_unmarshal_rows: null pointer");
    MX_REQUIRE(offsets_host[0] == 0, MX_ERR_SHAPE, "mx_unmarshal_rows: offsets[0] != 0");
    for (int64_t r = 0; r < nseg; ++r)
        MX_REQUIRE(offsets_host[r + 1] >= offsets_host[r], MX_ERR_SHAPE, "mx_unmarshal_rows: offsets decrease at %lld",
                   (long long)r);
    const int64_t total = offsets_host[nseg];
    const size_t vbytes = (size_t)total * elem_bytes;
    MX_REQUIRE(staging_bytes >= vbytes, MX_ERR_INVALID, "mx_unmarshal_rows: staging needs %zu bytes", vbytes);
    MX_REQUIRE(total == 0 || values_dev, MX_ERR_INVALID, "mx_unmarshal_rows: null values");
    if (vbytes) MX_TRY_HIP(hipMemcpyAsync(staging_host, values_dev, vbytes, hipMemcpyDeviceToHost, stream));
    MX_TRY_HIP(hipStreamSynchronize(stream));
    const char *st = (const char *)staging_host;
    for (int64_t r = 0; r < nseg; ++r) {
        const int64_t len = offsets_host[r + 1] - offsets_host[r];
        if (len > 0) {
            MX_REQUIRE(rows_host[r], MX_ERR_INVALID, "mx_unmarshal_rows: null row %lld", (long long)r);
            std::memcpy(rows_host[r], st + offsets_host[r] * elem_bytes, (size_t)len * elem_bytes);
        }
    }
    return MX_OK;
}

mx_status mx_records_to_fields(const void *aos_dev, int64_t n, int nfields, size_t field_bytes,
                               void *const *soa_fields_host, hipStream_t stream) {
    MX_REQUIRE(n >= 0, MX_ERR_SHAPE, "mx_records_to_fields: n < 0");
    MX_REQUIRE(nfields >= 1 && nfields <= kMaxFields, MX_ERR_INVALID, "mx_records_to_fields: 1..16 fields");
    MX_REQUIRE(field_bytes == 4 || field_bytes == 8, MX_ERR_INVALID, "mx_records_to_fields: fields of 4 or 8 bytes");
    if (n == 0) return MX_OK;
    MX_REQUIRE(aos_dev && soa_fields_host, MX_ERR_INVALID, "mx_records_to_fields: null pointer");
    FieldPtrs fp{};
    for (int j = 0; j < nfields; ++j) {
        MX_REQUIRE(soa_fields_host[j], MX_ERR_INVALID, "mx_records_to_fields: null field %d", j);
        fp.p[j] = soa_fields_host[j];
    }
    const DeviceInfo *d;
    if (mx_status st = device_info(&d)) return st;
    const int grid = grid_for(n, d);
    if (nfields == 4 && field_bytes == 4 && ((uintptr_t)aos_dev % 16) == 0)
        hipLaunchKernelGGL(k_aos4_to_soa, dim3(grid), dim3(NT), 0, stream, (const float4 *)aos_dev, n, fp);
    else if (field_bytes == 4)
        hipLaunchKernelGGL(k_aos_to_soa<uint32_t>, dim3(grid), dim3(NT), 0, stream, (const uint32_t *)aos_dev, n,
                           nfields, fp);
    else
        hipLaunchKernelGGL(k_aos_to_soa<uint64_t>, dim3(grid), dim3(NT), 0, stream, (const uint64_t *)aos_dev, n,
                           nfields, fp);
    return last_launch("mx_records_to_fields");
}

mx_status mx_offsets_regular(const int64_t *offsets_dev, int64_t nseg, int64_t *row_len_host, hipStream_t stream) {
    const char *who = "mx_offsets_regular";
    MX_REQUIRE(nseg >= 0, MX_ERR_SHAPE, "%s: nseg < 0", who);
    MX_REQUIRE(row_len_host, MX_ERR_INVALID, "%s: null output", who);
    *row_len_host = 0;
    if (nseg == 0) return MX_OK;
    MX_REQUIRE(offsets_dev, MX_ERR_INVALID, "%s: null offsets", who);
    const DeviceInfo *d;
    if (mx_status st = device_info(&d)) return st;
    long long *mm;
    {
        std::lock_guard<std::mutex> lk(g_range_mu);
        if (!g_range[d->device]) MX_TRY_HIP(hipMalloc(&g_range[d->device], 2 * sizeof(long long)));
        mm = g_range[d->device];
    }
    hipLaunchKernelGGL(k_range_init, dim3(1), dim3(1), 0, stream, mm);
    if (mx_status st = last_launch(who)) return st;
    hipLaunchKernelGGL(k_row_len_range, dim3(grid_for(nseg, d)), dim3(NT), 0, stream, offsets_dev, nseg, mm);
    if (mx_status st = last_launch(who)) return st;
    long long h[2];
    MX_TRY_HIP(hipMemcpyAsync(h, mm, sizeof h, hipMemcpyDeviceToHost, stream));
    MX_TRY_HIP(hipStreamSynchronize(stream));
    MX_REQUIRE(h[0] >= 0, MX_ERR_SHAPE, "%s: offsets decrease (a row of length %lld)", who, h[0]);
    MX_REQUIRE(h[0] == h[1], MX_ERR_SHAPE, "%s: irregular rows (lengths %lld .. %lld)", who, h[0], h[1]);
    *row_len_host = h[0];
    return MX_OK;
}

mx_status mx_fields_to_records(const void *const *soa_fields_host, int64_t n, int nfields,
                               size_t field_bytes, void *aos_dev, hipStream_t stream) {
    MX_REQUIRE(n >= 0, MX_ERR_SHAPE, "mx_fields_to_records: n < 0");
    MX_REQUIRE(nfields >= 1 && nfields <= kMaxFields, MX_ERR_INVALID, "mx_fields_to_records: 1..16 fields");
    MX_REQUIRE(field_bytes == 4 || field_bytes == 8, MX_ERR_INVALID, "mx_fields_to_records: fields of 4 or 8 bytes");
    if (n == 0) return MX_OK;
    MX_REQUIRE(aos_dev && soa_fields_host, MX_ERR_INVALID, "mx_fields_to_records: null pointer");
    FieldPtrs fp{};
    for (int j = 0; j < nfields; ++j) {
        MX_REQUIRE(soa_fields_host[j], MX_ERR_INVALID, "mx_fields_to_records: null field %d", j);
        fp.p[j] = const_cast<void *>(soa_fields_host[j]);
    }
    const DeviceInfo *d;
    if (mx_status st = device_info(&d)) return st;
    const int grid = grid_for(n, d);
    if (nfields == 4 && field_bytes == 4 && ((uintptr_t)aos_dev % 16) == 0)
        hipLaunchKernelGGL(k_soa_to_aos4, dim3(grid), dim3(NT), 0, stream, fp, n, (float4 *)aos_dev);
    else if (field_bytes == 4)
        hipLaunchKernelGGL(k_soa_to_aos<uint32_t>, dim3(grid), dim3(NT), 0, stream, fp, n, nfields,
                           (uint32_t *)aos_dev);
    else
        hipLaunchKernelGGL(k_soa_to_aos<uint64_t>, dim3(grid), dim3(NT), 0, stream, fp, n, nfields,
                           (uint64_t *)aos_dev);
    return last_launch("mx_fields_to_records");
}


mx_status mx_records_layout(const void *recs_host, int64_t nrec, size_t rec_bytes, const mx_field *fields,
                            int nfields, int64_t *counts_host, size_t *staging_bytes_host) {
    std::vector<FieldPlan> plan;
    size_t staging = 0;
    if (mx_status st = plan_records("mx_records_layout", recs_host, nrec, rec_bytes, fields, nfields, plan, &staging))
        return st;
    if (counts_host)
        for (int f = 0; f < nfields; ++f) counts_host[f] = plan[(size_t)f].count;
    if (staging_bytes_host) *staging_bytes_host = staging;
    return MX_OK;
}

mx_status mx_marshal_records(const void *recs_host, int64_t nrec, size_t rec_bytes, const mx_field *fields,
                             int nfields, void *staging_host, size_t staging_bytes, void *ws, size_t ws_bytes,
                             hipStream_t stream) {
    const char *who = "mx_marshal_records";
    std::vector<FieldPlan> plan;
    size_t need = 0;
    if (mx_status st = plan_records(who, recs_host, nrec, rec_bytes, fields, nfields, plan, &need)) return st;
    MX_REQUIRE(staging_host || need == 0, MX_ERR_INVALID, "%s: null staging", who);
    MX_REQUIRE(staging_bytes >= need, MX_ERR_INVALID, "%s: staging needs %zu bytes", who, need);
    for (int f = 0; f < nfields; ++f) {
        const mx_field &fd = fields[f];
        MX_REQUIRE(plan[(size_t)f].count == 0 || fd.values_dev, MX_ERR_INVALID, "%s: field %d: null values", who, f);
        if (fd.kind == MX_FIELD_SEQ)
            MX_REQUIRE(fd.offsets_dev && (nrec == 0 || fd.lengths_dev), MX_ERR_INVALID,
                       "%s: field %d: null lengths or offsets", who, f);
    }
    // the previous use of the staging buffer on this stream must be finished
    MX_TRY_HIP(hipStreamSynchronize(stream));
    char *st = (char *)staging_host;
    const char *recs = (const char *)recs_host;
    for (int f = 0; f < nfields; ++f) {
        const mx_field &fd = fields[f];
        const FieldPlan &p = plan[(size_t)f];
        const size_t eb = (size_t)fd.elem_bytes;
        if (fd.kind == MX_FIELD_SCALAR) {
            parallel_records(nrec, (int64_t)p.vbytes, [&](int64_t r0, int64_t r1) {
                for (int64_t r = r0; r < r1; ++r)
                    std::memcpy(st + p.vpos + (size_t)r * eb, recs + (size_t)r * rec_bytes + (size_t)fd.offset, eb);
            });
        } else {
            std::vector<const void *> rows((size_t)nrec);
            std::vector<int64_t> lens((size_t)nrec), starts((size_t)nrec + 1, 0);
            for (int64_t r = 0; r < nrec; ++r) {
                const mx_hseq h = seq_at(recs_host, rec_bytes, r, fd.offset);
                rows[(size_t)r] = h.data;
                lens[(size_t)r] = h.len;
                starts[(size_t)r + 1] = starts[(size_t)r] + h.len;
            }
            gather_rows(rows.data(), lens.data(), starts.data(), nrec, eb, st + p.vpos, p.count);
            if (nrec) std::memcpy(st + p.lpos, lens.data(), (size_t)nrec * 8);
        }
        if (p.vbytes) MX_TRY_HIP(hipMemcpyAsync(fd.values_dev, st + p.vpos, p.vbytes, hipMemcpyHostToDevice, stream));
        if (fd.kind == MX_FIELD_SEQ) {
            if (nrec)
                MX_TRY_HIP(hipMemcpyAsync(fd.lengths_dev, st + p.lpos, (size_t)nrec * 8, hipMemcpyHostToDevice, stream));
            if (mx_status s2 = lengths_to_offsets(fd.lengths_dev, nrec, fd.offsets_dev, ws, ws_bytes, stream)) return s2;
        }
    }
    return MX_OK;
}

mx_status mx_unmarshal_records(const mx_field *fields, int nfields, int64_t nrec, void *recs_host, size_t rec_bytes,
                               void *staging_host, size_t staging_bytes, hipStream_t stream) {
    const char *who = "mx_unmarshal_records";
    std::vector<FieldPlan> plan;
    size_t need = 0;
    if (mx_status st = plan_records(who, recs_host, nrec, rec_bytes, fields, nfields, plan, &need)) return st;
    MX_REQUIRE(staging_host || need == 0, MX_ERR_INVALID, "%s: null staging", who);
    MX_REQUIRE(staging_bytes >= need, MX_ERR_INVALID, "%s: staging needs %zu bytes", who, need);
    char *st = (char *)staging_host;
    for (int f = 0; f < nfields; ++f) {
        const mx_field &fd = fields[f];
        const FieldPlan &p = plan[(size_t)f];
        MX_REQUIRE(p.count == 0 || fd.values_dev, MX_ERR_INVALID, "%s: field %d: null values", who, f);
        if (p.vbytes) MX_TRY_HIP(hipMemcpyAsync(st + p.vpos, fd.values_dev, p.vbytes, hipMemcpyDeviceToHost, stream));
        if (fd.kind == MX_FIELD_SEQ) {
            MX_REQUIRE(fd.offsets_dev, MX_ERR_INVALID, "%s: field %d: null offsets", who, f);
            MX_TRY_HIP(hipMemcpyAsync(st + p.lpos, fd.offsets_dev, (size_t)(nrec + 1) * 8, hipMemcpyDeviceToHost,
                                      stream));
        }
    }
    MX_TRY_HIP(hipStreamSynchronize(stream));
    char *recs = (char *)recs_host;
    // every sequence's device length against the host record's, before any write
    for (int f = 0; f < nfields; ++f) {
        if (fields[f].kind != MX_FIELD_SEQ) continue;
        const int64_t *off = (const int64_t *)(st + plan[(size_t)f].lpos);
        MX_REQUIRE(off[0] == 0, MX_ERR_SHAPE, "%s: field %d: offsets[0] != 0", who, f);
        for (int64_t r = 0; r < nrec; ++r)
            MX_REQUIRE(off[r + 1] - off[r] == seq_at(recs_host, rec_bytes, r, fields[f].offset).len, MX_ERR_SHAPE,
                       "%s: field %d, record %lld: the host sequence's length differs from the device's", who, f,
                       (long long)r);
    }
    for (int f = 0; f < nfields; ++f) {
        const mx_field &fd = fields[f];
        const FieldPlan &p = plan[(size_t)f];
        const size_t eb = (size_t)fd.elem_bytes;
        if (fd.kind == MX_FIELD_SCALAR) {
            parallel_records(nrec, (int64_t)p.vbytes, [&](int64_t r0, int64_t r1) {
                for (int64_t r = r0; r < r1; ++r)
                    std::memcpy(recs + (size_t)r * rec_bytes + (size_t)fd.offset, st + p.vpos + (size_t)r * eb, eb);
            });
        } else {
            const int64_t *off = (const int64_t *)(st + p.lpos);
            parallel_records(nrec, (int64_t)p.vbytes, [&](int64_t r0, int64_t r1) {
                for (int64_t r = r0; r < r1; ++r) {
                    const mx_hseq h = seq_at(recs_host, rec_bytes, r, fd.offset);
                    if (h.len > 0) std::memcpy((void *)h.data, st + p.vpos + (size_t)off[r] * eb, (size_t)h.len * eb);
                }
            });
        }
    }
    return MX_OK;
}

}  // extern "C"
