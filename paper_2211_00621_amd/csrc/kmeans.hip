// k-means step as map (argmin-reduce) + reduce-by-key (the histo pattern of
// the paper's Parboil evaluation, Table 1), and the within-cluster SSE with its
// gradient with respect to the points.
//
//   label_i = the j minimising (dist(x_i, c_j), j) lexicographically
//   count_j = #{i : label_i = j},  sum_j = sum of x_i with label j
//   c'_j = sum_j / count_j, or c_j when count_j = 0
//
// Assignment on the matrix cores: argmin_j dist(x, c_j) = argmin_j f_j with
// f_j = |c_j|^2 - 2 x.c_j, 64 points x 64 centroids per wave (X straight from
// HBM into registers, -2C in LDS, the accumulators starting at the FP32
// |c_j|^2).  The products run in bfloat16 on v_mfma_f32_16x16x32_bf16, each
// FP32 operand split into a high and a middle part (v = v_h + v_m + v_l, each
// part the nearest bfloat16 to what is left: |v - v_h| <= 2^-8 |v|, |v_l| <=
// 2^-16 |v|): a.x is taken as a_h x_h + a_h x_m + a_m x_h, three 16x16x32
// products per tile against eight FP32 16x16x4 ones, each product exact in
// FP32.  The dropped terms (a_m x_m, a_h x_l, a_l x_h and smaller) are at most
// 3.02 2^-16 |a_t||x_t| per dimension, so at most 6.03 2^-16 |c||x| in all (a
// = -2c, Cauchy-Schwarz); the 3 DP FP32 additions of the three accumulations
// over DP padded dimensions (2 u each, u = 2^-24, allowing for the matrix
// core's own rounding) at most (6 DP / 256) 2^-16 times the sum of the
// magnitudes added, |c|^2 (1 + 2^-10) + 2.032 |c||x|; the FP32 |c|^2
// ((DP + 1) / 256) 2^-16 |c|^2; the candidate's index, carried in the six low
// mantissa bits with one chunk of 64 centroids (at most 63 ulp, 0.49 2^-16 of
// the value, |c|^2 + 2|c||x|; with more chunks its slot in the chunk, four
// bits, 0.12 2^-16).  So the computed values p_j satisfy |p_j - f_j| <= B =
// 2^-16 (XC |x| C + CC C^2) with C = max_j |c_j|, XC = 8.54 and CC = 1.37
// for DP = 32 and one chunk (10.06 and 2.25 for DP = 64).  With E = 2B: when the two smallest p differ by more
// than 2E the smallest is the exact, unique minimiser and also the binary64
// oracle's.  The bound is relative, so it needs the products above the
// subnormal range, where the matrix core may flush: below C = 2^-40 no label
// is certified here.  The other points (on the blob data about 2 % of them,
// where several centroids share a blob) go through up to three more stages:
// between their best two candidates in the FP32 direct form, when the third
// best is also above the margin; among all candidates in the FP32 direct
// form, four points at a time; and, for the few dozen per million left, in
// binary64 in the oracle's operation order -- subtract, square, add, no
// fused multiply-add -- taking the lexicographic minimum, so labels are
// bit-exact in all cases.
//
// Persistent waves: a fixed grid of at most kMaxBlocks blocks, each wave
// walking its own sequence of 64-point chunks and loading the next chunk's
// points while it certifies and adds the current one, so the stream of X from
// HBM overlaps the work.  The products run one block of 16 points at a time
// and the four lane groups' candidates are merged through lane swaps, not LDS,
// so that at d = 32, k = 64 three blocks of four waves fit a CU (168
// registers, 51.5 KB of LDS per block).
//
// Reduce-by-key from the registers that already hold the chunk: lane
// (g, l16) holds dimensions 8g..8g+7 of points mi*16 + l16 and adds them to
// wave-private LDS sums.  Lanes whose points share a label are separated into
// passes by their rank among equal labels, so no instruction has two lanes on
// one address; a wave's LDS operations execute in issue order, so the sums
// are the same on every run.  The block adds its waves in wave order and
// writes one partial per block; a finish kernel adds the block partials in
// block order in binary64, divides and writes the new centroids and the int64
// counts.  The grid does not depend on the device, so neither do the results.
#include <algorithm>
#include <atomic>
#include <cfloat>

#include "mx_internal.h"

namespace mx {
namespace {

constexpr int NT = 256;       // 4 waves
constexpr int kWaves = NT / kWave;
constexpr int kPtsWave = 64;  // points per wave chunk
constexpr int kMaxBlocks = 768; // persistent grid (three blocks per CU on 256 CUs)
constexpr int kMaxD = 64, kMaxK = 256, kMaxKD = 4096;
// finish kernel: a block owns kFinEntries entries (j, t), its kFinGroups thread
// groups take the block partials in turn
constexpr int kFinEntries = 8, kFinGroups = NT / kFinEntries;

// Per-wave LDS scratch in floats: the reduce-by-key's idle slots (DP / 32 x 2
// x 64 float4), which also hold four staged points (4 x DP), and with more
// than one centroid chunk the publication slots (4 x 64 float4).
__host__ __device__ constexpr int scr_floats(int DP, int KP) {
    return (KP > 64 && 4 * kPtsWave * 4 > DP * 16) ? 4 * kPtsWave * 4 : DP * 16;
}

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

// v = hi + mid + (a remainder of at most 2^-16 |v|), hi and mid bfloat16 (round
// to nearest even); each pair is converted once and its two high parts read
// back from the packed word (a bfloat16 is the top half of a float)
__device__ __forceinline__ void split_bf16(const float4 &u0, const float4 &u1, bf16x8 &hi, bf16x8 &mid) {
    const float v[8] = {u0.x, u0.y, u0.z, u0.w, u1.x, u1.y, u1.z, u1.w};
    unsigned hw[4], mw[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const unsigned h = __builtin_bit_cast(unsigned, __builtin_convertvector((f32x2){v[2 * e], v[2 * e + 1]}, bf16x2));
        const float h0 = __uint_as_float(h << 16), h1 = __uint_as_float(h & 0xffff0000u);
        hw[e] = h;
        mw[e] = __builtin_bit_cast(unsigned,
                                   __builtin_convertvector((f32x2){v[2 * e] - h0, v[2 * e + 1] - h1}, bf16x2));
    }
    typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
    hi = __builtin_bit_cast(bf16x8, (u32x4){hw[0], hw[1], hw[2], hw[3]});
    mid = __builtin_bit_cast(bf16x8, (u32x4){mw[0], mw[1], mw[2], mw[3]});
}

// inserts v into t1 <= t2 <= t3, keeping the three smallest (median forms: no
// canonicalising of bit-built values)
__device__ __forceinline__ void insert3(float &t1, float &t2, float &t3, float v) {
    t3 = __builtin_amdgcn_fmed3f(t2, t3, v);
    t2 = __builtin_amdgcn_fmed3f(t1, t2, v);
    t1 = __builtin_amdgcn_fmed3f(t1, v, -FLT_MAX);
}

// lanes 32..63 of a trade places with lanes 0..31 of b (v_permlane32_swap)
__device__ __forceinline__ void swap_halves(unsigned &a, unsigned &b) {
    const auto r = __builtin_amdgcn_permlane32_swap(a, b, false, false);
    a = r[0];
    b = r[1];
}
__device__ __forceinline__ void swap_halves(float &a, float &b) {
    unsigned ua = __float_as_uint(a), ub = __float_as_uint(b);
    swap_halves(ua, ub);
    a = __uint_as_float(ua);
    b = __uint_as_float(ub);
}

// the odd 16-lane rows of a trade places with the even rows of b
// (v_permlane16_swap)
__device__ __forceinline__ void swap_rows(unsigned &a, unsigned &b) {
    const auto r = __builtin_amdgcn_permlane16_swap(a, b, false, false);
    a = r[0];
    b = r[1];
}
__device__ __forceinline__ void swap_rows(float &a, float &b) {
    unsigned ua = __float_as_uint(a), ub = __float_as_uint(b);
    swap_rows(ua, ub);
    a = __uint_as_float(ua);
    b = __uint_as_float(ub);
}

// The words of the four lanes of this lane's 16-lane column (the same lane
// of rows 0..3): rows 2 (g >> 1) and 2 (g >> 1) + 1 by a row swap, then the
// other half's by a half swap.
__device__ __forceinline__ void column4(int v, int (&out)[4]) {
    unsigned w0 = (unsigned)v, w1 = w0;
    swap_rows(w0, w1);
    unsigned w2 = w0, w3 = w1;
    swap_halves(w0, w2);  // w0: row 0, w2: row 2
    swap_halves(w1, w3);  // w1: row 1, w3: row 3
    out[0] = (int)w0;
    out[1] = (int)w1;
    out[2] = (int)w2;
    out[3] = (int)w3;
}

// binary64 distance in the oracle's order: acc = acc + (x_t - c_t)^2, t ascending
__device__ __forceinline__ double dist64(const float *__restrict__ x, const float *c, int d) {
    double acc = 0.0;
    for (int t = 0; t < d; ++t) {
        const double diff = sub_rn((double)x[t], (double)c[t]);
        acc = add_rn(acc, mul_rn(diff, diff));
    }
    return acc;
}

// The same over the DP padded dimensions of an LDS row holding -2c (c = -m2 / 2
// exactly in binary64); past d both rows hold zeros, which add exact zeros.
template <int DP>
__device__ __forceinline__ double dist64_m2(const float *x, const float *m2) {
    double acc = 0.0;
    // two 16-byte groups of each row at a time: the rare paths that call
    // these keep few registers beside the chunk's
#pragma unroll 2
    for (int t = 0; t < DP; t += 4) {
        const float4 xv = *reinterpret_cast<const float4 *>(x + t);
        const float4 cv = *reinterpret_cast<const float4 *>(m2 + t);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const double diff = sub_rn((double)vget<float4, float>(xv, e), -0.5 * (double)vget<float4, float>(cv, e));
            acc = add_rn(acc, mul_rn(diff, diff));
        }
    }
    return acc;
}

// FP32 direct form sum (x_t - c_t)^2 over an LDS row holding -2c (c = -m2 / 2
// exactly); past d both rows hold zeros, which add exact zeros.
template <int DP>
__device__ __forceinline__ float dist32_m2(const float *x, const float *m2) {
    float acc = 0.f;
#pragma unroll 2
    for (int t = 0; t < DP; t += 4) {
        const float4 xv = *reinterpret_cast<const float4 *>(x + t);
        const float4 cv = *reinterpret_cast<const float4 *>(m2 + t);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const float diff = vget<float4, float>(xv, e) + 0.5f * vget<float4, float>(cv, e);
            acc += diff * diff;
        }
    }
    return acc;
}

struct KmArgs {
    const float *X;
    int64_t n;
    int d, k;
    const float *C;
    int32_t *labels;
    float *part_sums;   // [ceil(k*d / 8)][nblocks][8]: entry e of block b at (e / 8 * nblocks + b) * 8 + e % 8
    int *part_counts;   // [k][nblocks]
    unsigned long long *fallbacks;  // optional counter of binary64 recomputations
};

// Row stride of the LDS sums: d rounded up to 16 bytes.  When that is a
// multiple of 32 floats, row j keeps its 16-byte groups XOR-permuted by j mod 8
// within each aligned run of eight, so that one column of consecutive labels
// falls on different banks.
__host__ __device__ inline int sums_ld(int d) { return (d + 3) & ~3; }
__device__ __forceinline__ int sums_at(int j, int t, int ldd) {
    return j * ldd + ((ldd & 31) == 0 ? t ^ ((j & 7) << 2) : t);
}

// Orders this wave's LDS writes before its later LDS reads (a wave's LDS
// operations execute in order; this only keeps the compiler from moving them).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// X fragments of chunk c: point c*64 + mi*16 + l16, dims kc*32 + 8g .. +7.
// Branch-free, so the loads stay in flight while the current chunk is
// processed: points past n are read from the last point (their labels are
// never used) and dimensions past d from dimension d - 1 (the centroids are
// zero there, so only |x|^2 needs them zeroed, which mask_chunk does when the
// chunk is consumed).  VX: d == DP, X 16-byte aligned and fewer than 2^32
// 16-byte vectors in X (two 16-byte loads at 32-bit vector offsets).
template <int DP, bool VX>
__device__ __forceinline__ void load_chunk(float4 (&xa)[4][DP / 32][2], const KmArgs &a, int64_t c, int l16,
                                           int g) {
    const int d = a.d;
    if constexpr (VX) {
        // n * DP / 4 < 2^32, so the point index and the vector offset fit 32 bits
        const float4 *X4 = reinterpret_cast<const float4 *>(a.X);
        const uint32_t last = (uint32_t)a.n - 1u;
#pragma unroll
        for (int mi = 0; mi < 4; ++mi) {
            const uint32_t p = (uint32_t)c * (uint32_t)kPtsWave + (uint32_t)(mi * 16 + l16);
            const uint32_t v0 = min(p, last) * (uint32_t)(DP / 4) + (uint32_t)(2 * g);
#pragma unroll
            for (int kc = 0; kc < DP / 32; ++kc) {
                const float4 *q = X4 + (v0 + (uint32_t)(kc * 8));
                xa[mi][kc][0] = q[0];
                xa[mi][kc][1] = q[1];
            }
        }
        return;
    }
#pragma unroll
    for (int mi = 0; mi < 4; ++mi) {
        const int64_t p = c * kPtsWave + mi * 16 + l16;
        const int64_t pc = p < a.n ? p : a.n - 1;
#pragma unroll
        for (int kc = 0; kc < DP / 32; ++kc) {
            const int t0 = kc * 32 + 8 * g;
            {
                float v[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) v[e] = a.X[pc * d + (t0 + e < d ? t0 + e : d - 1)];
                xa[mi][kc][0] = make_float4(v[0], v[1], v[2], v[3]);
                xa[mi][kc][1] = make_float4(v[4], v[5], v[6], v[7]);
            }
        }
    }
}

// zeroes the dimensions past d (nothing to do when d == DP)
template <int DP, bool VX>
__device__ __forceinline__ void mask_chunk(float4 (&xa)[4][DP / 32][2], int d, int g) {
    if constexpr (!VX) {
#pragma unroll
        for (int mi = 0; mi < 4; ++mi)
#pragma unroll
            for (int kc = 0; kc < DP / 32; ++kc)
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int t = kc * 32 + 8 * g + 4 * h;
                    float4 &u = xa[mi][kc][h];
                    u.x = t + 0 < d ? u.x : 0.f;
                    u.y = t + 1 < d ? u.y : 0.f;
                    u.z = t + 2 < d ? u.z : 0.f;
                    u.w = t + 3 < d ? u.w : 0.f;
                }
    }
}

// DP: d padded to a multiple of 32; KP: k padded to a multiple of 64.
template <int DP, int KP, bool VX>
__global__ void __launch_bounds__(NT, (DP == 32 && KP == 64) ? (VX ? 3 : 2) : 1) k_kmeans_fused(KmArgs a) {
    constexpr int LDC = DP + 4;
    constexpr int LBITS = KP <= 64 ? 6 : KP <= 128 ? 7 : 8;  // bits of a label
    extern __shared__ __attribute__((aligned(16))) float smem[];
    const int d = a.d, k = a.k;
    const int ldd = VX ? DP : sums_ld(d);              // VX: d == DP
    float *Cs = smem;                                  // [KP][LDC]
    float *cnorm = Cs + KP * LDC;                      // [KP]
    float *sums_all = cnorm + KP;                      // [kWaves][k][ldd]
    int *counts_all = (int *)(sums_all + kWaves * k * ldd);  // [kWaves][k]
    float *scr = (float *)(counts_all + kWaves * k);   // [kWaves][scr_floats]
    __shared__ float cmax_s;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int l16 = lane & 15, g = lane >> 4;

    // the first chunk's points are in flight while the centroids are staged
    const int64_t nchunks = (a.n + kPtsWave - 1) / kPtsWave;
    const int64_t wstride = (int64_t)gridDim.x * kWaves;
    int64_t c = (int64_t)blockIdx.x * kWaves + wave;  // wave-uniform
    float4 xa[4][DP / 32][2];
    if (c < nchunks) load_chunk<DP, VX>(xa, a, c, l16, g);

    // -2 c into LDS (zero padded; the scaling is exact), then from those rows
    // |c|^2 (c = -m2 / 2 exactly wherever -2c is finite; where it is not,
    // |c|^2 overflows as well; padding centroids get FLT_MAX, finite so that
    // index packing keeps them ordered, and never below a real centroid's
    // value) and the largest norm
    for (int e = tid; e < KP * LDC; e += NT) {
        const int j = e / LDC, t = e - j * LDC;
        Cs[e] = (j < k && t < d) ? -2.0f * a.C[(int64_t)j * d + t] : 0.f;
    }
    for (int e = tid; e < kWaves * k * ldd; e += NT) sums_all[e] = 0.f;
    for (int e = tid; e < kWaves * k; e += NT) counts_all[e] = 0;
    __syncthreads();
    if (wave == 0) {
        float m = 0.f;
        for (int j = lane; j < KP; j += kWave) {
            // over the DP padded dimensions: past d the rows hold zeros, whose
            // squares add exact zeros
            float s = 0.f;
            if (j < k)
#pragma unroll
                for (int t = 0; t < DP; t += 4) {
                    const float4 u = *reinterpret_cast<const float4 *>(Cs + j * LDC + t);
                    const float v0 = -0.5f * u.x, v1 = -0.5f * u.y, v2 = -0.5f * u.z, v3 = -0.5f * u.w;
                    s += v0 * v0;
                    s += v1 * v1;
                    s += v2 * v2;
                    s += v3 * v3;
                }
            cnorm[j] = j < k ? s : FLT_MAX;
            if (j < k) m = fmaxf(m, s);
        }
        m = wave_reduce<Red<MX_MAX, float>>(m);
        if (lane == 0) cmax_s = sqrtf(m);
    }
    __syncthreads();
    const float cmax = cmax_s;
    // 2E = 4B = 2^-16 C (kXC |x| + kCC C): the bound's constants for DP
    // padded dimensions and kSlot = (2^bits - 1) / 128 for the index bits in
    // the values (six with one centroid chunk, else four), times four,
    // rounded up
    constexpr float kSlot = (KP == 64 ? 63.0f : 15.0f) / 128.0f;
    constexpr float kXC = 4.0f * (6.03f + 2.032f * (6.0f * DP / 256.0f) + 2.0f * kSlot) + 0.05f;
    constexpr float kCC = 4.0f * (1.001f * (6.0f * DP / 256.0f) + (DP + 1.0f) / 256.0f + kSlot) + 0.05f;
    const bool bound_ok = cmax >= 0x1p-40f;  // products above the subnormal range
    // A operands (-2c, rows ci*16 + l16 of centroid chunk cc, dimensions
    // kc*32 + 8g .. +7) as bfloat16 parts: held in registers for the whole
    // walk when there is one centroid chunk, else split per chunk
    auto a_ops = [&](int cc, int ci, int kc, bf16x8 &ah, bf16x8 &am) {
        const float *q = Cs + (cc * 64 + ci * 16 + l16) * LDC + kc * 32 + 8 * g;
        split_bf16(*reinterpret_cast<const float4 *>(q), *reinterpret_cast<const float4 *>(q + 4), ah, am);
    };
    bf16x8 areg_h[KP == 64 ? 4 : 1][DP / 32], areg_m[KP == 64 ? 4 : 1][DP / 32];
    if constexpr (KP == 64) {
#pragma unroll
        for (int ci = 0; ci < 4; ++ci)
#pragma unroll
            for (int kc = 0; kc < DP / 32; ++kc) a_ops(0, ci, kc, areg_h[ci][kc], areg_m[ci][kc]);
    }

    float *ws = sums_all + wave * k * ldd;
    int *wc = counts_all + wave * k;
    constexpr int kScr = scr_floats(DP, KP);
    float4 *pub = reinterpret_cast<float4 *>(scr + wave * kScr);  // scratch, 16-byte aligned

    for (; c < nchunks; c += wstride) {
        const int64_t p0 = c * kPtsWave;
        mask_chunk<DP, VX>(xa, d, g);

        // this lane's part of |x|^2 (its eight or sixteen dimensions)
        float xpart[4];
#pragma unroll
        for (int mi = 0; mi < 4; ++mi) {
            float s = 0.f;
#pragma unroll
            for (int kc = 0; kc < DP / 32; ++kc)
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const float4 u = xa[mi][kc][h];
                    s += u.x * u.x + u.y * u.y + u.z * u.z + u.w * u.w;
                }
            xpart[mi] = s;
        }

        // ---- f = |c|^2 - 2 c.x over chunks of 64 centroids.  The MFMA's A
        //      operand is -2c (centroid rows), its B operand the points and its
        //      accumulator starts at |c|^2, so lane (g, l16) ends with f for
        //      rows 4g + r (centroids) of column l16 (point) of each (centroid
        //      block ci, point block pi): 16 candidates per point in one lane.
        //      Each f carries its candidate's index (one chunk: ci*16 + r in
        //      its six low mantissa bits, the lane group's 4g added after the
        //      selection; more chunks: its slot ci*4 + r in four bits), so one
        //      minimum gives value and index, and medians of three keep the
        //      next smallest.  Then the four lane groups of each point are
        //      merged in a fixed order (lexicographic minimum).
        float m1, m2, m3 = INFINITY, xx;  // m3: the third smallest (one centroid chunk only)
        int mj, mj2 = -1;
        if constexpr (KP == 64) {
            // one point block at a time, so only its 16 accumulators are live
            v4f cn[4];  // |c|^2 of rows 4g .. 4g+3 of each centroid block: the first product's source
#pragma unroll
            for (int ci = 0; ci < 4; ++ci) {
                const float4 c4 = *reinterpret_cast<const float4 *>(cnorm + ci * 16 + 4 * g);
                cn[ci] = v4f{c4.x, c4.y, c4.z, c4.w};
            }
            float r1[4], r2[4], r3[4];
#pragma unroll
            for (int pi = 0; pi < 4; ++pi) {
                v4f acc[4];
#pragma unroll
                for (int kc = 0; kc < DP / 32; ++kc) {
                    // lane (g, l16) holds dimensions kc*32 + 8g .. +7 of point
                    // pi*16 + l16 (B operand) and of centroid row ci*16 + l16 (A)
                    bf16x8 bh, bm;
                    split_bf16(xa[pi][kc][0], xa[pi][kc][1], bh, bm);
#pragma unroll
                    for (int ci = 0; ci < 4; ++ci)
                        acc[ci] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(areg_h[ci][kc], bh, kc == 0 ? cn[ci] : acc[ci],
                                                                          0, 0, 0);
#pragma unroll
                    for (int ci = 0; ci < 4; ++ci)
                        acc[ci] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(areg_h[ci][kc], bm, acc[ci], 0, 0, 0);
#pragma unroll
                    for (int ci = 0; ci < 4; ++ci)
                        acc[ci] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(areg_m[ci][kc], bh, acc[ci], 0, 0, 0);
                }
                float b1 = INFINITY, b2 = INFINITY, b3 = INFINITY;
#pragma unroll
                for (int ci = 0; ci < 4; ++ci)
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        // bits 0-1 and 4-5 carry r and ci of the index
                        // ci*16 + 4g + r; bits 2-3 (the lane group's, equal
                        // for every candidate of this lane) are set below
                        insert3(b1, b2, b3, __uint_as_float((__float_as_uint(acc[ci][r]) & ~63u) | (unsigned)(ci * 16 + r)));
                // the same two bits in every value keep the lane's order
                const unsigned gb = 4u * (unsigned)g;
                r1[pi] = __uint_as_float(__float_as_uint(b1) | gb);
                r2[pi] = __uint_as_float(__float_as_uint(b2) | gb);
                r3[pi] = __uint_as_float(__float_as_uint(b3) | gb);
            }
            // The three smallest of the four lane groups' three smallest, in
            // registers: lanes l and l ^ 32 (groups g and g ^ 2) exchange half
            // their point blocks and merge, the lower half keeping blocks 0
            // and 1, the upper 2 and 3; then rows r and r ^ 1 (groups g and
            // g ^ 1) do the same, and row g is left with block g, whose
            // column l16 is point 16g + l16: the lane's own.  Every value
            // carries its whole index, so float order is (value, index)
            // order wherever the values differ by more than the index bits,
            // and the three smallest do not depend on the merge order.
            float xp[4];
#pragma unroll
            for (int mi = 0; mi < 4; ++mi) xp[mi] = xpart[mi];
#pragma unroll
            for (int pi = 0; pi < 2; ++pi) {
                swap_halves(r1[pi], r1[pi + 2]);
                swap_halves(r2[pi], r2[pi + 2]);
                swap_halves(r3[pi], r3[pi + 2]);
                swap_halves(xp[pi], xp[pi + 2]);
                insert3(r1[pi], r2[pi], r3[pi], r1[pi + 2]);
                insert3(r1[pi], r2[pi], r3[pi], r2[pi + 2]);
                insert3(r1[pi], r2[pi], r3[pi], r3[pi + 2]);
                xp[pi] += xp[pi + 2];
            }
            swap_rows(r1[0], r1[1]);
            swap_rows(r2[0], r2[1]);
            swap_rows(r3[0], r3[1]);
            swap_rows(xp[0], xp[1]);
            insert3(r1[0], r2[0], r3[0], r1[1]);
            insert3(r1[0], r2[0], r3[0], r2[1]);
            insert3(r1[0], r2[0], r3[0], r3[1]);
            m1 = r1[0];
            m2 = r2[0];
            m3 = r3[0];
            xx = xp[0] + xp[1];
            mj = (int)(__float_as_uint(m1) & 63u);
            mj2 = (int)(__float_as_uint(m2) & 63u);
        } else {
            float r1[4], r2[4];
            int ri[4];
#pragma unroll
            for (int cc = 0; cc < KP / 64; ++cc) {
                v4f acc[4][4];  // [ci][pi]
                v4f cn[4];
#pragma unroll
                for (int ci = 0; ci < 4; ++ci) {
                    const float4 c4 = *reinterpret_cast<const float4 *>(cnorm + cc * 64 + ci * 16 + 4 * g);
                    cn[ci] = v4f{c4.x, c4.y, c4.z, c4.w};
                }
#pragma unroll
                for (int kc = 0; kc < DP / 32; ++kc) {
                    bf16x8 bh[4], bm[4];
#pragma unroll
                    for (int pi = 0; pi < 4; ++pi) split_bf16(xa[pi][kc][0], xa[pi][kc][1], bh[pi], bm[pi]);
#pragma unroll
                    for (int ci = 0; ci < 4; ++ci) {
                        bf16x8 ah, am;
                        a_ops(cc, ci, kc, ah, am);
#pragma unroll
                        for (int pi = 0; pi < 4; ++pi)
                            acc[ci][pi] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[pi], kc == 0 ? cn[ci] : acc[ci][pi],
                                                                                  0, 0, 0);
#pragma unroll
                        for (int pi = 0; pi < 4; ++pi)
                            acc[ci][pi] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bm[pi], acc[ci][pi], 0, 0, 0);
#pragma unroll
                        for (int pi = 0; pi < 4; ++pi)
                            acc[ci][pi] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bh[pi], acc[ci][pi], 0, 0, 0);
                    }
                }
#pragma unroll
                for (int pi = 0; pi < 4; ++pi) {
                    float b1 = INFINITY, b2 = INFINITY;
#pragma unroll
                    for (int ci = 0; ci < 4; ++ci)
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const float f = __uint_as_float((__float_as_uint(acc[ci][pi][r]) & ~15u) | (unsigned)(ci * 4 + r));
                            // median forms: no canonicalising of the bit-built f
                            b2 = __builtin_amdgcn_fmed3f(b1, b2, f);
                            b1 = __builtin_amdgcn_fmed3f(b1, f, -FLT_MAX);
                        }
                    const int slot = (int)(__float_as_uint(b1) & 15u);
                    const int j1 = cc * 64 + (slot >> 2) * 16 + 4 * g + (slot & 3);
                    if (cc == 0) {
                        r1[pi] = b1; ri[pi] = j1; r2[pi] = b2;
                    } else {  // later centroid chunks have larger indices: ties keep the earlier
                        r2[pi] = fminf(fmaxf(r1[pi], b1), fminf(r2[pi], b2));
                        ri[pi] = b1 < r1[pi] ? j1 : ri[pi];
                        r1[pi] = fminf(r1[pi], b1);
                    }
                }
            }
            // every lane publishes (best, index, second, |x|^2 part) per
            // point; the point's lane merges the four lane groups in order
#pragma unroll
            for (int pi = 0; pi < 4; ++pi)
                pub[g * kPtsWave + pi * 16 + l16] = make_float4(r1[pi], __int_as_float(ri[pi]), r2[pi], xpart[pi]);
            wave_sync();
            float4 q = pub[lane];
            m1 = q.x;
            m2 = q.z;
            xx = q.w;
            mj = __float_as_int(q.y);
#pragma unroll
            for (int gg = 1; gg < 4; ++gg) {
                q = pub[gg * kPtsWave + lane];
                const int qj = __float_as_int(q.y);
                const bool tk = q.x < m1 || (q.x == m1 && qj < mj);
                m2 = fminf(fmaxf(m1, q.x), fminf(m2, q.z));
                mj = tk ? qj : mj;
                m1 = fminf(m1, q.x);
                xx += q.w;
            }
        }
        // next chunk's points, in flight while this one's labels are
        // certified and its points added (the last chunk reloads itself
        // rather than branch around the loads); issued after the products,
        // so the two chunks' registers are not live across them
        __builtin_amdgcn_sched_barrier(0);
        float4 xn[4][DP / 32][2];
        load_chunk<DP, VX>(xn, a, c + wstride < nchunks ? c + wstride : c, l16, g);
        int lrv;  // this lane's point: rank << 16 | label, or -1
        // ---- certify each label (lane = point); uncertified points are
        //      recomputed in binary64 by the whole wave, lanes over centroids
        {
            const int64_t p = p0 + lane;
            int label = -1;
            bool certified = true, two = false;
            if (p < a.n) {
                const float margin = bound_ok ? 0x1p-16f * cmax * (kXC * sqrtf(xx) + kCC * cmax) : INFINITY;
                certified = m2 - m1 > margin;
                // every candidate but the best two is at least 2E above the
                // best: the minimiser is one of those two
                two = KP == 64 && !certified && m3 - m1 > margin && mj2 >= 0;
                label = mj;
            }
            // ---- the best two, compared in the FP32 direct form by all
            //      lanes at once: lane (g, l16) adds (x_t - c_t)^2 over its
            //      dimensions for each of its points, the point's lane adds
            //      the four parts in lane-group order; within 2 (d + 3) u of
            //      the larger distance the point goes on to the stages below
            if constexpr (KP == 64) {
                if (__ballot(two)) {
                    // both indices of each point to the four lanes holding
                    // its dimensions
                    int vv[4];
                    column4(two ? (mj | (mj2 << 16)) : -1, vv);
                    float2 sd[4];
#pragma unroll
                    for (int mi = 0; mi < 4; ++mi) {
                        const int v = vv[mi];  // point mi * 16 + l16
                        sd[mi] = make_float2(0.f, 0.f);
                        if (v >= 0) {
                            const float *c1 = Cs + (v & 0xffff) * LDC, *c2 = Cs + (v >> 16) * LDC;
#pragma unroll
                            for (int kc = 0; kc < DP / 32; ++kc)
#pragma unroll
                                for (int h = 0; h < 2; ++h) {
                                    const int t = kc * 32 + 8 * g + 4 * h;
                                    const float4 xv = xa[mi][kc][h];
                                    const float4 u1 = *reinterpret_cast<const float4 *>(c1 + t);
                                    const float4 u2 = *reinterpret_cast<const float4 *>(c2 + t);
#pragma unroll
                                    for (int e = 0; e < 4; ++e) {
                                        const float x_ = vget<float4, float>(xv, e);
                                        const float d1 = x_ + 0.5f * vget<float4, float>(u1, e);
                                        const float d2 = x_ + 0.5f * vget<float4, float>(u2, e);
                                        sd[mi].x += d1 * d1;
                                        sd[mi].y += d2 * d2;
                                    }
                                }
                        }
                    }
                    // the four lane groups' parts to the point's lane, as in
                    // the merge above (a summation tree; the bound below
                    // holds for any order of the additions)
#pragma unroll
                    for (int pi = 0; pi < 2; ++pi) {
                        swap_halves(sd[pi].x, sd[pi + 2].x);
                        swap_halves(sd[pi].y, sd[pi + 2].y);
                        sd[pi].x += sd[pi + 2].x;
                        sd[pi].y += sd[pi + 2].y;
                    }
                    swap_rows(sd[0].x, sd[1].x);
                    swap_rows(sd[0].y, sd[1].y);
                    if (two) {
                        const float D1 = sd[0].x + sd[1].x, D2 = sd[0].y + sd[1].y;
                        // relative bound: subnormal squares add at most
                        // 2^-149 each, negligible once the larger sum is 2^-90
                        const float E2 = 2.0f * (float)(d + 3) * 5.9604645e-8f * fmaxf(D1, D2);
                        if (fabsf(D1 - D2) > 2.0f * E2 && fmaxf(D1, D2) >= 0x1p-90f) {
                            certified = true;
                            label = D1 < D2 ? mj : mj2;
                        }
                    }
                }
            }
            uint64_t todo = __ballot(!certified);
            // Uncertified points, four at a time: the points' coordinates go
            // from the registers that hold them (four lanes each) to this
            // wave's LDS scratch; row s of 16 lanes takes
            // point s, lane l of it centroids j = l, l + 16, ...: the FP32
            // direct form sum (x_t - c_t)^2 (c_t = -m2_t / 2 exactly), within
            // (d + 2) u (1 + u)^(d+2) of the exact value, with j in its eight
            // low bits (a change of at most 255 ulp, under 2^-15 of it; as
            // bits, non-negative floats order like unsigned integers, so no
            // denormal flushing can drop the index).  With E = 2 (d + 3 + 512)
            // u times the second smallest, a gap over 2E makes the smallest
            // the exact, unique minimiser.  The rest go to binary64 in the
            // oracle's order.
            float *xs = reinterpret_cast<float *>(pub);  // [4][DP]
            uint64_t todo64 = 0;
            while (todo) {
                int qs[4];
                int nq = 0;
#pragma unroll
                for (int s2 = 0; s2 < 4; ++s2) {
                    qs[s2] = todo ? __builtin_ctzll(todo) : -1;  // wave-uniform
                    if (todo) {
                        todo &= todo - 1;
                        ++nq;
                    }
                }
                wave_sync();
#pragma unroll
                for (int s2 = 0; s2 < 4; ++s2) {
                    const int q = qs[s2];
#pragma unroll
                    for (int mi = 0; mi < 4; ++mi)
                        if (q >= 0 && mi == (q >> 4) && l16 == (q & 15))
#pragma unroll
                            for (int kc = 0; kc < DP / 32; ++kc) {
                                *reinterpret_cast<float4 *>(xs + s2 * DP + kc * 32 + 8 * g) = xa[mi][kc][0];
                                *reinterpret_cast<float4 *>(xs + s2 * DP + kc * 32 + 8 * g + 4) = xa[mi][kc][1];
                            }
                }
                wave_sync();
                unsigned u1 = 0xffffffffu, u2 = 0xffffffffu;
                if (g < nq && cmax < INFINITY) {
                    for (int j = l16; j < k; j += 16) {
                        const unsigned v = (__float_as_uint(dist32_m2<DP>(xs + g * DP, Cs + j * LDC)) & ~255u) | (unsigned)j;
                        u2 = min(u2, max(u1, v));
                        u1 = min(u1, v);
                    }
                }
                // the two smallest over the 16 lanes of each row
#pragma unroll
                for (int st = 0; st < 4; ++st) {
                    unsigned o1, o2;
                    if (st == 0) { o1 = dpp_move<0xB1, 0xF>(u1, u1); o2 = dpp_move<0xB1, 0xF>(u2, u2); }
                    else if (st == 1) { o1 = dpp_move<0x4E, 0xF>(u1, u1); o2 = dpp_move<0x4E, 0xF>(u2, u2); }
                    else if (st == 2) { o1 = dpp_move<0x141, 0xF>(u1, u1); o2 = dpp_move<0x141, 0xF>(u2, u2); }
                    else { o1 = dpp_move<0x140, 0xF>(u1, u1); o2 = dpp_move<0x140, 0xF>(u2, u2); }
                    u2 = min(min(u2, o2), max(u1, o1));
                    u1 = min(u1, o1);
                }
                const float f1 = __uint_as_float(u1 & ~255u), f2 = __uint_as_float(u2 & ~255u);
                const float E2 = 2.0f * (float)(d + 3 + 512) * 5.9604645e-8f * f2;
                const bool ok = cmax < INFINITY && f2 - f1 > 2.0f * E2 && f2 >= 0x1p-90f;
                // every lane of row s holds point s's result
#pragma unroll
                for (int s2 = 0; s2 < 4; ++s2) {
                    if (qs[s2] < 0) break;
                    const int okq = __builtin_amdgcn_readlane((int)ok, 16 * s2);
                    const int jq = __builtin_amdgcn_readlane((int)(u1 & 255u), 16 * s2);
                    if (okq) {
                        if (lane == qs[s2]) label = jq;
                    } else {
                        todo64 |= 1ull << qs[s2];
                    }
                }
            }
            while (todo64) {
                const int q = __builtin_ctzll(todo64);  // wave-uniform
                todo64 &= todo64 - 1;
                wave_sync();
#pragma unroll
                for (int mi = 0; mi < 4; ++mi)
                    if (mi == (q >> 4) && l16 == (q & 15))
#pragma unroll
                        for (int kc = 0; kc < DP / 32; ++kc) {
                            *reinterpret_cast<float4 *>(xs + kc * 32 + 8 * g) = xa[mi][kc][0];
                            *reinterpret_cast<float4 *>(xs + kc * 32 + 8 * g + 4) = xa[mi][kc][1];
                        }
                wave_sync();
                const float *x = xs;
                if (a.fallbacks && lane == 0) atomicAdd(a.fallbacks, 1ull);
                double bd = INFINITY;
                int bj = 0x7fffffff;
                for (int j = lane; j < k; j += kWave) {
                    // -2c overflows only where |c|^2 does, which makes cmax infinite
                    const double dj = cmax < INFINITY ? dist64_m2<DP>(x, Cs + j * LDC) : dist64(x, a.C + (int64_t)j * d, d);
                    if (dj < bd || (dj == bd && j < bj)) { bd = dj; bj = j; }
                }
#pragma unroll
                for (int off = 32; off >= 1; off >>= 1) {
                    const double od = __shfl_xor(bd, off, kWave);
                    const int oj = __shfl_xor(bj, off, kWave);
                    if (od < bd || (od == bd && oj < bj)) { bd = od; bj = oj; }
                }
                if (lane == q) label = bj;
            }
            if (p < a.n) a.labels[p] = label;
            if (label >= 0) atomicAdd(&wc[label], 1);  // integer: order-free
            // rank among the chunk's earlier points with the same label: the
            // lanes with an equal label, found one label bit at a time
            const uint64_t valid = __ballot(label >= 0);
            uint32_t slo = (uint32_t)valid, shi = (uint32_t)(valid >> 32);
#pragma unroll
            for (int b = 0; b < LBITS; ++b) {
                // all ones where bit b of the label is set; the lanes that
                // agree with it on bit b are ~(ballot ^ m)
                const uint32_t m = (uint32_t)((int)((uint32_t)label << (31 - b)) >> 31);
                const uint64_t mb = __ballot(m != 0u);
                slo &= ~((uint32_t)mb ^ m);
                shi &= ~((uint32_t)(mb >> 32) ^ m);
            }
            const int rank = (int)__builtin_amdgcn_mbcnt_hi(shi, __builtin_amdgcn_mbcnt_lo(slo, 0u));
            lrv = label >= 0 ? (rank << 16) | label : -1;
        }
        wave_sync();
        // ---- reduce-by-key from registers.  Pass m adds every point whose
        //      rank among equal labels is m, so the lanes of one pass own
        //      distinct rows and a plain read-add-write is exact (LDS float
        //      atomics run about one lane per clock); each row receives its
        //      points in increasing index order.  A pass issues all its reads
        //      before its writes; lanes with nothing to add in it read and
        //      write their own slots in the wave's scratch.
        //      Dimensions past d hold zeros in xa, so a 16-byte group that
        //      ends within round4(d) (inside the row) is added whole; groups
        //      past it are skipped.
        {
            int Lm[4], Rm[4], lv[4];
            int rmax = -1;
            column4(lrv, lv);  // the words of points mi * 16 + l16
#pragma unroll
            for (int mi = 0; mi < 4; ++mi) {
                const int v = lv[mi];
                Lm[mi] = v & 0xffff;
                Rm[mi] = v >> 16;  // -1 for points past n
                rmax = max(rmax, Rm[mi]);
            }
            const int d4 = (d + 3) & ~3;
            float4 *junk = pub + lane;  // slot (kc, h) of this lane: junk[(kc * 2 + h) * 64]
            for (int m = 0; __ballot(rmax >= m); ++m) {
                // point blocks with nothing to add in this pass read one
                // broadcast slot and write nothing
                bool act[4];
#pragma unroll
                for (int mi = 0; mi < 4; ++mi) act[mi] = __ballot(Rm[mi] == m) != 0;
                // two point blocks at a time (the rows of a pass are distinct
                // over all four)
#pragma unroll
                for (int m0 = 0; m0 < 4; m0 += 2) {
                    float4 *dst[2][DP / 32][2];
                    float4 sm[2][DP / 32][2];
#pragma unroll
                    for (int u = 0; u < 2; ++u)
#pragma unroll
                        for (int kc = 0; kc < DP / 32; ++kc)
#pragma unroll
                            for (int h = 0; h < 2; ++h) {
                                const int mi = m0 + u, t = kc * 32 + 8 * g + 4 * h;
                                const bool live = Rm[mi] == m && (VX || t + 4 <= d4);
                                dst[u][kc][h] = live ? reinterpret_cast<float4 *>(ws + sums_at(Lm[mi], t, ldd))
                                                     : junk + (kc * 2 + h) * kPtsWave;
                                sm[u][kc][h] = *(act[mi] ? dst[u][kc][h] : pub);
                            }
#pragma unroll
                    for (int u = 0; u < 2; ++u)
                        if (act[m0 + u]) {
#pragma unroll
                            for (int kc = 0; kc < DP / 32; ++kc)
#pragma unroll
                                for (int h = 0; h < 2; ++h) {
                                    float4 v = sm[u][kc][h];
                                    const float4 x = xa[m0 + u][kc][h];
                                    v.x += x.x; v.y += x.y; v.z += x.z; v.w += x.w;
                                    *dst[u][kc][h] = v;
                                }
                        }
                }
            }
        }
        wave_sync();
#pragma unroll
        for (int mi = 0; mi < 4; ++mi)
#pragma unroll
            for (int kc = 0; kc < DP / 32; ++kc) {
                xa[mi][kc][0] = xn[mi][kc][0];
                xa[mi][kc][1] = xn[mi][kc][1];
            }
    }
    __syncthreads();
    // ---- block partial: waves added in wave order
    const int kd = k * d;
    // entry groups of 8 with the blocks side by side, so that the finish
    // kernel's waves read eight blocks' groups as 256 contiguous bytes
    float *ps = a.part_sums + (int64_t)blockIdx.x * kFinEntries;
    for (int e = tid; e < kd; e += NT) {
        const int j = e / d, t = e - j * d;
        const int at = sums_at(j, t, ldd);
        float s = sums_all[at];
#pragma unroll
        for (int w = 1; w < kWaves; ++w) s += sums_all[w * k * ldd + at];
        ps[(int64_t)(e / kFinEntries) * gridDim.x * kFinEntries + e % kFinEntries] = s;
    }
    int *pc = a.part_counts + blockIdx.x;  // label j at [j * gridDim.x]
    for (int j = tid; j < k; j += NT) {
        int cn = counts_all[j];
#pragma unroll
        for (int w = 1; w < kWaves; ++w) cn += counts_all[w * k + j];
        pc[(int64_t)j * gridDim.x] = cn;
    }
}

// Adds the block partials in a fixed order (binary64), divides, writes C' and
// counts.  A block owns 8 entries (j, t); its 32 thread groups take block
// partials b = group, group + 32, ... and the 32 group sums are added in group
// order, so the result does not depend on scheduling.  The partials of one
// entry group sit block after block, so a wave (eight groups) reads eight
// consecutive blocks' entries as 256 contiguous bytes, and their counts as
// eight consecutive ints.

__global__ void __launch_bounds__(NT) k_kmeans_finish(const float *__restrict__ part_sums,
                                                      const int *__restrict__ part_counts, int nblocks,
                                                      int d, int k, const float *__restrict__ C,
                                                      int64_t *__restrict__ counts, float *__restrict__ C_out) {
    __shared__ double ssum[kFinGroups][kFinEntries];
    __shared__ long long scnt[kFinGroups][kFinEntries];
    const int kd = k * d;
    const int le = threadIdx.x % kFinEntries, grp = threadIdx.x / kFinEntries;
    const int e = blockIdx.x * kFinEntries + le;
    const float *grp_sums = part_sums + (int64_t)blockIdx.x * nblocks * kFinEntries + le;  // block b at [b * 8]
    const int j = e < kd ? e / d : 0;
    const int *grp_counts = part_counts + (int64_t)j * nblocks;  // block b at [b]
    double s = 0.0;
    long long c = 0;
    if (e < kd) {
        int b = grp;
        for (; b + 7 * kFinGroups < nblocks; b += 8 * kFinGroups) {
            float p[8];
            int cq[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                p[i] = grp_sums[(int64_t)(b + i * kFinGroups) * kFinEntries];
                cq[i] = grp_counts[b + i * kFinGroups];
            }
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                s += (double)p[i];
                c += cq[i];
            }
        }
        for (; b < nblocks; b += kFinGroups) {
            s += (double)grp_sums[(int64_t)b * kFinEntries];
            c += grp_counts[b];
        }
    }
    ssum[grp][le] = s;
    scnt[grp][le] = c;
    __syncthreads();
    if (grp == 0 && e < kd) {
        double tot = 0.0;
        long long ctot = 0;
        for (int q = 0; q < kFinGroups; ++q) {
            tot += ssum[q][le];
            ctot += scnt[q][le];
        }
        C_out[e] = ctot > 0 ? (float)(tot / (double)ctot) : C[e];
        if (e == j * d) counts[j] = ctot;
    }
}

// ---------------------------------------------------------------- plain form
// assignment: one thread per point, FP32 distances read from global memory,
// the same certification (bound for the direct form) and binary64 fallback
__global__ void __launch_bounds__(NT) k_kmeans_assign_plain(const float *__restrict__ X, int64_t n, int d,
                                                            const float *__restrict__ C, int k,
                                                            int32_t *__restrict__ labels) {
    const int64_t p = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (p >= n) return;
    const float *x = X + p * d;
    float b1 = INFINITY, b2 = INFINITY;
    int i1 = 0;
    for (int j = 0; j < k; ++j) {
        float s = 0.f;
        for (int t = 0; t < d; ++t) {
            const float diff = x[t] - C[(int64_t)j * d + t];
            s += diff * diff;
        }
        if (s < b1) { b2 = b1; b1 = s; i1 = j; }
        else if (s < b2) b2 = s;
    }
    // |D~ - D| <= (d + 3) u D for the direct form; certify with a factor 2
    const float E = 2.0f * (float)(d + 3) * 5.9604645e-8f * b2;
    int label = i1;
    if (!(b2 - b1 > 2.0f * E)) {
        double bd = 0.0;
        label = -1;
        for (int j = 0; j < k; ++j) {
            const double dj = dist64(x, C + (int64_t)j * d, d);
            if (label < 0 || dj < bd) { bd = dj; label = j; }
        }
    }
    labels[p] = label;
}

__global__ void __launch_bounds__(NT) k_zero_words(uint32_t *__restrict__ p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (i < n) p[i] = 0u;
}

__global__ void __launch_bounds__(NT) k_kmeans_accum_plain(const float *__restrict__ X, int64_t n, int d,
                                                           const int32_t *__restrict__ labels,
                                                           float *__restrict__ sums, int *__restrict__ cnt) {
    const int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (e >= n * d) return;
    const int64_t p = e / d;
    const int t = (int)(e - p * d);
    const int l = labels[p];
    atomicAdd(&sums[(int64_t)l * d + t], X[e]);
    if (t == 0) atomicAdd(&cnt[l], 1);
}

__global__ void __launch_bounds__(NT) k_kmeans_divide_plain(const float *__restrict__ sums,
                                                            const int *__restrict__ cnt, int d, int k,
                                                            const float *__restrict__ C,
                                                            int64_t *__restrict__ counts, float *__restrict__ C_out) {
    const int e = blockIdx.x * NT + threadIdx.x;
    if (e >= k * d) return;
    const int j = e / d;
    const int c = cnt[j];
    C_out[e] = c > 0 ? sums[e] / (float)c : C[e];
    if (e == j * d) counts[j] = c;
}

// ---------------------------------------------------------------- SSE and its gradient
// Partial sums of (x - c_label)^2, one per block.  VEC: d % 4 == 0 and X, C
// 16-byte aligned (16-byte loads, the vector index split by 32-bit division
// when n*d/4 < 2^32, which it is for any X below 16 GiB).
template <bool VEC>
__global__ void __launch_bounds__(NT) k_sse_partial(const float *__restrict__ X, int64_t n, int d,
                                                    const float *__restrict__ C,
                                                    const int32_t *__restrict__ labels, float *__restrict__ part) {
    __shared__ float red[NT / kWave];
    float acc = 0.f;
    if constexpr (VEC) {
        const uint32_t dv = (uint32_t)d / 4, nv = (uint32_t)(n * d / 4);
        const float4 *X4 = reinterpret_cast<const float4 *>(X), *C4 = reinterpret_cast<const float4 *>(C);
        for (uint32_t i = blockIdx.x * NT + threadIdx.x; i < nv; i += gridDim.x * NT) {
            const uint32_t p = i / dv, q = i - p * dv;
            const float4 x = X4[i];
            const float4 c = C4[(uint32_t)labels[p] * dv + q];
            const float a = x.x - c.x, b = x.y - c.y, e = x.z - c.z, f = x.w - c.w;
            acc += (a * a + b * b) + (e * e + f * f);
        }
    } else {
        const int64_t total = n * d;
        for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < total; e += (int64_t)gridDim.x * NT) {
            const int64_t p = e / d;
            const float diff = X[e] - C[(int64_t)labels[p] * d + (e - p * d)];
            acc += diff * diff;
        }
    }
    acc = block_reduce<Red<MX_ADD, float>, NT>(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

__global__ void __launch_bounds__(NT) k_sse_final(const float *__restrict__ part, int nb, float *__restrict__ out) {
    __shared__ double red[NT / kWave];
    double acc = 0.0;
    for (int b = threadIdx.x; b < nb; b += NT) acc += (double)part[b];
    acc = block_reduce<Red<MX_ADD, double>, NT>(acc, red);
    if (threadIdx.x == 0) out[0] = (float)acc;
}

__global__ void __launch_bounds__(NT) k_sse_grad(const float *__restrict__ X, int64_t n, int d,
                                                 const float *__restrict__ C, const int32_t *__restrict__ labels,
                                                 const float *__restrict__ gscale, float *__restrict__ G, int vec) {
    const float g2 = 2.0f * gscale[0];
    const int64_t stride = (int64_t)gridDim.x * NT;
    if (vec) {  // d % 4 == 0, 16-byte aligned
        const int64_t nv = n * d / 4;
        const int dv = d / 4;
        for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < nv; i += stride) {
            const int64_t p = i / dv;
            const float4 x = reinterpret_cast<const float4 *>(X)[i];
            const float4 c = reinterpret_cast<const float4 *>(C)[(int64_t)labels[p] * dv + (i - p * dv)];
            reinterpret_cast<float4 *>(G)[i] =
                make_float4(g2 * (x.x - c.x), g2 * (x.y - c.y), g2 * (x.z - c.z), g2 * (x.w - c.w));
        }
    } else {
        for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < n * d; e += stride) {
            const int64_t p = e / d;
            G[e] = g2 * (X[e] - C[(int64_t)labels[p] * d + (e - p * d)]);
        }
    }
}

// ---------------------------------------------------------------- sizes and dispatch
int64_t fused_blocks(int64_t n) {
    const int64_t b = ceil_div(n > 0 ? n : 1, (int64_t)kWaves * kPtsWave);
    return b < kMaxBlocks ? b : kMaxBlocks;
}

size_t fused_lds_bytes(int DP, int KP, int k, int d) {
    return (size_t)KP * (DP + 4) * 4 + (size_t)KP * 4 + (size_t)kWaves * k * sums_ld(d) * 4 + (size_t)kWaves * k * 4 +
           (size_t)kWaves * scr_floats(DP, KP) * 4;
}

size_t ws_layout(int64_t n, int d, int k, size_t *sums_off, size_t *counts_off, size_t *plain_off) {
    const int64_t nb = fused_blocks(n);
    size_t off = kCounterBytes;
    *sums_off = off;
    off += align256((size_t)nb * (size_t)ceil_div(k * d, kFinEntries) * kFinEntries * 4);
    *counts_off = off;
    off += align256((size_t)nb * (size_t)k * 4);
    *plain_off = off;  // plain: sums [k*d] floats then counts [k] ints
    off += align256((size_t)k * d * 4) + align256((size_t)k * 4);
    return off;
}

mx_status check(const char *who, const float *X, int64_t n, int d, const float *C, int k) {
    MX_REQUIRE(n >= 0, MX_ERR_SHAPE, "%s: n < 0", who);
    MX_REQUIRE(d >= 1 && d <= kMaxD, MX_ERR_UNSUPPORTED, "%s: need 1 <= d <= %d", who, kMaxD);
    MX_REQUIRE(k >= 1 && k <= kMaxK && k * d <= kMaxKD, MX_ERR_UNSUPPORTED,
               "%s: need 1 <= k <= %d and k*d <= %d", who, kMaxK, kMaxKD);
    MX_REQUIRE(C && (n == 0 || X), MX_ERR_INVALID, "%s: null input", who);
    return MX_OK;
}

// Debug mode: number of binary64 recomputations in the last step (per process).
std::atomic<long long> g_last_fallbacks{-1};
unsigned long long *g_fb_counter[64] = {};

template <int DP, int KP>
void launch_fused(const KmArgs &a, int64_t nb, size_t lds, hipStream_t s) {
    if (a.d == DP && (uintptr_t)a.X % 16 == 0 && a.n * DP / 4 < (1LL << 32))
        hipLaunchKernelGGL((k_kmeans_fused<DP, KP, true>), dim3((unsigned)nb), dim3(NT), lds, s, a);
    else
        hipLaunchKernelGGL((k_kmeans_fused<DP, KP, false>), dim3((unsigned)nb), dim3(NT), lds, s, a);
}

}  // namespace
}  // namespace mx

using namespace mx;

extern "C" {

size_t mx_kmeans_workspace_bytes(int64_t n, int d, int k) {
    if (n < 0 || d < 1 || k < 1) return 0;
    size_t so, co, po;
    return align256(ws_layout(n, d, k, &so, &co, &po));
}

mx_status mx_kmeans_step_f32(const float *X_dev, int64_t n, int d, const float *C_dev, int k,
                             int32_t *labels_dev, int64_t *counts_dev, float *C_out_dev, void *ws,
                             size_t ws_bytes, hipStream_t stream) {
    const char *who = "mx_kmeans_step_f32";
    if (mx_status st = check(who, X_dev, n, d, C_dev, k)) return st;
    MX_REQUIRE(counts_dev && C_out_dev && (n == 0 || labels_dev), MX_ERR_INVALID, "%s: null output", who);
    MX_REQUIRE(C_out_dev != C_dev, MX_ERR_INVALID, "%s: C_out must not alias C", who);
    size_t so, co, po;
    const size_t need = align256(ws_layout(n, d, k, &so, &co, &po));
    MX_REQUIRE(ws && ws_bytes >= need && ((uintptr_t)ws & 255) == 0, MX_ERR_WORKSPACE,
               "%s: workspace needs %zu bytes, 256-byte aligned", who, need);
    const int64_t nb = fused_blocks(n);
    MX_REQUIRE(nb < (1LL << 31), MX_ERR_SHAPE, "%s: too many points", who);
    const int DP = d <= 32 ? 32 : 64;
    const int KP = (int)ceil_div(k, 64) * 64;
    const size_t lds = fused_lds_bytes(DP, KP, k, d);
    const DeviceInfo *dv;
    if (mx_status st = device_info(&dv)) return st;
    MX_REQUIRE(lds <= (size_t)dv->lds_bytes, MX_ERR_UNSUPPORTED,
               "%s: k = %d, d = %d needs %zu bytes of LDS (the device allows %d)", who, k, d, lds, dv->lds_bytes);
    KmArgs a{X_dev, n, d, k, C_dev, labels_dev, (float *)((char *)ws + so), (int *)((char *)ws + co), nullptr};
    const bool dbg = debug_mode();
    if (dbg) {
        if (!g_fb_counter[dv->device]) MX_TRY_HIP(hipMalloc(&g_fb_counter[dv->device], sizeof(unsigned long long)));
        MX_TRY_HIP(hipMemsetAsync(g_fb_counter[dv->device], 0, sizeof(unsigned long long), stream));
        a.fallbacks = g_fb_counter[dv->device];
    }
    if (n > 0) {
        if (DP == 32) {
            switch (KP) {
            case 64: launch_fused<32, 64>(a, nb, lds, stream); break;
            case 128: launch_fused<32, 128>(a, nb, lds, stream); break;
            case 192: launch_fused<32, 192>(a, nb, lds, stream); break;
            default: launch_fused<32, 256>(a, nb, lds, stream); break;
            }
        } else {
            switch (KP) {
            case 64: launch_fused<64, 64>(a, nb, lds, stream); break;
            default: launch_fused<64, 128>(a, nb, lds, stream); break;  // k*d <= 4096 bounds k to 64 at d = 64
            }
        }
        if (mx_status st = last_launch(who)) return st;
    }
    const int kd = k * d;
    hipLaunchKernelGGL(k_kmeans_finish, dim3((unsigned)ceil_div(kd, kFinEntries)), dim3(NT), 0, stream, a.part_sums,
                       a.part_counts, n > 0 ? (int)nb : 0, d, k, C_dev, counts_dev, C_out_dev);
    if (mx_status st = last_launch(who)) return st;
    if (dbg) {
        unsigned long long h = 0;
        MX_TRY_HIP(hipMemcpyAsync(&h, a.fallbacks, sizeof h, hipMemcpyDeviceToHost, stream));
        MX_TRY_HIP(hipStreamSynchronize(stream));
        g_last_fallbacks.store((long long)h);
    }
    return MX_OK;
}

int64_t mx_kmeans_debug_fallbacks(void) { return g_last_fallbacks.load(); }

mx_status mx_kmeans_step_plain_f32(const float *X_dev, int64_t n, int d, const float *C_dev, int k,
                                   int32_t *labels_dev, int64_t *counts_dev, float *C_out_dev, void *ws,
                                   size_t ws_bytes, hipStream_t stream) {
    const char *who = "mx_kmeans_step_plain_f32";
    if (mx_status st = check(who, X_dev, n, d, C_dev, k)) return st;
    MX_REQUIRE(counts_dev && C_out_dev && (n == 0 || labels_dev), MX_ERR_INVALID, "%s: null output", who);
    size_t so, co, po;
    const size_t need = align256(ws_layout(n, d, k, &so, &co, &po));
    MX_REQUIRE(ws && ws_bytes >= need && ((uintptr_t)ws & 255) == 0, MX_ERR_WORKSPACE,
               "%s: workspace needs %zu bytes, 256-byte aligned", who, need);
    float *sums = (float *)((char *)ws + po);
    int *cnt = (int *)((char *)sums + align256((size_t)k * d * 4));
    const int64_t words = (int64_t)(align256((size_t)k * d * 4) + align256((size_t)k * 4)) / 4;
    hipLaunchKernelGGL(k_zero_words, dim3((unsigned)ceil_div(words, NT)), dim3(NT), 0, stream, (uint32_t *)sums,
                       words);
    if (n > 0) {
        hipLaunchKernelGGL(k_kmeans_assign_plain, dim3((unsigned)ceil_div(n, NT)), dim3(NT), 0, stream, X_dev, n, d,
                           C_dev, k, labels_dev);
        hipLaunchKernelGGL(k_kmeans_accum_plain, dim3((unsigned)ceil_div(n * d, NT)), dim3(NT), 0, stream, X_dev, n,
                           d, labels_dev, sums, cnt);
    }
    hipLaunchKernelGGL(k_kmeans_divide_plain, dim3((unsigned)ceil_div(k * d, NT)), dim3(NT), 0, stream, sums, cnt,
                       d, k, C_dev, counts_dev, C_out_dev);
    return last_launch(who);
}

mx_status mx_kmeans_sse_f32(const float *X_dev, int64_t n, int d, const float *C_dev, const int32_t *labels_dev,
                            float *sse_dev, void *ws, size_t ws_bytes, hipStream_t stream) {
    const char *who = "mx_kmeans_sse_f32";
    MX_REQUIRE(n >= 0 && d >= 1, MX_ERR_SHAPE, "%s: bad sizes", who);
    MX_REQUIRE(sse_dev && C_dev && (n == 0 || (X_dev && labels_dev)), MX_ERR_INVALID, "%s: null pointer", who);
    const size_t need = kCounterBytes + align256(4 * 1024);
    MX_REQUIRE(ws && ws_bytes >= need && ((uintptr_t)ws & 255) == 0, MX_ERR_WORKSPACE,
               "%s: workspace needs %zu bytes, 256-byte aligned", who, need);
    float *part = (float *)((char *)ws + kCounterBytes);
    int nb = (int)std::min<int64_t>(1024, ceil_div(n * d > 0 ? n * d : 1, NT * 4));
    const bool vec = d % 4 == 0 && (uintptr_t)X_dev % 16 == 0 && (uintptr_t)C_dev % 16 == 0 && n * d / 4 < (1LL << 32);
    if (vec)
        hipLaunchKernelGGL(k_sse_partial<true>, dim3(nb), dim3(NT), 0, stream, X_dev, n, d, C_dev, labels_dev, part);
    else
        hipLaunchKernelGGL(k_sse_partial<false>, dim3(nb), dim3(NT), 0, stream, X_dev, n, d, C_dev, labels_dev, part);
    hipLaunchKernelGGL(k_sse_final, dim3(1), dim3(NT), 0, stream, part, nb, sse_dev);
    return last_launch(who);
}

mx_status mx_kmeans_sse_grad_f32(const float *X_dev, int64_t n, int d, const float *C_dev,
                                 const int32_t *labels_dev, const float *gscale_dev, float *G_dev,
                                 hipStream_t stream) {
    const char *who = "mx_kmeans_sse_grad_f32";
    MX_REQUIRE(n >= 0 && d >= 1, MX_ERR_SHAPE, "%s: bad sizes", who);
    if (n == 0) return MX_OK;
    MX_REQUIRE(X_dev && C_dev && labels_dev && gscale_dev && G_dev, MX_ERR_INVALID, "%s: null pointer", who);
    const DeviceInfo *dv;
    if (mx_status st = device_info(&dv)) return st;
    const int vec = (d % 4 == 0) && ((uintptr_t)X_dev % 16 == 0) && ((uintptr_t)C_dev % 16 == 0) &&
                    ((uintptr_t)G_dev % 16 == 0);
    const int64_t items = vec ? n * d / 4 : n * d;
    int64_t grid = ceil_div(items, NT);
    if (grid > (int64_t)dv->num_cus * 16) grid = (int64_t)dv->num_cus * 16;
    hipLaunchKernelGGL(k_sse_grad, dim3((unsigned)grid), dim3(NT), 0, stream, X_dev, n, d, C_dev, labels_dev,
                       gscale_dev, G_dev, vec);
    return last_launch(who);
}

}  // extern "C"
