// User-defined map bodies.  The source language's map and map2 take arbitrary
// first-order functions built from its arithmetic (Appendix A; the
// compilable subset of Section 4.2).  A body arrives as a straight-line
// register program; this file turns it into HIP source in which the body is
// ordinary inlined code -- a streaming map kernel, a fused map + reduce
// (partial pass plus a finish kernel in block order) and the reverse mode --
// compiles that source with hipRTC for the current device and keeps the
// module for the rest of the process.  A chain of operations then costs one
// pass over HBM instead of one pass (and one temporary) per operation, which
// is the point of accelerating whole expressions rather than single
// operators (Section 5.2).
//
// The reverse mode is generated from the same program: the forward values in
// SSA form, then the adjoints in reverse instruction order, each operand
// receiving the chain-rule term of the instruction that read it.
#include <hip/hiprtc.h>

#include <cinttypes>
#include <cmath>
#include <cstdio>
#include <memory>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "mx_internal.h"

struct mx_expr {
    std::vector<mx_xinsn> prog;
    int nin = 0, out_reg = 0;
    mx_dtype dtype = MX_F32;
    std::string src;
};

namespace mx {

// hipRTC: source -> code object for the current device -> module, cached per
// (device, source) for the life of the process.
mx_status rtc_module(const std::string &src, const char *name, hipModule_t *out) {
    static std::mutex mu;
    static std::unordered_map<std::string, hipModule_t> cache;
    int dev = 0;
    MX_TRY_HIP(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    MX_TRY_HIP(hipGetDeviceProperties(&prop, dev));
    const std::string key = std::to_string(dev) + "\n" + src;
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(key);
    if (it != cache.end()) {
        *out = it->second;
        return MX_OK;
    }
    hiprtcProgram prog;
    if (hiprtcCreateProgram(&prog, src.c_str(), name, 0, nullptr, nullptr) != HIPRTC_SUCCESS)
        return set_error(MX_ERR_HIP, "hiprtcCreateProgram failed");
    const std::string arch = std::string("--offload-arch=") + prop.gcnArchName;
    // no packed FP32 instructions in generated code either
    const char *opts[] = {arch.c_str(), "-O3", "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang",
                          "-packed-fp32-ops"};
    const hiprtcResult rc = hiprtcCompileProgram(prog, (int)(sizeof opts / sizeof opts[0]), opts);
    if (rc != HIPRTC_SUCCESS) {
        size_t ls = 0;
        hiprtcGetProgramLogSize(prog, &ls);
        std::string log(ls, '\0');
        if (ls) hiprtcGetProgramLog(prog, &log[0]);
        hiprtcDestroyProgram(&prog);
        return set_error(MX_ERR_HIP, "hipRTC failed to compile %s: %s", name, log.c_str());
    }
    size_t cs = 0;
    hiprtcGetCodeSize(prog, &cs);
    std::vector<char> code(cs);
    hiprtcGetCode(prog, code.data());
    hiprtcDestroyProgram(&prog);
    hipModule_t mod = nullptr;
    MX_TRY_HIP(hipModuleLoadData(&mod, code.data()));
    cache.emplace(key, mod);
    *out = mod;
    return MX_OK;
}

namespace {

constexpr int kRegs = 16, kMaxInsn = 64, kMaxIn = 4;
constexpr int NT = 256;          // threads per block of every generated kernel
constexpr int kGroupsPerIt = 4;  // vector groups per thread and loop iteration
constexpr int kMaxRedBlocks = 2048;  // eight per CU resident at once: one round, longer-lived threads

bool reads_a(int op) { return op >= MX_X_ADD; }
bool reads_b(int op) { return op >= MX_X_ADD && op <= MX_X_MAX; }

// ---------------------------------------------------------------- source generation
std::string literal(double v, mx_dtype dt) {
    if (dt == MX_F32) v = (double)(float)v;  // rounded to the element type
    if (std::isnan(v)) return "((T)__builtin_nan(\"\"))";
    if (std::isinf(v)) return v > 0 ? "((T)__builtin_huge_val())" : "((T)-__builtin_huge_val())";
    char buf[64];
    std::snprintf(buf, sizeof buf, "((T)%a)", v);
    return buf;
}

// The body's forward values, one SSA name per instruction (v<k>); src_a /
// src_b receive the instruction that produced each operand (-1: none).
std::string forward_lines(const std::vector<mx_xinsn> &p, mx_dtype dt, std::vector<int> &src_a,
                          std::vector<int> &src_b, int &out_src, int out_reg) {
    std::string s;
    int last[kRegs];
    for (int &l : last) l = -1;
    const int n = (int)p.size();
    src_a.assign(n, -1);
    src_b.assign(n, -1);
    auto v = [](int k) { return "v" + std::to_string(k); };
    for (int k = 0; k < n; ++k) {
        const mx_xinsn &q = p[k];
        if (reads_a(q.op)) src_a[k] = last[q.a];
        if (reads_b(q.op)) src_b[k] = last[q.b];
        const std::string a = reads_a(q.op) ? v(src_a[k]) : "", b = reads_b(q.op) ? v(src_b[k]) : "";
        std::string e;
        switch (q.op) {
        case MX_X_IN: e = "x" + std::to_string(q.a); break;
        case MX_X_CONST: e = literal(q.imm, dt); break;
        case MX_X_ADD: e = a + " + " + b; break;
        case MX_X_SUB: e = a + " - " + b; break;
        case MX_X_MUL: e = a + " * " + b; break;
        case MX_X_DIV: e = a + " / " + b; break;
        case MX_X_MIN: e = "(" + b + " < " + a + " ? " + b + " : " + a + ")"; break;
        case MX_X_MAX: e = "(" + b + " > " + a + " ? " + b + " : " + a + ")"; break;
        case MX_X_NEG: e = "-" + a; break;
        case MX_X_ABS: e = "(" + a + " < (T)0 ? -" + a + " : " + a + ")"; break;
        case MX_X_SQ: e = a + " * " + a; break;
        case MX_X_EXP: e = "exp(" + a + ")"; break;
        case MX_X_LOG: e = "log(" + a + ")"; break;
        case MX_X_SQRT: e = "sqrt(" + a + ")"; break;
        case MX_X_RSQRT: e = "(T)1 / sqrt(" + a + ")"; break;
        }
        s += "    const T " + v(k) + " = " + e + ";\n";
        last[q.dst] = k;
    }
    out_src = last[out_reg];
    return s;
}

std::string gen_source(const mx_expr &e) {
    const bool f32 = e.dtype == MX_F32;
    std::vector<int> sa, sb;
    int os = -1;
    const std::string fwd = forward_lines(e.prog, e.dtype, sa, sb, os, e.out_reg);
    const int n = (int)e.prog.size();

    // Reverse sweep.  Every SSA value k that the output can reach carries an
    // adjoint g<k> and a predicate r<k>: whether the output reaches it at
    // this element.  min / max pass their adjoint to the operand they
    // returned only, so which values are reached depends on the data; a term
    // is selected into an adjoint under its predicate rather than multiplied
    // by zero, so a subtree that is not reached (a log or a quotient at a
    // pole behind the branch not taken) contributes nothing, not 0 * inf.
    // Where no min / max lies on the way, the predicates are constants and
    // fold away.
    std::string rev;
    std::vector<char> declared(n, 0);
    auto g = [](int k) { return "g" + std::to_string(k); };
    auto r = [](int k) { return "r" + std::to_string(k); };
    auto v = [](int k) { return "v" + std::to_string(k); };
    // adjoint j gains term under predicate cond
    auto add_term = [&](int j, const std::string &cond, const std::string &term) {
        if (j < 0) return;
        if (!declared[j]) {
            rev += "    T " + g(j) + " = (T)0;\n    bool " + r(j) + " = false;\n";
            declared[j] = 1;
        }
        rev += "    if (" + cond + ") { " + g(j) + " = " + r(j) + " ? " + g(j) + " + " + term + " : " + term + "; " +
               r(j) + " = true; }\n";
    };
    rev += "    T " + g(os) + " = seed;\n    bool " + r(os) + " = true;\n";
    declared[os] = 1;
    bool gin_decl[kMaxIn] = {false, false, false, false};
    for (int k = n - 1; k >= 0; --k) {
        if (!declared[k]) continue;
        const mx_xinsn &q = e.prog[k];
        const std::string gk = g(k), vk = v(k), rk = r(k);
        const std::string va = sa[k] >= 0 ? v(sa[k]) : "", vb = sb[k] >= 0 ? v(sb[k]) : "";
        switch (q.op) {
        case MX_X_IN: {
            const std::string gi = "gi" + std::to_string(q.a), ri = "ri" + std::to_string(q.a);
            if (!gin_decl[q.a]) {
                rev += "    bool " + ri + " = false;\n";
                gin_decl[q.a] = true;
            }
            rev += "    if (" + rk + ") { " + gi + " = " + ri + " ? " + gi + " + " + gk + " : " + gk + "; " + ri +
                   " = true; }\n";
            break;
        }
        case MX_X_CONST: break;
        case MX_X_ADD: add_term(sa[k], rk, gk); add_term(sb[k], rk, gk); break;
        case MX_X_SUB: add_term(sa[k], rk, gk); add_term(sb[k], rk, "(-" + gk + ")"); break;
        case MX_X_MUL:
            add_term(sa[k], rk, "(" + gk + " * " + vb + ")");
            add_term(sb[k], rk, "(" + gk + " * " + va + ")");
            break;
        case MX_X_DIV:
            add_term(sa[k], rk, "(" + gk + " / " + vb + ")");
            add_term(sb[k], rk, "(-(" + gk + " * " + vk + " / " + vb + "))");
            break;
        case MX_X_MIN:
            add_term(sa[k], rk + " && !(" + vb + " < " + va + ")", gk);
            add_term(sb[k], rk + " && (" + vb + " < " + va + ")", gk);
            break;
        case MX_X_MAX:
            add_term(sa[k], rk + " && !(" + vb + " > " + va + ")", gk);
            add_term(sb[k], rk + " && (" + vb + " > " + va + ")", gk);
            break;
        case MX_X_NEG: add_term(sa[k], rk, "(-" + gk + ")"); break;
        case MX_X_ABS: add_term(sa[k], rk, "(" + va + " < (T)0 ? -" + gk + " : " + gk + ")"); break;
        case MX_X_SQ: add_term(sa[k], rk, "(" + gk + " * (" + va + " + " + va + "))"); break;
        case MX_X_EXP: add_term(sa[k], rk, "(" + gk + " * " + vk + ")"); break;
        case MX_X_LOG: add_term(sa[k], rk, "(" + gk + " / " + va + ")"); break;
        case MX_X_SQRT: add_term(sa[k], rk, "(" + gk + " / (" + vk + " + " + vk + "))"); break;
        case MX_X_RSQRT: add_term(sa[k], rk, "(-(" + gk + " * " + vk + " * " + vk + " * " + vk + ") * (T)0.5)"); break;
        }
    }

    std::string in_params;
    for (int k = 0; k < kMaxIn; ++k) in_params += std::string(k ? ", " : "") + "const T x" + std::to_string(k);

    std::string s;
    s += "// generated by the mx library from a straight-line map body\n";
    s += f32 ? "typedef float T;\ntypedef float4 VT;\n#define VW 4\n" : "typedef double T;\ntypedef double2 VT;\n#define VW 2\n";
    s += "#define NT " + std::to_string(NT) + "\n#define GPI " + std::to_string(kGroupsPerIt) + "\n";
    s += "#define NIN " + std::to_string(e.nin) + "\n";
    s += "#define SU (NIN >= 4 ? 2 : NIN >= 2 ? 4 : 8)\n";  // 16-byte groups per input in flight per lane
    s += "__device__ __forceinline__ T mx_body(" + in_params + ") {\n#pragma clang fp contract(off)\n" + fwd +
         "    return v" + std::to_string(os) + ";\n}\n";
    s += "__device__ __forceinline__ void mx_body_vjp(" + in_params +
         ", const T seed, T &gi0, T &gi1, T &gi2, T &gi3) {\n#pragma clang fp contract(off)\n" + fwd +
         "    gi0 = (T)0; gi1 = (T)0; gi2 = (T)0; gi3 = (T)0;\n" + rev + "}\n";
    s += R"(
__device__ __forceinline__ T mx_vget(const VT &v, int j) { return reinterpret_cast<const T *>(&v)[j]; }
__device__ __forceinline__ void mx_vset(VT &v, int j, T x) { reinterpret_cast<T *>(&v)[j] = x; }
#define MX_PTRS const T *__restrict__ p0, const T *__restrict__ p1, const T *__restrict__ p2, const T *__restrict__ p3
#define MX_VPTRS const VT *q0 = (const VT *)p0, *q1 = (const VT *)p1, *q2 = (const VT *)p2, *q3 = (const VT *)p3

// group j of VW elements of every input, read only for the inputs that exist
__device__ __forceinline__ void mx_load_group(MX_PTRS, long long j, VT (&a)[4]) {
    MX_VPTRS;
    if (NIN > 0) a[0] = q0[j];
    if (NIN > 1) a[1] = q1[j];
    if (NIN > 2) a[2] = q2[j];
    if (NIN > 3) a[3] = q3[j];
}
__device__ __forceinline__ T mx_body_at(const VT (&a)[4], int e) {
    return mx_body(NIN > 0 ? mx_vget(a[0], e) : (T)0, NIN > 1 ? mx_vget(a[1], e) : (T)0,
                   NIN > 2 ? mx_vget(a[2], e) : (T)0, NIN > 3 ? mx_vget(a[3], e) : (T)0);
}
__device__ __forceinline__ T mx_body_i(MX_PTRS, long long i) {
    return mx_body(NIN > 0 ? p0[i] : (T)0, NIN > 1 ? p1[i] : (T)0, NIN > 2 ? p2[i] : (T)0, NIN > 3 ? p3[i] : (T)0);
}

// out[i] = body(x_i).  vec: every pointer 16-byte aligned; then groups of VW
// elements, GPI groups in flight per thread, the tail element by element.
extern "C" __global__ void __launch_bounds__(NT) mx_xmap(MX_PTRS, T *__restrict__ out, long long n, int vec) {
    const long long tid = (long long)blockIdx.x * NT + threadIdx.x, nt = (long long)gridDim.x * NT;
    long long done = 0;
    if (vec) {
        const long long nv = n / VW;
        VT *qo = (VT *)out;
        long long j = tid;
        for (; j + (GPI - 1) * nt < nv; j += GPI * nt) {
            VT a[GPI][4];
#pragma unroll
            for (int u = 0; u < GPI; ++u) mx_load_group(p0, p1, p2, p3, j + u * nt, a[u]);
#pragma unroll
            for (int u = 0; u < GPI; ++u) {
                VT r;
#pragma unroll
                for (int e = 0; e < VW; ++e) mx_vset(r, e, mx_body_at(a[u], e));
                qo[j + u * nt] = r;
            }
        }
        for (; j < nv; j += nt) {
            VT a[4];
            mx_load_group(p0, p1, p2, p3, j, a);
            VT r;
#pragma unroll
            for (int e = 0; e < VW; ++e) mx_vset(r, e, mx_body_at(a, e));
            qo[j] = r;
        }
        done = nv * VW;
    }
    for (long long i = done + tid; i < n; i += nt) out[i] = mx_body_i(p0, p1, p2, p3, i);
}

// Reverse mode: gk[i] = seed_i * d body / d input k (null outputs skipped).
extern "C" __global__ void __launch_bounds__(NT) mx_xvjp(MX_PTRS, const T *__restrict__ gout,
                                                           const T *__restrict__ gscale, T *__restrict__ g0,
                                                           T *__restrict__ g1, T *__restrict__ g2,
                                                           T *__restrict__ g3, long long n, int vec) {
    const long long tid = (long long)blockIdx.x * NT + threadIdx.x, nt = (long long)gridDim.x * NT;
    const bool hg = gout != nullptr, hs = gscale != nullptr;
    const T gs = hs ? *gscale : (T)1;
    long long done = 0;
    if (vec) {
        const long long nv = n / VW;
        const VT *qg = (const VT *)gout;
        VT *r0 = (VT *)g0, *r1 = (VT *)g1, *r2 = (VT *)g2, *r3 = (VT *)g3;
        for (long long j = tid; j < nv; j += nt) {
            VT a[4];
            mx_load_group(p0, p1, p2, p3, j, a);
            VT go;
            if (hg) go = qg[j];
            VT o0, o1, o2, o3;
#pragma unroll
            for (int e = 0; e < VW; ++e) {
                const T seed = hg ? (hs ? mx_vget(go, e) * gs : mx_vget(go, e)) : gs;
                T d0, d1, d2, d3;
                mx_body_vjp(NIN > 0 ? mx_vget(a[0], e) : (T)0, NIN > 1 ? mx_vget(a[1], e) : (T)0,
                            NIN > 2 ? mx_vget(a[2], e) : (T)0, NIN > 3 ? mx_vget(a[3], e) : (T)0, seed, d0, d1,
                            d2, d3);
                mx_vset(o0, e, d0); mx_vset(o1, e, d1); mx_vset(o2, e, d2); mx_vset(o3, e, d3);
            }
            if (r0) r0[j] = o0;
            if (r1) r1[j] = o1;
            if (r2) r2[j] = o2;
            if (r3) r3[j] = o3;
        }
        done = nv * VW;
    }
    for (long long i = done + tid; i < n; i += nt) {
        const T seed = hg ? (hs ? gout[i] * gs : gout[i]) : gs;
        T d0, d1, d2, d3;
        mx_body_vjp(NIN > 0 ? p0[i] : (T)0, NIN > 1 ? p1[i] : (T)0, NIN > 2 ? p2[i] : (T)0,
                    NIN > 3 ? p3[i] : (T)0, seed, d0, d1, d2, d3);
        if (g0) g0[i] = d0;
        if (g1) g1[i] = d1;
        if (g2) g2[i] = d2;
        if (g3) g3[i] = d3;
    }
}

// loop n (\i -> out[idx[i]] = body(x_i)): one slot per iteration, slots
// outside [0, out_len) never written
extern "C" __global__ void __launch_bounds__(NT) mx_xscatter(MX_PTRS, const long long *__restrict__ idx,
                                                               T *__restrict__ out, long long n, long long out_len) {
    const long long tid = (long long)blockIdx.x * NT + threadIdx.x, nt = (long long)gridDim.x * NT;
    for (long long i = tid; i < n; i += nt) {
        const long long j = idx[i];
        const T v = mx_body_i(p0, p1, p2, p3, i);
        if (j >= 0 && j < out_len) out[j] = v;
    }
}
)";
    // fused map + reduce, one pair of kernels per operator
    const char *ops[4][3] = {{"add", "a + b", "(T)0"},
                             {"mul", "a * b", "(T)1"},
                             {"min", "(b < a ? b : a)", "((T)__builtin_huge_val())"},
                             {"max", "(b > a ? b : a)", "((T)-__builtin_huge_val())"}};
    for (auto &o : ops) {
        const std::string nm = o[0], ap = o[1], id = o[2];
        s += "__device__ __forceinline__ T mx_op_" + nm + "(T a, T b) {\n#pragma clang fp contract(off)\n    return " +
             ap + ";\n}\n";
        s += "__device__ __forceinline__ T mx_block_" + nm + R"((T v, T *sh) {
    // fixed tree over the wave, then the waves in order
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = mx_op_)" + nm + R"((v, __shfl_xor(v, o, 64));
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    T r = sh[0];
#pragma unroll
    for (int w = 1; w < NT / 64; ++w) r = mx_op_)" + nm + R"((r, sh[w]);
    return r;
}
// each thread folds its elements in a fixed order; one partial per block
extern "C" __global__ void __launch_bounds__(NT) mx_xred_)" + nm + R"((MX_PTRS, long long n, int vec, T *__restrict__ partial) {
    __shared__ T sh[NT / 64];
    const long long tid = (long long)blockIdx.x * NT + threadIdx.x, nt = (long long)gridDim.x * NT;
    T acc = )" + id + R"(;
    long long done = 0;
    if (vec) {
        const long long nv = n / VW;
        long long j = tid;
        for (; j + (GPI - 1) * nt < nv; j += GPI * nt) {
            VT a[GPI][4];
#pragma unroll
            for (int u = 0; u < GPI; ++u) mx_load_group(p0, p1, p2, p3, j + u * nt, a[u]);
#pragma unroll
            for (int u = 0; u < GPI; ++u)
#pragma unroll
                for (int e = 0; e < VW; ++e) acc = mx_op_)" + nm + R"((acc, mx_body_at(a[u], e));
        }
        for (; j < nv; j += nt) {
            VT a[4];
            mx_load_group(p0, p1, p2, p3, j, a);
#pragma unroll
            for (int e = 0; e < VW; ++e) acc = mx_op_)" + nm + R"((acc, mx_body_at(a, e));
        }
        done = nv * VW;
    }
    for (long long i = done + tid; i < n; i += nt) acc = mx_op_)" + nm + R"((acc, mx_body_i(p0, p1, p2, p3, i));
    const T r = mx_block_)" + nm + R"((acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = r;
}
// the partials in block order (thread t takes t, t + NT, ...), then ne op total
extern "C" __global__ void __launch_bounds__(NT) mx_xfin_)" + nm + R"((const T *__restrict__ partial, int nb, T ne, T *__restrict__ out) {
    __shared__ T sh[NT / 64];
    T acc = )" + id + R"(;
    for (int b = threadIdx.x; b < nb; b += NT) acc = mx_op_)" + nm + R"((acc, partial[b]);
    const T r = mx_block_)" + nm + R"((acc, sh);
    if (threadIdx.x == 0) *out = mx_op_)" + nm + R"((ne, r);
}
// Nested map (reduce op ne . map body) over ragged rows sharing `offsets`: a
// block takes rb consecutive rows (one contiguous span of elements), its four
// waves take contiguous quarters of the span's 16-byte groups, lanes
// interleaved; a thread folds the body values it visits into its current row
// (positions only increase, so rows never go back) and parks finished rows in
// its own LDS slot; each row's NT slots are then folded in a fixed order.
extern "C" __global__ void __launch_bounds__(NT) mx_xseg_)" + nm + R"((MX_PTRS, const long long *__restrict__ offsets,
                                                              long long nseg, int rb, T ne, T *__restrict__ out,
                                                              int vec) {
    extern __shared__ __attribute__((aligned(16))) unsigned char mx_lds[];
    long long *soff = (long long *)mx_lds;
    T *slot = (T *)(mx_lds + (((long long)(rb + 1) * 8 + 15) & ~15LL));
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const long long r0 = (long long)blockIdx.x * rb;
    const int nrows = (int)(nseg - r0 < rb ? nseg - r0 : rb);
    if (t <= nrows) soff[t] = offsets[r0 + t];
    for (int k = 0; k < nrows; ++k) slot[k * NT + t] = )" + id + R"(;
    __syncthreads();
    const long long S = soff[0], E = soff[nrows];
    int cur = 0;
    long long end = soff[1];
    T a = )" + id + R"(;
    auto take = [&](long long p, T x) {
        while (p >= end) {
            slot[cur * NT + t] = a;
            a = )" + id + R"(;
            ++cur;
            end = soff[cur + 1];
        }
        a = mx_op_)" + nm + R"((a, x);
    };
    // row (within the block) holding position p: row ends at or before p, one ballot
    auto row_of = [&](long long p) {
        const bool past = lane < nrows && soff[lane + 1] <= p;
        return __popcll(__ballot(past));
    };
    if (vec) {
        const long long vs = (S + VW - 1) / VW, ve = E / VW > vs ? E / VW : vs;
        const long long head_end = vs * VW < E ? vs * VW : E;
        const long long q = (ve - vs + 3) / 4;
        const long long cs = vs + w * q < ve ? vs + w * q : ve;
        const long long ce = cs + q < ve ? cs + q : ve;
        if (w == 0) {
            if (S + lane < head_end) take(S + lane, mx_body_i(p0, p1, p2, p3, S + lane));
        } else if (cs < ce) {
            cur = row_of(cs * VW);
            end = soff[cur + 1];
        }
        for (long long i = cs + lane; i < ce; i += SU * 64) {
            VT x[SU][4];
#pragma unroll
            for (int u = 0; u < SU; ++u)
                if (i + u * 64 < ce) mx_load_group(p0, p1, p2, p3, i + u * 64, x[u]);
#pragma unroll
            for (int u = 0; u < SU; ++u) {
                if (i + u * 64 < ce) {
                    const long long q0 = (i + u * 64) * VW;
                    if (q0 + VW - 1 < end) {
#pragma unroll
                        for (int j = 0; j < VW; ++j) a = mx_op_)" + nm + R"((a, mx_body_at(x[u], j));
                    } else {
#pragma unroll
                        for (int j = 0; j < VW; ++j) take(q0 + j, mx_body_at(x[u], j));
                    }
                }
            }
        }
        if (w == 3) {
            const long long tail_start = ve * VW > head_end ? ve * VW : head_end;
            if (cs >= ce && tail_start < E) {
                cur = row_of(tail_start);
                end = soff[cur + 1];
            }
            if (tail_start + lane < E) take(tail_start + lane, mx_body_i(p0, p1, p2, p3, tail_start + lane));
        }
    } else {
        for (long long i = S + t; i < E; i += NT) take(i, mx_body_i(p0, p1, p2, p3, i));
    }
    slot[cur * NT + t] = a;
    __syncthreads();
    for (int k = w; k < nrows; k += NT / 64) {
        T v = slot[k * NT + lane];
#pragma unroll
        for (int qq = 1; qq < NT / 64; ++qq) v = mx_op_)" + nm + R"((v, slot[k * NT + qq * 64 + lane]);
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) v = mx_op_)" + nm + R"((v, __shfl_xor(v, o, 64));
        if (lane == 0) out[r0 + k] = mx_op_)" + nm + R"((ne, v);
    }
}
)";
    }
    return s;
}

// ---------------------------------------------------------------- compiled modules
struct Compiled {
    hipModule_t mod = nullptr;
    hipFunction_t map = nullptr, vjp = nullptr, scatter = nullptr, red[4] = {}, fin[4] = {}, seg[4] = {};
};

std::mutex g_mu;
std::unordered_map<std::string, std::unique_ptr<Compiled>> g_cache;  // key: device + source

mx_status compile(const mx_expr &e, const Compiled **out) {
    int dev = 0;
    MX_TRY_HIP(hipGetDevice(&dev));
    const std::string key = std::to_string(dev) + "\n" + e.src;
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_cache.find(key);
    if (it != g_cache.end()) {
        *out = it->second.get();
        return MX_OK;
    }
    hipModule_t mod = nullptr;
    if (mx_status st = rtc_module(e.src, "mx_expr.hip", &mod)) return st;
    auto c = std::make_unique<Compiled>();
    c->mod = mod;
    MX_TRY_HIP(hipModuleGetFunction(&c->map, c->mod, "mx_xmap"));
    MX_TRY_HIP(hipModuleGetFunction(&c->vjp, c->mod, "mx_xvjp"));
    MX_TRY_HIP(hipModuleGetFunction(&c->scatter, c->mod, "mx_xscatter"));
    const char *nm[4] = {"add", "mul", "min", "max"};
    for (int o = 0; o < 4; ++o) {
        MX_TRY_HIP(hipModuleGetFunction(&c->red[o], c->mod, (std::string("mx_xred_") + nm[o]).c_str()));
        MX_TRY_HIP(hipModuleGetFunction(&c->fin[o], c->mod, (std::string("mx_xfin_") + nm[o]).c_str()));
        MX_TRY_HIP(hipModuleGetFunction(&c->seg[o], c->mod, (std::string("mx_xseg_") + nm[o]).c_str()));
    }
    *out = c.get();
    g_cache.emplace(key, std::move(c));
    return MX_OK;
}

mx_status launch(hipFunction_t f, int64_t blocks, hipStream_t s, void **args, const char *what,
                 unsigned lds = 0) {
    MX_TRY_HIP(hipModuleLaunchKernel(f, (unsigned)blocks, 1, 1, NT, 1, 1, lds, s, args, nullptr));
    (void)what;
    return MX_OK;
}

bool aligned16(const void *p) { return ((uintptr_t)p & 15) == 0; }

int64_t stream_blocks(int64_t n, int vw, int num_cus) {
    const int64_t b = ceil_div(n > 0 ? n : 1, (int64_t)NT * vw * kGroupsPerIt);
    const int64_t cap = (int64_t)num_cus * 8;
    return b < 1 ? 1 : (b > cap ? cap : b);
}

// the partial pass's grid depends only on n, so the result does not depend on the device
int64_t reduce_blocks(int64_t n, int vw) {
    const int64_t b = ceil_div(n > 0 ? n : 1, (int64_t)NT * vw * kGroupsPerIt);
    return b > kMaxRedBlocks ? kMaxRedBlocks : b;
}

// Debug mode of the indexed-write loop: every index in range and no slot hit
// twice.  counts[j] = number of iterations writing slot j (integer atomics).
__global__ void __launch_bounds__(NT) k_zero_u32(uint32_t *__restrict__ p, int64_t m) {
    const int64_t stride = (int64_t)gridDim.x * NT;
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < m; i += stride) p[i] = 0u;
}
__global__ void __launch_bounds__(NT) k_scatter_check(const long long *__restrict__ idx, int64_t n, int64_t out_len,
                                                      uint32_t *__restrict__ counts, uint32_t *__restrict__ flag) {
    const int64_t stride = (int64_t)gridDim.x * NT;
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += stride) {
        const long long j = idx[i];
        if (j < 0 || j >= out_len) atomicOr(flag, 1u);
        else if (atomicAdd(&counts[j], 1u) != 0u) atomicOr(flag, 2u);
    }
}

mx_status check_inputs(const mx_expr *e, const void *const *in_dev, int64_t n, const char *who) {
    MX_REQUIRE(e, MX_ERR_INVALID, "%s: null expression", who);
    MX_REQUIRE(n >= 0, MX_ERR_SHAPE, "%s: n < 0", who);
    MX_REQUIRE(in_dev || n == 0, MX_ERR_INVALID, "%s: null input list", who);
    if (n > 0)
        for (int k = 0; k < e->nin; ++k) MX_REQUIRE(in_dev[k], MX_ERR_INVALID, "%s: input %d is null", who, k);
    return MX_OK;
}

}  // namespace
}  // namespace mx

using namespace mx;

extern "C" {

mx_status mx_expr_create(const mx_xinsn *prog, int ninsn, int nin, int out_reg, mx_dtype dtype, mx_expr **out) {
    const char *who = "mx_expr_create";
    MX_REQUIRE(out, MX_ERR_INVALID, "%s: null output handle", who);
    *out = nullptr;
    MX_REQUIRE(prog, MX_ERR_INVALID, "%s: null program", who);
    MX_REQUIRE(ninsn >= 1 && ninsn <= kMaxInsn, MX_ERR_INVALID, "%s: need 1..%d instructions", who, kMaxInsn);
    MX_REQUIRE(nin >= 1 && nin <= kMaxIn, MX_ERR_INVALID, "%s: need 1..%d inputs", who, kMaxIn);
    MX_REQUIRE(out_reg >= 0 && out_reg < kRegs, MX_ERR_INVALID, "%s: out_reg %d out of range", who, out_reg);
    MX_REQUIRE(dtype == MX_F32 || dtype == MX_F64, MX_ERR_DTYPE, "%s: dtype must be MX_F32 or MX_F64", who);
    bool written[kRegs] = {};
    for (int k = 0; k < ninsn; ++k) {
        const mx_xinsn &q = prog[k];
        MX_REQUIRE(q.op >= MX_X_IN && q.op <= MX_X_RSQRT, MX_ERR_INVALID, "%s: instruction %d: bad op %d", who, k,
                   (int)q.op);
        MX_REQUIRE(q.dst >= 0 && q.dst < kRegs, MX_ERR_INVALID, "%s: instruction %d: bad dst", who, k);
        if (q.op == MX_X_IN)
            MX_REQUIRE(q.a >= 0 && q.a < nin, MX_ERR_INVALID, "%s: instruction %d: input %d of %d", who, k,
                       (int)q.a, nin);
        if (reads_a(q.op))
            MX_REQUIRE(q.a >= 0 && q.a < kRegs && written[q.a], MX_ERR_INVALID,
                       "%s: instruction %d reads r%d before it is written", who, k, (int)q.a);
        if (reads_b(q.op))
            MX_REQUIRE(q.b >= 0 && q.b < kRegs && written[q.b], MX_ERR_INVALID,
                       "%s: instruction %d reads r%d before it is written", who, k, (int)q.b);
        written[q.dst] = true;
    }
    MX_REQUIRE(written[out_reg], MX_ERR_INVALID, "%s: out_reg r%d is never written", who, out_reg);
    auto *e = new (std::nothrow) mx_expr;
    MX_REQUIRE(e, MX_ERR_INVALID, "%s: out of host memory", who);
    e->prog.assign(prog, prog + ninsn);
    e->nin = nin;
    e->out_reg = out_reg;
    e->dtype = dtype;
    e->src = gen_source(*e);
    *out = e;
    return MX_OK;
}

mx_status mx_expr_destroy(mx_expr *e) {
    delete e;
    return MX_OK;
}

const char *mx_expr_source(const mx_expr *e) { return e ? e->src.c_str() : nullptr; }

mx_status mx_expr_prepare(mx_expr *e) {
    MX_REQUIRE(e, MX_ERR_INVALID, "mx_expr_prepare: null expression");
    const Compiled *c;
    return compile(*e, &c);
}

mx_status mx_expr_map(mx_expr *e, const void *const *in_dev, int64_t n, void *out_dev, hipStream_t stream) {
    const char *who = "mx_expr_map";
    if (mx_status st = check_inputs(e, in_dev, n, who)) return st;
    MX_REQUIRE(out_dev || n == 0, MX_ERR_INVALID, "%s: null output", who);
    if (n == 0) return MX_OK;
    const Compiled *c;
    if (mx_status st = compile(*e, &c)) return st;
    const DeviceInfo *dv;
    if (mx_status st = device_info(&dv)) return st;
    const void *p[kMaxIn] = {};
    bool al = aligned16(out_dev);
    for (int k = 0; k < e->nin; ++k) {
        p[k] = in_dev[k];
        al = al && aligned16(p[k]);
    }
    const int vw = e->dtype == MX_F32 ? 4 : 2;
    int vec = al ? 1 : 0;
    long long nn = n;
    void *args[] = {&p[0], &p[1], &p[2], &p[3], &out_dev, &nn, &vec};
    return launch(c->map, stream_blocks(n, vw, dv->num_cus), stream, args, who);
}

size_t mx_expr_workspace_bytes(const mx_expr *e, int64_t n) {
    (void)n;
    if (!e) return 0;
    return align256(kCounterBytes + (size_t)kMaxRedBlocks * dtype_size(e->dtype));
}

mx_status mx_expr_map_reduce(mx_expr *e, mx_redop op, const void *const *in_dev, int64_t n, const void *ne_host,
                             void *out_dev, void *ws, size_t ws_bytes, hipStream_t stream) {
    const char *who = "mx_expr_map_reduce";
    if (mx_status st = check_inputs(e, in_dev, n, who)) return st;
    MX_REQUIRE(op >= MX_ADD && op <= MX_MAX, MX_ERR_INVALID, "%s: bad reduce operator %d", who, (int)op);
    MX_REQUIRE(ne_host && out_dev, MX_ERR_INVALID, "%s: null ne or output", who);
    const size_t need = mx_expr_workspace_bytes(e, n);
    MX_REQUIRE(ws && ws_bytes >= need && ((uintptr_t)ws & 255) == 0, MX_ERR_WORKSPACE,
               "%s: workspace needs %zu bytes, 256-byte aligned", who, need);
    const Compiled *c;
    if (mx_status st = compile(*e, &c)) return st;
    const void *p[kMaxIn] = {};
    bool al = true;
    for (int k = 0; k < e->nin && n > 0; ++k) {
        p[k] = in_dev[k];
        al = al && aligned16(p[k]);
    }
    const int vw = e->dtype == MX_F32 ? 4 : 2;
    int vec = al ? 1 : 0;
    long long nn = n;
    void *partial = (char *)ws + kCounterBytes;
    const int64_t nb = n > 0 ? reduce_blocks(n, vw) : 0;
    if (nb > 0) {
        void *args[] = {&p[0], &p[1], &p[2], &p[3], &nn, &vec, &partial};
        if (mx_status st = launch(c->red[op], nb, stream, args, who)) return st;
    }
    int nbi = (int)nb;
    if (e->dtype == MX_F32) {
        float ne = *(const float *)ne_host;
        void *args[] = {&partial, &nbi, &ne, &out_dev};
        return launch(c->fin[op], 1, stream, args, who);
    }
    double ne = *(const double *)ne_host;
    void *args[] = {&partial, &nbi, &ne, &out_dev};
    return launch(c->fin[op], 1, stream, args, who);
}

mx_status mx_expr_segmented_reduce(mx_expr *e, mx_redop op, const void *const *in_dev, const int64_t *offsets_dev,
                                   int64_t nseg, const void *ne_host, void *out_dev, hipStream_t stream) {
    const char *who = "mx_expr_segmented_reduce";
    MX_REQUIRE(e, MX_ERR_INVALID, "%s: null expression", who);
    MX_REQUIRE(nseg >= 0, MX_ERR_SHAPE, "%s: nseg < 0", who);
    MX_REQUIRE(op >= MX_ADD && op <= MX_MAX, MX_ERR_INVALID, "%s: bad reduce operator %d", who, (int)op);
    if (nseg == 0) return MX_OK;
    MX_REQUIRE(in_dev && offsets_dev && ne_host && out_dev, MX_ERR_INVALID, "%s: null pointer", who);
    for (int k = 0; k < e->nin; ++k) MX_REQUIRE(in_dev[k], MX_ERR_INVALID, "%s: input %d is null", who, k);
    if (debug_mode())
        if (mx_status st = check_offsets_debug(who, offsets_dev, nseg, stream)) return st;
    const Compiled *c;
    if (mx_status st = compile(*e, &c)) return st;
    const DeviceInfo *dv;
    if (mx_status st = device_info(&dv)) return st;
    const void *p[kMaxIn] = {};
    bool al = true;
    for (int k = 0; k < e->nin; ++k) {
        p[k] = in_dev[k];
        al = al && aligned16(p[k]);
    }
    const int rb = segmented_rows_per_block(nseg, dv);
    const int64_t grid = ceil_div(nseg, rb);
    MX_REQUIRE(grid <= 0x7fffffff, MX_ERR_SHAPE, "%s: too many rows", who);
    const unsigned lds = (unsigned)((((size_t)rb + 1) * 8 + 15) / 16 * 16 + (size_t)rb * NT * dtype_size(e->dtype));
    int vec = al ? 1 : 0, rbi = rb;
    long long ns = nseg;
    const void *off = offsets_dev;
    if (e->dtype == MX_F32) {
        float ne = *(const float *)ne_host;
        void *args[] = {&p[0], &p[1], &p[2], &p[3], &off, &ns, &rbi, &ne, &out_dev, &vec};
        return launch(c->seg[op], grid, stream, args, who, lds);
    }
    double ne = *(const double *)ne_host;
    void *args[] = {&p[0], &p[1], &p[2], &p[3], &off, &ns, &rbi, &ne, &out_dev, &vec};
    return launch(c->seg[op], grid, stream, args, who, lds);
}

size_t mx_expr_loop_workspace_bytes(int64_t out_len) {
    if (out_len < 0) return 0;
    return align256(kCounterBytes + (size_t)out_len * sizeof(uint32_t));
}

mx_status mx_expr_loop_scatter(mx_expr *e, const void *const *in_dev, int64_t n, const int64_t *index_dev,
                               void *out_dev, int64_t out_len, void *ws, size_t ws_bytes, hipStream_t stream) {
    const char *who = "mx_expr_loop_scatter";
    if (mx_status st = check_inputs(e, in_dev, n, who)) return st;
    MX_REQUIRE(out_len >= 0, MX_ERR_SHAPE, "%s: out_len < 0", who);
    if (n == 0) return MX_OK;
    MX_REQUIRE(index_dev && (out_dev || out_len == 0), MX_ERR_INVALID, "%s: null index or output", who);
    const DeviceInfo *dv;
    if (mx_status st = device_info(&dv)) return st;
    const int grid = (int)stream_blocks(n, 1, dv->num_cus);
    if (debug_mode()) {
        const size_t need = mx_expr_loop_workspace_bytes(out_len);
        MX_REQUIRE(ws && ws_bytes >= need && ((uintptr_t)ws & 255) == 0, MX_ERR_WORKSPACE,
                   "%s: debug mode needs a workspace of %zu bytes, 256-byte aligned", who, need);
        uint32_t *flag = (uint32_t *)ws, *counts = (uint32_t *)((char *)ws + kCounterBytes);
        hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(NT), 0, stream, flag, (int64_t)1);
        if (out_len > 0)
            hipLaunchKernelGGL(k_zero_u32, dim3((unsigned)stream_blocks(out_len, 1, dv->num_cus)), dim3(NT), 0,
                               stream, counts, out_len);
        hipLaunchKernelGGL(k_scatter_check, dim3(grid), dim3(NT), 0, stream, (const long long *)index_dev, n,
                           out_len, counts, flag);
        if (mx_status st = last_launch(who)) return st;
        uint32_t h = 0;
        MX_TRY_HIP(hipMemcpyAsync(&h, flag, sizeof h, hipMemcpyDeviceToHost, stream));
        MX_TRY_HIP(hipStreamSynchronize(stream));
        MX_REQUIRE(!(h & 1u), MX_ERR_SHAPE, "%s: an index is outside [0, %lld)", who, (long long)out_len);
        MX_REQUIRE(!(h & 2u), MX_ERR_SHAPE, "%s: two iterations write the same slot", who);
    }
    const Compiled *c;
    if (mx_status st = compile(*e, &c)) return st;
    const void *p[kMaxIn] = {};
    for (int k = 0; k < e->nin; ++k) p[k] = in_dev[k];
    long long nn = n, ol = out_len;
    const void *ix = index_dev;
    void *args[] = {&p[0], &p[1], &p[2], &p[3], &ix, &out_dev, &nn, &ol};
    return launch(c->scatter, grid, stream, args, who);
}

mx_status mx_expr_vjp(mx_expr *e, const void *const *in_dev, int64_t n, const void *gout_dev,
                      const void *gscale_dev, void *const *gin_dev, hipStream_t stream) {
    const char *who = "mx_expr_vjp";
    if (mx_status st = check_inputs(e, in_dev, n, who)) return st;
    MX_REQUIRE(gin_dev, MX_ERR_INVALID, "%s: null gradient list", who);
    if (n == 0) return MX_OK;
    const Compiled *c;
    if (mx_status st = compile(*e, &c)) return st;
    const DeviceInfo *dv;
    if (mx_status st = device_info(&dv)) return st;
    const void *p[kMaxIn] = {};
    void *gk[kMaxIn] = {};
    bool al = gout_dev == nullptr || aligned16(gout_dev);
    for (int k = 0; k < e->nin; ++k) {
        p[k] = in_dev[k];
        gk[k] = gin_dev[k];
        al = al && aligned16(p[k]) && (gk[k] == nullptr || aligned16(gk[k]));
    }
    const int vw = e->dtype == MX_F32 ? 4 : 2;
    int vec = al ? 1 : 0;
    long long nn = n;
    void *args[] = {&p[0], &p[1], &p[2], &p[3], &gout_dev, &gscale_dev, &gk[0], &gk[1], &gk[2], &gk[3], &nn, &vec};
    return launch(c->vjp, stream_blocks(n, vw, dv->num_cus), stream, args, who);
}

}  // extern "C"
