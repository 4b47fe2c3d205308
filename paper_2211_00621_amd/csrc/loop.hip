// The general parallel loop of the CUDA backend (Appendix A, Source
// Language): `loop n f` runs f i for every i in [0, n) in an undefined order,
// and f reads and writes tensors through tensorGet / tensorSet -- Listing 1's
// in-place axpy is one.  A loop body arrives as a straight-line program over
// an integer and a float register file; this file turns it into HIP source
// (one SSA value per instruction, the tensors' element types and ranks baked
// in), compiles it with hipRTC and launches one thread per iteration,
// grid-strided.
//
// The same body is generated three times, as a template on the mode: the
// run itself, and the two trace passes of debug mode, which write nothing:
// the first claims every slot an iteration sets (atomicCAS of the iteration
// number into a per-slot owner word: a second iteration finding the slot
// taken is a write-write conflict), the second checks every slot an
// iteration gets against those owners (a read-write conflict).  A trace pass
// keeps the iteration's own sets in registers, and a later get of the same
// slot takes the value from there, so the indices it computes are the ones
// the run computes.  Indices outside their dimension make a get yield 0 and
// a set write nothing in every mode; debug mode reports them.
#include <cinttypes>
#include <cmath>
#include <cstdio>
#include <mutex>
#include <string>
#include <vector>

#include "mx_internal.h"

struct mx_loop {
    std::vector<mx_linsn> prog;
    std::vector<mx_ltype> tensors;
    mx_dtype ftype = MX_F32;
    unsigned set_mask = 0;  // tensors the body sets
    std::string src;
    hipFunction_t fn[3] = {nullptr, nullptr, nullptr};
    int fn_device = -1;
    std::mutex mu;
};

namespace mx {
namespace {

constexpr int NT = 256;
constexpr int kRegs = 64, kMaxInsn = 256, kMaxTensors = 8;

bool is_int_type(mx_dtype d) { return d == MX_I32 || d == MX_I64; }
const char *elem_name(mx_dtype d) {
    switch (d) {
    case MX_F32: return "float";
    case MX_F64: return "double";
    case MX_I32: return "int";
    case MX_I64: return "long long";
    }
    return "?";
}
bool float_op(int op) { return op >= MX_X_CONST && op <= MX_X_RSQRT; }
bool float_binary(int op) { return op >= MX_X_ADD && op <= MX_X_MAX; }
bool int_binary(int op) { return op >= MX_L_IADD && op <= MX_L_IMAX; }
bool is_get(int op) { return op == MX_L_FGET || op == MX_L_IGET; }
bool is_set(int op) { return op == MX_L_FSET || op == MX_L_ISET; }

mx_status validate(const mx_linsn *p, int n, const mx_ltype *ts, int nt, mx_dtype ft) {
    MX_REQUIRE(n >= 1 && n <= kMaxInsn, MX_ERR_INVALID, "mx_loop_create: 1..%d instructions", kMaxInsn);
    MX_REQUIRE(nt >= 0 && nt <= kMaxTensors && (nt == 0 || ts), MX_ERR_INVALID, "mx_loop_create: 0..%d tensors",
               kMaxTensors);
    MX_REQUIRE(ft == MX_F32 || ft == MX_F64, MX_ERR_DTYPE, "mx_loop_create: the float type is F32 or F64");
    for (int t = 0; t < nt; ++t) {
        MX_REQUIRE(dtype_valid(ts[t].dtype), MX_ERR_DTYPE, "mx_loop_create: tensor %d: bad element type", t);
        MX_REQUIRE(ts[t].rank >= 1 && ts[t].rank <= 3, MX_ERR_INVALID, "mx_loop_create: tensor %d: rank 1..3", t);
    }
    auto reg = [](int r) { return r >= 0 && r < kRegs; };
    for (int k = 0; k < n; ++k) {
        const mx_linsn &q = p[k];
        const int op = q.op;
        const bool known = float_op(op) || (op >= MX_L_ITER && op <= MX_L_I2F) || is_get(op) || is_set(op);
        MX_REQUIRE(known, MX_ERR_INVALID, "mx_loop_create: instruction %d: unknown op %d", k, op);
        if (!is_set(op)) MX_REQUIRE(reg(q.dst), MX_ERR_INVALID, "mx_loop_create: instruction %d: bad dst", k);
        if (float_op(op) && op != MX_X_CONST) {
            MX_REQUIRE(reg(q.a) && (!float_binary(op) || reg(q.b)), MX_ERR_INVALID,
                       "mx_loop_create: instruction %d: bad operand", k);
        }
        if (int_binary(op)) MX_REQUIRE(reg(q.a) && reg(q.b), MX_ERR_INVALID, "mx_loop_create: instruction %d: bad operand", k);
        if (op == MX_L_INEG || op == MX_L_I2F) MX_REQUIRE(reg(q.a), MX_ERR_INVALID, "mx_loop_create: instruction %d: bad operand", k);
        if (is_get(op) || is_set(op)) {
            MX_REQUIRE(q.tensor >= 0 && q.tensor < nt, MX_ERR_INVALID, "mx_loop_create: instruction %d: no tensor %d",
                       k, q.tensor);
            const mx_ltype &tt = ts[q.tensor];
            const bool want_int = op == MX_L_IGET || op == MX_L_ISET;
            MX_REQUIRE(is_int_type(tt.dtype) == want_int, MX_ERR_DTYPE,
                       "mx_loop_create: instruction %d: tensor %d has the other element kind", k, q.tensor);
            MX_REQUIRE(reg(q.a) && (tt.rank < 2 || reg(q.b)) && (tt.rank < 3 || reg(q.c)), MX_ERR_INVALID,
                       "mx_loop_create: instruction %d: bad index register", k);
            if (is_set(op)) MX_REQUIRE(reg(q.src), MX_ERR_INVALID, "mx_loop_create: instruction %d: bad src", k);
        }
    }
    return MX_OK;
}

std::string ilit(int64_t v) {
    char buf[48];
    std::snprintf(buf, sizeof buf, "((long long)0x%" PRIx64 "ULL)", (uint64_t)v);
    return buf;
}

std::string flit(double v, mx_dtype ft) {
    if (ft == MX_F32) v = (double)(float)v;
    if (std::isnan(v)) return "((T)__builtin_nan(\"\"))";
    if (std::isinf(v)) return v > 0 ? "((T)__builtin_huge_val())" : "((T)-__builtin_huge_val())";
    char buf[64];
    std::snprintf(buf, sizeof buf, "((T)%a)", v);
    return buf;
}

std::string gen_source(const mx_loop &l) {
    const int n = (int)l.prog.size();
    std::string b;  // body lines
    int li[kRegs], lf[kRegs];
    for (int r = 0; r < kRegs; ++r) li[r] = lf[r] = -1;
    auto I = [&](int r) { return li[r] < 0 ? std::string("izero") : "i" + std::to_string(li[r]); };
    auto F = [&](int r) { return lf[r] < 0 ? std::string("fzero") : "f" + std::to_string(lf[r]); };
    std::vector<int> sets;  // instruction numbers of the sets so far
    auto slot = [&](const mx_linsn &q, int k) {
        const mx_ltype &tt = l.tensors[q.tensor];
        std::string e = "mx_slot(A.t[" + std::to_string(q.tensor) + "], " + std::to_string(tt.rank) + ", " + I(q.a);
        e += ", " + (tt.rank >= 2 ? I(q.b) : std::string("0LL")) + ", " + (tt.rank >= 3 ? I(q.c) : std::string("0LL")) + ")";
        return "    const long long q" + std::to_string(k) + " = " + e + ";\n    bad |= q" + std::to_string(k) +
               " < 0 ? 1u : 0u;\n";
    };
    for (int k = 0; k < n; ++k) {
        const mx_linsn &q = l.prog[k];
        const std::string K = std::to_string(k);
        const int op = q.op;
        if (float_op(op)) {
            const std::string a = op != MX_X_CONST ? F(q.a) : "", c = float_binary(op) ? F(q.b) : "";
            std::string e;
            switch (op) {
            case MX_X_CONST: e = flit(q.fimm, l.ftype); break;
            case MX_X_ADD: e = a + " + " + c; break;
            case MX_X_SUB: e = a + " - " + c; break;
            case MX_X_MUL: e = a + " * " + c; break;
            case MX_X_DIV: e = a + " / " + c; break;
            case MX_X_MIN: e = "(" + c + " < " + a + " ? " + c + " : " + a + ")"; break;
            case MX_X_MAX: e = "(" + c + " > " + a + " ? " + c + " : " + a + ")"; break;
            case MX_X_NEG: e = "-" + a; break;
            case MX_X_ABS: e = "(" + a + " < (T)0 ? -" + a + " : " + a + ")"; break;
            case MX_X_SQ: e = a + " * " + a; break;
            case MX_X_EXP: e = "exp(" + a + ")"; break;
            case MX_X_LOG: e = "log(" + a + ")"; break;
            case MX_X_SQRT: e = "sqrt(" + a + ")"; break;
            case MX_X_RSQRT: e = "(T)1 / sqrt(" + a + ")"; break;
            }
            b += "    const T f" + K + " = " + e + ";\n";
            lf[q.dst] = k;
            continue;
        }
        switch (op) {
        case MX_L_ITER: b += "    const long long i" + K + " = it;\n"; li[q.dst] = k; break;
        case MX_L_ICONST: b += "    const long long i" + K + " = " + ilit(q.iimm) + ";\n"; li[q.dst] = k; break;
        case MX_L_IADD:
        case MX_L_ISUB:
        case MX_L_IMUL: {
            const char *o = op == MX_L_IADD ? " + " : op == MX_L_ISUB ? " - " : " * ";
            b += "    const long long i" + K + " = (long long)((unsigned long long)" + I(q.a) + o +
                 "(unsigned long long)" + I(q.b) + ");\n";
            li[q.dst] = k;
            break;
        }
        case MX_L_IDIV: b += "    const long long i" + K + " = mx_idiv(" + I(q.a) + ", " + I(q.b) + ");\n"; li[q.dst] = k; break;
        case MX_L_IMOD: b += "    const long long i" + K + " = mx_imod(" + I(q.a) + ", " + I(q.b) + ");\n"; li[q.dst] = k; break;
        case MX_L_IMIN:
            b += "    const long long i" + K + " = " + I(q.b) + " < " + I(q.a) + " ? " + I(q.b) + " : " + I(q.a) + ";\n";
            li[q.dst] = k;
            break;
        case MX_L_IMAX:
            b += "    const long long i" + K + " = " + I(q.b) + " > " + I(q.a) + " ? " + I(q.b) + " : " + I(q.a) + ";\n";
            li[q.dst] = k;
            break;
        case MX_L_INEG:
            b += "    const long long i" + K + " = (long long)(0ULL - (unsigned long long)" + I(q.a) + ");\n";
            li[q.dst] = k;
            break;
        case MX_L_I2F: b += "    const T f" + K + " = (T)" + I(q.a) + ";\n"; lf[q.dst] = k; break;
        case MX_L_FGET:
        case MX_L_IGET: {
            const mx_ltype &tt = l.tensors[q.tensor];
            const bool fl = op == MX_L_FGET;
            const std::string v = (fl ? "f" : "i") + K, ty = fl ? "T" : "long long", el = elem_name(tt.dtype);
            const std::string tn = std::to_string(q.tensor);
            b += slot(q, k);
            b += "    " + ty + " " + v + " = (" + ty + ")0;\n";
            b += "    if (q" + K + " >= 0) {\n";
            // trace modes: the iteration's own earlier sets of this tensor, latest first
            std::string chain = "        ";
            for (auto it = sets.rbegin(); it != sets.rend(); ++it) {
                if (l.prog[*it].tensor != q.tensor) continue;
                const std::string P = std::to_string(*it);
                chain += "if (MODE != 0 && q" + P + " == q" + K + ") " + v + " = (" + ty + ")ov" + P + ";\n        else ";
            }
            b += chain + v + " = (" + ty + ")((const " + el + " *)A.t[" + tn + "].p)[q" + K + "];\n";
            if (l.set_mask >> q.tensor & 1u) {
                b += "        if (MODE == 2) { const unsigned long long o = A.own[" + tn + "][q" + K +
                     "]; if (o != 0ULL && o != (unsigned long long)(it + 1)) bad |= 4u; }\n";
            }
            b += "    }\n";
            (fl ? lf : li)[q.dst] = k;
            break;
        }
        case MX_L_FSET:
        case MX_L_ISET: {
            const mx_ltype &tt = l.tensors[q.tensor];
            const std::string el = elem_name(tt.dtype), tn = std::to_string(q.tensor);
            std::string val;
            if (op == MX_L_FSET) val = "(" + el + ")" + F(q.src);
            else if (tt.dtype == MX_I32) val = "(int)(unsigned)(unsigned long long)" + I(q.src);
            else val = I(q.src);
            b += slot(q, k);
            b += "    const " + el + " ov" + K + " = " + val + ";\n";
            b += "    if (q" + K + " >= 0) {\n";
            b += "        if (MODE == 0) ((" + el + " *)A.t[" + tn + "].p)[q" + K + "] = ov" + K + ";\n";
            b += "        if (MODE == 1) { const unsigned long long o = atomicCAS(&A.own[" + tn + "][q" + K +
                 "], 0ULL, (unsigned long long)(it + 1)); if (o != 0ULL && o != (unsigned long long)(it + 1)) bad |= 2u; }\n";
            b += "    }\n";
            sets.push_back(k);
            break;
        }
        }
    }

    std::string s;
    s += "// generated by the mx library from a parallel loop body\n";
    s += l.ftype == MX_F32 ? "typedef float T;\n" : "typedef double T;\n";
    s += "#define NT " + std::to_string(NT) + "\n";
    s += R"(struct MxT { void *p; long long d0, d1, d2; };
struct MxArgs { MxT t[8]; unsigned long long *own[8]; long long n; unsigned *err; };
__device__ __forceinline__ long long mx_idiv(long long a, long long b) {
    return b == 0 ? 0LL : b == -1 ? (long long)(0ULL - (unsigned long long)a) : a / (b == 0 ? 1LL : b);
}
__device__ __forceinline__ long long mx_imod(long long a, long long b) {
    return (b == 0 || b == -1) ? 0LL : a % (b == 0 ? 1LL : b);
}
// row-major slot of a rank-r index, -1 when an index is outside its dimension
__device__ __forceinline__ long long mx_slot(const MxT &t, int r, long long i0, long long i1, long long i2) {
    if (i0 < 0 || i0 >= t.d0) return -1;
    if (r == 1) return i0;
    if (i1 < 0 || i1 >= t.d1) return -1;
    if (r == 2) return i0 * t.d1 + i1;
    if (i2 < 0 || i2 >= t.d2) return -1;
    return (i0 * t.d1 + i1) * t.d2 + i2;
}
// one iteration; MODE 0 runs it, 1 and 2 trace it (no writes): flags 1 an
// index out of range, 2 a slot another iteration sets, 4 a slot read that
// another iteration sets
template <int MODE> __device__ __forceinline__ unsigned mx_iter(const MxArgs &A, const long long it) {
#pragma clang fp contract(off)
    unsigned bad = 0u;
    const long long izero = 0LL;
    const T fzero = (T)0;
    (void)izero; (void)fzero;
)";
    s += b;
    s += "    return bad;\n}\n";
    for (int m = 0; m < 3; ++m) {
        const std::string M = std::to_string(m);
        s += "extern \"C\" __global__ void __launch_bounds__(NT) mx_loop_" + M + "(MxArgs A) {\n"
             "    unsigned bad = 0u;\n"
             "    const long long stride = (long long)gridDim.x * NT;\n"
             "    for (long long it = (long long)blockIdx.x * NT + threadIdx.x; it < A.n; it += stride) bad |= mx_iter<" +
             M + ">(A, it);\n"
             "    if (bad && A.err) atomicOr(A.err, bad);\n}\n";
    }
    return s;
}

struct Args {
    struct T { void *p; long long d0, d1, d2; } t[8];
    unsigned long long *own[8];
    long long n;
    unsigned *err;
};
static_assert(sizeof(Args) == 8 * 32 + 8 * 8 + 8 + 8, "kernel argument layout");

int64_t numel(const mx_ltype &tt, const mx_ltensor &x) {
    int64_t m = 1;
    for (int k = 0; k < tt.rank; ++k) m *= x.dims[k];
    return m;
}

mx_status functions(mx_loop *l, hipFunction_t out[3]) {
    int dev = 0;
    MX_TRY_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(l->mu);
    if (l->fn_device != dev) {
        hipModule_t mod = nullptr;
        if (mx_status st = rtc_module(l->src, "mx_loop.hip", &mod)) return st;
        for (int m = 0; m < 3; ++m)
            MX_TRY_HIP(hipModuleGetFunction(&l->fn[m], mod, ("mx_loop_" + std::to_string(m)).c_str()));
        l->fn_device = dev;
    }
    for (int m = 0; m < 3; ++m) out[m] = l->fn[m];
    return MX_OK;
}

size_t own_bytes(const mx_loop *l, const mx_ltensor *ts, int t) {
    return (l->set_mask >> t & 1u) ? align256((size_t)numel(l->tensors[t], ts[t]) * 8) : 0;
}

}  // namespace
}  // namespace mx

using namespace mx;

extern "C" {

mx_status mx_loop_create(const mx_linsn *prog, int ninsn, const mx_ltype *tensors, int ntensors, mx_dtype float_type,
                         mx_loop **out) {
    MX_REQUIRE(out && prog, MX_ERR_INVALID, "mx_loop_create: null argument");
    if (mx_status st = validate(prog, ninsn, tensors, ntensors, float_type)) return st;
    auto *l = new mx_loop();
    l->prog.assign(prog, prog + ninsn);
    if (ntensors) l->tensors.assign(tensors, tensors + ntensors);
    l->ftype = float_type;
    for (const mx_linsn &q : l->prog)
        if (is_set(q.op)) l->set_mask |= 1u << q.tensor;
    l->src = gen_source(*l);
    *out = l;
    return MX_OK;
}

mx_status mx_loop_destroy(mx_loop *l) {
    delete l;
    return MX_OK;
}

mx_status mx_loop_prepare(mx_loop *l) {
    MX_REQUIRE(l, MX_ERR_INVALID, "mx_loop_prepare: null loop");
    hipFunction_t f[3];
    return functions(l, f);
}

const char *mx_loop_source(const mx_loop *l) { return l ? l->src.c_str() : ""; }

size_t mx_loop_workspace_bytes(const mx_loop *l, const mx_ltensor *tensors) {
    if (!l || (!tensors && !l->tensors.empty())) return 0;
    size_t b = kCounterBytes;
    for (int t = 0; t < (int)l->tensors.size(); ++t) b += own_bytes(l, tensors, t);
    return b;
}

mx_status mx_loop_run(mx_loop *l, int64_t n, const mx_ltensor *tensors, void *ws, size_t ws_bytes,
                      hipStream_t stream) {
    const char *who = "mx_loop_run";
    MX_REQUIRE(l, MX_ERR_INVALID, "%s: null loop", who);
    MX_REQUIRE(n >= 0, MX_ERR_SHAPE, "%s: n < 0", who);
    const int nt = (int)l->tensors.size();
    MX_REQUIRE(nt == 0 || tensors, MX_ERR_INVALID, "%s: null tensor list", who);
    Args A{};
    for (int t = 0; t < nt; ++t) {
        const mx_ltype &tt = l->tensors[t];
        for (int k = 0; k < tt.rank; ++k)
            MX_REQUIRE(tensors[t].dims[k] >= 0, MX_ERR_SHAPE, "%s: tensor %d: negative dimension", who, t);
        const int64_t m = numel(tt, tensors[t]);
        MX_REQUIRE(m == 0 || tensors[t].data, MX_ERR_INVALID, "%s: tensor %d: null data", who, t);
        A.t[t].p = tensors[t].data;
        A.t[t].d0 = tensors[t].dims[0];
        A.t[t].d1 = tt.rank >= 2 ? tensors[t].dims[1] : 1;
        A.t[t].d2 = tt.rank >= 3 ? tensors[t].dims[2] : 1;
    }
    A.n = n;
    if (n == 0) return MX_OK;
    hipFunction_t f[3];
    if (mx_status st = functions(l, f)) return st;
    const DeviceInfo *d;
    if (mx_status st = device_info(&d)) return st;
    int64_t grid = ceil_div(n, NT);
    if (grid > (int64_t)d->num_cus * 8) grid = (int64_t)d->num_cus * 8;
    void *params[] = {&A};
    if (debug_mode()) {
        const size_t need = mx_loop_workspace_bytes(l, tensors);
        MX_REQUIRE(ws && ws_bytes >= need && ((uintptr_t)ws & 255) == 0, MX_ERR_WORKSPACE,
                   "%s: debug mode needs a workspace of %zu bytes, 256-byte aligned", who, need);
        MX_TRY_HIP(hipMemsetAsync(ws, 0, need, stream));
        size_t off = kCounterBytes;
        for (int t = 0; t < nt; ++t) {
            if (l->set_mask >> t & 1u) A.own[t] = (unsigned long long *)((char *)ws + off);
            off += own_bytes(l, tensors, t);
        }
        A.err = (unsigned *)ws;
        for (int m = 1; m <= 2; ++m)
            MX_TRY_HIP(hipModuleLaunchKernel(f[m], (unsigned)grid, 1, 1, NT, 1, 1, 0, stream, params, nullptr));
        unsigned flags = 0;
        MX_TRY_HIP(hipMemcpyAsync(&flags, ws, sizeof flags, hipMemcpyDeviceToHost, stream));
        MX_TRY_HIP(hipStreamSynchronize(stream));
        if (flags)
            return set_error(MX_ERR_SHAPE, "%s: %s%s%s (nothing written)", who,
                             (flags & 1u) ? "an index outside its dimension; " : "",
                             (flags & 2u) ? "a slot set by two iterations; " : "",
                             (flags & 4u) ? "a slot set by one iteration and read by another; " : "");
        A.err = nullptr;
        for (int t = 0; t < 8; ++t) A.own[t] = nullptr;
    }
    MX_TRY_HIP(hipModuleLaunchKernel(f[0], (unsigned)grid, 1, 1, NT, 1, 1, 0, stream, params, nullptr));
    if (debug_mode()) MX_TRY_HIP(hipStreamSynchronize(stream));
    return MX_OK;
}

}  // extern "C"
