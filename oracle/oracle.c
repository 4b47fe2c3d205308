/*
 * Oracle for the accelerated-expression primitives -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, sequential CPU interpreter of what the parallel keywords of
 * the paper's source language compute (Appendix A, the Futhark and CUDA
 * extensions of the core language; Figure "Extensions of expressions"):
 *
 *   map f s        apply f to every element of s
 *   map2 f s1 s2   apply f elementwise to two sequences of equal length
 *   reduce f ne s  combine s with the associative f and neutral element ne;
 *                  evaluated here as the sequential left fold (Listing 1 uses
 *                  `reduce addi 0` and `foldl addi 0` interchangeably, and the
 *                  dynamic assumptions of Appendix "Dynamic Assumptions" make
 *                  every bracketing give the same value)
 *   flatten s      concatenation of inner sequences
 *   loop n f       f i for every i in [0, n); run here in ascending order
 *
 * Every floating-point quantity is carried in IEEE binary64 and every integer in
 * int64 (the paper's compiler always uses 64-bit integers, Section 5.1).  Build
 * with -O2 -ffp-contract=off and without -ffast-math, so each operation below
 * is one correctly rounded IEEE operation in the order written.
 *
 * The config programs (dot product, ragged row sums, dense map-map-reduce,
 * N-body loop, k-means step, batched dot/matvec) are written as compositions
 * of these combinators, with no blocking, fusion or reordering.
 *
 * Only tests, the smoke check and the bench's CPU-baseline leg may call this
 * code.  It shares no source with the GPU library.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---- operator tables (numbering mirrors the public enum values so that the
 *      same integer names the same operator on both sides; the code is separate) */
enum { OR_ADD = 0, OR_MUL = 1, OR_MIN = 2, OR_MAX = 3 };
enum { OR_U_ID = 0, OR_U_NEG = 1, OR_U_ABS = 2, OR_U_SQ = 3, OR_U_AFFINE = 4,
       OR_U_EXP = 5, OR_U_LOG = 6, OR_U_SQRT = 7, OR_U_RSQRT = 8 };
enum { OR_B_ADD = 0, OR_B_SUB = 1, OR_B_MUL = 2, OR_B_DIV = 3, OR_B_MIN = 4, OR_B_MAX = 5 };

/* ------------------------------------------------------------------------ */
/* Binary operators f : T -> T -> T used as reduce operators.                */
/* ------------------------------------------------------------------------ */
static double red_f64(int op, double x, double y)
{
    switch (op) {
    case OR_ADD: return x + y;
    case OR_MUL: return x * y;
    case OR_MIN: return y < x ? y : x;
    case OR_MAX: return y > x ? y : x;
    }
    return NAN;
}

static int64_t red_i64(int op, int64_t x, int64_t y)
{
    /* two's-complement wrap-around, computed in unsigned arithmetic */
    switch (op) {
    case OR_ADD: return (int64_t)((uint64_t)x + (uint64_t)y);
    case OR_MUL: return (int64_t)((uint64_t)x * (uint64_t)y);
    case OR_MIN: return y < x ? y : x;
    case OR_MAX: return y > x ? y : x;
    }
    return 0;
}

/* Map bodies.  AFFINE is x -> p0*x + p1 (a lambda with two captured
 * constants, e.g. the body `muli c (addi x 1)` of Listing 2 is p0 = p1 = c). */
static double un_f64(int f, double x, double p0, double p1)
{
    switch (f) {
    case OR_U_ID: return x;
    case OR_U_NEG: return -x;
    case OR_U_ABS: return fabs(x);
    case OR_U_SQ: return x * x;
    case OR_U_AFFINE: return p0 * x + p1;
    case OR_U_EXP: return exp(x);
    case OR_U_LOG: return log(x);
    case OR_U_SQRT: return sqrt(x);
    case OR_U_RSQRT: return 1.0 / sqrt(x);
    }
    return NAN;
}

static int64_t un_i64(int f, int64_t x, int64_t p0, int64_t p1)
{
    switch (f) {
    case OR_U_ID: return x;
    case OR_U_NEG: return (int64_t)(0u - (uint64_t)x);
    case OR_U_ABS: return x < 0 ? (int64_t)(0u - (uint64_t)x) : x;
    case OR_U_SQ: return (int64_t)((uint64_t)x * (uint64_t)x);
    case OR_U_AFFINE: return (int64_t)((uint64_t)p0 * (uint64_t)x + (uint64_t)p1);
    }
    return 0;
}

static double bin_f64(int f, double x, double y)
{
    switch (f) {
    case OR_B_ADD: return x + y;
    case OR_B_SUB: return x - y;
    case OR_B_MUL: return x * y;
    case OR_B_DIV: return x / y;
    case OR_B_MIN: return y < x ? y : x;
    case OR_B_MAX: return y > x ? y : x;
    }
    return NAN;
}

static int64_t bin_i64(int f, int64_t x, int64_t y)
{
    switch (f) {
    case OR_B_ADD: return (int64_t)((uint64_t)x + (uint64_t)y);
    case OR_B_SUB: return (int64_t)((uint64_t)x - (uint64_t)y);
    case OR_B_MUL: return (int64_t)((uint64_t)x * (uint64_t)y);
    case OR_B_MIN: return y < x ? y : x;
    case OR_B_MAX: return y > x ? y : x;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* map / map2 (Appendix A: `map e1 e2`, `map2 e1 e2 e3`)                     */
/* ------------------------------------------------------------------------ */
void or_map_f64(int f, double p0, double p1, const double *s, int64_t n, double *out)
{
    for (int64_t i = 0; i < n; ++i) out[i] = un_f64(f, s[i], p0, p1);
}

void or_map_i64(int f, int64_t p0, int64_t p1, const int64_t *s, int64_t n, int64_t *out)
{
    for (int64_t i = 0; i < n; ++i) out[i] = un_i64(f, s[i], p0, p1);
}

void or_map2_f64(int f, const double *s1, const double *s2, int64_t n, double *out)
{
    for (int64_t i = 0; i < n; ++i) out[i] = bin_f64(f, s1[i], s2[i]);
}

void or_map2_i64(int f, const int64_t *s1, const int64_t *s2, int64_t n, int64_t *out)
{
    for (int64_t i = 0; i < n; ++i) out[i] = bin_i64(f, s1[i], s2[i]);
}

/* ------------------------------------------------------------------------ */
/* reduce f ne s = foldl f ne s (Appendix A `reduce`; Listing 1)             */
/* ------------------------------------------------------------------------ */
double or_foldl_f64(int op, double ne, const double *s, int64_t n)
{
    double acc = ne;
    for (int64_t i = 0; i < n; ++i) acc = red_f64(op, acc, s[i]);
    return acc;
}

int64_t or_foldl_i64(int op, int64_t ne, const int64_t *s, int64_t n)
{
    int64_t acc = ne;
    for (int64_t i = 0; i < n; ++i) acc = red_i64(op, acc, s[i]);
    return acc;
}

/* The fused form of Listing 2 and of a dot product: reduce op ne (map2 f a b),
 * computed literally as the map2 into a temporary and then the fold. */
double or_map2_foldl_f64(int f, int op, double ne, const double *a, const double *b, int64_t n)
{
    double *tmp = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    or_map2_f64(f, a, b, n, tmp);
    double r = or_foldl_f64(op, ne, tmp, n);
    free(tmp);
    return r;
}

int64_t or_map2_foldl_i64(int f, int op, int64_t ne, const int64_t *a, const int64_t *b, int64_t n)
{
    int64_t *tmp = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    or_map2_i64(f, a, b, n, tmp);
    int64_t r = or_foldl_i64(op, ne, tmp, n);
    free(tmp);
    return r;
}

/* ------------------------------------------------------------------------ */
/* Marshaling of a ragged sequence [[T]] (Section 4.3): the flat layout is    */
/* the concatenation of the rows (what `flatten` returns) plus offsets, where */
/* offsets[0] = 0 and offsets[r+1] = offsets[r] + |row r|.                    */
/* ------------------------------------------------------------------------ */
void or_offsets_from_lengths(const int64_t *lengths, int64_t nseg, int64_t *offsets)
{
    offsets[0] = 0;
    for (int64_t r = 0; r < nseg; ++r) offsets[r + 1] = offsets[r] + lengths[r];
}

/* map (reduce op ne) over the rows of a marshalled ragged sequence */
void or_segmented_foldl_f64(int op, double ne, const double *values, const int64_t *offsets,
                            int64_t nseg, double *out)
{
    for (int64_t r = 0; r < nseg; ++r)
        out[r] = or_foldl_f64(op, ne, values + offsets[r], offsets[r + 1] - offsets[r]);
}

void or_segmented_foldl_i64(int op, int64_t ne, const int64_t *values, const int64_t *offsets,
                            int64_t nseg, int64_t *out)
{
    for (int64_t r = 0; r < nseg; ++r)
        out[r] = or_foldl_i64(op, ne, values + offsets[r], offsets[r + 1] - offsets[r]);
}

/* Reverse of the row sum map (reduce (+) 0): every element of row r receives
 * the upstream gradient of out[r] (the adjoint of a sum is a broadcast). */
void or_segmented_sum_adjoint_f64(const double *gout, const int64_t *offsets, int64_t nseg,
                                  double *gvalues)
{
    for (int64_t r = 0; r < nseg; ++r)
        for (int64_t e = offsets[r]; e < offsets[r + 1]; ++e) gvalues[e] = gout[r];
}

/* Reverse of reduce op ne s (derived; the paper has no reverse mode): the
 * gradient of y = foldl op ne s with respect to every element of s, times
 * the upstream gradient g.
 *   op = +        every element receives g (the adjoint of a sum is a
 *                 broadcast).
 *   op = min/max  the fold replaces its accumulator only when an element is
 *                 strictly below (above) it, so y is the element at which the
 *                 last replacement happened -- the lowest index attaining the
 *                 extreme -- or ne itself when no element improves on it.
 *                 That element receives g, every other element 0 (y does not
 *                 depend on them where the values differ).
 *   op = *        not defined here (returns -1). */
int or_reduce_adjoint_f64(int op, double ne, const double *s, int64_t n, double g, double *gs)
{
    if (op == OR_ADD) {
        for (int64_t i = 0; i < n; ++i) gs[i] = g;
        return 0;
    }
    if (op != OR_MIN && op != OR_MAX) return -1;
    double acc = ne;
    int64_t arg = -1;
    for (int64_t i = 0; i < n; ++i) {
        const int better = op == OR_MIN ? s[i] < acc : s[i] > acc;
        if (better) {
            acc = s[i];
            arg = i;
        }
    }
    for (int64_t i = 0; i < n; ++i) gs[i] = 0.0;
    if (arg >= 0) gs[arg] = g;
    return 0;
}

/* ... and of map (reduce op ne) over the rows of a marshalled ragged
 * sequence: row r's elements receive the reverse of its reduce with the
 * upstream gradient gout[r]. */
int or_segmented_reduce_adjoint_f64(int op, double ne, const double *values, const int64_t *offsets, int64_t nseg,
                                    const double *gout, double *gvalues)
{
    for (int64_t r = 0; r < nseg; ++r) {
        const int rc = or_reduce_adjoint_f64(op, ne, values + offsets[r], offsets[r + 1] - offsets[r], gout[r],
                                             gvalues + offsets[r]);
        if (rc) return rc;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Dense nested map-map-reduce (the sgemm pattern of Table 1):               */
/*   C[i][j] = reduce (+) 0 (map2 (*) (row i of op(A)) (column j of op(B)))  */
/* op(A) is A (M x K row-major) or, with ta = 1, the transpose of A stored   */
/* K x M row-major; likewise op(B) is K x N, or with tb = 1 stored N x K.    */
/* ------------------------------------------------------------------------ */
void or_matmul_f64(const double *A, const double *B, double *C, int64_t M, int64_t N,
                   int64_t K, int ta, int tb)
{
    double *row = (double *)malloc(sizeof(double) * (size_t)(K > 0 ? K : 1));
    double *col = (double *)malloc(sizeof(double) * (size_t)(K > 0 ? K : 1));
    for (int64_t i = 0; i < M; ++i) {
        for (int64_t k = 0; k < K; ++k) row[k] = ta ? A[k * M + i] : A[i * K + k];
        for (int64_t j = 0; j < N; ++j) {
            for (int64_t k = 0; k < K; ++k) col[k] = tb ? B[j * K + k] : B[k * N + j];
            C[i * N + j] = or_map2_foldl_f64(OR_B_MUL, OR_ADD, 0.0, row, col, K);
        }
    }
    free(row);
    free(col);
}

/* ------------------------------------------------------------------------ */
/* Sequential loop around a pairwise map(reduce): gravitational N-body with  */
/* Plummer softening, integrated by explicit (forward) Euler.  This is the   */
/* ODE-solver pattern of the CUDA-backend evaluation (Table 2).              */
/*   a_i = G * sum_j m_j d_ij (|d_ij|^2 + eps2)^(-3/2),  d_ij = x_j - x_i    */
/*   x_{t+1} = x_t + dt v_t,   v_{t+1} = v_t + dt a(x_t)                     */
/* The fold over j runs over every body including j = i, whose term is       */
/* exactly zero because d_ii = 0.                                            */
/* Layout: x is [N][3], m is [N].                                            */
/* ------------------------------------------------------------------------ */
void or_nbody_accel(const double *x, const double *m, int64_t N, double eps2, double G,
                    double *acc)
{
    for (int64_t i = 0; i < N; ++i) {
        double ax = 0.0, ay = 0.0, az = 0.0;
        for (int64_t j = 0; j < N; ++j) {
            double dx = x[3 * j + 0] - x[3 * i + 0];
            double dy = x[3 * j + 1] - x[3 * i + 1];
            double dz = x[3 * j + 2] - x[3 * i + 2];
            double s = dx * dx + dy * dy + dz * dz + eps2;
            double phi = 1.0 / (s * sqrt(s));
            double w = G * m[j] * phi;
            ax = ax + w * dx;
            ay = ay + w * dy;
            az = az + w * dz;
        }
        acc[3 * i + 0] = ax;
        acc[3 * i + 1] = ay;
        acc[3 * i + 2] = az;
    }
}

/* One forward-Euler step: both updates read the state at time t. */
void or_nbody_step(const double *x, const double *v, const double *m, int64_t N, double eps2,
                   double G, double dt, double *x_out, double *v_out)
{
    double *a = (double *)malloc(sizeof(double) * (size_t)(3 * (N > 0 ? N : 1)));
    or_nbody_accel(x, m, N, eps2, G, a);
    for (int64_t c = 0; c < 3 * N; ++c) {
        x_out[c] = x[c] + dt * v[c];
        v_out[c] = v[c] + dt * a[c];
    }
    free(a);
}

/* Kinetic energy 1/2 * sum_i m_i |v_i|^2 as a left fold over bodies. */
double or_nbody_kinetic(const double *v, const double *m, int64_t N)
{
    double ke = 0.0;
    for (int64_t i = 0; i < N; ++i) {
        double v2 = v[3 * i] * v[3 * i] + v[3 * i + 1] * v[3 * i + 1] + v[3 * i + 2] * v[3 * i + 2];
        ke = ke + 0.5 * m[i] * v2;
    }
    return ke;
}

/* Forward loop of nsteps; writes the final state.  If traj_x is not NULL it
 * receives x_t for t = 0 .. nsteps (layout [nsteps+1][N][3]). */
void or_nbody_forward(const double *x0, const double *v0, const double *m, int64_t N,
                      double eps2, double G, double dt, int64_t nsteps, double *x_out,
                      double *v_out, double *traj_x)
{
    size_t bytes = sizeof(double) * (size_t)(3 * (N > 0 ? N : 1));
    double *x = (double *)malloc(bytes), *v = (double *)malloc(bytes);
    double *xn = (double *)malloc(bytes), *vn = (double *)malloc(bytes);
    memcpy(x, x0, sizeof(double) * (size_t)(3 * N));
    memcpy(v, v0, sizeof(double) * (size_t)(3 * N));
    for (int64_t t = 0; t < nsteps; ++t) {
        if (traj_x) memcpy(traj_x + t * 3 * N, x, sizeof(double) * (size_t)(3 * N));
        or_nbody_step(x, v, m, N, eps2, G, dt, xn, vn);
        double *tx = x; x = xn; xn = tx;
        double *tv = v; v = vn; vn = tv;
    }
    if (traj_x) memcpy(traj_x + nsteps * 3 * N, x, sizeof(double) * (size_t)(3 * N));
    memcpy(x_out, x, sizeof(double) * (size_t)(3 * N));
    memcpy(v_out, v, sizeof(double) * (size_t)(3 * N));
    free(x); free(v); free(xn); free(vn);
}

/* Transposed-Jacobian product of the acceleration map, out = J_a(x)^T abar.
 * Differentiating a_i gives, for d = x_j - x_k, s = |d|^2 + eps2,
 *   M_kj = s^(-3/2) I - 3 s^(-5/2) d d^T   (symmetric in k and j),
 *   out_k = G * sum_j M_kj (m_k abar_j - m_j abar_k),
 * folded over j = 0..N-1 (the j = k term is exactly zero). */
void or_nbody_accel_vjp(const double *x, const double *m, int64_t N, double eps2, double G,
                        const double *abar, double *out)
{
    for (int64_t k = 0; k < N; ++k) {
        double ox = 0.0, oy = 0.0, oz = 0.0;
        for (int64_t j = 0; j < N; ++j) {
            double dx = x[3 * j + 0] - x[3 * k + 0];
            double dy = x[3 * j + 1] - x[3 * k + 1];
            double dz = x[3 * j + 2] - x[3 * k + 2];
            double s = dx * dx + dy * dy + dz * dz + eps2;
            double phi = 1.0 / (s * sqrt(s));
            double psi = 3.0 * phi / s;
            double wx = m[k] * abar[3 * j + 0] - m[j] * abar[3 * k + 0];
            double wy = m[k] * abar[3 * j + 1] - m[j] * abar[3 * k + 1];
            double wz = m[k] * abar[3 * j + 2] - m[j] * abar[3 * k + 2];
            double dw = dx * wx + dy * wy + dz * wz;
            ox = ox + G * (phi * wx - psi * dx * dw);
            oy = oy + G * (phi * wy - psi * dy * dw);
            oz = oz + G * (phi * wz - psi * dz * dw);
        }
        out[3 * k + 0] = ox;
        out[3 * k + 1] = oy;
        out[3 * k + 2] = oz;
    }
}

/* One reverse step of the discrete adjoint of forward Euler:
 *   xbar_t = xbar_{t+1} + dt * J_a(x_t)^T vbar_{t+1}
 *   vbar_t = vbar_{t+1} + dt * xbar_{t+1}                                   */
static void adjoint_step(const double *x_t, const double *m, int64_t N, double eps2, double G,
                         double dt, double *xbar, double *vbar, double *tmp)
{
    or_nbody_accel_vjp(x_t, m, N, eps2, G, vbar, tmp);
    for (int64_t c = 0; c < 3 * N; ++c) {
        double xb_new = xbar[c] + dt * tmp[c];
        double vb_new = vbar[c] + dt * xbar[c];
        xbar[c] = xb_new;
        vbar[c] = vb_new;
    }
}

/* Gradient of the final kinetic energy with respect to the initial positions
 * (and velocities), reverse sweep over a full tape of x_t. */
double or_nbody_ke_grad_tape(const double *x0, const double *v0, const double *m, int64_t N,
                             double eps2, double G, double dt, int64_t nsteps, double *gx0,
                             double *gv0)
{
    size_t n3 = (size_t)(3 * (N > 0 ? N : 1));
    double *traj = (double *)malloc(sizeof(double) * n3 * (size_t)(nsteps + 1));
    double *xT = (double *)malloc(sizeof(double) * n3), *vT = (double *)malloc(sizeof(double) * n3);
    double *tmp = (double *)malloc(sizeof(double) * n3);
    or_nbody_forward(x0, v0, m, N, eps2, G, dt, nsteps, xT, vT, traj);
    double ke = or_nbody_kinetic(vT, m, N);
    for (int64_t i = 0; i < N; ++i)
        for (int c = 0; c < 3; ++c) {
            gx0[3 * i + c] = 0.0;
            gv0[3 * i + c] = m[i] * vT[3 * i + c];
        }
    for (int64_t t = nsteps - 1; t >= 0; --t)
        adjoint_step(traj + t * 3 * N, m, N, eps2, G, dt, gx0, gv0, tmp);
    free(traj); free(xT); free(vT); free(tmp);
    return ke;
}

/* Same gradient with checkpoints of (x, v) every k steps; each segment is
 * recomputed forward from its checkpoint before its reverse sweep. */
double or_nbody_ke_grad_ckpt(const double *x0, const double *v0, const double *m, int64_t N,
                             double eps2, double G, double dt, int64_t nsteps, int64_t k,
                             double *gx0, double *gv0)
{
    int64_t nck = (nsteps + k - 1) / k;
    size_t n3 = (size_t)(3 * (N > 0 ? N : 1));
    double *ckx = (double *)malloc(sizeof(double) * n3 * (size_t)(nck > 0 ? nck : 1));
    double *ckv = (double *)malloc(sizeof(double) * n3 * (size_t)(nck > 0 ? nck : 1));
    double *x = (double *)malloc(sizeof(double) * n3), *v = (double *)malloc(sizeof(double) * n3);
    double *xn = (double *)malloc(sizeof(double) * n3), *vn = (double *)malloc(sizeof(double) * n3);
    double *seg = (double *)malloc(sizeof(double) * n3 * (size_t)k);
    double *tmp = (double *)malloc(sizeof(double) * n3);
    memcpy(x, x0, sizeof(double) * n3);
    memcpy(v, v0, sizeof(double) * n3);
    for (int64_t t = 0; t < nsteps; ++t) {
        if (t % k == 0) {
            memcpy(ckx + (t / k) * 3 * N, x, sizeof(double) * (size_t)(3 * N));
            memcpy(ckv + (t / k) * 3 * N, v, sizeof(double) * (size_t)(3 * N));
        }
        or_nbody_step(x, v, m, N, eps2, G, dt, xn, vn);
        double *tx = x; x = xn; xn = tx;
        double *tv = v; v = vn; vn = tv;
    }
    double ke = or_nbody_kinetic(v, m, N);
    for (int64_t i = 0; i < N; ++i)
        for (int c = 0; c < 3; ++c) {
            gx0[3 * i + c] = 0.0;
            gv0[3 * i + c] = m[i] * v[3 * i + c];
        }
    for (int64_t c0 = nck - 1; c0 >= 0; --c0) {
        int64_t t0 = c0 * k, t1 = t0 + k < nsteps ? t0 + k : nsteps;
        memcpy(x, ckx + c0 * 3 * N, sizeof(double) * (size_t)(3 * N));
        memcpy(v, ckv + c0 * 3 * N, sizeof(double) * (size_t)(3 * N));
        for (int64_t t = t0; t < t1; ++t) {
            memcpy(seg + (t - t0) * 3 * N, x, sizeof(double) * (size_t)(3 * N));
            or_nbody_step(x, v, m, N, eps2, G, dt, xn, vn);
            double *tx = x; x = xn; xn = tx;
            double *tv = v; v = vn; vn = tv;
        }
        for (int64_t t = t1 - 1; t >= t0; --t)
            adjoint_step(seg + (t - t0) * 3 * N, m, N, eps2, G, dt, gx0, gv0, tmp);
    }
    free(ckx); free(ckv); free(x); free(v); free(xn); free(vn); free(seg); free(tmp);
    return ke;
}

/* ------------------------------------------------------------------------ */
/* k-means step: map (argmin-reduce) + reduce-by-key (the histo pattern).    */
/*   dist(i, j) = foldl (+) 0 over dims d of (x_id - c_jd)^2                 */
/*   label_i    = the j minimising (dist(i, j), j) lexicographically         */
/*   count_j    = #{i : label_i = j},   sum_j = foldl (+) 0 of x_i, label j  */
/*   c'_j       = sum_j / count_j, or c_j if count_j = 0                     */
/* X is [n][d] and C is [k][d], both row-major.                              */
/* ------------------------------------------------------------------------ */
double or_sqdist(const double *x, const double *c, int64_t d)
{
    double acc = 0.0;
    for (int64_t t = 0; t < d; ++t) {
        double diff = x[t] - c[t];
        acc = acc + diff * diff;
    }
    return acc;
}

void or_kmeans_assign(const double *X, int64_t n, int64_t d, const double *C, int64_t k,
                      int32_t *labels)
{
    for (int64_t i = 0; i < n; ++i) {
        double best = 0.0;
        int64_t arg = -1;
        for (int64_t j = 0; j < k; ++j) {
            double dj = or_sqdist(X + i * d, C + j * d, d);
            /* (value, index) lexicographic minimum: strict < keeps the lowest index */
            if (arg < 0 || dj < best) { best = dj; arg = j; }
        }
        labels[i] = (int32_t)arg;
    }
}

void or_kmeans_update(const double *X, int64_t n, int64_t d, const int32_t *labels, int64_t k,
                      const double *C_old, int64_t *counts, double *sums, double *C_new)
{
    for (int64_t j = 0; j < k; ++j) {
        counts[j] = 0;
        for (int64_t t = 0; t < d; ++t) sums[j * d + t] = 0.0;
    }
    for (int64_t i = 0; i < n; ++i) {
        int64_t j = labels[i];
        counts[j] = counts[j] + 1;
        for (int64_t t = 0; t < d; ++t) sums[j * d + t] = sums[j * d + t] + X[i * d + t];
    }
    for (int64_t j = 0; j < k; ++j)
        for (int64_t t = 0; t < d; ++t)
            C_new[j * d + t] = counts[j] > 0 ? sums[j * d + t] / (double)counts[j] : C_old[j * d + t];
}

/* Within-cluster sum of squares SSE = sum_i dist(x_i, c_{label_i}) and its
 * gradient with respect to the points, dSSE/dx_i = 2 (x_i - c_{label_i})
 * (labels and centroids held fixed). */
double or_kmeans_sse(const double *X, int64_t n, int64_t d, const double *C,
                     const int32_t *labels)
{
    double acc = 0.0;
    for (int64_t i = 0; i < n; ++i) acc = acc + or_sqdist(X + i * d, C + (int64_t)labels[i] * d, d);
    return acc;
}

void or_kmeans_sse_grad(const double *X, int64_t n, int64_t d, const double *C,
                        const int32_t *labels, double gscale, double *G)
{
    for (int64_t i = 0; i < n; ++i)
        for (int64_t t = 0; t < d; ++t)
            G[i * d + t] = gscale * (2.0 * (X[i * d + t] - C[(int64_t)labels[i] * d + t]));
}

/* ------------------------------------------------------------------------ */
/* Batched independent expressions: each task is evaluated on its own by the  */
/* single-expression definitions above.  Task rows of the table are          */
/* (kind, rows, cols, a_off, b_off, out_off); kind 0 = dot, 1 = matvec.      */
/* ------------------------------------------------------------------------ */
void or_batch_forward(const int64_t *table, int64_t ntasks, const double *A, const double *B,
                      double *out)
{
    for (int64_t t = 0; t < ntasks; ++t) {
        const int64_t *r = table + 6 * t;
        int64_t kind = r[0], rows = r[1], cols = r[2];
        const double *a = A + r[3], *b = B + r[4];
        double *o = out + r[5];
        if (kind == 0) {
            o[0] = or_map2_foldl_f64(OR_B_MUL, OR_ADD, 0.0, a, b, cols);
        } else {
            for (int64_t i = 0; i < rows; ++i)
                o[i] = or_map2_foldl_f64(OR_B_MUL, OR_ADD, 0.0, a + i * cols, b, cols);
        }
    }
}

/* Reverse of each task.  dot: (gA, gB) = (g * b, g * a).  matvec y = A x:
 * gA = g x^T (outer product) and gx = A^T g, the latter as a fold over rows. */
void or_batch_backward(const int64_t *table, int64_t ntasks, const double *A, const double *B,
                       const double *gout, double *gA, double *gB)
{
    for (int64_t t = 0; t < ntasks; ++t) {
        const int64_t *r = table + 6 * t;
        int64_t kind = r[0], rows = r[1], cols = r[2];
        const double *a = A + r[3], *b = B + r[4], *g = gout + r[5];
        double *ga = gA + r[3], *gb = gB + r[4];
        if (kind == 0) {
            for (int64_t i = 0; i < cols; ++i) {
                ga[i] = g[0] * b[i];
                gb[i] = g[0] * a[i];
            }
        } else {
            for (int64_t i = 0; i < rows; ++i)
                for (int64_t c = 0; c < cols; ++c) ga[i * cols + c] = g[i] * b[c];
            for (int64_t c = 0; c < cols; ++c) {
                double acc = 0.0;
                for (int64_t i = 0; i < rows; ++i) acc = acc + a[i * cols + c] * g[i];
                gb[c] = acc;
            }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* User-defined map bodies.  The source language's map and map2 take any    */
/* first-order function built from the language's arithmetic (Appendix A;   */
/* Section 4.2).  A body is a straight-line program over registers          */
/* r0..r15: each instruction (op, dst, a, b, imm) writes r[dst].  The       */
/* interpreter runs it once per element, in binary64.                       */
/* ------------------------------------------------------------------------ */
enum { OR_X_IN = 0, OR_X_CONST = 1, OR_X_ADD = 2, OR_X_SUB = 3, OR_X_MUL = 4, OR_X_DIV = 5,
       OR_X_MIN = 6, OR_X_MAX = 7, OR_X_NEG = 8, OR_X_ABS = 9, OR_X_SQ = 10, OR_X_EXP = 11,
       OR_X_LOG = 12, OR_X_SQRT = 13, OR_X_RSQRT = 14 };
#define OR_X_REGS 16
#define OR_X_MAXINSN 64

/* one instruction on values already read from the registers */
static double x_apply(int op, double va, double vb, double imm, double in)
{
    switch (op) {
    case OR_X_IN: return in;
    case OR_X_CONST: return imm;
    case OR_X_ADD: return va + vb;
    case OR_X_SUB: return va - vb;
    case OR_X_MUL: return va * vb;
    case OR_X_DIV: return va / vb;
    case OR_X_MIN: return vb < va ? vb : va;
    case OR_X_MAX: return vb > va ? vb : va;
    case OR_X_NEG: return -va;
    case OR_X_ABS: return va < 0.0 ? -va : va;
    case OR_X_SQ: return va * va;
    case OR_X_EXP: return exp(va);
    case OR_X_LOG: return log(va);
    case OR_X_SQRT: return sqrt(va);
    case OR_X_RSQRT: return 1.0 / sqrt(va);
    }
    return NAN;
}

/* Evaluates the body at element i of the inputs X[k*n + i] (k < nin); the
 * value of every instruction goes to val[] (indexed by instruction), and the
 * instruction that produced each operand to src_a[] / src_b[]. */
static double x_eval(const int32_t *code, const double *imm, int ninsn, int out_reg, const double *X,
                     int64_t n, int64_t i, double *val, int *src_a, int *src_b, int *out_src)
{
    double r[OR_X_REGS];
    int last[OR_X_REGS];
    for (int q = 0; q < OR_X_REGS; ++q) { r[q] = 0.0; last[q] = -1; }
    for (int k = 0; k < ninsn; ++k) {
        const int op = code[4 * k], dst = code[4 * k + 1], a = code[4 * k + 2], b = code[4 * k + 3];
        const int reads_a = op >= OR_X_ADD, reads_b = op >= OR_X_ADD && op <= OR_X_MAX;
        const double va = reads_a ? r[a] : 0.0, vb = reads_b ? r[b] : 0.0;
        const double in = op == OR_X_IN ? X[(int64_t)a * n + i] : 0.0;
        src_a[k] = reads_a ? last[a] : -1;
        src_b[k] = reads_b ? last[b] : -1;
        val[k] = x_apply(op, va, vb, imm[k], in);
        r[dst] = val[k];
        last[dst] = k;
    }
    *out_src = last[out_reg];
    return r[out_reg];
}

void or_expr_map_f64(const int32_t *code, const double *imm, int ninsn, int out_reg, const double *X, int64_t n,
                     double *out)
{
    double val[OR_X_MAXINSN];
    int sa[OR_X_MAXINSN], sb[OR_X_MAXINSN], os;
    for (int64_t i = 0; i < n; ++i) out[i] = x_eval(code, imm, ninsn, out_reg, X, n, i, val, sa, sb, &os);
}

/* reduce op ne (map body s): the sequential left fold of the body's values */
double or_expr_map_foldl_f64(int op, double ne, const int32_t *code, const double *imm, int ninsn, int out_reg,
                             const double *X, int64_t n)
{
    double val[OR_X_MAXINSN];
    int sa[OR_X_MAXINSN], sb[OR_X_MAXINSN], os;
    double acc = ne;
    for (int64_t i = 0; i < n; ++i)
        acc = red_f64(op, acc, x_eval(code, imm, ninsn, out_reg, X, n, i, val, sa, sb, &os));
    return acc;
}

/* Reverse mode of the body at every element: G[k*n + i] = s_i * d body / d
 * input k, with s_i = (gout ? gout[i] : 1) * (gscale ? *gscale : 1).  Adjoints
 * flow from the output back through the instructions in reverse order; an
 * operand receives the chain-rule term of the instruction that read it,
 * terms added in that reverse order.  min / max are locally one of their
 * operands, so their derivative is that of the operand they returned: it
 * alone receives the adjoint and the other operand receives nothing (its
 * subtree is not reached from this use, so a non-finite partial inside it,
 * such as 1/c or log c at c = 0, leaves the gradient untouched).  abs passes
 * the adjoint to x with the sign of the branch taken.  Instructions the
 * output does not depend on pass nothing. */
void or_expr_vjp_f64(const int32_t *code, const double *imm, int ninsn, int nin, int out_reg, const double *X,
                     int64_t n, const double *gout, const double *gscale, double *G)
{
    double val[OR_X_MAXINSN], adj[OR_X_MAXINSN];
    int sa[OR_X_MAXINSN], sb[OR_X_MAXINSN], reached[OR_X_MAXINSN], os;
    for (int64_t i = 0; i < n; ++i) {
        x_eval(code, imm, ninsn, out_reg, X, n, i, val, sa, sb, &os);
        for (int k = 0; k < ninsn; ++k) { adj[k] = 0.0; reached[k] = 0; }
        double seed = gout ? gout[i] : 1.0;
        if (gscale) seed = gout ? seed * gscale[0] : gscale[0];
        double gin[4] = {0.0, 0.0, 0.0, 0.0};
        int gin_set[4] = {0, 0, 0, 0};
        if (os >= 0) { adj[os] = seed; reached[os] = 1; }
        for (int k = ninsn - 1; k >= 0; --k) {
            if (!reached[k]) continue;
            const int op = code[4 * k];
            const double g = adj[k], vk = val[k];
            const int ja = sa[k], jb = sb[k];
            const double va = ja >= 0 ? val[ja] : 0.0, vb = jb >= 0 ? val[jb] : 0.0;
            double ca = 0.0, cb = 0.0;  /* terms for operands a and b */
            int ta = 0, tb = 0;         /* which operands receive a term */
            switch (op) {
            case OR_X_IN: {
                const int a = code[4 * k + 2];
                gin[a] = gin_set[a] ? gin[a] + g : g;
                gin_set[a] = 1;
                break;
            }
            case OR_X_CONST: break;
            case OR_X_ADD: ca = g; cb = g; ta = tb = 1; break;
            case OR_X_SUB: ca = g; cb = -g; ta = tb = 1; break;
            case OR_X_MUL: ca = g * vb; cb = g * va; ta = tb = 1; break;
            case OR_X_DIV: ca = g / vb; cb = -(g * vk / vb); ta = tb = 1; break;
            case OR_X_MIN: if (vb < va) { cb = g; tb = 1; } else { ca = g; ta = 1; } break;
            case OR_X_MAX: if (vb > va) { cb = g; tb = 1; } else { ca = g; ta = 1; } break;
            case OR_X_NEG: ca = -g; ta = 1; break;
            case OR_X_ABS: ca = va < 0.0 ? -g : g; ta = 1; break;
            case OR_X_SQ: ca = g * (va + va); ta = 1; break;
            case OR_X_EXP: ca = g * vk; ta = 1; break;
            case OR_X_LOG: ca = g / va; ta = 1; break;
            case OR_X_SQRT: ca = g / (vk + vk); ta = 1; break;
            case OR_X_RSQRT: ca = -(g * vk * vk * vk) * 0.5; ta = 1; break;
            }
            /* operand a's term first, then b's (a MUL of a value by itself adds both) */
            if (ta && ja >= 0) { adj[ja] = reached[ja] ? adj[ja] + ca : ca; reached[ja] = 1; }
            if (tb && jb >= 0) { adj[jb] = reached[jb] ? adj[jb] + cb : cb; reached[jb] = 1; }
        }
        for (int a = 0; a < nin; ++a) G[(int64_t)a * n + i] = gin[a];
    }
}

/* loop n (\i -> tensorSet out idx[i] (body x_i)): the CUDA backend's parallel
 * loop over i (Appendix A, Source Language: `loop n f` calls f i for every i
 * in [0, n) in an undefined order), here run sequentially in ascending i.
 * Slots outside [0, out_len) are not written. */
void or_expr_loop_scatter_f64(const int32_t *code, const double *imm, int ninsn, int out_reg, const double *X,
                              int64_t n, const int64_t *idx, double *out, int64_t out_len)
{
    double val[OR_X_MAXINSN];
    int sa[OR_X_MAXINSN], sb[OR_X_MAXINSN], os;
    for (int64_t i = 0; i < n; ++i) {
        const int64_t j = idx[i];
        const double v = x_eval(code, imm, ninsn, out_reg, X, n, i, val, sa, sb, &os);
        if (j >= 0 && j < out_len) out[j] = v;
    }
}

/* ------------------------------------------------------------------------ */
/* The general parallel loop (Appendix A, Source Language: `loop n f` calls  */
/* f i for every i in [0, n) in an undefined order; f reads and writes       */
/* tensors with tensorGet / tensorSet, as in Listing 1's in-place axpy).     */
/* The body is a straight-line program over 64 int64 registers and 64       */
/* binary64 registers; tensors (rank 1..3, row-major) hold binary64 (float   */
/* element types) or int64 (integer element types, an I32 tensor keeping    */
/* its stores wrapped to 32 bits) values.                                   */
/* ------------------------------------------------------------------------ */
enum { OR_L_ITER = 32, OR_L_ICONST = 33, OR_L_IADD = 34, OR_L_ISUB = 35, OR_L_IMUL = 36, OR_L_IDIV = 37,
       OR_L_IMOD = 38, OR_L_IMIN = 39, OR_L_IMAX = 40, OR_L_INEG = 41, OR_L_I2F = 42,
       OR_L_FGET = 48, OR_L_IGET = 49, OR_L_FSET = 50, OR_L_ISET = 51 };
#define OR_L_REGS 64
#define OR_L_MAXSET 256

typedef struct {
    int ntensors;
    const int *is_int, *is32, *rank;
    const int64_t *dims;   /* 3 per tensor */
    void *const *data;     /* double * or int64_t * */
} or_tensors;

/* integer division truncating toward zero, 0 for a zero divisor, wrapping
 * INT64_MIN / -1 */
static int64_t l_idiv(int64_t a, int64_t b)
{
    if (b == 0) return 0;
    if (b == -1) return (int64_t)(0 - (uint64_t)a);
    return a / b;
}

static int64_t l_imod(int64_t a, int64_t b)
{
    if (b == 0 || b == -1) return 0;
    return a % b;
}

/* slot of tensor t at the index registers, -1 when out of range */
static int64_t l_slot(const or_tensors *T, int t, int64_t i0, int64_t i1, int64_t i2)
{
    const int64_t *d = T->dims + 3 * t;
    const int r = T->rank[t];
    if (i0 < 0 || i0 >= d[0]) return -1;
    if (r == 1) return i0;
    if (i1 < 0 || i1 >= d[1]) return -1;
    if (r == 2) return i0 * d[1] + i1;
    if (i2 < 0 || i2 >= d[2]) return -1;
    return (i0 * d[1] + i1) * d[2] + i2;
}

static int64_t l_numel(const or_tensors *T, int t)
{
    int64_t m = 1;
    for (int k = 0; k < T->rank[t]; ++k) m *= T->dims[3 * t + k];
    return m;
}

/* One iteration.  mode 0: run (gets and sets on the tensors).  mode 1 and 2
 * trace it without writing: sets go to a private log that later gets of the
 * same iteration read first.  mode 1 claims every set slot for iteration
 * it in owner[t] (0 = free, it + 1 = taken) and flags 2 when another
 * iteration holds it; mode 2 flags 4 for a get of a slot another iteration
 * owns.  Returns the flags, bit 0 for an index out of range. */
static int l_exec(const int32_t *code, const int64_t *iimm, const double *fimm, int ninsn, const or_tensors *T,
                  int64_t it, int mode, int64_t *const *owner)
{
    int64_t ir[OR_L_REGS];
    double fr[OR_L_REGS];
    int logt[OR_L_MAXSET];
    int64_t logs[OR_L_MAXSET], logi[OR_L_MAXSET];
    double logf[OR_L_MAXSET];
    int nlog = 0, flags = 0;
    for (int q = 0; q < OR_L_REGS; ++q) { ir[q] = 0; fr[q] = 0.0; }
    for (int k = 0; k < ninsn; ++k) {
        const int32_t *c = code + 8 * k;
        const int op = c[0], dst = c[1], a = c[2], b = c[3], cc = c[4], src = c[5], t = c[6];
        switch (op) {
        case OR_L_ITER: ir[dst] = it; break;
        case OR_L_ICONST: ir[dst] = iimm[k]; break;
        case OR_L_IADD: ir[dst] = (int64_t)((uint64_t)ir[a] + (uint64_t)ir[b]); break;
        case OR_L_ISUB: ir[dst] = (int64_t)((uint64_t)ir[a] - (uint64_t)ir[b]); break;
        case OR_L_IMUL: ir[dst] = (int64_t)((uint64_t)ir[a] * (uint64_t)ir[b]); break;
        case OR_L_IDIV: ir[dst] = l_idiv(ir[a], ir[b]); break;
        case OR_L_IMOD: ir[dst] = l_imod(ir[a], ir[b]); break;
        case OR_L_IMIN: ir[dst] = ir[b] < ir[a] ? ir[b] : ir[a]; break;
        case OR_L_IMAX: ir[dst] = ir[b] > ir[a] ? ir[b] : ir[a]; break;
        case OR_L_INEG: ir[dst] = (int64_t)(0 - (uint64_t)ir[a]); break;
        case OR_L_I2F: fr[dst] = (double)ir[a]; break;
        case OR_L_FGET:
        case OR_L_IGET: {
            const int64_t sl = l_slot(T, t, ir[a], ir[b], ir[cc]);
            double fv = 0.0;
            int64_t iv = 0;
            if (sl < 0) {
                flags |= 1;
            } else {
                int hit = 0;
                for (int e = nlog - 1; e >= 0 && !hit; --e)
                    if (logt[e] == t && logs[e] == sl) { fv = logf[e]; iv = logi[e]; hit = 1; }
                if (!hit) {
                    if (T->is_int[t]) iv = ((const int64_t *)T->data[t])[sl];
                    else fv = ((const double *)T->data[t])[sl];
                }
                if (mode == 2 && owner[t] && owner[t][sl] != 0 && owner[t][sl] != it + 1) flags |= 4;
            }
            if (op == OR_L_FGET) fr[dst] = fv;
            else ir[dst] = iv;
            break;
        }
        case OR_L_FSET:
        case OR_L_ISET: {
            const int64_t sl = l_slot(T, t, ir[a], ir[b], ir[cc]);
            if (sl < 0) { flags |= 1; break; }
            int64_t iv = op == OR_L_ISET ? ir[src] : 0;
            if (op == OR_L_ISET && T->is32[t]) iv = (int64_t)(int32_t)(uint32_t)(uint64_t)iv;
            const double fv = op == OR_L_FSET ? fr[src] : 0.0;
            if (mode == 0) {
                if (T->is_int[t]) ((int64_t *)T->data[t])[sl] = iv;
                else ((double *)T->data[t])[sl] = fv;
            } else {
                if (nlog < OR_L_MAXSET) { logt[nlog] = t; logs[nlog] = sl; logi[nlog] = iv; logf[nlog] = fv; ++nlog; }
                if (mode == 1) {
                    if (owner[t][sl] == 0) owner[t][sl] = it + 1;
                    else if (owner[t][sl] != it + 1) flags |= 2;
                }
            }
            break;
        }
        default:  /* float arithmetic: the map-body operators on float registers */
            if (op == OR_X_CONST) fr[dst] = fimm[k];
            else fr[dst] = x_apply(op, fr[a], op >= OR_X_ADD && op <= OR_X_MAX ? fr[b] : 0.0, 0.0, 0.0);
            break;
        }
    }
    return flags;
}

/* loop n f: iterations in the order given (NULL: ascending).  Returns bit 0
 * when an index was out of range (that get gave 0, that set wrote nothing). */
int or_loop_run(const int32_t *code, const int64_t *iimm, const double *fimm, int ninsn, int ntensors,
                const int *is_int, const int *is32, const int *rank, const int64_t *dims, void *const *data,
                int64_t n, const int64_t *order)
{
    const or_tensors T = {ntensors, is_int, is32, rank, dims, data};
    int flags = 0;
    for (int64_t j = 0; j < n; ++j) flags |= l_exec(code, iimm, fimm, ninsn, &T, order ? order[j] : j, 0, NULL);
    return flags;
}

/* The debug-mode check: every iteration traced from the tensors as they are
 * before the loop (its own earlier sets visible to its own gets), nothing
 * written.  Flags: 1 an index out of range, 2 a slot set by two iterations,
 * 4 a slot one iteration sets and another reads. */
int or_loop_check(const int32_t *code, const int64_t *iimm, const double *fimm, int ninsn, int ntensors,
                  const int *is_int, const int *is32, const int *rank, const int64_t *dims, void *const *data,
                  int64_t n)
{
    const or_tensors T = {ntensors, is_int, is32, rank, dims, data};
    int64_t *owner[8] = {0};
    int flags = 0;
    for (int k = 0; k < ninsn; ++k) {
        const int op = code[8 * k], t = code[8 * k + 6];
        if ((op == OR_L_FSET || op == OR_L_ISET) && !owner[t])
            owner[t] = (int64_t *)calloc((size_t)(l_numel(&T, t) > 0 ? l_numel(&T, t) : 1), sizeof(int64_t));
    }
    for (int64_t i = 0; i < n; ++i) flags |= l_exec(code, iimm, fimm, ninsn, &T, i, 1, owner);
    for (int64_t i = 0; i < n; ++i) flags |= l_exec(code, iimm, fimm, ninsn, &T, i, 2, owner);
    for (int t = 0; t < 8; ++t) free(owner[t]);
    return flags;
}

/* ------------------------------------------------------------------------ */
/* Kernels of the shapes in the paper's Parboil comparison (Table 1), on     */
/* synthetic inputs (the datasets are not available).                        */
/* ------------------------------------------------------------------------ */

/* histo: reduce-by-key of keys into bins, counts[k] = #{i : keys[i] = k};
 * keys >= nbins fall in no bin. */
void or_histogram_u32(const uint32_t *keys, int64_t n, int64_t nbins, int64_t *counts)
{
    for (int64_t k = 0; k < nbins; ++k) counts[k] = 0;
    for (int64_t i = 0; i < n; ++i)
        if ((int64_t)keys[i] < nbins) counts[keys[i]] = counts[keys[i]] + 1;
}

/* stencil: one Jacobi sweep of the 7-point stencil on an nx x ny x nz grid
 * (x fastest): at interior points out = c1 * (sum of the six neighbours,
 * added x-, x+, y-, y+, z-, z+) - c0 * centre; boundary points are copied. */
void or_stencil7(const double *in, int64_t nx, int64_t ny, int64_t nz, double c0, double c1, double *out)
{
    for (int64_t z = 0; z < nz; ++z)
        for (int64_t y = 0; y < ny; ++y)
            for (int64_t x = 0; x < nx; ++x) {
                const int64_t i = (z * ny + y) * nx + x;
                if (x == 0 || y == 0 || z == 0 || x == nx - 1 || y == ny - 1 || z == nz - 1) {
                    out[i] = in[i];
                    continue;
                }
                double s = in[i - 1];
                s = s + in[i + 1];
                s = s + in[i - nx];
                s = s + in[i + nx];
                s = s + in[i - nx * ny];
                s = s + in[i + nx * ny];
                out[i] = c1 * s - c0 * in[i];
            }
}

/* mri-q: for every voxel x_i, with arg = 2 pi (kx_k x + ky_k y + kz_k z),
 * Qr_i = sum_k phi_k cos(arg), Qi_i = sum_k phi_k sin(arg), k ascending. */
void or_mriq(const double *kx, const double *ky, const double *kz, const double *phi, int64_t nk,
             const double *x, const double *y, const double *z, int64_t nx, double *qr, double *qi)
{
    const double two_pi = 6.283185307179586476925286766559;
    for (int64_t i = 0; i < nx; ++i) {
        double ar = 0.0, ai = 0.0;
        for (int64_t k = 0; k < nk; ++k) {
            const double arg = two_pi * (kx[k] * x[i] + ky[k] * y[i] + kz[k] * z[i]);
            ar = ar + phi[k] * cos(arg);
            ai = ai + phi[k] * sin(arg);
        }
        qr[i] = ar;
        qi[i] = ai;
    }
}

/* tpacf: angular pair counts.  Points are unit vectors (x, y, z) in
 * binary32; a pair's similarity is the binary32 dot product x1 x2 + y1 y2 +
 * z1 z2 (three products and two additions, each rounded to binary32 -- the
 * precision the kernel decides in).  With the decreasing binary32 bin edges
 * e_0 > ... > e_{m-1} (cosines of increasing angles), a pair falls in bin
 * #{b : d < e_b}, one of m + 1 bins.  self != 0: pairs i < j of set 1 only;
 * else all pairs of set 1 x set 2. */
void or_tpacf(const float *x1, const float *y1, const float *z1, int64_t n1, const float *x2, const float *y2,
              const float *z2, int64_t n2, int self, const float *edges, int m, int64_t *counts)
{
    for (int b = 0; b <= m; ++b) counts[b] = 0;
    for (int64_t i = 0; i < n1; ++i) {
        const int64_t j0 = self ? i + 1 : 0, jn = self ? n1 : n2;
        for (int64_t j = j0; j < jn; ++j) {
            const float xj = self ? x1[j] : x2[j], yj = self ? y1[j] : y2[j], zj = self ? z1[j] : z2[j];
            float d = x1[i] * xj;
            d = d + y1[i] * yj;
            d = d + z1[i] * zj;
            int bin = 0;
            for (int b = 0; b < m; ++b) bin += d < edges[b];
            counts[bin] = counts[bin] + 1;
        }
    }
}
