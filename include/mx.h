/*
 * mx.h -- C ABI of the MI355X (gfx950) data-parallel primitives for
 * accelerated expressions.
 *
 * The paper marks an expression `accelerate e`; its free variables are
 * marshalled from the host language's representation into flat backend arrays,
 * the expression's parallel keywords (map, map2, reduce, flatten, loop) run on
 * the GPU, and the result is marshalled back (Sections 2.1, 4.3; Appendix A).
 * This library is the run-time half of that scheme for one GPU: each entry
 * point evaluates one parallel keyword, or one fixed composition of them, on
 * flat device arrays.  There is no compiler: operators are enumerations, since
 * accelerated code may not pass higher-order functions (Section 4.4,
 * Appendix "Static Rules").
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Return value: MX_OK (0) or a negative mx_status.  On error nothing was
 *   launched, except MX_ERR_HIP, which reports a failed HIP call; the text of
 *   the last error of the calling thread is returned by mx_last_error().
 * - Pointers named *_dev or documented "device" are device addresses in the
 *   current HIP device's memory; pointers named *_host are host addresses.
 *   The caller owns every buffer (inputs, outputs and workspaces).  The library
 *   never frees caller memory and calls no allocator on the launch path
 *   (mx_batch_plan_create is the documented exception).
 * - Every call is asynchronous on the given stream (0 = the null stream) unless
 *   documented otherwise.  Scalar results are written to device memory.
 * - Sizes are element counts of type int64_t; n = 0 is valid everywhere and
 *   yields the empty result (a reduce of an empty sequence returns ne).
 * - Reduction operators must be associative and ne must be their neutral
 *   element; this is the caller's responsibility, as in the paper (Appendix
 *   "Dynamic Assumptions").  For any associative op the result equals the left
 *   fold foldl op ne s; integer results are exact (two's-complement wrap);
 *   floating-point results are one bracketing of that fold, fixed for a given
 *   size and launch configuration, so repeated calls are bit-identical.
 * - Debug mode (mx_set_debug(1)) adds the dynamic checks of the paper's debug
 *   compilation mode (Section 2.2; Appendix "Dynamic Assumptions"): ragged
 *   offsets are validated on the device before use and the stream is
 *   synchronised to report violations as MX_ERR_SHAPE.  Accelerate mode (the
 *   default) omits those checks.
 * - Workspaces: entry points taking (ws, ws_bytes) need at least
 *   mx_workspace_bytes(kind, ...) bytes of device memory, 256-byte aligned, which
 *   must be zero-filled before its first use.  Every successful call leaves the
 *   workspace's counters zero again, so one buffer can be reused (and captured in
 *   a HIP graph) without clearing.  A buffer serves one workspace kind: other
 *   kinds leave partial results in it.  Calls that share a workspace must be
 *   ordered on one stream.
 */
#ifndef MX_H
#define MX_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum mx_status {
    MX_OK = 0,
    MX_ERR_INVALID = -1,     /* null pointer, bad enum or flag, bad alignment */
    MX_ERR_SHAPE = -2,       /* mismatched lengths, bad offsets, size limits */
    MX_ERR_DTYPE = -3,       /* unsupported element type for this entry point */
    MX_ERR_UNSUPPORTED = -4, /* valid request that this library does not implement */
    MX_ERR_HIP = -5,         /* a HIP runtime call failed */
    MX_ERR_WORKSPACE = -6    /* workspace missing or too small */
} mx_status;

/* Element types.  Integers accumulate in int64 (the paper's compiler always
 * uses 64-bit integers, Section 5.1); I32 inputs widen to I64 results. */
typedef enum mx_dtype { MX_F32 = 0, MX_F64 = 1, MX_I32 = 2, MX_I64 = 3 } mx_dtype;

/* Associative, commutative reduce operators. */
typedef enum mx_redop { MX_ADD = 0, MX_MUL = 1, MX_MIN = 2, MX_MAX = 3 } mx_redop;

/* Map bodies.  MX_U_AFFINE is x -> p0 * x + p1 with two captured constants
 * (Listing 2's `muli c (addi x 1)` is p0 = p1 = c).  EXP, LOG, SQRT and RSQRT
 * are floating-point only. */
typedef enum mx_unop {
    MX_U_ID = 0, MX_U_NEG = 1, MX_U_ABS = 2, MX_U_SQ = 3, MX_U_AFFINE = 4,
    MX_U_EXP = 5, MX_U_LOG = 6, MX_U_SQRT = 7, MX_U_RSQRT = 8
} mx_unop;

/* map2 bodies.  MX_B_DIV is floating-point only. */
typedef enum mx_binop {
    MX_B_ADD = 0, MX_B_SUB = 1, MX_B_MUL = 2, MX_B_DIV = 3, MX_B_MIN = 4, MX_B_MAX = 5
} mx_binop;

/* Workspace kinds for mx_workspace_bytes (other entry points have their own
 * size queries next to them). */
typedef enum mx_ws_kind {
    MX_WS_REDUCE = 0,   /* mx_reduce, mx_map2_reduce: n = sequence length */
    MX_WS_SCAN = 1,     /* mx_lengths_to_offsets, mx_marshal_rows: n = number of rows */
    MX_WS_HISTOGRAM = 2, /* mx_histogram_u32: n = number of keys, aux = nbins; 0 = none used */
    MX_WS_SEGMENTED = 3  /* mx_segmented_reduce: n = number of values (any dtype) */
} mx_ws_kind;

/* ======================================================================= */
/* Runtime                                                                  */
/* ======================================================================= */

/* Selects `device` as the current HIP device of the calling thread and caches
 * its properties (compute-unit count, LDS size).  Optional: every entry point
 * initialises the current device lazily.  Errors: MX_ERR_HIP. */
mx_status mx_init(int device);

/* Text of the last error raised on the calling thread ("" if none).  The
 * pointer stays valid until the thread's next failing call. */
const char *mx_last_error(void);

/* Library version string, e.g. "mx 0.1.0 gfx950". */
const char *mx_version(void);

/* Debug mode on (1) or off (0), process-wide.  See the header comment. */
mx_status mx_set_debug(int on);
int mx_get_debug(void);

/* Bytes of device workspace an entry point of the given kind needs for n
 * elements (aux as documented per kind).  Always a multiple of 256. */
size_t mx_workspace_bytes(mx_ws_kind kind, int64_t n, int64_t aux);

/* Plain device-to-device copy of n 32-bit words through the library's
 * streaming kernel (the reference kernel used to calibrate hardware byte
 * counters).  dst and src must not overlap.  Errors: MX_ERR_INVALID. */
mx_status mx_copy32(const void *src_dev, void *dst_dev, int64_t n, hipStream_t stream);

/* Read-only streaming pass over n 32-bit words (the measured ceiling that
 * the memory-bound kernels are compared with): block b reads contiguous 16 KB
 * chunks b, b + B, ... in 16-byte loads (B = min(chunks, MX_STREAM_READ_SLOTS):
 * one chunk per block up to 256 MiB) and stores the XOR of its words into
 * xor_dev[b] with a plain store (no atomics, which would slow the pass);
 * xor_dev is a device array of MX_STREAM_READ_SLOTS uint32 the caller
 * zero-fills first, and the XOR of all slots is the XOR of all n words.  src
 * must be 16-byte aligned.  Errors: MX_ERR_INVALID, MX_ERR_SHAPE. */
#define MX_STREAM_READ_SLOTS 16384
mx_status mx_stream_read(const void *src_dev, int64_t n, uint32_t *xor_dev, hipStream_t stream);

/* ======================================================================= */
/* Marshaling (Section 4.3): nested sequences -> flat values + offsets      */
/* ======================================================================= */

/* Exclusive scan of row lengths into offsets (device):
 *   offsets[0] = 0, offsets[r+1] = offsets[r] + lengths[r],  r < nseg,
 * i.e. the offsets array of the flat layout of a ragged sequence [[T]].
 * lengths: int64[nseg] device; offsets: int64[nseg+1] device (may not alias
 * lengths).  Negative lengths are the caller's error (checked in debug mode,
 * MX_ERR_SHAPE); offsets must stay below 2^62.  Workspace kind MX_WS_SCAN with
 * n = nseg (unused for nseg <= 1024); the call leaves it all zero again.
 * One pass over the lengths: tiles of 1024 rows (4096 beyond 65 536 rows)
 * chained by decoupled look-back through status words in the workspace. */
mx_status mx_lengths_to_offsets(const int64_t *lengths_dev, int64_t nseg, int64_t *offsets_dev,
                                void *ws, size_t ws_bytes, hipStream_t stream);

/* Marshals a ragged sequence held as nseg separate host rows (the host
 * language's boxed representation) into the flat device layout: the rows are
 * gathered, in order, into the caller's pinned host staging buffer by host
 * threads, copied to values_dev with one host-to-device transfer, and the
 * offsets are computed on the device by mx_lengths_to_offsets.
 *   rows_host[r]      host pointer to lengths_host[r] elements of elem_bytes
 *   staging_host      pinned host memory (hipHostMalloc) of at least
 *                     round_up(sum(lengths) * elem_bytes, 256) + nseg * 8 bytes
 *   values_dev        device, sum(lengths) * elem_bytes bytes
 *   lengths_dev       device int64[nseg] (receives a copy of lengths_host)
 *   offsets_dev       device int64[nseg + 1]
 * The call first waits for work already queued on the stream (an earlier
 * transfer may still read the staging buffer); the staging buffer must then
 * stay untouched until the stream has passed this call.  Workspace kind
 * MX_WS_SCAN with n = nseg.  Errors: MX_ERR_INVALID,
 * MX_ERR_WORKSPACE, MX_ERR_HIP. */
mx_status mx_marshal_rows(const void *const *rows_host, const int64_t *lengths_host, int64_t nseg,
                          size_t elem_bytes, void *staging_host, size_t staging_bytes,
                          void *values_dev, int64_t *lengths_dev, int64_t *offsets_dev, void *ws,
                          size_t ws_bytes, hipStream_t stream);

/* Inverse of mx_marshal_rows: copies the flat device values back and scatters
 * row r into rows_host[r] (offsets_host[r] .. offsets_host[r+1]).  Synchronous:
 * waits for the stream.  staging_host: pinned host buffer of at least
 * offsets_host[nseg] * elem_bytes bytes.  Errors: MX_ERR_INVALID, MX_ERR_HIP. */
mx_status mx_unmarshal_rows(const void *values_dev, const int64_t *offsets_host, int64_t nseg,
                            size_t elem_bytes, void *staging_host, size_t staging_bytes,
                            void *const *rows_host, hipStream_t stream);

/* Records {l_1 = e_1, ..., l_f = e_f} with f fields of 4 or 8 bytes each:
 * array-of-records (interleaved, record i field j at aos[i*f + j]) <-> one
 * flat device array per field (field j of record i at soa[j][i]).
 * soa_fields_host is a host array of f device pointers.  1 <= f <= 16.
 * Errors: MX_ERR_INVALID. */
mx_status mx_records_to_fields(const void *aos_dev, int64_t n, int nfields, size_t field_bytes,
                               void *const *soa_fields_host, hipStream_t stream);
mx_status mx_fields_to_records(const void *const *soa_fields_host, int64_t n, int nfields,
                               size_t field_bytes, void *aos_dev, hipStream_t stream);

/* Sequences of records whose fields are scalars or sequences (the record
 * types {l_1 : T_1, ..., l_f : T_f} of Appendix A allow T_i = [T]; Section
 * 4.3 marshals accelerated bindings by their types).  The host records are
 * nrec structs of rec_bytes each; field f sits at byte offset fields[f].offset
 * of a record: a scalar of elem_bytes, or an mx_hseq (pointer and length of
 * the record's sequence).  Field-wise device layout: a scalar field is one
 * array of nrec values (values_dev); a sequence field is the concatenation of
 * every record's sequence in record order (values_dev), their lengths
 * (lengths_dev, int64[nrec]) and offsets (offsets_dev, int64[nrec + 1], the
 * exclusive scan of the lengths, computed on the device). */
typedef struct {
    const void *data;  /* host: len elements of the field's elem_bytes */
    int64_t len;
} mx_hseq;
typedef enum { MX_FIELD_SCALAR = 0, MX_FIELD_SEQ = 1 } mx_field_kind;
typedef struct {
    int32_t kind;          /* mx_field_kind */
    int32_t elem_bytes;    /* 1, 2, 4 or 8 */
    int64_t offset;        /* byte offset of the field in a host record */
    void *values_dev;      /* device: nrec values, or the sum of the lengths */
    int64_t *lengths_dev;  /* sequence fields: device int64[nrec]; else NULL */
    int64_t *offsets_dev;  /* sequence fields: device int64[nrec + 1]; else NULL */
} mx_field;

/* For every field its element count (nrec for a scalar field, the sum of the
 * records' lengths for a sequence field) into counts_host[f], and the bytes of
 * pinned host staging that mx_marshal_records and mx_unmarshal_records need.
 * Errors: MX_ERR_INVALID (bad field description, null sequence data with a
 * positive length), MX_ERR_SHAPE (negative length). */
mx_status mx_records_layout(const void *recs_host, int64_t nrec, size_t rec_bytes, const mx_field *fields,
                            int nfields, int64_t *counts_host, size_t *staging_bytes_host);

/* Marshals the records field by field: host threads gather every field into
 * the pinned staging buffer, one host-to-device copy per field (and per
 * sequence field one for its lengths), then the offsets of each sequence field
 * by the device scan (mx_lengths_to_offsets; workspace kind MX_WS_SCAN with
 * n = nrec, reused field after field).  Waits for earlier work on the stream
 * before it refills the staging buffer, which must then stay untouched until
 * the stream has passed this call.  1 <= nfields <= 16. */
mx_status mx_marshal_records(const void *recs_host, int64_t nrec, size_t rec_bytes, const mx_field *fields,
                             int nfields, void *staging_host, size_t staging_bytes, void *ws, size_t ws_bytes,
                             hipStream_t stream);

/* The inverse: copies every field back and writes the host records -- scalar
 * fields into the records, sequence fields into the host memory each record's
 * mx_hseq points to, whose len must equal the device length of that record's
 * sequence (MX_ERR_SHAPE otherwise; checked before any record is written).
 * Synchronous.  Staging: the bytes mx_records_layout gives for the records. */
mx_status mx_unmarshal_records(const mx_field *fields, int nfields, int64_t nrec, void *recs_host, size_t rec_bytes,
                               void *staging_host, size_t staging_bytes, hipStream_t stream);

/* `map flatten` over a depth-3 ragged sequence [[[T]]] given by outer offsets
 * (nouter+1 entries, counting middle rows) and inner offsets (counting values):
 * the flattened inner rows of outer element i span values
 * inner[outer[i]] .. inner[outer[i+1]], so out[i] = inner[outer[i]] for
 * i <= nouter.  Flattening the outermost level itself needs no call (drop the
 * outer offsets).  All pointers device.  Errors: MX_ERR_INVALID. */
mx_status mx_compose_offsets(const int64_t *outer_dev, int64_t nouter, const int64_t *inner_dev,
                             int64_t *out_dev, hipStream_t stream);

/* Regularity of one nesting level: succeeds when every row of the offsets
 * array (device, nseg + 1 entries) has the same length, returned in
 * *row_len_host (0 for nseg = 0); MX_ERR_SHAPE when the rows are ragged or the
 * offsets decrease.  Tensors (rank <= 3) are nested sequences whose levels
 * are all regular (the paper's Futhark backend accepts only those, Section
 * 4.3); this is the check that turns a marshalled nesting into a tensor
 * shape.  Synchronous: waits for the stream.  Keeps one 16-byte device
 * buffer per device for the process. */
mx_status mx_offsets_regular(const int64_t *offsets_dev, int64_t nseg, int64_t *row_len_host, hipStream_t stream);

/* ======================================================================= */
/* map / map2 (Appendix A)                                                  */
/* ======================================================================= */

/* out[i] = f(x[i]) for i < n.  dtype is the element type of x; out has the
 * accumulator type (F32->F32, F64->F64, I32->I64, I64->I64).  params_host
 * points to two values of the output type (p0, p1), used by MX_U_AFFINE; may
 * be NULL otherwise.  out may alias x when the types have equal size.
 * Errors: MX_ERR_INVALID, MX_ERR_DTYPE (float-only f on an integer type). */
mx_status mx_map(mx_unop f, mx_dtype dtype, const void *x_dev, int64_t n, const void *params_host,
                 void *out_dev, hipStream_t stream);

/* out[i] = f(a[i], b[i]) for i < n, both inputs of type dtype, out of the
 * accumulator type; map2 requires sequences of equal length, so the caller
 * passes one n.  out may alias a or b when the types have equal size (the
 * in-place update of Listing 1's axpy loop).  Errors: MX_ERR_INVALID,
 * MX_ERR_DTYPE. */
mx_status mx_map2(mx_binop f, mx_dtype dtype, const void *a_dev, const void *b_dev, int64_t n,
                  void *out_dev, hipStream_t stream);

/* ======================================================================= */
/* reduce (Appendix A; Appendix "Dynamic Assumptions" for associativity)    */
/* ======================================================================= */

/* *out = reduce op ne x = foldl op ne x, as op(ne, tree_op(x)).
 * ne_host: one host value of the accumulator type.  out_dev: one device value
 * of the accumulator type.  Workspace kind MX_WS_REDUCE with n.
 * Errors: MX_ERR_INVALID, MX_ERR_DTYPE, MX_ERR_WORKSPACE. */
mx_status mx_reduce(mx_redop op, mx_dtype dtype, const void *x_dev, int64_t n, const void *ne_host,
                    void *out_dev, void *ws, size_t ws_bytes, hipStream_t stream);

/* Fused *out = reduce op ne (map2 f a b) without materialising the map2
 * result (the dot product is f = MX_B_MUL, op = MX_ADD; Listing 2 composes a
 * map with a reduce the same way).  I32 inputs are widened before f.
 * Workspace kind MX_WS_REDUCE with n.  Errors as mx_reduce. */
mx_status mx_map2_reduce(mx_binop f, mx_redop op, mx_dtype dtype, const void *a_dev,
                         const void *b_dev, int64_t n, const void *ne_host, void *out_dev, void *ws,
                         size_t ws_bytes, hipStream_t stream);

/* Reverse of the fused dot product *out = sum_i a[i] * b[i] (F32 only):
 * ga[i] = g * b[i], gb[i] = g * a[i] with g = *gout_dev (device scalar), so no
 * host synchronisation is needed.  ga/gb may be NULL to skip that gradient.
 * Errors: MX_ERR_INVALID. */
mx_status mx_dot_adjoint_f32(const float *a_dev, const float *b_dev, int64_t n,
                             const float *gout_dev, float *ga_dev, float *gb_dev,
                             hipStream_t stream);

/* Reverse of y = reduce op ne x (F32; derived, the paper has no reverse
 * mode) with upstream gradient g = *gout_dev (a device float):
 *   MX_ADD            gx[i] = g for every i (a broadcast).
 *   MX_MIN / MX_MAX   the left fold replaces its accumulator only when an
 *                     element is strictly below (above) it, so y is the element
 *                     at the lowest index attaining the extreme, or ne when no
 *                     element improves on ne (ties with ne included, and a NaN
 *                     ne); that element gets g, all others 0.  NaN elements
 *                     are never chosen.  The index is exact and deterministic.
 *   MX_MUL            MX_ERR_UNSUPPORTED.
 * ne_host: one host float (the forward call's ne).  gx must not alias x.
 * Workspace (MIN / MAX only; may be NULL for ADD): kind MX_WS_REDUCE with n.
 * Two launches for MIN / MAX (per-block arg pairs with gx zero-filled, then
 * one block writes g at the arg).  Errors: MX_ERR_INVALID, MX_ERR_SHAPE,
 * MX_ERR_WORKSPACE, MX_ERR_UNSUPPORTED. */
mx_status mx_reduce_adjoint_f32(mx_redop op, const float *x_dev, int64_t n, const float *ne_host,
                                const float *gout_dev, float *gx_dev, void *ws, size_t ws_bytes,
                                hipStream_t stream);

/* ======================================================================= */
/* Nested map (reduce) over a ragged sequence                               */
/* ======================================================================= */
/* The parallel keywords nest (Appendix A, Source Language: map applies a
 * function to every element of a sequence, reduce folds a sequence with an
 * associative operator and its neutral element), so map (reduce op ne) over a
 * sequence of sequences reduces every inner sequence; marshaling (Section
 * 4.3) lays the rows out as one flat value array plus offsets.  The rows may
 * differ in length: the dynamic assumptions that make Futhark's nested arrays
 * regular (Appendix, Dynamic Assumptions) are not needed here. */

/* out[r] = reduce op ne (row r) for r < nseg, where row r is
 * values[offsets[r] .. offsets[r+1]) of the flat layout made by marshaling.
 * values: device, nvalues elements of dtype.  offsets: device int64[nseg+1],
 * non-decreasing, offsets[0] = 0, offsets[nseg] = nvalues (all three
 * validated in debug mode).  Empty rows give ne.  out: device, accumulator
 * type, nseg values.
 * Two schedules, chosen from nseg and nvalues alone: with at least 32 rows
 * per compute unit and at most 16384 values per row on average, blocks take
 * up to 8 consecutive rows each and stream their span (row-span path);
 * otherwise the values are split evenly: each block streams a range of 16 KB
 * chunks, owns the rows that start in it, and rows that run more than a chunk
 * past its range are split across blocks, whose parts are combined in order
 * through the workspace.  Either way the fold order depends only on the
 * offsets, so results repeat bit for bit (for floating point they may differ
 * in the last bits from mx_segmented_reduce_plain's left fold).
 * Workspace: mx_workspace_bytes(MX_WS_SEGMENTED, nvalues, 0) bytes, 256-byte
 * aligned, zero-filled before first use (the call leaves it zero again); NULL
 * is accepted when nvalues <= 2048.  Calls that share a workspace must not
 * overlap.  Errors: MX_ERR_INVALID, MX_ERR_DTYPE, MX_ERR_WORKSPACE,
 * MX_ERR_SHAPE (nvalues < 0; bad offsets in debug mode). */
mx_status mx_segmented_reduce(mx_redop op, mx_dtype dtype, const void *values_dev, int64_t nvalues,
                              const int64_t *offsets_dev, int64_t nseg, const void *ne_host, void *out_dev,
                              void *ws, size_t ws_bytes, hipStream_t stream);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): mx_segmented_reduce without
 * a workspace argument.  The split-row slots live in a 1 MiB device array
 * built into the library, one copy per device, held until the process ends;
 * its address is looked up once per device (in mx_init, else on the first
 * call there).  No allocation of any kind happens in the call.  Accepts
 * nvalues up to mx_segmented_noalloc_max_values() (about 59.6 M, for any
 * dtype) and rejects larger inputs with MX_ERR_WORKSPACE.  Every call on one
 * device shares that device's array: calls that overlap on one device (two
 * streams, two threads) race and must not be issued.  A small fill kernel
 * clears the part of the array a call uses before its reduce, so two launches
 * per call.  Results equal mx_segmented_reduce's bit for bit (same kernels,
 * same schedule).  Other errors as mx_segmented_reduce. */
mx_status mx_segmented_reduce_noalloc(mx_redop op, mx_dtype dtype, const void *values_dev, int64_t nvalues,
                                      const int64_t *offsets_dev, int64_t nseg, const void *ne_host, void *out_dev,
                                      hipStream_t stream);
/* The largest nvalues mx_segmented_reduce_noalloc accepts. */
int64_t mx_segmented_noalloc_max_values(void);

/* Reference "plain" form of mx_segmented_reduce: one thread folds one row
 * sequentially, left to right from ne (no load balancing, uncoalesced, no
 * workspace).  Same contract otherwise. */
mx_status mx_segmented_reduce_plain(mx_redop op, mx_dtype dtype, const void *values_dev, int64_t nvalues,
                                    const int64_t *offsets_dev, int64_t nseg, const void *ne_host,
                                    void *out_dev, hipStream_t stream);

/* Reverse of the row sums out[r] = sum(row r) (F32): every element of row r
 * receives gout[r]: gvalues[e] = gout[r] for offsets[r] <= e < offsets[r+1].
 * gvalues: device float[nvalues], offsets[nseg] = nvalues (debug mode checks
 * it).  Same two schedules as mx_segmented_reduce (no row needs a second
 * block here: every block writes only its own span or range).
 * Errors: MX_ERR_INVALID, MX_ERR_SHAPE. */
mx_status mx_segmented_sum_adjoint_f32(const float *gout_dev, const int64_t *offsets_dev, int64_t nseg,
                                       float *gvalues_dev, int64_t nvalues, hipStream_t stream);

/* Reverse of out[r] = reduce op ne (row r) (F32): row r receives the reverse
 * of its reduce (as mx_reduce_adjoint_f32) with upstream gradient gout[r]:
 * MX_ADD broadcasts gout[r] over the row (mx_segmented_sum_adjoint_f32;
 * values may then be NULL), MX_MIN / MX_MAX put gout[r] at the row's arg
 * element and 0 elsewhere (one wave per row).  gout: device float[nseg];
 * values and gvalues: device float[nvalues] with nvalues = offsets[nseg];
 * gvalues must not alias values.  Errors:
 * MX_ERR_INVALID, MX_ERR_SHAPE (debug mode), MX_ERR_UNSUPPORTED (MX_MUL). */
mx_status mx_segmented_reduce_adjoint_f32(mx_redop op, const float *values_dev, int64_t nvalues,
                                          const int64_t *offsets_dev, int64_t nseg, const float *ne_host,
                                          const float *gout_dev, float *gvalues_dev, hipStream_t stream);

/* ======================================================================= */
/* Dense nested map (map (reduce (+) 0 (map2 (*) row col))) -- FP32 on MFMA */
/* ======================================================================= */
/* The same keywords nested twice over regular data (Appendix A, Source
 * Language): map over the rows of A of map over the columns of B of
 * reduce (+) 0 (map2 (*) row col) -- the matrix product the paper's sgemm
 * benchmarks compute (Section 5.1, Table 1).  Regular nesting is what the
 * Futhark backend requires of nested sequences (Appendix, Dynamic
 * Assumptions); here it is a dense contraction and runs on the matrix cores. */

/* C[i][j] = sum_k op(A)[i][k] * op(B)[k][j], i < M, j < N, k < K, FP32 inputs
 * and FP32 accumulation on the matrix cores.  Row-major, densely packed:
 * op(A) = A stored M x K (ta = 0) or its transpose stored K x M (ta = 1);
 * op(B) = B stored K x N (tb = 0) or its transpose stored N x K (tb = 1).
 * C (M x N) must not alias A or B.  The reverse of C = A B is
 * dA = dC B^T (ta = 0, tb = 1) and dB = A^T dC (ta = 1, tb = 0).
 * Errors: MX_ERR_INVALID. */
mx_status mx_map_map_reduce_f32(int ta, int tb, int64_t M, int64_t N, int64_t K, const float *A_dev,
                                const float *B_dev, float *C_dev, hipStream_t stream);

/* Reference "plain" form: one thread per output element folding over k from
 * global memory.  Same contract. */
mx_status mx_map_map_reduce_plain_f32(int ta, int tb, int64_t M, int64_t N, int64_t K,
                                      const float *A_dev, const float *B_dev, float *C_dev,
                                      hipStream_t stream);

/* ======================================================================= */
/* Sequential loops around map (reduce): N-body (the ODE-solver pattern of   */
/* the paper's CUDA-backend evaluation, Table 2) and its adjoint             */
/* ======================================================================= */
/* Bodies are float4 records (x, y, z, m) -- the record {x, y, z, m} marshalled
 * as one 16-byte element -- and velocities / adjoints are float4 (x, y, z, 0).
 * All pointers are device pointers, 16-byte aligned.  Gravitational
 * acceleration with Plummer softening eps2 > 0:
 *   a_i = G sum_j m_j d_ij (|d_ij|^2 + eps2)^(-3/2),  d_ij = x_j - x_i,
 * a map over bodies of a reduce over bodies (the j = i term is zero).
 * Forward Euler: x_{t+1} = x_t + dt v_t, v_{t+1} = v_t + dt a(x_t).
 * The pair loop is split into slices of j; slice partials are added in slice
 * order, so results are deterministic and independent of the device.
 * Pair entry points need a workspace of mx_nbody_pair_workspace_bytes(n). */
size_t mx_nbody_pair_workspace_bytes(int64_t n);

/* acc4[i] = (a_i, 0).  Errors: MX_ERR_INVALID, MX_ERR_SHAPE, MX_ERR_WORKSPACE. */
mx_status mx_nbody_accel_f32(const float *pos4_dev, int64_t n, float eps2, float G, float *acc4_dev,
                             void *ws, size_t ws_bytes, hipStream_t stream);

/* One fused Euler step (pair loop, slice sum and update).  Outputs must not
 * alias inputs.  Errors as mx_nbody_accel_f32. */
mx_status mx_nbody_step_f32(const float *pos4_dev, const float *vel4_dev, int64_t n, float eps2, float G,
                            float dt, float *pos4_out_dev, float *vel4_out_dev, void *ws, size_t ws_bytes,
                            hipStream_t stream);

/* Reference "plain" form of one step: an untiled pair loop reading bodies from
 * global memory (one thread per body, no j split) into acc4_dev, then a
 * separate update kernel. */
mx_status mx_nbody_step_plain_f32(const float *pos4_dev, const float *vel4_dev, int64_t n, float eps2,
                                  float G, float dt, float *acc4_dev, float *pos4_out_dev,
                                  float *vel4_out_dev, hipStream_t stream);

/* Transposed-Jacobian product of the acceleration map:
 *   out_k = G sum_j M_kj (m_k abar_j - m_j abar_k),
 *   M_kj = s^(-3/2) I - 3 s^(-5/2) d d^T,  d = x_j - x_k,  s = |d|^2 + eps2.
 * Errors as mx_nbody_accel_f32. */
mx_status mx_nbody_accel_vjp_f32(const float *pos4_dev, const float *abar4_dev, int64_t n, float eps2,
                                 float G, float *out4_dev, void *ws, size_t ws_bytes, hipStream_t stream);

/* One reverse step of the discrete adjoint of the Euler step at state x_t:
 *   xbar_t = xbar_{t+1} + dt J_a(x_t)^T vbar_{t+1},  vbar_t = vbar_{t+1} + dt xbar_{t+1}.
 * Outputs must not alias inputs. */
mx_status mx_nbody_adjoint_step_f32(const float *pos4_dev, const float *xbar4_dev, const float *vbar4_dev,
                                    int64_t n, float eps2, float G, float dt, float *xbar4_out_dev,
                                    float *vbar4_out_dev, void *ws, size_t ws_bytes, hipStream_t stream);

/* Kinetic energy 1/2 sum_i m_i |v_i|^2 into one device float. */
mx_status mx_nbody_kinetic_f32(const float *pos4_dev, const float *vel4_dev, int64_t n, float *ke_dev,
                               hipStream_t stream);

/* The loop and its reverse: runs nsteps Euler steps from (pos4, vel4), writes
 * the final kinetic energy to ke_dev, and the gradients of that energy with
 * respect to the initial positions (gx4) and velocities (gv4) by the reverse
 * sweep of the discrete adjoint, storing states only every ckpt_every steps
 * and recomputing each segment forward before its reverse sweep.  The
 * recomputation reproduces the forward states bit for bit.  Launches only
 * (no allocation, no host synchronisation), so the call can be captured in a
 * HIP graph.  1 <= ckpt_every <= 64.  Workspace: mx_nbody_workspace_bytes. */
size_t mx_nbody_workspace_bytes(int64_t n, int nsteps, int ckpt_every);
mx_status mx_nbody_ke_grad_f32(const float *pos4_dev, const float *vel4_dev, int64_t n, float eps2, float G,
                               float dt, int nsteps, int ckpt_every, float *ke_dev, float *gx4_dev,
                               float *gv4_dev, void *ws, size_t ws_bytes, hipStream_t stream);

/* The same loop split at the kinetic energy, for callers that want the
 * gradient later or not at all (an autograd forward and backward):
 * mx_nbody_ke_f32 runs the forward loop, leaves the checkpoints and the final
 * state in ws and writes KE; mx_nbody_ke_vjp_f32, given the same inputs and
 * the ws that call left untouched, runs the checkpointed reverse sweep seeded
 * with g m v_T, g = *gscale_dev (a device float; NULL means 1), and writes
 * g dKE/dx0 and g dKE/dv0.  With gscale_dev NULL the two calls give the
 * gradients of mx_nbody_ke_grad_f32 bit for bit.  Same arguments, workspace
 * size and errors as mx_nbody_ke_grad_f32; n = 0 writes KE = 0. */
mx_status mx_nbody_ke_f32(const float *pos4_dev, const float *vel4_dev, int64_t n, float eps2, float G, float dt,
                          int nsteps, int ckpt_every, float *ke_dev, void *ws, size_t ws_bytes,
                          hipStream_t stream);
mx_status mx_nbody_ke_vjp_f32(const float *pos4_dev, const float *vel4_dev, int64_t n, float eps2, float G,
                              float dt, int nsteps, int ckpt_every, const float *gscale_dev, float *gx4_dev,
                              float *gv4_dev, void *ws, size_t ws_bytes, hipStream_t stream);

/* ======================================================================= */
/* k-means step: map (argmin-reduce) + reduce-by-key (the histo pattern of  */
/* the paper's Parboil evaluation, Table 1)                                  */
/* ======================================================================= */
/* X: n x d row-major float32 points; C: k x d float32 centroids (device).
 *   labels[i]  = the j minimising (dist(x_i, c_j), j) lexicographically, with
 *                dist the squared Euclidean distance: bit-exact to the binary64
 *                definition (an FP32 matrix-core filter whose error bound is
 *                certified per point, binary64 recomputation otherwise)
 *   counts[j]  = #{i : labels[i] = j}                      (int64, exact)
 *   C_out[j]   = mean of the points labelled j, or C[j] when count is 0
 * Supported sizes: 1 <= d <= 64, 1 <= k <= 256, k * d <= 4096, else
 * MX_ERR_UNSUPPORTED.  The step's workgroups need up to 133 KiB of LDS (at
 * d = 17, k = 240), within the 160 KiB a gfx950 workgroup may use; a device
 * that allows less rejects the larger shapes with MX_ERR_UNSUPPORTED.  Deterministic: no float atomics.  C_out must not alias
 * C.  Workspace: mx_kmeans_workspace_bytes(n, d, k), zero-filled once. */
size_t mx_kmeans_workspace_bytes(int64_t n, int d, int k);
mx_status mx_kmeans_step_f32(const float *X_dev, int64_t n, int d, const float *C_dev, int k,
                             int32_t *labels_dev, int64_t *counts_dev, float *C_out_dev, void *ws,
                             size_t ws_bytes, hipStream_t stream);

/* Debug mode only: the number of points whose label the last
 * mx_kmeans_step_f32 call (in debug mode) recomputed in binary64 because the
 * FP32 margin was not certified; -1 before any such call. */
int64_t mx_kmeans_debug_fallbacks(void);

/* Reference "plain" form: one thread per point with distances from global
 * memory (same certified labels), then float atomics for the sums (result
 * order not fixed), then a divide kernel.  Same contract otherwise. */
mx_status mx_kmeans_step_plain_f32(const float *X_dev, int64_t n, int d, const float *C_dev, int k,
                                   int32_t *labels_dev, int64_t *counts_dev, float *C_out_dev, void *ws,
                                   size_t ws_bytes, hipStream_t stream);

/* Within-cluster sum of squares sum_i |x_i - C[labels[i]]|^2 into one device
 * float.  Workspace of at least 256 + 4096 bytes, 256-byte aligned. */
mx_status mx_kmeans_sse_f32(const float *X_dev, int64_t n, int d, const float *C_dev, const int32_t *labels_dev,
                            float *sse_dev, void *ws, size_t ws_bytes, hipStream_t stream);

/* Its gradient with respect to the points (labels and centroids held fixed):
 * G[i] = g * 2 (x_i - C[labels[i]]) with g = *gscale_dev, the upstream
 * gradient of the SSE (device scalar). */
mx_status mx_kmeans_sse_grad_f32(const float *X_dev, int64_t n, int d, const float *C_dev,
                                 const int32_t *labels_dev, const float *gscale_dev, float *G_dev,
                                 hipStream_t stream);

/* ======================================================================= */
/* Batches of uneven independent expressions in one persistent launch       */
/* ======================================================================= */
/* The paper observes that acceleration pays off when work is concentrated in
 * few `accelerate` uses and that small problems leave the GPU idle (Section
 * 5.2).  A batch evaluates many small independent expressions together.
 * Task table (host, int64, one row of 6 per task):
 *   (kind, rows, cols, a_off, b_off, out_off)
 *   kind 0, dot:    out[out_off] = sum_i A[a_off + i] * B[b_off + i], i < cols
 *                   (rows must be 1)
 *   kind 1, matvec: out[out_off + r] = sum_c A[a_off + r*cols + c] * B[b_off + c]
 * over three float32 device pools A, B and out.  Tasks may not overlap in
 * their outputs.  Reverse (upstream gradient gout shaped like out):
 *   dot:    gA[a_off + i] = g * B[b_off + i], gB[b_off + i] = g * A[a_off + i]
 *   matvec: gA[a_off + r*cols + c] = g[r] * B[b_off + c],
 *           gB[b_off + c] = sum_r A[a_off + r*cols + c] * g[r].
 * A plan cuts tasks into tiles of equal bytes, longest first: dots into
 * ranges of tile_elems elements, matvecs into whole-row ranges of about
 * 2 * tile_elems elements (one streamed operand instead of two);
 * forward and backward each run as one persistent launch (blocks_per_cu blocks
 * per compute unit pulling tiles with an atomic ticket) plus one combine
 * launch that adds multi-tile partials in tile order.  Results are
 * deterministic for a given configuration. */
typedef struct mx_batch_config {
    int32_t tile_elems;     /* >= 4096; default 16384 */
    int32_t blocks_per_cu;  /* 1 .. 32; default 8 */
    int32_t reserved[2];
} mx_batch_config;
typedef struct mx_batch_plan mx_batch_plan;

/* Builds a plan (host work plus small device tables: the documented
 * allocation outside the launch path).  cfg may be NULL for defaults.
 * Errors: MX_ERR_INVALID, MX_ERR_SHAPE (bad task row), MX_ERR_HIP. */
mx_status mx_batch_plan_create(const int64_t *table_host, int64_t ntasks, const mx_batch_config *cfg,
                               mx_batch_plan **plan);
mx_status mx_batch_plan_destroy(mx_batch_plan *plan);

/* Workspace for forward, backward and autotuning with any configuration. */
size_t mx_batch_workspace_bytes(const mx_batch_plan *plan);
mx_status mx_batch_get_config(const mx_batch_plan *plan, mx_batch_config *cfg);
mx_status mx_batch_set_config(mx_batch_plan *plan, const mx_batch_config *cfg);

mx_status mx_batch_forward(const mx_batch_plan *plan, const float *A_dev, const float *B_dev, float *out_dev,
                           void *ws, size_t ws_bytes, hipStream_t stream);
mx_status mx_batch_backward(const mx_batch_plan *plan, const float *A_dev, const float *B_dev, const float *gout_dev,
                            float *gA_dev, float *gB_dev, void *ws, size_t ws_bytes, hipStream_t stream);

/* Reference "plain" forms: one launch per task. */
mx_status mx_batch_forward_plain(const mx_batch_plan *plan, const float *A_dev, const float *B_dev, float *out_dev,
                                 hipStream_t stream);
mx_status mx_batch_backward_plain(const mx_batch_plan *plan, const float *A_dev, const float *B_dev,
                                  const float *gout_dev, float *gA_dev, float *gB_dev, hipStream_t stream);

/* Picks tile_elems in {4096 .. 65536} and blocks_per_cu in {2, 4, 8, 16} by
 * timing forward + backward on the given buffers (which it overwrites), and
 * sets it on the plan.  If cache_path (may be NULL) names a JSON-lines file
 * holding an entry for this task shape and device, that entry is used without
 * timing; otherwise the choice is appended to it.  Synchronises the stream.
 * The chosen configuration is returned in *chosen (may be NULL). */
mx_status mx_batch_autotune(mx_batch_plan *plan, const float *A_dev, const float *B_dev, float *out_dev,
                            const float *gout_dev, float *gA_dev, float *gB_dev, void *ws, size_t ws_bytes,
                            const char *cache_path, hipStream_t stream, mx_batch_config *chosen);

/* ======================================================================= */
/* Parboil-shaped kernels (the paper's Table 1 comparison, synthetic data)  */
/* ======================================================================= */
/* histo: counts[k] = #{i : keys[i] = k} for k < nbins (keys >= nbins fall in
 * no bin), a reduce-by-key with integer counts.  counts: nbins uint32 device
 * entries, overwritten.  0 <= n < 2^32 - 1.  Few bins (<= 32768) are counted
 * in per-block LDS histograms and flushed.  More bins, up to 2^27: with a
 * workspace of mx_workspace_bytes(MX_WS_HISTOGRAM, n, nbins) bytes (zero-
 * filled before first use, 256-byte aligned; the call leaves its counters at
 * zero) the keys are first grouped by bucket of 2^11..2^15 bins and each
 * bucket is counted in LDS by one block; with ws = NULL, or past 2^27 bins,
 * by global atomics (slow: every key is a memory-side atomic).  ws is unused
 * when the size query returns 0.  Integer additions commute: the result does
 * not depend on the order.  Errors: MX_ERR_SHAPE, MX_ERR_INVALID,
 * MX_ERR_WORKSPACE. */
mx_status mx_histogram_u32(const uint32_t *keys_dev, int64_t n, int64_t nbins, uint32_t *counts_dev, void *ws,
                           size_t ws_bytes, hipStream_t stream);

/* stencil: one Jacobi sweep of the 7-point stencil on an nx x ny x nz float32
 * grid (x fastest): out = c1 * (x- + x+ + y- + y+ + z- + z+, added in that
 * order) - c0 * centre at interior points, every operation rounded on its
 * own; boundary points are copied.  in and out must not overlap.
 * Errors: MX_ERR_SHAPE (an empty grid, a plane or nz beyond the launch
 * limits), MX_ERR_INVALID (null or identical grids). */
mx_status mx_stencil7_f32(const float *in_dev, float *out_dev, int64_t nx, int64_t ny, int64_t nz, float c0,
                          float c1, hipStream_t stream);

/* mri-q: for voxels (x_i, y_i, z_i) and samples (kx_k, ky_k, kz_k, phi_k),
 * Qr_i = sum_k phi_k cos(2 pi t_ik), Qi_i = sum_k phi_k sin(2 pi t_ik),
 * t_ik = kx_k x_i + ky_k y_i + kz_k z_i (FP32, samples in order; sin and cos
 * of 2 pi t from the hardware sine and cosine of the exactly reduced
 * revolution t - rint(t), absolute error at most 1.26e-7 as measured against
 * binary64).  Errors: MX_ERR_SHAPE, MX_ERR_INVALID. */
mx_status mx_mriq_f32(const float *kx_dev, const float *ky_dev, const float *kz_dev, const float *phi_dev,
                      int64_t nk, const float *x_dev, const float *y_dev, const float *z_dev, int64_t nv,
                      float *qr_dev, float *qi_dev, hipStream_t stream);

/* tpacf: angular pair counts of unit vectors (x, y, z) in float32.  A pair's
 * similarity is the float32 dot product x1 x2 + y1 y2 + z1 z2 (each product
 * and addition rounded on its own); with the decreasing float32 edges
 * e_0 > ... > e_{m-1} (cosines of increasing angles, device array, m <= 32)
 * the pair falls in bin #{b : d < e_b}, one of m + 1 bins (found by binary
 * search, so edges that increase anywhere give undefined bins); counts: m + 1
 * int64 device entries, overwritten.  self_pairs != 0: the pairs i < j of set
 * 1 (set 2 ignored); else all pairs of set 1 x set 2.  Integer counts,
 * bit-exact and order-free.  Errors: MX_ERR_SHAPE, MX_ERR_UNSUPPORTED (m >
 * 32), MX_ERR_INVALID. */
mx_status mx_tpacf_f32(const float *x1_dev, const float *y1_dev, const float *z1_dev, int64_t n1,
                       const float *x2_dev, const float *y2_dev, const float *z2_dev, int64_t n2, int self_pairs,
                       const float *edges_dev, int nedges, int64_t *counts_dev, hipStream_t stream);

/* ======================================================================= */
/* User-defined map bodies                                                   */
/* ======================================================================= */
/* The source language's map and map2 take any first-order function built
 * from its arithmetic (Appendix A; the compilable subset of Section 4.2),
 * not only the fixed bodies above.  A body here is a straight-line program
 * over registers r0..r15 of the element type, one instruction
 *   { op, dst, a, b, imm }   writing r[dst]:
 *   MX_X_IN      r[dst] = element i of input array a        (0 <= a < nin)
 *   MX_X_CONST   r[dst] = imm, rounded to the element type
 *   MX_X_ADD .. MX_X_MAX       r[dst] = r[a] op r[b]
 *                (MIN: r[b] < r[a] ? r[b] : r[a]; MAX likewise with >)
 *   MX_X_NEG .. MX_X_RSQRT     r[dst] = f(r[a])
 *                (NEG -x; ABS x < 0 ? -x : x; SQ x*x; RSQRT 1/sqrt(x))
 * Every operation is rounded on its own (no fused multiply-add), as in the
 * map bodies above.  The body's value is r[out_reg] after the last
 * instruction.
 *
 * mx_expr_create checks the program (1..64 instructions, registers read only
 * after being written, out_reg written, 1 <= nin <= 4, dtype MX_F32 or
 * MX_F64; else MX_ERR_INVALID / MX_ERR_DTYPE) and generates HIP source in
 * which the body is inlined code: a map kernel, a fused map + reduce (one
 * partial pass over a grid that depends only on n, a finish kernel in block
 * order: deterministic), and the reverse mode.  The source is compiled with
 * hipRTC for the current device's architecture on first use and cached for
 * the life of the process (per source text and device), so a chain of
 * operations costs one pass over HBM.  The handle owns host memory only;
 * compiled modules stay loaded until the process ends.  Input and output
 * arrays are device arrays of n elements of the program's dtype; outputs
 * must not overlap inputs. */
typedef enum {
    MX_X_IN = 0, MX_X_CONST = 1,
    MX_X_ADD = 2, MX_X_SUB = 3, MX_X_MUL = 4, MX_X_DIV = 5, MX_X_MIN = 6, MX_X_MAX = 7,
    MX_X_NEG = 8, MX_X_ABS = 9, MX_X_SQ = 10, MX_X_EXP = 11, MX_X_LOG = 12, MX_X_SQRT = 13, MX_X_RSQRT = 14
} mx_xop;
typedef struct {
    int32_t op, dst, a, b;
    double imm;
} mx_xinsn;
typedef struct mx_expr mx_expr;

mx_status mx_expr_create(const mx_xinsn *prog, int ninsn, int nin, int out_reg, mx_dtype dtype, mx_expr **out);
mx_status mx_expr_destroy(mx_expr *e);
/* Compiles the kernels for the current device now (otherwise the first call
 * that needs them does), so that later calls only launch; call it before
 * capturing the expression's launches into a graph. */
mx_status mx_expr_prepare(mx_expr *e);
/* The generated HIP source (owned by the handle; valid until it is destroyed). */
const char *mx_expr_source(const mx_expr *e);

/* out[i] = body(in[0][i], .., in[nin-1][i]).  in_dev: host array of nin
 * device pointers. */
mx_status mx_expr_map(mx_expr *e, const void *const *in_dev, int64_t n, void *out_dev, hipStream_t stream);

/* *out_dev = ne op body(x_0) op body(x_1) ... (reduce of the map, fused; ne
 * from host memory, of the element type).  n = 0 gives ne.  Workspace:
 * mx_expr_workspace_bytes(e, n), 256-byte aligned. */
size_t mx_expr_workspace_bytes(const mx_expr *e, int64_t n);
mx_status mx_expr_map_reduce(mx_expr *e, mx_redop op, const void *const *in_dev, int64_t n, const void *ne_host,
                             void *out_dev, void *ws, size_t ws_bytes, hipStream_t stream);

/* Nested map (reduce op ne . map body) over ragged rows (Listing 2's shape
 * with any body): out[r] = ne op body(x_i) op ... over the elements i of row
 * r, i in [offsets[r], offsets[r+1]); every input is a device array (not
 * NULL, even when all rows are empty) of offsets[nseg] elements laid out by
 * the same int64 device offsets (nseg + 1 entries,
 * offsets[0] = 0, non-decreasing; checked on the device in debug mode).  An
 * empty row gives ne.  Same block-span schedule as mx_segmented_reduce, with
 * the body applied as each element is loaded (no temporary); deterministic.
 * The reverse of a row sum with a body is mx_segmented_sum_adjoint_f32 (the
 * row gradients broadcast over the elements) then mx_expr_vjp with that as
 * gout. */
mx_status mx_expr_segmented_reduce(mx_expr *e, mx_redop op, const void *const *in_dev, const int64_t *offsets_dev,
                                   int64_t nseg, const void *ne_host, void *out_dev, hipStream_t stream);

/* The parallel loop of the CUDA backend (Appendix A, Source Language: `loop n f`
 * calls f i for every i in [0, n) in an undefined order; here f writes tensor slots): for every i < n, out[index[i]] = body(x_i).
 * Iterations run in parallel in no particular order, so the result is defined
 * when the indices are distinct -- the user's guarantee, as in the paper.
 * index: n int64 device entries; out: out_len device elements, slots no index
 * names keep their values; indices outside [0, out_len) are never written.
 * In debug mode the library first checks, on the device, that every index is
 * in range and no slot is written twice (MX_ERR_SHAPE otherwise; nothing is
 * written then), using ws of mx_expr_loop_workspace_bytes(out_len) bytes
 * (256-byte aligned; may be NULL outside debug mode), and synchronises. */
size_t mx_expr_loop_workspace_bytes(int64_t out_len);
mx_status mx_expr_loop_scatter(mx_expr *e, const void *const *in_dev, int64_t n, const int64_t *index_dev,
                               void *out_dev, int64_t out_len, void *ws, size_t ws_bytes, hipStream_t stream);

/* Reverse mode: gin[k][i] = s_i * d body / d input k at element i, with
 * s_i = (gout ? gout[i] : 1) * (gscale ? *gscale : 1) (gout a device array of
 * n, gscale a device scalar; either may be NULL).  The adjoint flows back
 * through the instructions in reverse order; min / max pass it to the
 * operand they returned only (the other operand, and the values behind it
 * that nothing else uses, receive nothing: a pole on the branch not taken
 * leaves the gradient finite), abs to x with the sign of the branch taken;
 * instructions the output does not depend on pass nothing.  gin_dev: host
 * array of nin device pointers, NULL entries skipped.  With gout = NULL and
 * gscale the upstream gradient of a map + reduce (+) this is that reduce's
 * adjoint. */
mx_status mx_expr_vjp(mx_expr *e, const void *const *in_dev, int64_t n, const void *gout_dev,
                      const void *gscale_dev, void *const *gin_dev, hipStream_t stream);

/* ======================================================================= */
/* The general parallel loop (Appendix A, Source Language: `loop n f` runs  */
/* f i for every i in [0, n) in an undefined order; f reads and writes      */
/* tensors through tensorGet / tensorSet -- Listing 1's in-place axpy)      */
/* ======================================================================= */
/* A loop body is a straight-line program over two register files: 64 integer
 * registers (int64, two's-complement wrap-around) and 64 float registers of
 * the loop's float type T (F32 or F64), all starting at 0 in every
 * iteration.  Tensors (the paper's Tensor[Int] / Tensor[Float], rank 1 to 3
 * -- the default maximum rank of Appendix "Dynamic Assumptions") are numbered
 * 0..ntensors-1 (at most 8), each with an element type (F32, F64, I32, I64)
 * and a rank fixed when the loop is created; their data and dimensions are
 * given per run, row-major (the last index fastest).
 *
 *   MX_L_ITER           i[dst] = the iteration number i
 *   MX_L_ICONST         i[dst] = iimm
 *   MX_L_IADD .. IMAX   i[dst] = i[a] op i[b]; IDIV truncates toward zero and
 *                       IMOD is the remainder of that division (a - (a/b) b);
 *                       a zero divisor gives 0 for both; INT64_MIN / -1
 *                       wraps to INT64_MIN
 *   MX_L_INEG           i[dst] = -i[a]
 *   MX_L_I2F            f[dst] = i[a] rounded to T
 *   the map-body codes MX_X_CONST .. MX_X_RSQRT act on the float registers:
 *                       f[dst] = fimm (rounded to T), f[a] op f[b], f(f[a])
 *   MX_L_FGET / IGET    f[dst] / i[dst] = tensor[t][i[a]] (rank 1),
 *                       [i[a], i[b]] (rank 2), [i[a], i[b], i[c]] (rank 3);
 *                       a float tensor for FGET, an integer one for IGET
 *   MX_L_FSET / ISET    tensor[t][index as above] = f[src] / i[src], rounded
 *                       (F32) or wrapped (I32) to the element type
 *
 * Within an iteration the instructions take effect in program order (a get
 * after a set of the same slot sees the stored value).  Iterations run in
 * parallel in no particular order: the result is defined when no slot that
 * one iteration writes is written or read by another -- the user's
 * guarantee, as in the paper.  An index outside its dimension makes a get
 * yield 0 and a set write nothing (never a fault).  Debug mode
 * (mx_set_debug) first traces every iteration without writing anything --
 * the indices as the iteration computes them, its own earlier sets
 * included -- and fails with MX_ERR_SHAPE, before anything is written, when
 * an index is out of range, two iterations set one slot, or an iteration
 * reads a slot another one sets; it uses the workspace of
 * mx_loop_workspace_bytes (one int64 per element of every tensor the body
 * sets, 256-byte aligned; NULL is fine outside debug mode) and synchronises.
 * The body is compiled (hipRTC) into HIP source on first use per device. */
typedef enum {
    MX_L_ITER = 32, MX_L_ICONST = 33,
    MX_L_IADD = 34, MX_L_ISUB = 35, MX_L_IMUL = 36, MX_L_IDIV = 37, MX_L_IMOD = 38, MX_L_IMIN = 39, MX_L_IMAX = 40,
    MX_L_INEG = 41, MX_L_I2F = 42,
    MX_L_FGET = 48, MX_L_IGET = 49, MX_L_FSET = 50, MX_L_ISET = 51
} mx_lop;
typedef struct {
    int32_t op, dst, a, b, c, src, tensor, reserved;  /* reserved: 0 */
    int64_t iimm;
    double fimm;
} mx_linsn;
typedef struct {
    mx_dtype dtype;
    int32_t rank;  /* 1..3 */
} mx_ltype;
typedef struct {
    void *data;       /* device, dims[0] * .. * dims[rank-1] elements */
    int64_t dims[3];  /* entries past the rank are ignored */
} mx_ltensor;
typedef struct mx_loop mx_loop;

/* At most 256 instructions, 8 tensors, registers 0..63.  Checks operands,
 * register files, tensor numbers and element kinds.  Errors: MX_ERR_INVALID,
 * MX_ERR_DTYPE. */
mx_status mx_loop_create(const mx_linsn *prog, int ninsn, const mx_ltype *tensors, int ntensors, mx_dtype float_type,
                         mx_loop **out);
mx_status mx_loop_destroy(mx_loop *l);
mx_status mx_loop_prepare(mx_loop *l);
const char *mx_loop_source(const mx_loop *l);
size_t mx_loop_workspace_bytes(const mx_loop *l, const mx_ltensor *tensors);
/* Runs loop n f with tensors (host array of ntensors descriptors).  Errors:
 * MX_ERR_INVALID, MX_ERR_SHAPE (negative sizes; debug-mode findings),
 * MX_ERR_WORKSPACE (debug mode), MX_ERR_HIP. */
mx_status mx_loop_run(mx_loop *l, int64_t n, const mx_ltensor *tensors, void *ws, size_t ws_bytes,
                      hipStream_t stream);

/* ======================================================================= */
/* HIP graphs of launch sequences (loop bodies, forward + backward passes)  */
/* ======================================================================= */
/* Any sequence of this library's launches on one stream can be captured once
 * and replayed: mx_graph_begin starts capturing `stream` (which must not be the
 * null stream), the following entry points record their kernels instead of
 * running them, and mx_graph_end instantiates the graph.  Capture entry points
 * that only launch (debug mode off; no marshal / unmarshal / plan creation).
 * A replay reuses the captured pointers and sizes. */
typedef struct mx_graph mx_graph;
mx_status mx_graph_begin(hipStream_t stream);
mx_status mx_graph_end(hipStream_t stream, mx_graph **graph);
mx_status mx_graph_launch(mx_graph *graph, hipStream_t stream);
mx_status mx_graph_destroy(mx_graph *graph);

#ifdef __cplusplus
}
#endif

#endif /* MX_H */
