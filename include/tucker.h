/*
 * tucker.h - C ABI of the MI355X (gfx950) ST-HOSVD Tucker compression library.
 *
 * Method: sequentially truncated higher-order SVD (ST-HOSVD) as stated in
 * Ballard, Klinvex & Kolda, "TuckerMPI" (ACM TOMS), Algorithm 1: for each mode
 * n in a caller-chosen order, form the Gram matrix S = Y_(n) Y_(n)^T of the
 * current working tensor (Algorithm 2), take its eigendecomposition, keep the
 * smallest number R_n of leading eigenvectors whose discarded eigenvalues sum
 * to at most eps^2 ||X||^2 / N (eq. Un), and shrink the working tensor with
 * Y <- Y x_n U_n^T (Algorithm 3).  The result satisfies
 * ||X - X^|| <= eps ||X|| (Corollary 1).  Reconstruction of a sub-tensor is a
 * chain of mode products in a flop-minimising order (Sec. 8).
 *
 * Layout (Sec. 4.1, eq. idxtolin): every tensor is a flat array in the
 * "natural descending" order: element (i_0,...,i_{N-1}) sits at
 * sum_n i_n * prod_{k<n} I_k  (mode 0 fastest).  A C-ordered array of shape
 * (I_{N-1},...,I_0) has identical bytes.  Factor matrices U_n are I_n x R_n,
 * column-major (element (i,r) at i + r*I_n), FP64.
 *
 * Pointers: "device" pointers are HIP device memory of the current device;
 * "host" pointers are ordinary host memory.  Sizes are element counts unless
 * stated.  Every call returns a tucker_status; on error no output is produced,
 * nothing leaks, and tucker_last_error() returns a message (thread-local).
 *
 * Streams: work is enqueued on the caller's stream.  Calls that must learn a
 * data-dependent size (the truncation ranks) synchronise that stream.
 */
#ifndef TUCKER_H
#define TUCKER_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TUCKER_OK = 0,
  TUCKER_EINVAL = 1,       /* invalid argument (shape, eps, order, null pointer, non-finite data) */
  TUCKER_ENOMEM = 2,       /* device memory could not be allocated */
  TUCKER_EHIP = 3,         /* a HIP runtime call failed; message holds its error string */
  TUCKER_ENOCONV = 4,      /* an eigenvalue iteration exceeded its iteration cap */
  TUCKER_EUNSUPPORTED = 5  /* combination not supported (e.g. no gfx950 device) */
} tucker_status;

typedef enum { TUCKER_F32 = 0, TUCKER_F64 = 1 } tucker_dtype;

/* Arithmetic of the Gram step.  FP64 is the reference path.  The reduced
 * forms keep the eigensolve, ||X||^2 and the truncation decision in FP64 and
 * carry the working tensor in FP32, with FP32 MFMA products in its mode
 * products; they are not part of the paper (which is FP64 only) and each
 * result's error is reported against the FP64 path.
 *   FP32   : FP32 MFMA products, FP32 accumulation within groups of 32
 *            columns of the unfolding, group sums accumulated in FP64.
 *   BF16X3 : each FP32 value split as x = b0 + b1 + r in bfloat16
 *            (b0 = bf16(x), b1 = bf16(x - b0)); products b1*b0' + b0*b1' +
 *            b0*b0' on BF16 MFMA, FP32 accumulation within groups of 256
 *            columns, FP64 across groups (Henry, Tang & Heinecke, ARITH
 *            2019).  The dropped b1*b1' term makes the Gram a slight
 *            under-estimate (relative ~1e-6).
 *   BF16X6 : three pieces b0, b1, b2 and the six products b2*b0' + b0*b2' +
 *            b1*b1' + b1*b0' + b0*b1' + b0*b0', FP32 accumulation within
 *            groups of 32 columns, FP64 across groups.
 *   AUTO   : the cheapest form whose predicted error of the truncation's tail
 *            sums, delta * ||X||^2, is at most 1% of the slack of a 1.05 eps
 *            target, (1.05^2 - 1) eps^2 ||X||^2 / N; delta = 2^-16/3 for
 *            BF16X3 (its bias) and 2^-23 for FP32 (the FP32 rounding of the
 *            working tensor and the accumulation); else FP64.  FP64 data and
 *            the fixed-rank form (no error target) always take FP64.  So FP32
 *            is chosen for eps >= 0.0108 sqrt(N), BF16X3 for eps >= 0.0705
 *            sqrt(N).  tucker_gram_precision reports the choice.
 * Range handling (per-slice scaling): every reduced Gram is checked on the
 * device.  If an entry is not finite, its trace differs from the FP64 sum of
 * squares of the working tensor by more than 1e-3 relative, or a diagonal
 * entry's mean square lies outside [2^-100, 2^100] (squares near the FP32
 * underflow or overflow range), the Gram of that mode is redone on a copy of
 * the working tensor in which every hyperslice of mode n (every row of the
 * unfolding) is divided by a power of two near its largest magnitude, and S
 * is multiplied back exactly (tucker_gram_scaled reports it); if that check
 * fails as well, the Gram is recomputed in FP64 (tucker_gram_precision). */
typedef enum {
  TUCKER_GRAM_FP64 = 0,
  TUCKER_GRAM_FP32 = 1,
  TUCKER_GRAM_BF16X3 = 2,
  TUCKER_GRAM_BF16X6 = 3,
  TUCKER_GRAM_AUTO = 4
} tucker_gram_prec;

/* Device memory allocator hook.  By default the library takes device memory
 * from its own stream-ordered caching pool (hipMalloc when nothing cached
 * fits).  With an allocator set, every block (handles, batch plans, scratch)
 * comes from alloc(bytes, ctx, stream), where `stream` is the stream the
 * block will be used on, and goes back through free(ptr, ctx, stream) in
 * stream order: the allocator may hand the block to later work on that
 * stream without synchronisation, as a caching allocator like PyTorch's
 * does.  alloc returns NULL when it cannot satisfy the request (the call then
 * fails with TUCKER_ENOMEM).  A block is returned to the allocator that
 * produced it, even after the setting changes.  The callbacks are called
 * from the calling thread, never concurrently for one call. */
typedef struct {
  void* (*alloc)(size_t bytes, void* ctx, hipStream_t stream);
  void (*free)(void* ptr, void* ctx, hipStream_t stream);
  void* ctx;
} tucker_allocator;

/* Set (a) or clear (NULL: the built-in pool) the allocator for all later
 * allocations of the library in this process.  EINVAL if a callback is NULL. */
tucker_status tucker_set_allocator(const tucker_allocator* a);
/* Return the built-in pool's idle blocks of the current device to HIP
 * (synchronises the device first: work in flight may still read them). */
tucker_status tucker_empty_cache(void);

typedef struct tucker_t tucker_t; /* opaque result handle */

#define TUCKER_MAX_MODES 16

/* ------------------------------------------------------------------------
 * Compression
 * ------------------------------------------------------------------------ */

/* ST-HOSVD of one tensor (Algorithm 1).
 *   data       device, prod(dims) values of `dtype`, natural descending; read only.
 *   dims       host, N sizes, each >= 1; 1 <= N <= TUCKER_MAX_MODES.
 *   eps        relative error target, finite and >= 0.
 *   mode_order host, N ints: a permutation of 0..N-1 giving the order in which
 *              modes are processed (Sec. 7 discusses the choice); NULL = 0..N-1.
 *   prec       Gram arithmetic (see tucker_gram_prec).  TUCKER_GRAM_FP64 keeps
 *              the working tensor in FP64 (FP64 MFMA products throughout);
 *              the reduced forms need dtype == TUCKER_F32 and keep the working
 *              tensor and the core in FP32; AUTO chooses.
 *   stream     HIP stream for all work (0 = default stream).
 *   out        receives a new handle owning core, factors, eigenvalues and
 *              ranks; release it with tucker_free.
 * Errors: EINVAL for bad arguments or non-finite ||X||^2; ENOMEM (predicted
 *         before the launches, see tucker_sthosvd_memory, or from a failed
 *         allocation); EHIP; ENOCONV if the eigensolver exceeded its
 *         iteration cap; EUNSUPPORTED for a mode above 2304 (the largest
 *         matrix of the eigensolver).
 * Waits once per mode for the rank R_n, which is read back while that mode's
 * eigenvectors are being formed, and synchronises `stream` before returning. */
tucker_status tucker_sthosvd(const void* data, tucker_dtype dtype, const int64_t* dims, int N,
                             double eps, const int* mode_order, tucker_gram_prec prec,
                             hipStream_t stream, tucker_t** out);

/* Fixed-rank ST-HOSVD (Sec. 9.4.1: the user gives the core size and the error
 * follows): as tucker_sthosvd with R_n = min(ranks[n], J_n) in place of the
 * eq. Un rule.  ranks: host, N values >= 1.  tucker_discarded reports the
 * discarded energy per mode (their sum is ||X - X^||^2).  With FP64 Grams
 * the whole compression is enqueued without a host round trip and `stream`
 * is synchronised once at the end; reduced forms read the range check back
 * per mode.  AUTO takes FP64 here (there is no error target). */
tucker_status tucker_sthosvd_ranks(const void* data, tucker_dtype dtype, const int64_t* dims, int N,
                                   const int64_t* ranks, const int* mode_order, tucker_gram_prec prec,
                                   hipStream_t stream, tucker_t** out);

/* Mode order by predicted cost (host only).  The cost model of Sec. 7: the
 * step that processes mode n does (J_n^2 + 2 R_n J_n) K flops (its Gram, with
 * the symmetric count, and its mode product), K the product of the other
 * current sizes; the eigensolve's (10/3) I_n^3 does not depend on the order.
 *   ranks   host, N values (given or estimated core sizes, capped at I_n):
 *           the order of least total flops, found exactly by dynamic
 *           programming over the sets of processed modes (2^N N steps); ties
 *           keep the first minimum found.  NULL (ranks unknown, the eps
 *           rule): increasing I_n, ties by mode index, which is the optimum
 *           when every mode shrinks by the same factor (later steps work on
 *           smaller tensors, so the larger modes go last).
 *   order_out host, N ints; flops_out host, the predicted flops (0 when ranks
 *           is NULL), may be NULL. */
tucker_status tucker_sthosvd_order(int N, const int64_t* dims, const int64_t* ranks, int* order_out,
                                   double* flops_out);

/* Predicted device memory of a compression (host only; the input tensor
 * is not counted): the handle's factors and eigenvalues, the Gram and
 * eigensolver workspaces, and the largest pair of working tensors with the
 * scratch of one step.  ranks: host, N values, or NULL for an upper bound
 * (no truncation).  prec: FP64 or a reduced form.  tucker_sthosvd and
 * tucker_sthosvd_ranks compare this prediction (the whole run for given
 * ranks, else the first step, then each next working tensor once its rank is
 * known) with the free device memory plus the pool's idle blocks, and return
 * TUCKER_ENOMEM before launching work that would not fit. */
tucker_status tucker_sthosvd_memory(tucker_dtype dtype, const int64_t* dims, int N, const int64_t* ranks,
                                    const int* mode_order, tucker_gram_prec prec, size_t* bytes);

/* Handle accessors.  Pointers returned are owned by the handle and valid until
 * tucker_free.  All of them are cheap and do not synchronise. */
int tucker_ndims(const tucker_t* t);
/* host out[N]: the original sizes I_n / the ranks R_n. */
tucker_status tucker_dims(const tucker_t* t, int64_t* dims_out);
tucker_status tucker_ranks(const tucker_t* t, int64_t* ranks_out);
/* host out[N]: mode_order used. */
tucker_status tucker_mode_order(const tucker_t* t, int* order_out);
/* Core G (device, prod(R) values of *dtype, natural descending). */
const void* tucker_core(const tucker_t* t, tucker_dtype* dtype);
/* Factor U_n (device, I_n x R_n column-major FP64, orthonormal columns; in
 * each column the entry of largest magnitude is positive, lowest row on ties). */
const double* tucker_factor(const tucker_t* t, int n);
/* Eigenvalues of mode n's Gram matrix (device, FP64, descending); count in
 * *count = J_n, the size of mode n of the working tensor when it was processed. */
const double* tucker_eigenvalues(const tucker_t* t, int n, int64_t* count);
/* ||X||^2 in FP64. */
double tucker_norm2(const tucker_t* t);
/* host out[N]: per mode, the sum of the discarded (clamped) eigenvalues;
 * by Corollary 1 their total is ||X - X^||^2 (up to rounding). */
tucker_status tucker_discarded(const tucker_t* t, double* disc_out);
/* host out[4*N]: per mode (in mode index order) milliseconds, measured with HIP
 * events on the call's stream: [4n+0] Gram step (main kernel, split-K
 * reduction, norm), [4n+1] eigensolve + truncation, [4n+2] TTM, [4n+3] the
 * main Gram kernel alone. */
tucker_status tucker_timings(const tucker_t* t, double* ms_out);
/* host out[N]: per mode, the Gram arithmetic actually used: the requested
 * one (AUTO resolved), or TUCKER_GRAM_FP64 where the range handling fell back
 * to it. */
tucker_status tucker_gram_precision(const tucker_t* t, tucker_gram_prec* prec_out);
/* host out[N]: per mode, 1 if its Gram ran on the per-slice scaled copy. */
tucker_status tucker_gram_scaled(const tucker_t* t, int* scaled_out);
void tucker_free(tucker_t* t);

/* A handle from a given Tucker model (core G, factors U_n), e.g. one
 * compressed elsewhere and moved to this machine for reconstruction (Sec. 8).
 *   core     device, prod(ranks) values of core_dtype, natural descending.
 *   dims     host, N original sizes I_n >= 1.  ranks: host, N values, 1 <= R_n <= I_n.
 *   factors  host array of N device pointers; U_n is I_n x R_n column-major FP64.
 * Everything is copied into handle-owned memory (synchronises `stream`); the
 * handle has no eigenvalues (count 0), zero norm and discarded energies, and
 * its Gram precision entries read FP64.  Errors: EINVAL, ENOMEM, EHIP. */
tucker_status tucker_create(const void* core, tucker_dtype core_dtype, const int64_t* dims, const int64_t* ranks,
                            int N, const double* const* factors, hipStream_t stream, tucker_t** out);

/* ------------------------------------------------------------------------
 * Reconstruction (Sec. 8): X^[begin:end) = G x_0 U_0[b_0:e_0,:] ... x_{N-1} U_{N-1}[b:e,:]
 * ------------------------------------------------------------------------ */

/* Index ranges are the RANGE operators with step 1 of tucker_reconstruct_ops
 * (post-processing attached with tucker_set_postprocess is applied).
 * begin/end  host, N each; half-open index ranges 0 <= begin_n < end_n <= I_n;
 *            NULL means the full range.
 * order      host, N ints, permutation giving the order of the mode products;
 *            NULL = the flop-minimising order of tucker_reconstruct_order.
 * out        device, caller-allocated, prod(end-begin) values of out_dtype,
 *            natural descending.
 * Products are FP64 MFMA, except that an FP32 core (reduced-precision
 * compression) reconstructed into FP32 output uses FP32 MFMA products.
 * Scratch for intermediate results is taken from the device's stream-ordered
 * pool and released before return (stream order).  The call may use any
 * stream: tucker_free then orders the release of the handle's memory after
 * the work enqueued here. */
tucker_status tucker_reconstruct(const tucker_t* t, const int64_t* begin, const int64_t* end,
                                 const int* order, void* out, tucker_dtype out_dtype,
                                 hipStream_t stream);

/* Flop-minimising order of a Multi-TTM G (sizes R) -> Z (sizes K), Sec. 8:
 * mode i precedes mode j when K_i R_i R_j + K_i R_j K_j < R_i R_j K_j + R_i K_i K_j,
 * i.e. sorting by 1/R_i - 1/K_i ascending (ties: lower mode first).
 * ranks, out_sizes: host, N each, >= 1.  order_out: host, N ints.  Host only. */
tucker_status tucker_reconstruct_order(int N, const int64_t* ranks, const int64_t* out_sizes,
                                       int* order_out);

/* ------------------------------------------------------------------------
 * Reconstruction through per-mode linear operators (Sec. 8): the result is
 *   Z = G x_0 (C_0^T U_0) x_1 (C_1^T U_1) ... x_{N-1} (C_{N-1}^T U_{N-1}),
 * i.e. the operator C_n^T (K_n x I_n) applied along every mode of X^.  The
 * paper's examples: down-sampling a mode by averaging neighbouring indices,
 * selecting one variable or one time step, and all-ones operators for a
 * summary statistic (the mean of one variable over space and time).
 * ------------------------------------------------------------------------ */
typedef enum {
  TUCKER_OP_IDENTITY = 0, /* every row (K_n = I_n) */
  TUCKER_OP_RANGE = 1,    /* rows begin, begin+step, ... below end: K_n = ceil((end-begin)/step) */
  TUCKER_OP_AVERAGE = 2,  /* down-sampling by averaging: output k is the mean of rows
                             [begin + k*step, min(begin + (k+1)*step, end)); K_n = ceil((end-begin)/step) */
  TUCKER_OP_SUM = 3,      /* one output, the sum of rows [begin, end): K_n = 1 */
  TUCKER_OP_MEAN = 4,     /* one output, their mean: K_n = 1 */
  TUCKER_OP_MATRIX = 5    /* a given operator: `matrix` (device, FP64) holds C_n^T, `rows` x I_n, row-major */
} tucker_op_kind;

typedef struct {
  int kind;             /* tucker_op_kind */
  int64_t begin, end;   /* RANGE, AVERAGE, SUM, MEAN: 0 <= begin < end <= I_n */
  int64_t step;         /* RANGE: stride >= 1; AVERAGE: window width >= 1 */
  int64_t rows;         /* MATRIX: K_n >= 1 */
  const double* matrix; /* MATRIX: device pointer; read during the call */
} tucker_op;

/* Order rules for the mode products of a reconstruction (Sec. 8).
 *   FLOPS : mode i precedes mode j when K_i R_i R_j + K_i R_j K_j < R_i R_j K_j + R_i K_i K_j
 *           (tucker_reconstruct_order);
 *   MEMORY: smallest temporary footprint: the intermediate after a product grows
 *           by K_i / R_i, so modes are taken by increasing K_i / R_i, i.e. mode i
 *           precedes mode j when R_i / K_i > R_j / K_j (ties: lower mode first).
 *           The paper prints this comparison with the opposite sign; its own
 *           measurements (the order 43120 using the least memory on both SP
 *           scenarios) follow the rule as stated here. */
typedef enum { TUCKER_ORDER_FLOPS = 0, TUCKER_ORDER_MEMORY = 1 } tucker_order_rule;

/* K_n of an operator applied to a mode of size I (host only); EINVAL for an
 * invalid operator. */
tucker_status tucker_op_size(const tucker_op* op, int64_t I, int64_t* K);

/* Order of the mode products for ranks R and output sizes K under `rule`
 * (host only; ranks, out_sizes >= 1; order_out: N ints). */
tucker_status tucker_reconstruct_order_rule(int N, const int64_t* ranks, const int64_t* out_sizes,
                                            tucker_order_rule rule, int* order_out);

/* Z as above.
 *   ops        host, N operators (NULL = identity on every mode).
 *   order      host, N ints, a permutation (the order of the mode products);
 *              NULL = by `rule`.
 *   out        device, caller-allocated, prod(K_n) values of out_dtype,
 *              natural descending.
 * The mode-n factor C_n^T U_n is formed on the device (FP64) first; then the
 * mode products run as in tucker_reconstruct.  Post-processing stored with
 * tucker_set_postprocess is applied (see there).
 * Errors: EINVAL (handle, operators, order, dtype, out), ENOMEM, EHIP. */
tucker_status tucker_reconstruct_ops(const tucker_t* t, const tucker_op* ops, const int* order,
                                     tucker_order_rule rule, void* out, tucker_dtype out_dtype,
                                     hipStream_t stream);

/* ------------------------------------------------------------------------
 * Pre- and post-processing by hyperslice (Sec. 3.5).  A hyperslice of mode n
 * is the set of elements with one fixed index i_n (for a variable mode: all
 * values of one variable).  Statistics are gathered per hyperslice, one
 * affine map per hyperslice shifts and/or scales its values before
 * compression, and the stored vectors undo the map after reconstruction.
 * ------------------------------------------------------------------------ */
#define TUCKER_NSTATS 6
typedef enum {
  TUCKER_STAT_MEAN = 0,
  TUCKER_STAT_STD = 1,   /* standard deviation, dividing by the element count */
  TUCKER_STAT_MIN = 2,
  TUCKER_STAT_MAX = 3,
  TUCKER_STAT_NORM1 = 4, /* sum of |x| */
  TUCKER_STAT_NORM2 = 5  /* sqrt(sum of x^2) */
} tucker_stat;

/* Statistics of the I_n hyperslices of mode n of X (device, natural
 * descending, `dtype`): stats (device) receives TUCKER_NSTATS x I_n doubles,
 * stats[s * I_n + i] for statistic s of slice i.  Accumulated in FP64 in a
 * fixed order (two passes over X: the mean first).  Asynchronous. */
tucker_status tucker_slice_stats(const void* X, tucker_dtype dtype, const int64_t* dims, int N, int n,
                                 double* stats, hipStream_t stream);

/* The two pre-processing methods of Sec. 3.5, from the statistics above:
 *   STANDARDIZE: shift = mean, scale = standard deviation;
 *   MAX        : shift = 0,    scale = max |x|.
 * A zero scale (a constant slice) becomes 1.  stats, shift, scale: device,
 * J values each for shift and scale.  Asynchronous. */
typedef enum { TUCKER_SCALE_STANDARDIZE = 0, TUCKER_SCALE_MAX = 1 } tucker_scale_method;
tucker_status tucker_scaling_vectors(const double* stats, int64_t J, tucker_scale_method method, double* shift,
                                     double* scale, hipStream_t stream);

/* Y = (X - shift_i) / scale_i on every element of hyperslice i of mode n
 * (inverse == 0), or Y = X * scale_i + shift_i with one rounding (inverse != 0),
 * computed in FP64 and rounded once to ydtype.  X and Y: device, natural
 * descending; Y may be X when the dtypes agree (in place).  shift, scale:
 * device, I_n values; scale entries must be non-zero.  Asynchronous. */
tucker_status tucker_slice_transform(const void* X, tucker_dtype xdtype, const int64_t* dims, int N, int n,
                                     const double* shift, const double* scale, int inverse, void* Y,
                                     tucker_dtype ydtype, hipStream_t stream);

/* Statistics, vectors and forward map in one call: Y = the pre-processed X
 * (Y may be X), shift and scale (device, I_n values each) receive the vectors
 * to store with the compressed tensor.  Asynchronous. */
tucker_status tucker_preprocess(const void* X, tucker_dtype xdtype, const int64_t* dims, int N, int n,
                                tucker_scale_method method, void* Y, tucker_dtype ydtype, double* shift,
                                double* scale, hipStream_t stream);

/* Attach the pre-processing of mode n to a handle (copies I_n values of
 * shift and scale, device pointers; shift may be NULL for a pure scaling).
 * Every later reconstruction returns data in the original units: the scale is
 * folded into the mode-n factor (C_n^T diag(scale) U_n) and the shift adds the
 * separable term (C_n^T shift) x prod_{m != n} (C_m^T 1).  Synchronises
 * `stream`. */
tucker_status tucker_set_postprocess(tucker_t* t, int n, const double* shift, const double* scale,
                                     hipStream_t stream);

/* ------------------------------------------------------------------------
 * Batching form (not in the paper): many independent tensors of the same
 * order N, every mode size <= 128, compressed together.  A plan binds the
 * data pointers and sizes and owns all device memory; running it only
 * enqueues kernels on the stream (no allocation, no synchronisation, no
 * memset), so a run may be captured in a HIP graph and replayed.  Ranks are
 * decided on the device (device-side sizes); each step is one batched Gram,
 * one batched eigensolve + truncation and one batched TTM over all tensors.
 * Tile sizes of the batched Gram and TTM are chosen by timing candidates on
 * the first plan of a shape class (count, N, precision, input type, total
 * size to within 2x) and remembered for the process.
 * ------------------------------------------------------------------------ */
typedef struct tucker_batch tucker_batch;

/*   count      number of tensors, 1 .. 4194303 (2^22 - 1).
 *   data       host array of `count` device pointers (natural descending, `dtype`).
 *   dims       host, count x N sizes (tensor t's sizes at dims + t*N), each 1..128.
 *   eps, mode_order, prec: as for tucker_sthosvd (the order is shared; AUTO
 *              is resolved once for the batch).
 *   stream     used for the plan's uploads and its tuning runs; synchronised.
 * Errors: EINVAL (arguments), EUNSUPPORTED (a size above 128, or more than 2^23 Gram or
 *         2^24 product work items in a step), ENOMEM, EHIP. */
tucker_status tucker_batch_create(int count, const void* const* data, tucker_dtype dtype,
                                  const int64_t* dims, int N, double eps, const int* mode_order,
                                  tucker_gram_prec prec, hipStream_t stream, tucker_batch** out);
/* Enqueue the whole compression on `stream` (capturable; reads the data
 * pointers given at creation each time it runs). */
tucker_status tucker_batch_run(tucker_batch* b, hipStream_t stream);
/* tucker_batch_create followed by tucker_batch_run. */
tucker_status tucker_sthosvd_batched(int count, const void* const* data, tucker_dtype dtype,
                                     const int64_t* dims, int N, double eps, const int* mode_order,
                                     tucker_gram_prec prec, hipStream_t stream, tucker_batch** out);
/* Results of the last run; each call synchronises the stream given to the
 * last tucker_batch_run (after replaying a captured run on another stream,
 * synchronise that stream first).  host out[count*N] ranks; host out[count]
 * ||X_t||^2. */
tucker_status tucker_batch_ranks(tucker_batch* b, int64_t* ranks_out);
tucker_status tucker_batch_norm2(tucker_batch* b, double* norm2_out);
/* Tensor i of the last run as a standalone handle (copies of its core,
 * factors and eigenvalues); release with tucker_free. */
tucker_status tucker_batch_item(tucker_batch* b, int i, tucker_t** out);
/* host out[count]: per tensor of the last run, bit 0 (1) if its data holds a
 * non-finite value (its results are then meaningless), bit 1 (2) if a
 * reduced-precision Gram of it failed the range check and was recomputed in
 * FP64 on the device (the batched form's range handling: checked per tensor
 * and step against the FP64 sum of squares of its working tensor, as in
 * tucker_gram_prec).  Synchronises as tucker_batch_ranks. */
tucker_status tucker_batch_status(tucker_batch* b, int* status_out);
/* The chosen tiles: Gram chunks per work item, TTM 64-column tiles per item. */
tucker_status tucker_batch_tiles(const tucker_batch* b, int* gram_chunks, int* ttm_tiles);
/* Synchronises the last run's stream, then releases everything. */
void tucker_batch_free(tucker_batch* b);

/* ------------------------------------------------------------------------
 * Single steps of the path, for testing and for callers composing their own
 * loop.  All pointers are device pointers except dims (host).
 * ------------------------------------------------------------------------ */

/* S = Y_(n) Y_(n)^T (Algorithm 2) for Y of sizes dims (natural descending) in
 * `dtype`; S is J_n x J_n FP64, full symmetric.  If norm2 is non-NULL, the
 * FP64 sum of squares of Y is written to it (device, one double).
 * prec selects the arithmetic; the reduced forms need dtype == TUCKER_F32 and
 * are not range-guarded here. */
tucker_status tucker_gram(const void* Y, tucker_dtype dtype, const int64_t* dims, int N, int n,
                          tucker_gram_prec prec, double* S, double* norm2, hipStream_t stream);

/* Eigendecomposition of a J x J symmetric FP64 matrix S (device, read only)
 * followed by the truncation rule eq. Un with threshold thr:
 *   lam  device, J values, eigenvalues in descending order;
 *   U    device, J x J column-major: columns 0..R-1 receive the leading
 *        eigenvectors (sign convention as for tucker_factor); the rest is scratch;
 *   R    device, one int64: the chosen rank (1 <= R <= J);
 *   disc device, one double: sum of the discarded (clamped) eigenvalues.
 * Errors: EINVAL for J outside 1..2304 (the largest matrix of the
 * eigensolver), a NULL pointer or a negative or non-finite thr.
 * Does not synchronise. */
tucker_status tucker_eig_truncate(const double* S, int64_t J, double thr, double* lam, double* U,
                                  int64_t* R, double* disc, hipStream_t stream);

/* tucker_eig_truncate without any allocation, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, kernels and results as
 * tucker_eig_truncate; the eigensolver's workspace is a static device array
 * of the library sized for J <= 1024 (16.8 MB per device, held until the
 * process ends), so J above 1024 is rejected with EINVAL.  The first call on
 * a device looks up the array's device address.  Every call on a device uses
 * that device's one workspace: calls that overlap on one device (different
 * streams, or host threads) race and must be serialised by the caller. */
tucker_status tucker_eig_truncate_noalloc(const double* S, int64_t J, double thr, double* lam, double* U,
                                          int64_t* R, double* disc, hipStream_t stream);

/* Mode product Z = Y x_n M (Sec. 2.2.3, Algorithm 3), M a K x J_n FP64
 * matrix with element (k,j) at M[k*msk + j*msj]; Z has the sizes of Y with
 * mode n replaced by K, in `zdtype`.  Y in `ydtype`.  fp32_products != 0
 * rounds M and Y to FP32 and uses FP32 MFMA products (FP32 accumulation);
 * otherwise products and accumulation are FP64. */
tucker_status tucker_ttm(const void* Y, tucker_dtype ydtype, const int64_t* dims, int N, int n,
                         const double* M, int64_t K, int64_t msk, int64_t msj, void* Z,
                         tucker_dtype zdtype, int fp32_products, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Diagnostics
 * ------------------------------------------------------------------------ */
const char* tucker_last_error(void);
const char* tucker_version(void);

#ifdef __cplusplus
}
#endif
#endif /* TUCKER_H */
