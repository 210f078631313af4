/* sketch.h - C ABI of the MI355X sketching library (libhsketch.so).
 *
 * The library computes the randomized sketches used by adaptive HSS
 * construction (Yaniv, Ghysels, Malik, Boateng, Li, arXiv 2302.01977):
 *   S  = A R     (section 1: post-multiplication of A by a tall random n x d R)
 *   S' = A^T R   (section 1: needed for the row space when A is nonsymmetric;
 *                 A is real here, so A^* = A^T)
 * where R = [R_0 | R_1 | ...] is a Gaussian, SJLT or SRHT operator (section 2.4),
 * grown block by block as Algorithm 1 appends JL-Operator(dd, n) columns.
 *
 * Conventions for every entry point
 *   - Return value: SK_OK (0) or a negative status; nothing throws across the ABI.
 *     sketch_last_error() returns a thread-local message for the last failure.
 *   - Matrices are column-major with an explicit leading dimension (in elements).
 *   - "device" pointers are HIP device allocations owned by the caller; the
 *     library never frees them.  "host" pointers are ordinary host memory.
 *   - stream is a hipStream_t (NULL = the default stream).  Compute calls only
 *     enqueue work and return; they do not synchronise the host.  Calls marked
 *     "synchronises" wait for the stream before returning.
 *   - One stream per context at a time: the compute calls (sketch_apply,
 *     sketch_extend, sketch_rerun, sketch_adjoint, sketch_apply_batched) keep
 *     split-source partial sums and other scratch in the context's workspace.
 *     Calls made through one context must be ordered on one stream (or the
 *     caller orders their streams with events); two streams running compute
 *     calls of one context at the same time race on that workspace.  Use one
 *     context per concurrent stream.  A context is used by one host thread at a
 *     time.
 *   - Operator entries are a pure function of (seed, block, index): see the
 *     counter layout in paper_2302_01977_amd/csrc/spec.hpp.  Each block is its
 *     own JL operator normalised by its own width w_b (Gaussian N(0, 1/w_b),
 *     SJLT +-1/sqrt(alpha), SRHT +-1/sqrt(w_b)).
 */
#ifndef HSKETCH_SKETCH_H
#define HSKETCH_SKETCH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define SK_OK 0
#define SK_EINVAL (-1)       /* bad argument: NULL pointer, ld < rows, width <= 0, alpha does not divide a width, ... */
#define SK_EUNSUPPORTED (-2) /* valid request this build does not implement (e.g. the batched call with an SRHT operator) */
#define SK_ENOMEM (-3)       /* device or host allocation failed */
#define SK_EHIP (-4)         /* a HIP runtime call failed; the message carries hipGetErrorString */
#define SK_ESTATE (-5)       /* released, foreign or corrupted handle/context */

/* operator kinds (section 2.4) */
#define SK_GAUSSIAN 0 /* i.i.d. N(0, 1/w_b) entries (values on the bfloat16 grid) */
#define SK_SJLT 1     /* block construction: alpha chunks of w_b/alpha columns, one +-1/sqrt(alpha) per chunk and row */
#define SK_SRHT 2     /* R = D H P / sqrt(w_b)-scaled; D Rademacher, H Sylvester-Hadamard (natural order) of dimension
                         nu = 2^ceil(log2 n) restricted to its first n rows, P uniform samples of [nu] */

/* element types of A and of the sketches */
#define SK_F64 0
#define SK_F32 1

/* Gaussian arithmetic (ignored by SJLT and SRHT, which add in the element type) */
#define SK_PREC_NATIVE 0 /* FP64 A: FP64 matrix cores; FP32 A: FP64 matrix cores on promoted values */
#define SK_PREC_BF16 1   /* FP32 A rounded to bf16, bf16 matrix cores, FP32 accumulation */
#define SK_PREC_BF16X3 2 /* FP32 A split exactly into three bf16 parts, three bf16 products, FP32 accumulation */

/* input kinds */
#define SK_DENSE 0  /* stored matrix A */
#define SK_POINTS 1 /* matrix-free Gaussian kernel K_ij = exp(-|x_i - x_j|^2 / (2 h^2)) + shift * delta_ij */

typedef struct sk_ctx sk_ctx;       /* per-device state: properties, workspace, tuning table */
typedef struct sk_handle sk_handle; /* one operator R = [R_0 | R_1 | ...] and its device metadata */

typedef struct {
  int32_t input;     /* SK_DENSE or SK_POINTS */
  int32_t dtype;     /* SK_F64 or SK_F32 (SK_POINTS: SK_F32) */
  int64_t m, n, lda; /* DENSE: A is m x n column-major, lda >= max(1, m) */
  const void *A;     /* DENSE: device pointer to A */
  int32_t symmetric; /* DENSE: nonzero = A is symmetric, S' is not formed */
  int32_t dim;       /* POINTS: coordinates per point, 1..4 */
  const float *X;    /* POINTS: device pointer, N x dim row-major FP32 */
  int64_t N;         /* POINTS: number of points; the kernel matrix is N x N */
  float h;           /* POINTS: bandwidth h > 0 */
  float shift;       /* POINTS: diagonal shift */
} sk_input;

/* SJLT constructions (section 2.4.3) */
#define SK_SJLT_BLOCK 0 /* alpha chunks of w_b/alpha columns, one nonzero per chunk and row */
#define SK_SJLT_GRAPH 1 /* alpha distinct columns per row drawn uniformly from the w_b columns of the block */

typedef struct {
  int32_t kind;         /* SK_GAUSSIAN, SK_SJLT or SK_SRHT */
  int32_t alpha;        /* SJLT: nonzeros per row, 1..32 (block construction: must divide every block width;
                           graph construction: at most every block width) */
  int32_t construction; /* SJLT: SK_SJLT_BLOCK or SK_SJLT_GRAPH; others: 0 */
  int32_t prec;         /* SK_PREC_* (Gaussian only) */
  int32_t flags;        /* reserved, must be 0 */
} sk_op_desc;

typedef struct {
  void *S;      /* device, m x d_new column-major, element type = dtype; never NULL */
  int64_t ldS;  /* >= m */
  void *St;     /* device, n x d_new column-major, or NULL: S' not formed */
  int64_t ldSt; /* >= n when St != NULL */
} sk_output;

#define SK_INIT_PROFILE 1u /* sketch_init flag: launch timing on from the start (see sketch_profile_enable) */

/* sketch_init: create a context on HIP device `device` (section 1: the sketch is
 * the preprocessing step of the compression).  *ctx receives the new context.
 * flags: 0 or SK_INIT_PROFILE; other bits are rejected.
 * Errors: SK_EINVAL (ctx NULL, device out of range, unknown flags), SK_EHIP. */
int sketch_init(sk_ctx **ctx, int32_t device, uint32_t flags);

/* sketch_finalize: destroy a context created by sketch_init; every handle made
 * from it must have been released.  Synchronises the device.  SK_ESTATE if ctx
 * is not a live context. */
int sketch_finalize(sk_ctx *ctx);

/* sketch_last_error: message describing the last failed call on this thread
 * (empty string if none).  The pointer stays valid until the next call. */
const char *sketch_last_error(void);

/* sketch_apply: draw block 0 of R (width d) from `seed` and compute
 *   S = A R  into out->S (m x d), and, if out->St != NULL, S' = A^T R into out->St
 *   (n x d; requires m == n and a nonsymmetric input)           -- section 1, eq. S <- A R
 * For SK_POINTS, S = K(X, h) R with K generated on the fly (N x N never stored).
 * *h receives a new handle owning the operator metadata (release with
 * sketch_release).  d > 0; SJLT with the block construction needs alpha | d, with
 * the graph construction alpha <= d; the SJLT and SRHT kernels need d % 16 == 0;
 * SRHT takes any n (H = H_nu, nu = 2^ceil(log2 n), section 7.2).  Asynchronous on `stream`.
 * Errors: SK_EINVAL, SK_EUNSUPPORTED, SK_ENOMEM, SK_EHIP. */
int sketch_apply(sk_ctx *ctx, const sk_input *in, const sk_op_desc *op, int32_t d, uint64_t seed,
                 const sk_output *out, sk_handle **h, void *stream);

/* sketch_extend: append `nblocks` blocks of width dd to R (Algorithm 1, extension
 * step: R <- [R, Rbar], S <- [S, A Rbar]) and compute only the new columns,
 * all new blocks in one pass over A.  out_new->S receives the m x (nblocks*dd)
 * new columns of S (and out_new->St those of S' when not NULL).  The input must
 * be the same matrix the handle was applied to.  Asynchronous. */
int sketch_extend(sk_handle *h, const sk_input *in, int32_t dd, int32_t nblocks,
                  const sk_output *out_new, void *stream);

/* sketch_rerun: redraw every block of the operator from `seed` (same widths) and
 * recompute all d columns of S (and S') in one pass; allocates nothing once the
 * handle exists.  out holds all d columns.  Asynchronous. */
int sketch_rerun(sk_handle *h, const sk_input *in, uint64_t seed, const sk_output *out, void *stream);

/* sketch_rerun_static: sketch_rerun for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments and results as sketch_rerun, bit for bit;
 * it allocates and frees nothing (no hipMalloc, hipFree or allocating library
 * routine; launch timing is not recorded).  The kernels' scratch (partial sums
 * of a split source range) lives in a fixed device array of 64 MiB that the
 * library holds on every GPU it runs on until the process ends.  A call whose
 * scratch would exceed 64 MiB fails with SK_EINVAL and a message giving both
 * sizes; the handle then keeps its previous operator (its metadata is
 * regenerated on `stream`).  Every call on one GPU shares that GPU's array and
 * it keeps the last call's contents: calls that overlap on one GPU, from any
 * context or stream, race; order them on one stream.  Asynchronous. */
int sketch_rerun_static(sk_handle *h, const sk_input *in, uint64_t seed, const sk_output *out, void *stream);

/* sketch_adjoint: backward of the sketch for the operator blocks
 * [block0, block0 + nblocks) (their columns, in order, are the columns of dS).
 *   DENSE (SJLT): dA = dS R^T (the adjoint of A -> A R), m x n, overwritten;
 *                 dS is m x (sum of the blocks' widths), lddS >= m, lddA >= m.
 *   POINTS (SJLT): with dS = W = dL/dS for S = K(X, h) R, writes
 *                 dX = dL/dX (N x dim row-major, FP32, device) and
 *                 *dh = dL/dh (one FP64 value, device), K recomputed tile by tile:
 *                 dL/dx_i = -(1/h^2) sum_j (G_ij + G_ji) K_ij (x_i - x_j),
 *                 dL/dh = sum_ij G_ij K_ij |x_i - x_j|^2 / h^3, G = W R^T.
 *                 Requires alpha <= 16 and blocks of at most 256 columns;
 *                 more blocks (over 16 hash codes per point or 256 columns in
 *                 all) are processed in groups, the gradient summed in FP64.
 * The input must be the one the handle was applied to.  Asynchronous; uses the
 * context workspace (calls sharing a context must be ordered on one stream).
 * Errors: SK_EINVAL, SK_EUNSUPPORTED (other operator kinds), SK_ENOMEM, SK_EHIP. */
int sketch_adjoint(sk_handle *h, const sk_input *in, int32_t block0, int32_t nblocks, const void *dS, int64_t lddS,
                   void *dA, int64_t lddA, float *dX, double *dh, void *stream);

/* sketch_width: current total width d and number of blocks of the operator. */
int sketch_width(const sk_handle *h, int32_t *d, int32_t *nblocks);

/* sketch_release: free the operator metadata of a handle.  Synchronises the
 * device before freeing.  SK_ESTATE for a released or foreign handle. */
int sketch_release(sk_handle *h);

/* sketch_get_rows: host evaluation of R(i0:i1, j0:j1) in FP64, column-major
 * (out[(i - i0) + (j - j0) * ldo]), from the operator definition.
 * Algorithm 1 needs R(I_tau, iota) for the diagonal-block corrections of the
 * local sketches; section 7.2 gives the SRHT element formula used here.
 * Requires 0 <= i0 <= i1 <= n, 0 <= j0 <= j1 <= d, ldo >= i1 - i0. */
int sketch_get_rows(const sk_handle *h, int64_t i0, int64_t i1, int64_t j0, int64_t j1, double *out,
                    int64_t ldo);

/* sketch_get_sjlt: copy the device-generated hash of SJLT block `block` to host:
 * codes[k * alpha + c] = (column inside the block << 1) | negative, for every row
 * k < n and c < alpha (section 6.1: R = (B+ - B-)/sqrt(alpha)); block
 * construction: c is the chunk; graph construction: c is the draw step.
 * Synchronises.  SK_EINVAL if the handle is not SJLT or block is out of range. */
int sketch_get_sjlt(const sk_handle *h, int32_t block, uint32_t *codes);

/* sketch_get_srht: copy the device-generated SRHT data to host: D[k] in {+1,-1}
 * for k < n (if D != NULL) and mu[j - j0] for global columns j0 <= j < j1 (if mu
 * != NULL).  Section 7: D and P are stored as vectors, H is never formed.
 * Synchronises. */
int sketch_get_srht(const sk_handle *h, int8_t *D, uint32_t *mu, int32_t j0, int32_t j1);

/* sketch_get_gaussian: copy the device-generated unscaled Gaussian draws of
 * block `block` (n x w_b, column-major, bfloat16 bit patterns) to host.
 * Synchronises. */
int sketch_get_gaussian(const sk_handle *h, int32_t block, uint16_t *bits);

/* sketch_profile_enable: when on != 0, every kernel launch made through this
 * context is bracketed by HIP events recorded on the launch's own stream (the
 * measurement behind achieved bandwidth; no effect on results). */
int sketch_profile_enable(sk_ctx *ctx, int32_t on);

/* sketch_profile_read: total elapsed milliseconds (*ms) and number of launches
 * (*count) recorded for the kernel family `name` ("sjlt_gather",
 * "sjlt_gather_t", "sjlt_reduce", "sjlt_meta", ...) since the last reset;
 * reset != 0 clears every record.  Synchronises on the recorded events. */
int sketch_profile_read(sk_ctx *ctx, const char *name, double *ms, int64_t *count, int32_t reset);

/* ---- batched sketches ----------------------------------------------------
 * Many independent stored matrices, each compressed adaptively with its own
 * SJLT operator grown in blocks of dd columns (Algorithm 1's extension step
 * S <- [S, A Rbar], run for a whole batch).  Round r draws block r of every
 * operator whose target width d[i] exceeds r * dd and computes
 *   S_i(:, r dd : (r+1) dd) = A_i R_i,r   (and S'_i = A_i^T R_i,r when St != NULL)
 * in one persistent launch over all (matrix, row tile) work items, after four
 * batched operator-generation launches.  Operators are identical to the ones
 * sketch_apply/sketch_extend draw for (seed[i], blocks of width dd, alpha). */
typedef struct sk_batch sk_batch;

#define SK_BATCH_GRAPH 1    /* capture each round in a HIP graph on first run, replay it afterwards */
#define SK_BATCH_AUTOTUNE 2 /* time the candidate tile shapes on this batch and keep the fastest
                               (cached in the context per batch signature); synchronises */

/* sketch_batch_create: plan a batch of `count` SK_DENSE matrices ins[i] (one
 * dtype; m, n <= 2^31 - 1; S' needs m == n) with final widths d[i] (positive
 * multiples of dd), block width dd in {64, 128, 256}, alpha | dd, operator seeds
 * seeds[i] and outputs outs[i] (S: m_i x d[i], ldS >= m_i; St: n_i x d[i] or
 * NULL).  The input and output buffers must stay valid for the batch's life:
 * their addresses are recorded (and baked into the graphs).  Allocates the
 * operator metadata of every (matrix, block); uploads on `stream` and
 * synchronises it.  *b receives the batch; release with sketch_batch_destroy.
 * Errors: SK_EINVAL, SK_EUNSUPPORTED (other block widths), SK_ENOMEM, SK_EHIP. */
int sketch_batch_create(sk_ctx *ctx, const sk_input *ins, int32_t count, const int32_t *d, int32_t dd,
                        int32_t alpha, const uint64_t *seeds, const sk_output *outs, int32_t flags, sk_batch **b,
                        void *stream);

/* sketch_batch_run: run rounds [r0, r1) in order on `stream` (asynchronous).
 * With SK_BATCH_GRAPH the first run of a round captures it (on a private
 * stream) and every run launches the instantiated graph. */
int sketch_batch_run(sk_batch *b, int32_t r0, int32_t r1, void *stream);

/* sketch_batch_reseed: new operator seeds for the following runs (the graphs
 * read them from device memory).  Synchronises `stream`. */
int sketch_batch_reseed(sk_batch *b, const uint64_t *seeds, void *stream);

/* sketch_batch_info: number of rounds and the tile shape in use:
 * shape[0..3] = (sources per chunk, waves per workgroup, columns per wave, rows
 * per lane). */
int sketch_batch_info(const sk_batch *b, int32_t *nrounds, int32_t *shape);

/* sketch_batch_mode: how round `round` runs: SK_ROUND_EAGER (the batch was made
 * without SK_BATCH_GRAPH), SK_ROUND_NOT_CAPTURED (graph mode, not run yet),
 * SK_ROUND_GRAPH (replays its captured graph) or SK_ROUND_CAPTURE_FAILED (the
 * runtime refused the capture or its instantiation; the round runs launch by
 * launch with the same kernels and arguments, so results are unchanged). */
#define SK_ROUND_EAGER 0
#define SK_ROUND_NOT_CAPTURED 1
#define SK_ROUND_GRAPH 2
#define SK_ROUND_CAPTURE_FAILED 3
int sketch_batch_mode(const sk_batch *b, int32_t round, int32_t *mode);

/* sketch_batch_destroy: free the batch (synchronises the device). */
int sketch_batch_destroy(sk_batch *b);

/* sketch_apply_batched: one call for a whole batch (Algorithm 1's extension step
 * run for many independent matrices): plans the batch exactly as
 * sketch_batch_create (same arguments, op->kind must be SK_SJLT with the block
 * construction and op->alpha its alpha; flags = SK_BATCH_GRAPH and/or
 * SK_BATCH_AUTOTUNE), runs every round, frees the batch, and, when hs != NULL,
 * stores in hs[i] a handle holding matrix i's operator (d[i] / dd blocks of
 * width dd drawn from seeds[i], the operator sketch_apply(dd) followed by
 * sketch_extend(dd) would draw), so that the caller can extend, query or
 * differentiate it later; each handle must be released.  Synchronises the
 * device.  On failure no handle is returned.
 * Errors: as sketch_batch_create; SK_EUNSUPPORTED for other operators. */
int sketch_apply_batched(sk_ctx *ctx, const sk_input *ins, const sk_op_desc *op, const int32_t *d, int32_t dd,
                         const uint64_t *seeds, const sk_output *outs, int32_t count, int32_t flags, sk_handle **hs,
                         void *stream);

/* ---- per-node HSS work on the device ---------------------------------------
 * Batched FP64 kernels for the node-level steps of Algorithm 1 (appendix "HSS
 * Algorithm Detailed Description"): the local sketches S_tau = S(I_tau, iota) -
 * D_tau R(I_tau, iota) and their internal-node forms (products and row
 * selections), the QR of the first d columns and the projection of the next dd
 * columns for the stopping test of section 3 (eq. "stopping_criteria-1"), the
 * interpolative decomposition by column-pivoted QR, and the local operators
 * R_tau = U_tau^T R(...).  Each call takes a host array of `count` descriptors,
 * one per node (sizes may differ), and enqueues the batch on `stream` with the
 * descriptors in the kernel arguments (one launch per 40-96 descriptors); it
 * does not wait for the device, and the host array may be reused on return.  All
 * matrices are FP64, column-major, in device memory owned by the caller.
 * Errors: SK_ESTATE (context), SK_EINVAL (a descriptor out of range; its index
 * is in the message), SK_EHIP. */
typedef struct {
  int32_t m, n, k;        /* C is m x n; op(A) is m x k, op(B) k x n */
  int32_t transA, transB; /* nonzero: op(X) = X^T */
  double alpha, beta;     /* C = beta C + alpha op(A) op(B); beta = 0 ignores C's old values */
  const double *A;
  int64_t lda;
  const double *B;
  int64_t ldb;
  double *C;
  int64_t ldc;
} sk_gemm_desc;
int sketch_batched_gemm(sk_ctx *ctx, const sk_gemm_desc *descs, int32_t count, void *stream);

/* Householder QR of A (m x n, overwritten: R above the diagonal, reflectors
 * below); rdiag[j] = |R_jj| for j < r = min(m, n) <= 1024; when Q != NULL the
 * explicit Q (m x r, ldq >= m) with A = Q R. */
typedef struct {
  int32_t m, n;
  double *A;
  int64_t lda;
  double *rdiag;
  double *Q;
  int64_t ldq;
} sk_qr_desc;
int sketch_batched_qr(sk_ctx *ctx, const sk_qr_desc *descs, int32_t count, void *stream);

/* Interpolative decomposition M ~ M(:, J) Y of M (p x q, overwritten) by
 * column-pivoted Householder QR: column norms recomputed exactly at each step,
 * pivot = first column of maximal norm, stop at the first k with norm <
 * max(eps_a, eps_r |R_00|).  Writes *rank = k (device int), perm[0:q] (J =
 * perm[0:k]) and Y (k x q, ldy >= min(p, q)) with Y(:, J) = I and the other
 * columns R11^{-1} R12. */
typedef struct {
  int32_t p, q;
  double *M;
  int64_t ldm;
  double eps_r, eps_a;
  int32_t *perm;
  int32_t *rank;
  double *Y;
  int64_t ldy;
} sk_id_desc;
int sketch_batched_id(sk_ctx *ctx, const sk_id_desc *descs, int32_t count, void *stream);

/* *out = ||A||_F for A m x n (device scalar) */
typedef struct {
  int32_t m, n;
  const double *A;
  int64_t lda;
  double *out;
} sk_norm_desc;
int sketch_batched_norm(sk_ctx *ctx, const sk_norm_desc *descs, int32_t count, void *stream);

/* dst(i, j) = src(r_i, c_j), r_i = rows[i] (or row0 + i when rows is NULL),
 * c_j = cols[j] (or col0 + j): row selections and submatrices such as
 * B = A(I~, I~') (dst m x n, ldd >= m; rows / cols device int64 arrays); with
 * trans != 0 the transpose, dst(i, j) = src(c_j, r_i). */
typedef struct {
  int32_t m, n;
  int32_t trans;
  const double *src;
  int64_t lds;
  const int64_t *rows;
  const int64_t *cols;
  int64_t row0, col0;
  double *dst;
  int64_t ldd;
} sk_gather_desc;
int sketch_batched_gather(sk_ctx *ctx, const sk_gather_desc *descs, int32_t count, void *stream);

/* sketch_get_rows_device: R(i0:i1, j0:j1) in FP64 written to device memory
 * (out[(i - i0) + (j - j0) * ldo]) from the handle's device metadata (the
 * leaf corrections D_tau R(I_tau, iota) and local operators of Algorithm 1).
 * Asynchronous on `stream`; out is caller-owned device memory.
 * Errors: SK_ESTATE (not a live handle), SK_EINVAL (rows outside [0, n),
 * columns outside [0, d), out NULL for a non-empty range, ldo < i1 - i0),
 * SK_EHIP. */
int sketch_get_rows_device(const sk_handle *h, int64_t i0, int64_t i1, int64_t j0, int64_t j1, double *out,
                           int64_t ldo, void *stream);

/* ---- operator state (checkpoint / resume) ---------------------------------
 * An operator is a pure function of (kind, alpha, construction, precision,
 * element type, input kind, n, seed, table chunk sizes, block widths): Algorithm
 * 1's JL-Operator(d, n) per block, drawn from the seed.  The state holds those
 * fields (a few hundred bytes, host memory, with a checksum); importing it
 * regenerates every block's device metadata, so a resumed handle extends,
 * reruns and differentiates exactly as the original would. */

/* sketch_state_export: with buf == NULL, *len receives the size of the state;
 * otherwise writes the state of h to buf (host, *len bytes available) and sets
 * *len to the bytes written.  Host only; no device work.
 * Errors: SK_ESTATE (bad handle), SK_EINVAL (len NULL or buffer too small). */
int sketch_state_export(const sk_handle *h, void *buf, size_t *len);

/* sketch_state_import: a new handle on ctx from a state written by
 * sketch_state_export (host buffer of len bytes); generates its metadata on the
 * device and synchronises.  Release with sketch_release.
 * Errors: SK_EINVAL (not a state, wrong version, size or checksum, fields out of
 * range), SK_EUNSUPPORTED, SK_ENOMEM, SK_EHIP. */
int sketch_state_import(sk_ctx *ctx, const void *buf, size_t len, sk_handle **h);

/* ---- test hooks (callers: test suites that exercise failure handling) ------
 * sketch_test_hook(ctx, SK_HOOK_FAIL_ALLOC, k): the k-th device allocation made
 *   for ctx from now on (k >= 1; 1 = the next one) fails with SK_ENOMEM as if
 *   the device were full; k = 0 disarms.
 * sketch_test_hook(ctx, SK_HOOK_FAIL_GRAPH, on): while on != 0, graph capture
 *   in sketch_batch_run fails as if the runtime refused it (the round then runs
 *   launch by launch, see sketch_batch_mode).
 * sketch_test_poison_lds(ctx, pattern, stream): enqueue a kernel that fills the
 *   whole 160 KB LDS of each workgroup on every CU with `pattern`, so that the
 *   next kernels start on LDS holding those bits (checks that no kernel reads
 *   LDS it did not write).  Asynchronous. */
#define SK_HOOK_FAIL_ALLOC 1
#define SK_HOOK_FAIL_GRAPH 2
int sketch_test_hook(sk_ctx *ctx, int32_t hook, int64_t arg);
int sketch_test_poison_lds(sk_ctx *ctx, uint32_t pattern, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* HSKETCH_SKETCH_H */
