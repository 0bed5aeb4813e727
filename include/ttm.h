/*
 * ttm.h -- C interface of libttm, the MI355X (gfx950) library for the chain of
 * mode-n tensor-times-matrix products on dense 3-way tensors.
 *
 * Operator (mode-n product, the directional operator the paper applies along
 * one direction of a 3D field, Sec. 4.2 Eq. (cfds), here with one dense factor
 * per mode):
 *
 *     Y = X x1 A x2 B x3 C,
 *     Y[j1,j2,j3] = sum_{i1,i2,i3} A[j1,i1] * B[j2,i2] * C[j3,i3] * X[i1,i2,i3]
 *
 * Layout.  Every tensor is dense and row-major (C order):
 *     X  [I1][I2][I3]  (i3 contiguous)     Y  [J1][J2][J3]
 *     A  [J1][I1]      B  [J2][I2]         C  [J3][I3]
 * No mode unfolding is ever materialised: each contraction reads its operand
 * through strides, and operand transposes happen in registers or LDS.
 *
 * Memory.  Every tensor pointer is a device pointer owned by the caller; the
 * library never allocates or frees caller tensors.  Scratch space comes from a
 * caller-owned device workspace whose size the *_workspace_size queries give.
 * The only library-owned memory is a batched plan (host and device metadata),
 * created by ttm_batched_plan_create and freed by ttm_batched_plan_destroy.
 *
 * Ordering.  Every compute call is asynchronous and ordered on the caller's
 * HIP stream (passed as an opaque pointer; NULL is the null stream).  The
 * compute calls neither synchronise nor allocate, so they may be captured into
 * a HIP graph.  A device fault surfaces at the caller's next synchronisation.
 *
 * Errors.  Arguments are validated before anything is launched; on error a
 * negative ttm_status is returned and nothing has been written.
 *
 * Threads.  Calls are re-entrant; a plan is immutable after creation except
 * for its autotuned choice, which ttm_batched_autotune sets.
 */
#ifndef TTM_H
#define TTM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TTM_OK = 0,
    TTM_ERR_INVALID_ARG = -1,  /* null pointer, non-positive size, bad alignment */
    TTM_ERR_UNSUPPORTED = -2,  /* dtype/math combination or size not provided */
    TTM_ERR_WORKSPACE = -3,    /* workspace missing or smaller than required */
    TTM_ERR_ALIAS = -4,        /* an output overlaps an input */
    TTM_ERR_HIP = -5           /* the HIP runtime reported an error */
} ttm_status;

typedef enum { TTM_F64 = 0, TTM_F32 = 1, TTM_BF16 = 2 } ttm_dtype;

/*
 * Arithmetic of a call.
 *  F64    : double products, double accumulation.
 *  F32    : float products, float accumulation (FP32 matrix cores).
 *  BF16   : every operand rounded to bfloat16 (round to nearest even) before
 *           each product, float accumulation; intermediates are re-rounded to
 *           bfloat16 when they become the next product's operand.
 *  BF16X3 : every float operand v is split into hi = rne_bf16(v) and
 *           lo = rne_bf16(v - hi); a product is formed as hi*hi' + hi*lo' +
 *           lo*hi' on bfloat16 matrix cores with float accumulation, and
 *           intermediates stay float and are split again.  The split
 *           keeps about 16 significant bits of every operand, so the error
 *           is about 2^-17 times the sum of the magnitudes of the terms of an
 *           output: near float's on well-conditioned data (relative error
 *           about 7e-6 on the 1024^3 -> 128^3 Gaussian workload), but up to
 *           about 2^-17 times the condition number where terms cancel (about
 *           4e-5 for the compact-scheme derivative factors of Sec. 4.2,
 *           whose sums cancel heavily).  Runs at bfloat16 matrix-core rates.
 */
typedef enum { TTM_MATH_F64 = 0, TTM_MATH_F32 = 1, TTM_MATH_BF16 = 2, TTM_MATH_BF16X3 = 3 } ttm_math;

/* Sizes of one chain: X is I[0] x I[1] x I[2], Y is J[0] x J[1] x J[2]. */
typedef struct { int64_t I[3]; int64_t J[3]; } ttm_shape;

typedef struct ttm_batched_plan ttm_batched_plan;

/* Human-readable name of a status code (static string, never NULL). */
const char *ttm_status_string(int status);

/* Library version as major*10000 + minor*100 + patch. */
int ttm_version(void);

/*
 * Slab-kernel selection (process-wide), a measurement and test hook that
 * compares the implementations of the fused mode-3/mode-2 step; results of
 * every selection agree with the operator above.  Changing it while another
 * thread runs ttm_chain only changes which kernel that call launches.
 *   0 (default): with bf16 X, the bf16 or bf16x3 form and four column
 *      waves (J3 above 32), where rows are 16-byte aligned, I3 a multiple
 *      of 64 and the i2 range of a workgroup at least 256 rows (the grid
 *      splits I2 into ranges of a multiple of 128 rows so as to reach about
 *      1024 workgroups), the kernel of 3; otherwise, where X is already in the
 *      operand format with 16-byte aligned rows and I3 a multiple of 256
 *      bytes, the kernel of 2; the register-staged kernel elsewhere;
 *   1: the register-staged kernel everywhere;
 *   2: direct-to-LDS, 256-byte chunks, two stages, with the fragments of C
 *      loaded from L2 by every wave (where it applies, else as 1);
 *   3: direct-to-LDS for both X and C, eight waves over 256-row tiles,
 *      128-byte chunks, three X stages and two C stages (where the
 *      conditions of 0 hold, else as 1).
 * Returns TTM_ERR_INVALID_ARG for any other value.
 */
int ttm_set_slab_kernel(int mode);

/*
 * Supported (x_dtype, f_dtype, y_dtype, math) combinations of ttm_chain:
 *   (F64,  F64, F64, F64)
 *   (F32,  F32, F32, F32)   (F32, F32, F32, BF16)   (F32, F32, F32, BF16X3)
 *   (BF16, F32, F32, F32)   (BF16, F32, F32, BF16)  (BF16, F32, F32, BF16X3)
 * Anything else returns TTM_ERR_UNSUPPORTED.
 */
int ttm_chain_supported(int x_dtype, int f_dtype, int y_dtype, int math);

/* Bytes of device workspace ttm_chain needs for this shape and arithmetic
 * (0 for an invalid or unsupported request). */
size_t ttm_chain_workspace_size(const ttm_shape *shape, int x_dtype, int math);

/*
 * Y = X x1 A x2 B x3 C (the chain written out above).
 *
 * shape     : sizes, every I[n] >= 1 and J[n] >= 1.
 * X         : device, x_dtype, [I1][I2][I3], 16-byte aligned.
 * A, B, C   : device, f_dtype, [J1][I1], [J2][I2], [J3][I3], 4-byte aligned.
 * Y         : device, y_dtype, [J1][J2][J3], must not overlap any input or ws.
 * ws        : device workspace of at least ttm_chain_workspace_size bytes,
 *             16-byte aligned; its contents on entry are ignored.
 * stream    : hipStream_t (opaque), NULL for the null stream.
 *
 * The contracted mode order inside the library is 3, then 2, then 1 (the
 * contiguous mode first); mode products on distinct modes commute, so this is
 * the same operator.  Results are deterministic: a repeated call with the same
 * inputs gives bitwise-identical output.
 */
int ttm_chain(const ttm_shape *shape,
              const void *X, int x_dtype,
              const void *A, const void *B, const void *C, int f_dtype,
              void *Y, int y_dtype, int math,
              void *ws, size_t ws_bytes, void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * computation and results as ttm_chain (the same kernels, bit for bit), with
 * the workspace taken from a scratch array the library holds on each GPU
 * instead of a caller buffer.  The call itself allocates nothing.
 *
 * Scratch: TTM_NOALLOC_SCRATCH_BYTES bytes of device memory per GPU, part of
 * the library's device code (it exists on a GPU once the library's kernels
 * are loaded there, and is held until the process ends).  Shapes whose
 * ttm_chain_workspace_size exceeds it return TTM_ERR_WORKSPACE (the
 * 1024^3 -> 128^3 bf16x3 chain needs about 82 MiB and must use ttm_chain;
 * 512^3 -> 64^3 fits).  The first call on a GPU looks up the array's device
 * address (no allocation); make that first call outside graph capture.
 *
 * Every call on one GPU uses the same scratch: calls that overlap in time on
 * one GPU (on different streams, or from different threads without
 * ordering) race and give wrong results.  Calls ordered on one stream are
 * safe.  Arguments, layout and errors otherwise as for ttm_chain.
 */
#define TTM_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int ttm_chain_noalloc(const ttm_shape *shape,
                      const void *X, int x_dtype,
                      const void *A, const void *B, const void *C, int f_dtype,
                      void *Y, int y_dtype, int math, void *stream);

/*
 * Gradient of a scalar loss L through the chain, given G = dL/dY:
 *     dX = G x1 A^T x2 B^T x3 C^T
 *     dA[j1,i1] = sum_{j2,j3} G[j1,j2,j3] (X x2 B x3 C)[i1,j2,j3]
 *     dB[j2,i2] = sum_{j1,j3} G[j1,j2,j3] (X x1 A x3 C)[j1,i2,j3]
 *     dC[j3,i3] = sum_{j1,j2} G[j1,j2,j3] (X x1 A x2 B)[j1,j2,i3]
 * All tensors have one dtype, `dtype`, with math F64 for F64 data and F32 for
 * F32 data (matrix-core products in that precision).  G is [J1][J2][J3];
 * dX, dA, dB, dC have the shapes
 * of X, A, B, C and each may be NULL when not wanted (at least one must be
 * given).  Outputs are overwritten (not accumulated) and must not overlap any
 * input, each other, or ws.  Alignment and stream as for ttm_chain.
 */
size_t ttm_chain_backward_workspace_size(const ttm_shape *shape, int dtype, int math);
int ttm_chain_backward(const ttm_shape *shape, const void *G,
                       const void *X, const void *A, const void *B, const void *C, int dtype,
                       void *dX, void *dA, void *dB, void *dC, int math,
                       void *ws, size_t ws_bytes, void *stream);

/*
 * Batched chains over `count` independent cuboids (ragged sizes), run by one
 * persistent kernel launch.  One wavefront takes one cuboid at a time with
 * one lane per fiber of each mode (the paper's grouping of independent lines
 * onto the lanes of one unit, Sec. 4.1); cuboids are dealt to the waves
 * longest first, each to the wave with the least work so far (LPT).
 *
 * dims_host : host array of count x 6 int64, per cuboid (I1,I2,I3,J1,J2,J3),
 *             every entry in [1, 16].
 * dtype     : F32 (math F32) or F64 (math F64).
 * tune_cache: path of a JSON cache of autotuned launch shapes, or NULL.  When
 *             the file holds an entry for this device and workload class it is
 *             used; otherwise built-in defaults apply until ttm_batched_autotune.
 * Buffers   : X, A, B, C, Y are the cuboids' tensors stored back to back in
 *             cuboid order (each row-major as in ttm_chain); cuboid k starts at
 *             the running sum of the element counts of cuboids 0..k-1.
 *             ttm_batched_plan_totals reports the total element counts.
 * Creating a plan allocates host memory and device metadata (the cuboid
 * descriptors in the order the waves take them, and each wave's first
 * entry) and copies it synchronously on `stream`; destroy frees both.
 */
int ttm_batched_plan_create(int64_t count, const int64_t *dims_host, int dtype, int math,
                            const char *tune_cache, void *stream, ttm_batched_plan **out);
int ttm_batched_plan_destroy(ttm_batched_plan *plan);

/* totals[5] = elements of (X, A, B, C, Y) over all cuboids. */
int ttm_batched_plan_totals(const ttm_batched_plan *plan, int64_t *totals);

/* Y_k = X_k x1 A_k x2 B_k x3 C_k for every cuboid k, one launch on `stream`.
 * Needs no workspace.  Y must not overlap the inputs. */
int ttm_chain_batched(const ttm_batched_plan *plan, const void *X, const void *A,
                      const void *B, const void *C, void *Y, void *stream);

/*
 * Same computation replayed from a HIP graph owned by the plan.  The graph
 * holds the single persistent-kernel node; it is instantiated on first use and
 * its node arguments are updated in place when the buffers change.  Not
 * thread-safe for one plan (the graph is shared).
 */
int ttm_chain_batched_graph(ttm_batched_plan *plan, const void *X, const void *A,
                            const void *B, const void *C, void *Y, void *stream);

/*
 * Reference launch pattern for comparison: one kernel launch per cuboid
 * (count launches).  Same results as ttm_chain_batched.
 */
int ttm_chain_batched_loop(const ttm_batched_plan *plan, const void *X, const void *A,
                           const void *B, const void *C, void *Y, void *stream);

/*
 * Autotune the batched launch: times every candidate (kernel variant, block
 * size, resident blocks per compute unit) on the given buffers with HIP
 * events, each timed launch on a cold last-level cache (a 512 MiB buffer the
 * call allocates is rewritten before it), rebuilds the LPT assignment for
 * each candidate's wave count, keeps the fastest in the plan, and, when the
 * plan has a tune_cache path, rewrites that JSON file.  Synchronises
 * `stream`.  Y is overwritten.  best_ms_out (nullable) receives the chosen
 * candidate's mean time in ms.
 */
int ttm_batched_autotune(ttm_batched_plan *plan, const void *X, const void *A,
                         const void *B, const void *C, void *Y, void *stream,
                         int reps, double *best_ms_out);

/* The plan's current launch shape (out holds 4 ints): out[0] = threads per
 * block, out[1] = resident blocks per compute unit, out[2] = total blocks,
 * out[3] = kernel variant (float, mode products on the vector units: 0
 * keeps the next cuboid's inputs in registers at two waves per SIMD, 1 and 2
 * run three and four waves per SIMD without; on the matrix cores: 3 at three
 * waves per SIMD with a shorter prefetch, 4 at four without; double: every
 * variant runs the same kernel). */
int ttm_batched_plan_config(const ttm_batched_plan *plan, int *out);

/* Pins the plan's launch shape, as the autotuner does with its choice:
 * threads per block (64, 128 or 256), resident blocks per compute unit (at
 * least 1 and at most what LDS and the variant's registers allow) and the
 * variant (0 to 4, as in ttm_batched_plan_config).  Rebuilds the
 * assignment of cuboids to waves (synchronising `stream`).  The results of
 * every shape are identical among the vector-unit variants (0-2) and among
 * the matrix-core variants (3, 4); the two families sum the terms of each
 * output in different orders (both to float rounding of the exact result).
 * TTM_ERR_INVALID_ARG for a shape outside these ranges, TTM_ERR_HIP. */
int ttm_batched_plan_set_config(ttm_batched_plan *plan, int threads, int blocks_per_cu, int variant,
                                void *stream);

/*
 * The compact sixth-order first derivative of Sec. 4.2, Eq. (cfds), on a
 * periodic grid, applied along one mode of a 3-way field:
 *
 *   alpha y_{i-1} + y_i + alpha y_{i+1} = a (x_{i+1} - x_{i-1}) / (2h)
 *                                       + b (x_{i+2} - x_{i-2}) / (4h)
 *
 * for every fiber along `mode`, indices taken modulo n = dims[mode-1], i.e.
 * Y = X x_mode D with D = A_c^-1 B_c (A_c the cyclic tridiagonal left side,
 * B_c the cyclic five-point right side), evaluated without forming D: the
 * right-hand side is built on the fly and the cyclic tridiagonal system
 * (Sec. 2.1) is solved in one of two ways.  Fibers of at least 2K points
 * and a multiple of 8 (K = 40 for F64, 24 for F32), whose coefficient alpha
 * makes rho^K below the
 * rounding unit (rho = (1 - sqrt(1 - 4 alpha^2)) / (2 alpha); alpha = 1/3
 * gives 0.382) take a single pass: A_c factors as a product of two cyclic
 * first-order operators whose inverses are recursions that forget their
 * start after K points (the diagonal dominance of Sec. 4.2), so each point
 * is read once and written once; the result equals the exact solve up to
 * rounding.  Other fibers take the periodic Thomas algorithm (forward and
 * backward sweeps through Y).  The paper's values are alpha = 1/3,
 * a = 14/9, b = 1/9.
 */
typedef struct {
    double alpha, a, b, h;   /* |alpha| < 1/2 (diagonal dominance); h != 0 */
} ttm_compact_coef;

/* Workspace bytes for fibers of n points (n >= 3) in dtype F64 or F32; 0 if
 * unsupported. */
size_t ttm_compact_workspace_size(int64_t n, int dtype);

/*
 * Y = the scheme applied along `mode` (1, 2 or 3) of X.
 *   dims   host array (I1, I2, I3), each >= 1, dims[mode-1] >= 3
 *   X, Y   device, row-major [I1][I2][I3] of dtype (F64 or F32), aligned to
 *          the element size; Y must not overlap X or the workspace
 *   coef   host pointer, read during the call
 *   ws     device workspace of ttm_compact_workspace_size(dims[mode-1], dtype)
 *          bytes (16-byte aligned); it holds the fiber-independent coefficients
 *          of the Thomas sweeps (the preprocessing the paper does once per
 *          operator, Sec. 4.2), computed on the device on `stream`; the
 *          single pass does not read it
 *   prepared  0: compute the coefficients into ws first (a short sequential
 *          kernel, about 0.1 ms for 512 points); 1: ws already holds them
 *          from an earlier call with the same fiber length, coef and dtype
 *          (not checked: other contents give wrong results, never a fault)
 * Arithmetic in dtype.  Errors: TTM_ERR_INVALID_ARG (null pointer, mode out of
 * range, sizes, non-finite or non-dominant coefficients, misalignment),
 * TTM_ERR_UNSUPPORTED (dtype, fibers shorter than 3), TTM_ERR_WORKSPACE,
 * TTM_ERR_ALIAS, TTM_ERR_HIP; nothing is launched on an error.
 */
int ttm_compact_apply(const int64_t *dims, int mode, const void *X, void *Y, int dtype,
                      const ttm_compact_coef *coef, void *ws, size_t ws_bytes, int prepared, void *stream);

/*
 * Truncated HOSVD factors (the Tucker factors the chain applies): for each
 * mode n, the J[n] leading left singular vectors of the unfolding X_(n), as
 * the rows of an J[n] x I[n] factor, computed in FP64 on the GPU: the Gram
 * matrix X_(n) X_(n)^T on the FP64 matrix cores, then its symmetric
 * eigendecomposition by the cyclic Jacobi method (one workgroup per mode, the
 * three modes in one launch).  Rows come
 * in decreasing order of their eigenvalue (squared singular value), each
 * with its entry of largest magnitude positive.  X x1 A x2 B x3 C with these
 * factors (ttm_chain) is the Tucker core.
 *   shape  I[n] in [1, 128], J[n] in [1, I[n]]
 *   X      device, F64, [I1][I2][I3]
 *   A,B,C  device, F64, [J1][I1], [J2][I2], [J3][I3]
 *   evals  device, F64, I1 + I2 + I3 values (nullable): every eigenvalue of
 *          each mode's Gram matrix, decreasing, mode 1 first
 *   ws     ttm_hosvd_workspace_size(shape) bytes, 16-byte aligned
 * Where eigenvalues repeat, the corresponding vectors are any orthonormal
 * basis of their space.  Errors: TTM_ERR_INVALID_ARG, TTM_ERR_UNSUPPORTED
 * (a mode longer than 128), TTM_ERR_WORKSPACE, TTM_ERR_ALIAS, TTM_ERR_HIP.
 */
size_t ttm_hosvd_workspace_size(const ttm_shape *shape);
int ttm_hosvd(const ttm_shape *shape, const void *X, void *A, void *B, void *C, void *evals, void *ws,
              size_t ws_bytes, void *stream);

/*
 * A field moved between directional layouts (Sec. 4.1: each direction has
 * its own layout, in which that direction's lines are contiguous, and Sec.
 * 5.3 counts these reorders in the data movement of a transport step):
 *
 *   Y[i_perm[0]][i_perm[1]][i_perm[2]] = X[i0][i1][i2]      (accumulate = 0)
 *   Y[i_perm[0]][i_perm[1]][i_perm[2]] += X[i0][i1][i2]     (accumulate != 0)
 *
 * i.e. Y's axis k is X's axis perm[k]; the accumulating form adds a
 * direction's result into another layout, in the element type.
 *   dims   host array (n0, n1, n2) of X, each in [1, 2^31]
 *   perm   host array, a permutation of {0, 1, 2}
 *   X, Y   device, row-major, dtype F32 or F64, aligned to the element size;
 *          Y has dims (n_perm[0], n_perm[1], n_perm[2]) and must not overlap X
 * The copy is bit-exact (elements move as bytes).  Errors:
 * TTM_ERR_INVALID_ARG (null pointer, sizes, perm, misalignment),
 * TTM_ERR_UNSUPPORTED (dtype, grid limits), TTM_ERR_ALIAS, TTM_ERR_HIP.
 */
int ttm_reorder(const int64_t *dims, const int *perm, const void *X, void *Y, int dtype, int accumulate,
                void *stream);

/*
 * Plain device-to-device copy of `bytes` (a multiple of 16; both pointers
 * 16-byte aligned, not overlapping) on `stream`: the practical HBM bandwidth
 * ceiling for the roofline, and the known-size reference for byte counters.
 */
int ttm_stream_copy(void *dst, const void *src, size_t bytes, void *stream);

/*
 * Per-kernel timing for measurement.  When enabled, every kernel the library
 * launches is bracketed by HIP events recorded on the launch stream (do not
 * enable it while capturing a graph).  ttm_timing_collect synchronises those
 * events and returns, for up to `max` kernel names, the name (entry n at
 * names + 64*n, NUL-terminated, so `names` holds 64*max bytes), the number of
 * launches and their summed duration in ms; it then clears the record.
 * Returns the number of entries written, or a negative status.
 */
int ttm_timing_enable(int on);
int ttm_timing_collect(char *names, int64_t *counts, double *total_ms, int max);

#ifdef __cplusplus
}
#endif
#endif /* TTM_H */
