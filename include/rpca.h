/*
 * rpca.h -- C ABI of the MI355X (gfx950) randomized block-Lanczos PCA library.
 *
 * The method is the six-step algorithm of Halko, Martinsson, Shkolnisky and
 * Tygert, "An algorithm for the principal component analysis of large data
 * sets", Section 3 ("Summary of the algorithm"), run out-of-core the way
 * Section 4 describes, with the data matrix A touched only by streaming
 * products with tall, skinny blocks:
 *
 *   Step 1   H^(0) = A G,  H^(j) = A (A^T H^(j-1)), j = 1..i      (eqs. first_prod..last_prod)
 *            H = [H^(0) | ... | H^(i)]                            (eq. product23)
 *   Step 2   H = Q R, Q with (i+1) l orthonormal columns           (eq. good_approx23)
 *   Step 3   T = A^T Q                                             (eq. product_t3)
 *   Step 4   T = V~ S~ W^T, S~ non-increasing                      (eq. svd_small3)
 *   Step 5   U~ = Q W                                              (eq. product33)
 *   Step 6   U, S, V = leading k columns / k x k block
 *
 * so that ||A - U S V^T||_2 is close to sigma_{k+1} (eq. sort_of_svd).
 *
 * Conventions for every entry point:
 *   - No call throws, aborts or exits; each returns an rpca_status.
 *   - Matrices are row-major with an explicit leading dimension (elements).
 *   - "device" pointers are HIP device memory of the plan's device;
 *     "pinned host" pointers come from hipHostMalloc (or equivalent).
 *   - The caller owns every pointer it passes; the plan owns its workspace
 *     and frees it in rpca_destroy.  A plan is bound to one HIP stream and
 *     must not be used from two threads at once.
 *   - Calls that produce results block until those results are complete on
 *     the plan's stream.
 */
#ifndef RPCA_H
#define RPCA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RPCA_OK = 0,
  RPCA_ERR_INVALID_ARG = 1,   /* a precondition below is violated */
  RPCA_ERR_UNSUPPORTED = 2,   /* valid request the library does not implement */
  RPCA_ERR_OUT_OF_MEMORY = 3, /* workspace allocation failed */
  RPCA_ERR_HIP = 4,           /* a HIP runtime call failed; code in rpca_stats.hip_error */
  RPCA_ERR_CALLBACK = 5,      /* the panel callback returned non-zero */
  RPCA_ERR_NONFINITE = 6,     /* NaN or Inf met in the data or the iterates */
  RPCA_ERR_QR_BREAKDOWN = 7,  /* H (or T) numerically rank deficient beyond the fallback */
  RPCA_ERR_NO_STATE = 8,      /* rpca_backward / rpca_get_state without a kept forward */
  RPCA_ERR_SCRATCH_LIMIT = 9  /* rpca_quantize_noalloc: the scratch would exceed its fixed size */
} rpca_status;

/* How A is stored.  Every format is row-major m x n with leading dimension lda.
 *   F32        float
 *   BF16       bfloat16 bit patterns (uint16_t)
 *   FP8_E4M3   OCP e4m3 bytes (uint8_t); entry (r, c) is q(r, c) * col_scale[c]
 *   BF16_HILO  two bfloat16 planes: hi at A, lo at A + m*lda; entry = hi + lo
 * The three low-precision formats (not part of the paper, which stores
 * float32; they trade accuracy of the stored A for bytes moved) need A 16-byte
 * aligned and lda a multiple of 16; entries between n and lda are ignored.
 * Their products run on bfloat16 matrix cores with float accumulation, the
 * float operand carried as a bfloat16 hi + lo pair (16 significant bits).   */
typedef enum {
  RPCA_A_F32 = 0,
  RPCA_A_BF16 = 1,
  RPCA_A_FP8_E4M3 = 2,
  RPCA_A_BF16_HILO = 3
} rpca_storage;

/* Where A lives (Section 4: storage on disk vs. on-the-fly evaluation).
 *   DEVICE           A resident in HBM
 *   HOST_PINNED      A in pinned host memory, streamed by row panels
 *   CALLBACK         rows produced on demand on the host by an rpca_panel_cb
 *                    (Section 4.1), copied to the device panel by panel
 *   DEVICE_CALLBACK  rows produced on demand on the device by an
 *                    rpca_device_panel_cb registered with
 *                    rpca_set_device_panel_cb (Section 4.1 without a host
 *                    link: every pass regenerates the rows it reads)      */
typedef enum {
  RPCA_SRC_DEVICE = 0,
  RPCA_SRC_HOST_PINNED = 1,
  RPCA_SRC_CALLBACK = 2,
  RPCA_SRC_DEVICE_CALLBACK = 3
} rpca_source;

enum {
  RPCA_FLAG_KEEP_STATE = 1u << 0,  /* keep H, Q, R, T, W, ... for rpca_backward / rpca_get_state */
  RPCA_FLAG_PROFILE = 1u << 1,     /* time every stage with HIP events (rpca_stats.ms_*) */
  RPCA_FLAG_FORCE_FALLBACK = 1u << 2, /* take the shifted Cholesky-QR fallback for Step 2 */
  RPCA_FLAG_NO_RESCALE = 1u << 3,  /* do not rescale the power iterates (Section 3, overflow remark) */
  /* float32 A only, DEVICE source, n even: form the float32 products of the
   * passes over A (Steps 1 and 3) on bfloat16 matrix cores, each float32
   * operand split by round-to-nearest into three bfloat16 parts and the six
   * products of combined order <= 2 accumulated in float32 (dropped terms and
   * split residuals below 2^-22 of each product, the rounding level of a
   * float32 product).  UNSUPPORTED for other storage, sources or odd n.  A
   * matrix that is not 16-byte aligned with lda % 4 == 0 uses the float32
   * matrix-core kernels instead.                                              */
  RPCA_FLAG_SPLIT_BF16 = 1u << 4,
  /* float32 A only, DEVICE source: carry Step 1 (the blocks
   * H^(0..i) of eqs. first_prod .. last_prod and the products A^T H^(j)) in
   * float64 on the FP64 matrix cores, each float32 entry of A exact in
   * float64, and keep H in float64 for Step 2 -- the arithmetic of the
   * paper's experiments (A stored in single precision, computations in
   * double, Section 6).  Needed when the spectrum spans a wide range above
   * sigma_{k+1} and has a long, heavy tail, as in the paper's first example:
   * float32 products then lose the directions that the later blocks carry
   * below ~1e-7 of the leading ones.  Centring enters as exact float64
   * rank-one corrections with the column means of a separate float64
   * column-sum pass.  Step 3 stays on the float32 kernels.  UNSUPPORTED with
   * other storage or sources, SPLIT_BF16 or KEEP_STATE.                     */
  RPCA_FLAG_FP64_STEP1 = 1u << 5,
  /* Step 2 by Householder QR (a TSQR reduction tree over row blocks, Q formed
   * from the reflectors) instead of Cholesky QR; it is otherwise the last
   * fallback, for every L = (i+1) l <= 1024 the plan accepts.  The first
   * Householder Step 2 of a plan allocates the tree's workspace (about
   * 4 L^2 doubles per level-0 block, at most 2048 blocks), kept until
   * rpca_destroy; OUT_OF_MEMORY if that fails.                             */
  RPCA_FLAG_FORCE_HOUSEHOLDER = 1u << 6,
  /* Run each power step of Step 1 (eqs. second_prod .. last_prod) as one
   * fused kernel that reads A once: H^(j) and the adjoint partial sums of
   * A^T H^(j) come from the same read of each row block (Section 4.1), the
   * columns split over the compute units of one or two XCDs, the partial
   * sums of H^(j) combined between them through device-coherent atomics.
   * Without the flag a power step is a forward launch and an adjoint launch
   * (two reads of A).  Taken for float32 A in device memory (no SPLIT_BF16 /
   * FP64_STEP1, m >= n, i >= 1, m >= 32768, l + 1 <= 64, n <= 20480) on a
   * device of 256 compute units in 8 XCDs with cooperative launch; the plan
   * checks the layout once with a launch without rows and otherwise keeps
   * the two launches (rpca_stats.fused_launches stays 0).                   */
  RPCA_FLAG_FUSED = 1u << 7
};

typedef struct {
  int64_t m, n;        /* A is m x n.  Section 3 takes n <= m and applies the method to A^T
                          otherwise: for m < n the plan factors B = A~^T (n x m, float32 A in
                          device memory, no KEEP_STATE / SPLIT_BF16 / FP64_STEP1) and returns
                          U, V of A (U = V_B, V = U_B); the sign rule then applies to u_j */
  int32_t k;           /* rank of the approximation, 1 <= k < n */
  int32_t l;           /* block width, l >= k */
  int32_t i;           /* power steps, i >= 0, with (i+1) l <= n - k (Section 3) */
  int32_t storage;     /* rpca_storage */
  int32_t source;      /* rpca_source */
  int32_t center;      /* 1: factor A - 1 mu^T with mu the column means of A (Introduction) */
  int64_t panel_rows;  /* rows per streamed panel for HOST_PINNED / CALLBACK / DEVICE_CALLBACK; 0 = automatic */
  uint64_t seed;       /* G from Philox4x32-10 + Box-Muller when rpca_factor gets G == NULL */
  uint32_t flags;      /* RPCA_FLAG_* */
  int32_t device;      /* HIP device ordinal the plan runs on */
} rpca_desc;

/* Fills rows [row0, row0+nrows) of A into dst (pinned host memory owned by the
 * plan, leading dimension ld elements, in the plan's storage format).  For
 * FP8_E4M3 the callback also writes the n column scales into col_scale on its
 * first call (col_scale is NULL on later calls).  Returns 0 on success; any
 * other value aborts rpca_factor with RPCA_ERR_CALLBACK.  Section 4.1: rows
 * are evaluated on demand and every contribution of a row is made at once.  */
typedef int (*rpca_panel_cb)(void* user, int64_t row0, int64_t nrows, void* dst, int64_t ld,
                             float* col_scale);

typedef struct rpca_plan_s* rpca_plan_t;

/* Enqueues, on hip_stream (a hipStream_t owned by the plan), device work that
 * writes rows [row0, row0+nrows) of A as float32 into dst (device memory owned
 * by the plan, nrows x ld, ld >= n), and returns 0; any other value aborts
 * rpca_factor with RPCA_ERR_CALLBACK.  The callback runs on the thread that
 * called rpca_factor; it must only enqueue work on hip_stream (no device-wide
 * synchronisation, no work on other streams that dst depends on).  It is
 * called once per panel per pass, panels in row order, and the same rows must
 * come back identical in every pass (Section 4.1: rows evaluated on demand,
 * every contribution of a row made at once; Section 6.1, third example: regenerated rows
 * restart their generator from the same seed).                              */
typedef int (*rpca_device_panel_cb)(void* user, int64_t row0, int64_t nrows, float* dst, int64_t ld,
                                    void* hip_stream);
/* Timing and counters of the last rpca_factor call.  Without PROFILE only
 * ms_total and the counters are filled; with PROFILE the ms_* stages are the
 * times between HIP events recorded on the plan's stream at the stage
 * boundaries, and the kernel times are event pairs around the panel kernels. */
typedef struct {
  double ms_total;       /* entry to results ready, host clock */
  double ms_colmean;     /* column-mean pass or pass-0 shift (centering), HIP events */
  double ms_power;       /* Step 1: all power passes, HIP events */
  double ms_qr;          /* Step 2, HIP events */
  double ms_tpass;       /* Step 3, HIP events */
  double ms_small_svd;   /* Step 4, HIP events */
  double ms_assemble;    /* Steps 5-6, HIP events */
  double ms_fwd_kernel;  /* summed duration of the A X panel kernels (event timed) */
  double ms_adj_kernel;  /* summed duration of the A^T Z panel kernels (event timed) */
  int64_t fwd_launches;  /* number of A X kernel launches timed above */
  int64_t adj_launches;  /* number of A^T Z kernel launches timed above */
  int64_t a_bytes_read;  /* bytes of A the panel kernels read: a_reads full reads of
                            the stored matrix, plus the rows of the pass-0 shift */
  int64_t h2d_bytes;     /* bytes of A moved host -> device (streamed sources) */
  int32_t qr_fallback;   /* Step 2: 0 Cholesky QR twice; 1 shifted Cholesky QR three times;
                            2 shifted rounds repeated until plain Cholesky QR applies;
                            3 Householder TSQR */
  int32_t eig_vectors;   /* eigenvectors computed in Step 4 (k, or L when state is kept) */
  int32_t hip_error;     /* raw hipError_t of the last RPCA_ERR_HIP */
  int32_t passes;        /* passes of the schedule: i power steps, one A X pass, one
                            A^T Q pass (i + 2), plus a column-mean pass when one is made */
  double ms_tpass_kernel;  /* the Step 3 (T pass) launches among ms_adj_kernel (event timed) */
  int64_t tpass_launches;  /* number of those launches */
  int32_t a_reads;       /* full reads of A the kernels made: a power step run as a
                            forward launch and an adjoint launch reads A twice, a
                            streamed panel or a fused power step once */
  int32_t reserved;
  double ms_fused_kernel;  /* summed duration of the single-read power-step kernels (event timed) */
  int64_t fused_launches;  /* number of those launches */
} rpca_stats;

/* Creates a plan for the problem in *desc, bound to hip_stream (a hipStream_t,
 * NULL = the null stream) on desc->device, and allocates its workspace
 * (O((i+1) l (m+n)) entries, Section 4: only Steps 1 and 3 touch A).
 * Errors: INVALID_ARG when desc is NULL, out is NULL, or the Section 3
 * parameter rules fail for s = min(m, n) (1 <= k < s, l >= k, (i+1) l <= s - k,
 * i >= 0); UNSUPPORTED for (i+1) l > 1024, an unknown storage/source, or
 * m < n with a storage, source or flag the transposed problem does not take;
 * OUT_OF_MEMORY / HIP when allocation fails.  On error *out is NULL.      */
rpca_status rpca_plan(const rpca_desc* desc, void* hip_stream, rpca_plan_t* out);

/* Computes U (m x k), S (k, non-increasing, >= 0) and V (n x k) of Steps 1-6.
 *   A          DEVICE: device pointer; HOST_PINNED: pinned host pointer;
 *              CALLBACK, DEVICE_CALLBACK: ignored (may be NULL).  Format per
 *              desc->storage.
 *   lda        leading dimension of A in elements (>= n).
 *   col_scale  FP8_E4M3 only: n device floats (DEVICE) or host floats
 *              (HOST_PINNED); NULL otherwise.
 *   cb, user   CALLBACK source only (DEVICE_CALLBACK plans use the generator
 *              registered by rpca_set_device_panel_cb; INVALID_ARG without one).
 *   G          min(m, n) x l device floats (row-major, leading dimension l),
 *              the Gaussian test matrix of Step 1 (m < n: of the problem of
 *              A^T, whose columns are the m rows of A); NULL = generate from desc->seed
 *              with Philox4x32-10 (counter = element index r*l+c >> 1, stream 1,
 *              key = seed) and Box-Muller, rounded to float.
 *   U, ldu     device, m x k floats, ldu >= k.
 *   S          device, k floats.
 *   V, ldv     device, n x k floats, ldv >= k.
 * Column j of U and V is signed so that the largest-magnitude entry of v_j is
 * positive.  The schedule has i + 2 passes (one A^T(A X) per power step, one
 * A X pass, one A^T Q pass); in device memory a power step is a forward and an
 * adjoint launch, so A is read 2i + 2 times (rpca_stats.a_reads), once per
 * pass when it is streamed by panels.  Centring adds a column-mean pass for
 * streamed sources, for i = 0 and for FP64 Step 1; otherwise it is folded
 * into pass 0.
 * Low-precision storage: with centring the column means come from the
 * stored values (times col_scale for FP8) and enter only through the exact
 * rank-one correction.
 * Errors: INVALID_ARG for NULL or misaligned pointers or short leading
 * dimensions (low-precision formats: A not 16-byte aligned or lda % 16 != 0,
 * FP8_E4M3 without col_scale); CALLBACK; NONFINITE; QR_BREAKDOWN; HIP.     */
rpca_status rpca_factor(rpca_plan_t plan, const void* A, int64_t lda, const float* col_scale,
                        rpca_panel_cb cb, void* user, const float* G,
                        float* U, int64_t ldu, float* S, float* V, int64_t ldv);

/* Reverse-mode derivative of rpca_factor with G held fixed (the paper has no
 * derivative; this is the exact adjoint of Steps 1-6 as computed).  Needs a
 * preceding rpca_factor with RPCA_FLAG_KEEP_STATE and the same A still valid.
 *   gS  (k), gU (m x k, ldgu), gV (n x k, ldgv): device cotangents of S, U, V
 *       (any may be NULL = zero).
 *   dA  (m x n, ldda): device floats receiving dL/dA, formed as P Y^T from
 *       rank-(3i+2)l float64 factors rounded to float32, with float32-level
 *       products (three-part bfloat16 splits, six products per term).
 * The first call allocates the reverse-sweep workspace, kept until
 * rpca_destroy.  Blocks the calling thread until dA is written.
 * Errors: NO_STATE, INVALID_ARG, UNSUPPORTED (storage other than F32,
 * streamed sources), OUT_OF_MEMORY, NONFINITE (an entry of dA is not finite:
 * the derivative is not defined at this A, e.g. tied leading singular values
 * or a Step 2 factor singular to working precision; dA is still written),
 * HIP.                                                                     */
rpca_status rpca_backward(rpca_plan_t plan, const float* gS, const float* gU, int64_t ldgu,
                          const float* gV, int64_t ldgv, float* dA, int64_t ldda);

/* Appendix estimator p_{j,q}(D) of ||D||_2 for D = A~ - U S V^T (A~ = A, or
 * A - 1 mu^T when the plan centres), with q start vectors of iid N(0,1)
 * entries (Philox stream 9 under `seed`) and j power steps (the paper uses
 * j = 6 and q = k).  U (m x k), S (k), V (n x k) are device floats as
 * rpca_factor returns them; A as in rpca_factor (DEVICE source only).
 * *estimate receives the estimate (host double).  Allocates its O((m+n) q)
 * workspace on each call and frees it before returning; blocks the calling
 * thread until done.
 * Errors: INVALID_ARG (NULL pointers, j < 1, q < 1 or q > 1024, short leading
 * dimensions), UNSUPPORTED (storage other than F32, streamed sources),
 * NO_STATE (centring plan without a preceding rpca_factor), OUT_OF_MEMORY,
 * HIP.                                                                     */
rpca_status rpca_residual(rpca_plan_t plan, const void* A, int64_t lda, const float* col_scale,
                          const float* U, int64_t ldu, const float* S, const float* V, int64_t ldv,
                          int32_t j, int32_t q, uint64_t seed, double* estimate);

/* Converts a device float matrix A (m x n, lda) into a stored format of
 * rpca_storage (BF16, FP8_E4M3 or BF16_HILO), writing out (device, m x ldo
 * elements, 2 m ldo for BF16_HILO; 16-byte aligned, ldo >= n, ldo % 16 == 0;
 * columns n .. ldo-1 are written as zero).  With a shift, a = A[r][c] - shift[c]
 * (float32) is stored instead of A[r][c]:
 *   shift_mode 0: no shift (shift may be NULL);
 *   shift_mode 1: shift is n device floats given by the caller;
 *   shift_mode 2: shift (n device floats) receives fl32 of the column means of
 *                 A (float64 sums) and is then used.
 * Column-mean centring of the stored matrix removes any shift, so a shifted
 * copy factored with desc.center = 1 gives the centred PCA of the data while
 * the stored bits carry the spread instead of the mean.
 * Rounding (the definitions the library's tests check bit for bit):
 *   BF16 / BF16_HILO: round to nearest, ties to even; lo = bf16(a - hi).
 *   FP8_E4M3: per-column scale c_j = fl32(max_r |a_rj| / 448) (1 when the
 *   column is zero) written to col_scale (n device floats); code =
 *   e4m3(fl32(a / c_j)) rounded to nearest, ties to the even code, saturated
 *   at +-448 (never NaN).
 * Blocks the calling thread until done (allocates small scratch).
 * Errors: INVALID_ARG (F32 or unknown storage, NULL pointers, short or
 * unaligned leading dimensions, bad shift_mode); OUT_OF_MEMORY; HIP.        */
rpca_status rpca_quantize(int32_t storage, int64_t m, int64_t n, const float* A, int64_t lda,
                          void* out, int64_t ldo, float* col_scale, float* shift, int32_t shift_mode,
                          void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * conversion as rpca_quantize, with the same arguments, rules and output
 * bits, but no device allocation and no host-side wait.  Its scratch (per-row-
 * split column sums and maxima: n * (12 * splits + 8) bytes, splits =
 * ceil(m / 4096) up to 256) is taken from a fixed device array of
 * RPCA_NOALLOC_SCRATCH_BYTES per GPU, held until the process ends; a request
 * that needs more returns RPCA_ERR_SCRATCH_LIMIT (e.g. n above ~10900 once
 * m >= 2^20, above ~1.67 million for m <= 4096).  The kernels are enqueued on
 * hip_stream and the call returns without waiting.  Every call on one GPU
 * uses that GPU's one array and nothing in it needs clearing between calls:
 * calls on the same stream are ordered, but calls that overlap in time on one
 * GPU (other streams or threads) race on the scratch.
 * Errors: as rpca_quantize (INVALID_ARG, HIP for a failed launch or symbol
 * lookup), plus SCRATCH_LIMIT; never OUT_OF_MEMORY.                         */
#define RPCA_NOALLOC_SCRATCH_BYTES (32u << 20)
rpca_status rpca_quantize_noalloc(int32_t storage, int64_t m, int64_t n, const float* A, int64_t lda,
                                  void* out, int64_t ldo, float* col_scale, float* shift,
                                  int32_t shift_mode, void* hip_stream);

/* Intermediate results kept by KEEP_STATE (device copies into dst):
 *   RPCA_STATE_H      m x L floats, the blocks H^(j) each multiplied by a
 *                     positive scalar (rpca_get_state(RPCA_STATE_HSCALE))
 *   RPCA_STATE_HSCALE i+1 doubles: the block scalars
 *   RPCA_STATE_Q      m x L doubles (Step 2)
 *   RPCA_STATE_T      n x L doubles (Step 3)
 *   RPCA_STATE_SIGMA  L doubles, S~ of Step 4
 *   RPCA_STATE_W      L x L doubles, W of Step 4 (columns in S~ order; only the
 *                     first k columns are computed unless KEEP_STATE was set)
 *   RPCA_STATE_MU     n doubles, column means (centering)
 *   RPCA_STATE_H64    m x L doubles, the float64 blocks of an FP64_STEP1 plan
 *                     (scaled as RPCA_STATE_H; RPCA_STATE_H is then NO_STATE)
 * ld is the destination leading dimension in elements (>= column count).   */
enum {
  RPCA_STATE_H = 0,
  RPCA_STATE_HSCALE = 1,
  RPCA_STATE_Q = 2,
  RPCA_STATE_T = 3,
  RPCA_STATE_SIGMA = 4,
  RPCA_STATE_W = 5,
  RPCA_STATE_MU = 6,
  RPCA_STATE_H64 = 7
};
rpca_status rpca_get_state(rpca_plan_t plan, int32_t which, void* dst, int64_t ld);

/* Copies the statistics of the last call into *out. */
rpca_status rpca_get_stats(rpca_plan_t plan, rpca_stats* out);

/* Static description of a status code (never NULL). */
const char* rpca_status_str(rpca_status s);

/* Registers the row generator of a DEVICE_CALLBACK plan (replacing any earlier
 * one); user is passed back unchanged.  The plan's panel buffers are filled on
 * a second stream of the plan, double-buffered against the panel kernels.
 * Errors: INVALID_ARG (NULL plan or cb), UNSUPPORTED (plan of another source). */
rpca_status rpca_set_device_panel_cb(rpca_plan_t plan, rpca_device_panel_cb cb, void* user);

/* Frees the plan and its workspace; NULL is ignored. */
void rpca_destroy(rpca_plan_t plan);

#ifdef __cplusplus
}
#endif

#endif /* RPCA_H */
