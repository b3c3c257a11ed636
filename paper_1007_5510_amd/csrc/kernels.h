// Host-side launch interface of the library's kernels (internal, not ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rpca {

// ---------------------------------------------------------------- panel products
struct FwdArgs {              // Z = alpha ((A - 1 s^T) Xt^T - 1 corr^T)
  const void* A = nullptr;    // m x n row-major, storage per kernel family
  int64_t lda = 0, m = 0, n = 0;
  const float* shift = nullptr;   // n (padded to x4, zero tail) or null
  const float* Xt = nullptr;      // ncols x ldx (padded rows zero beyond n)
  int64_t ldx = 0;
  int ncols = 0;
  const float* corr = nullptr;    // ncols or null
  const double* alpha = nullptr;  // device scalar or null
  float* Z = nullptr;
  int64_t ldz = 0;
  bool vec = false;               // A 16-byte aligned and lda % 4 == 0
  // K split: ksplit > 1 writes partial sums P[s][r][c] (ldp >= ncols rounded up to
  // 64, split_stride >= m * ldp) and reduces them into Z; kchunk per split
  int ksplit = 1;
  int64_t kchunk = 0;
  float* P = nullptr;
  int64_t ldp = 0, split_stride = 0;
  // optional events recorded around the main product kernel only
  hipEvent_t ev_begin = nullptr, ev_end = nullptr;
  // low-precision storage: X split into bfloat16 hi/lo planes (cpad x ldxs,
  // column scales already folded in) and the hi -> lo plane distance of A
  const uint16_t* Xh = nullptr;
  const uint16_t* Xl = nullptr;
  int64_t ldxs = 0;
  int64_t plane = 0;  // BF16_HILO: elements between the hi and lo planes
  // float32 A on bfloat16 matrix cores: X split into three bfloat16 planes
  // (cpad x ldxs3 each, xplane3 elements apart)
  const uint16_t* X3 = nullptr;
  int64_t ldxs3 = 0, xplane3 = 0;
};

struct AdjArgs {              // P_s = ((A_s - 1 s^T)^T Z_s)^T, s = 0..nsplit-1
  const void* A = nullptr;
  int64_t lda = 0, m = 0, n = 0;
  const float* shift = nullptr;
  const float* Z = nullptr;       // m x ncols (ldz)
  int64_t ldz = 0;
  int ncols = 0;
  int64_t rows_per_split = 0;     // multiple of 4
  int nsplit = 0;
  bool ones = false;              // float32 kernel: row ncols of each P_s = column sums of A_s - 1 s^T
  float* P = nullptr;             // [nsplit][ncols][ldp]
  int64_t ldp = 0, split_stride = 0;
  bool vec = false;
  hipEvent_t ev_begin = nullptr, ev_end = nullptr;
  // low-precision storage: Z split into transposed, row-permuted bfloat16
  // hi/lo planes (cpad x ldzs)
  const uint16_t* Zh = nullptr;
  const uint16_t* Zl = nullptr;
  int64_t ldzs = 0;
  int cpad_z = 0;  // rows of the Z planes (>= every Z column the kernel's tiles read)
  int64_t plane = 0;
  // float32 A on bfloat16 matrix cores: Z transposed and split into three
  // bfloat16 planes (cpad x ldzs3 each, zplane3 elements apart)
  const uint16_t* Z3 = nullptr;
  int64_t ldzs3 = 0, zplane3 = 0;
};

// One power step of Step 1 on a single read of float32 A (panel_fused.hip): Z as the forward
// product writes it and the adjoint partial sums of ngroups * nseg row segments as the adjoint
// product writes them (P[split][ncols (+1 with ones)][ldp]).  Cooperative launch of
// ngroups * gsize workgroups, one per CU, grouped by XCD.
struct FusedArgs {
  const void* A = nullptr;
  int64_t lda = 0, m = 0, n = 0;
  const float* shift = nullptr;
  const float* Xt = nullptr;
  int64_t ldx = 0;
  int ncols = 0;
  bool ones = false;
  const float* corr = nullptr;
  const double* alpha = nullptr;
  float* Z = nullptr;
  int64_t ldz = 0;
  float* P = nullptr;
  int64_t ldp = 0, split_stride = 0;
  int ngroups = 0, gsize = 0;      // groups of compute units and their size (gsize = xcc_per_group * cu_per_xcc)
  int xcc_per_group = 0, cu_per_xcc = 0;
  int64_t rows_per_group = 0;      // multiple of 16, ngroups * rows_per_group >= m
  int nseg = 1;                    // row segments per group (partial sums each)
  int64_t seg_rows = 0;            // multiple of 16, nseg * seg_rows >= rows_per_group
  bool vec = false;
  unsigned* ws = nullptr;          // fused_ws_words() words
  float* xpart = nullptr;          // fused_xpart_floats(gsize) floats
  float* xred = nullptr;           // fused_xred_floats() floats
  hipEvent_t ev_begin = nullptr, ev_end = nullptr;
};
size_t fused_ws_words();
size_t fused_xpart_floats(int gsize);
size_t fused_xred_floats();
bool fused_fits(int64_t n, int ncols, bool ones, int ngroups, int gsize);
int fused_max_tiles_per_member();
hipError_t launch_fused_f32(const FusedArgs& a, hipStream_t st);

hipError_t launch_fwd_f32(const FwdArgs& a, hipStream_t st);
// K split for the forward product over `slots` concurrent blocks
void fwd_split(int64_t m, int64_t n, int64_t slots, int* ksplit, int64_t* kchunk);
// row split of the adjoint product over `slots` concurrent blocks
void adj_split(int64_t m, int64_t n, int ncols, int64_t slots, int* nsplit, int64_t* rows_per_split);
hipError_t launch_adj_f32(const AdjArgs& a, hipStream_t st);
// float64 reduction of the forward K-split partials into Z (with alpha and corr)
hipError_t launch_fwd_reduce(const FwdArgs& a, int ksplit, hipStream_t st);
// float32 products on bfloat16 matrix cores with a three-way operand split (panel_x6.hip)
hipError_t launch_split3_x(const float* Xt, int64_t ldx, int64_t n, int ncols, int cpad, uint16_t* Xp, int64_t ldxs,
                           int64_t plane, hipStream_t st);
hipError_t launch_split3_zt(const float* Z, int64_t ldz, int64_t m, int ncols, bool ones, int cpad, uint16_t* Zp,
                            int64_t ldzs, int64_t plane, hipStream_t st);
hipError_t launch_fwd_x6(const FwdArgs& a, hipStream_t st);
// three-part bfloat16 split of X (rows x cols) in the K-step-major layout of the rank-K product:
// part q of X[r][k] at ((3 (k / 16) + q) rows_pad + r) 16 + k % 16, zero for r < rows_pad, k < kp
// outside X; Xp holds 3 rows_pad kp entries
hipError_t launch_split3_rows(const float* X, int64_t ldx, int64_t rows, int cols, int64_t rows_pad, int kp,
                              uint16_t* Xp, hipStream_t st);
// O = P Y^T (m x n, ld ldo) from the split of P (rows_pad = mpad, m rounded up to 256) and of Y
// (rows_pad = npad >= n rounded up to 256), kp a multiple of 32; *nonfinite |= 1 when an entry of
// O is not finite
hipError_t launch_outer_x6(const uint16_t* Pp, int64_t mpad, const uint16_t* Yp, int64_t npad, int kp, int64_t m,
                           int64_t n, float* O, int64_t ldo, int* nonfinite, hipStream_t st);
// 65 to 192 output columns (with rows_per_split % 32 == 0 and planes at least that wide) go to the
// one-read wide kernel, others to 64-column tiles
hipError_t launch_adj_x6(const AdjArgs& a, hipStream_t st);
hipError_t launch_fwd_lowp(int storage, const FwdArgs& a, hipStream_t st);
hipError_t launch_adj_lowp(int storage, const AdjArgs& a, hipStream_t st);
void fwd_split_lp(int storage, int64_t m, int64_t n, int64_t slots, int* ksplit, int64_t* kchunk);
void adj_split_lp(int storage, int64_t m, int64_t n, int ncols, int64_t slots, int* nsplit,
                  int64_t* rows_per_split);
// hi/lo bfloat16 planes of (col_scale o Xt): cpad x ldxs (ldxs % 64 == 0, cpad % 64 == 0)
hipError_t launch_split_x(const float* Xt, int64_t ldx, int64_t n, int ncols, const float* col_scale,
                          uint16_t* Xh, uint16_t* Xl, int64_t ldxs, int cpad, hipStream_t st);
// transposed, row-permuted hi/lo bfloat16 planes of Z: cpad x ldzs (ldzs % 32 == 0)
hipError_t launch_split_zt(const float* Z, int64_t ldz, int64_t m, int ncols, uint16_t* Zh, uint16_t* Zl,
                           int64_t ldzs, int cpad, hipStream_t st, bool ones = false);
// quantisers of the stored formats (see rpca_quantize)
hipError_t launch_quantize(int storage, int64_t m, int64_t n, const float* A, int64_t lda, const float* shift,
                           void* out, int64_t ldo, float* col_scale, float* amax_part, int nsplit,
                           int64_t rows_per_split, hipStream_t st);

// ---------------------------------------------------------------- float64 Step 1 (panel_f64.hip)
constexpr int F64_RT = 4;    // forward: 16-row tiles per wave (a block of 4 waves takes 256 rows)
constexpr int F64_KST = 32;  // forward: K per LDS stage
constexpr int F64_RS = 32;   // adjoint: rows per stage

struct Fwd64Args {             // Z = alpha A Xt^T, float32 A, float64 X and Z
  const float* A = nullptr;    // m x n row-major (lda)
  int64_t lda = 0, m = 0, n = 0;
  const double* Xt = nullptr;  // ncols x ldx, ldx even and >= n + F64_KST, zero past n
  int64_t ldx = 0;
  int ncols = 0;
  const double* alpha = nullptr;  // device scalar or null
  const double* corr = nullptr;   // ncols or null: Z = alpha (A Xt^T - 1 corr^T)
  double* Z = nullptr;
  int64_t ldz = 0;
  bool vec = false;            // A 16-byte aligned and lda % 4 == 0
  int ksplit = 1;              // > 1: partials P[s][r][c] (ldp >= ncols), kchunk % F64_KST == 0
  int64_t kchunk = 0;
  double* P = nullptr;
  int64_t ldp = 0, split_stride = 0;
  hipEvent_t ev_begin = nullptr, ev_end = nullptr;
};

struct Adj64Args {             // P_s = (A_s^T Z_s)^T, float32 A, float64 Z and P
  const float* A = nullptr;
  int64_t lda = 0, m = 0, n = 0;
  const double* Z = nullptr;   // m x ncols (ldz)
  int64_t ldz = 0;
  int ncols = 0;
  int64_t rows_per_split = 0;
  int nsplit = 0;
  double* P = nullptr;         // [nsplit][ncols][ldp], 32-byte aligned, ldp % 4 == 0
  int64_t ldp = 0, split_stride = 0;
  bool vec = false;
  hipEvent_t ev_begin = nullptr, ev_end = nullptr;
};

hipError_t launch_fwd64(const Fwd64Args& a, hipStream_t st);
hipError_t launch_adj64(const Adj64Args& a, hipStream_t st);
// Xt[j][c] = sum_s P[s][j][c] - d[c] zsum[j] (d, zsum null: no correction) in float64; per-block sums of
// squares into sq_part
hipError_t launch_reduce_x64(const double* P, int nsplit, int64_t split_stride, int64_t ldp, int ncols, int64_t n,
                             const double* d, const double* zsum, double* Xt, int64_t ldx, double* sq_part,
                             int* n_sq_part, hipStream_t st);
// corr[j] = sum_c d[c] Xt[j][c] (float64 X)
hipError_t launch_dot_rows64(const double* d, const double* Xt, int64_t ldx, int64_t n, int ncols, double* corr,
                             hipStream_t st);
// part[s][c] = sum over rows of split s of X[r][c] (float64 X, rows x cols, ld)
hipError_t launch_colsum_f64(const double* X, int64_t ld, int64_t rows, int cols, int64_t rows_per_split,
                             int nsplit, double* part, hipStream_t st);
hipError_t launch_check_finite_f64(const double* X, int64_t rows, int cols, int64_t ld, int* flag, hipStream_t st);
void fwd64_split(int64_t m, int64_t n, int ncols, int64_t slots, int* ksplit, int64_t* kchunk);
void adj64_split(int64_t m, int64_t n, int ncols, int64_t slots, int* nsplit, int64_t* rows_per_split);

// ---------------------------------------------------------------- Householder TSQR (qr_householder.hip)
// Level of the reduction tree: rows_total rows of X (ld L) in nb blocks of bu rows (the last block takes
// the remainder; every block has >= L rows).  factor: reflectors in place, tau[k L + j], R of block k to
// Rout + k L L.  apply: Yout rows of block k = Q_k [C_k; 0], C_k = rows [k L, (k+1) L) of Cin (identity
// when Cin is null).
hipError_t launch_hh_factor(double* X, int64_t rows_total, int64_t bu, int nb, int L, double* tau, double* Rout,
                            hipStream_t st);
hipError_t launch_hh_apply(const double* X, int64_t rows_total, int64_t bu, int nb, int L, const double* tau,
                           const double* Cin, double* Yout, hipStream_t st);
// per-workgroup LDS of the device for the two kernels above; whether blocks of maxrows rows fit
void set_hh_lds_limit(size_t bytes);
bool hh_fits(int L, int64_t maxrows);

// ---------------------------------------------------------------- auxiliary
// FP64 column sums of a row-major matrix in a given storage: part[s][c] over row splits.
hipError_t launch_colsum(int storage, const void* X, int64_t ld, int64_t rows, int64_t cols,
                         const float* col_scale, int64_t plane, int64_t rows_per_split, int nsplit,
                         double* part, hipStream_t st);
// out[c] = scale * sum_s part[s][c]; optional fl32 copy and residual d = out - fl32(out).
hipError_t launch_colsum_reduce(const double* part, int nsplit, int64_t cols, double scale, double* out,
                                float* out_f32, double* resid, hipStream_t st);
// Xt[c][r] = normal(seed, stream 1, r*l + c) rounded to float (G of Step 1).
hipError_t launch_gen_G(uint64_t seed, int64_t n, int l, float* Xt, int64_t ldx, hipStream_t st);
// Xt[c][r] = G[r][c]
hipError_t launch_transpose_G(const float* G, int64_t ldg, int64_t n, int l, float* Xt, int64_t ldx,
                              hipStream_t st);
// corr[j] = sum_c d[c] Xt[j][c]
hipError_t launch_dot_rows(const double* d, const float* Xt, int64_t ldx, int64_t n, int ncols, float* corr,
                           hipStream_t st);
// Xt[j][c] = sum_s P[s][j][c] - d[c] zsum[j]; per-block sums of squares into sq_part
hipError_t launch_reduce_y(const float* P, int nsplit, int64_t split_stride, int64_t ldp, int ncols, int64_t n,
                           const float* col_scale, const double* d, const double* zsum, float* Xt, int64_t ldx,
                           double* sq_part, int* n_sq_part, hipStream_t st);
// alpha = 1/sqrt(sum of sq_part) (1 when zero or rescaling is off); nonfinite flag
hipError_t launch_finish_scale(const double* sq_part, int n_part, bool rescale, double* alpha, int* flag,
                               hipStream_t st);
// T[c][j] = sum_s P[s][j][c] - d[c] qsum[j]  (T row-major n x ncols, FP64)
hipError_t launch_reduce_t(const float* P, int nsplit, int64_t split_stride, int64_t ldp, int ncols, int64_t n,
                           const float* col_scale, const double* d, const double* qsum, double* T, int64_t ldt,
                           hipStream_t st);
// the same reductions from a single float64 accumulator (streamed passes)
hipError_t launch_reduce_y64(const double* P, int64_t ldp, int ncols, int64_t n, const double* d, const double* zsum,
                             float* Xt, int64_t ldx, double* sq_part, int* n_sq_part, hipStream_t st);
hipError_t launch_reduce_t64(const double* P, int64_t ldp, int ncols, int64_t n, const double* d, const double* qsum,
                             double* T, int64_t ldt, hipStream_t st);
// acc[r][c] += sum_s part[s][r][c] over rows x cols (leading dimension ld)
hipError_t launch_accumulate_parts(bool f64, const void* part, int nsplit, int64_t split_stride, int64_t rows,
                                   int64_t cols, int64_t ld, double* acc, hipStream_t st);
// centring fused into pass 0: d0 = colsum(A - 1 s0^T)/m from row `row` of the adjoint partials,
// mu = s0 + d0, shift <- fl32(mu), dres = mu - fl32(mu)
// low-precision storage: mu[c] = cs[c] (cs null: 1) * sum_s P[s][row][c] / m, the column means of
// the stored matrix from the column sums an implicit ones column left in row `row` of the partials
hipError_t launch_pass0_mean_lp(const float* P, int nsplit, int64_t split_stride, int64_t ldp, int row, int64_t n,
                                int64_t m, const float* cs, double* mu, hipStream_t st);
hipError_t launch_pass0_center(const float* P, int nsplit, int64_t split_stride, int64_t ldp, int row, int64_t n,
                               int64_t m, float* shift, double* d0, double* mu, double* dres, hipStream_t st);
// X[r][c] -= corr[c]
hipError_t launch_sub_cols(float* X, int64_t ldx, int64_t rows, int cols, const float* corr, hipStream_t st);
// flag |= nonfinite(x) over a float matrix
hipError_t launch_check_finite_f32(const float* X, int64_t rows, int64_t cols, int64_t ld, int* flag,
                                   hipStream_t st);
hipError_t launch_fill_f64(double* p, int64_t count, double v, hipStream_t st);
hipError_t launch_fill_u32(unsigned* p, int64_t count, unsigned v, hipStream_t st);
// out[r][c] = X[r][c] - colsum[c] * inv_rows, float64 (projects the column sums out)
hipError_t launch_center_cols(const float* X, int64_t ldx, int64_t rows, int64_t cols, const double* colsum,
                              double inv_rows, double* out, int64_t ldo, hipStream_t st);

// ---------------------------------------------------------------- small FP64 algebra
// part[s][i][j] = sum over rows of split s of X[r][i] X[r][j]
hipError_t launch_gram(bool x_is_f64, const void* X, int64_t ldx, int64_t rows, int L, int64_t rows_per_split,
                       int nsplit, double* part, hipStream_t st);
// W = sum_s part[s] (+ shift * I when shift_from_trace: shift = coef * trace)
hipError_t launch_gram_reduce(const double* part, int nsplit, int L, double* W, double shift_coef,
                              hipStream_t st);
// per-workgroup LDS limit used to pick LDS-resident variants of the single-workgroup kernels
void set_max_lds(size_t bytes);
// W (L x L) -> upper R with W = R^T R in place; flag set on breakdown
hipError_t launch_cholesky(double* W, int L, double rel_tol, int* flag, hipStream_t st);
// Rinv = R^-1 (upper)
hipError_t launch_triinv(const double* R, int L, double* Rinv, hipStream_t st);
// Cholesky (as launch_cholesky) and R^-1 (as launch_triinv) in one launch, for L <= 1024
bool cholinv_fits(int L);
hipError_t launch_cholinv(double* W, int L, double rel_tol, int* flag, double* Rinv, hipStream_t st);
// C = A B (A: M x K float or double, B: K x N double), optional upper-triangular B,
// column scale, FP64 and/or FP32 outputs
hipError_t launch_gemm64(bool a_is_f64, const void* A, int64_t lda, const double* B, int64_t ldb, int64_t M,
                         int N, int K, bool b_upper, const double* colscale, double* C, int64_t ldc, float* C32,
                         int64_t ldc32, hipStream_t st, const double* Cin = nullptr, int64_t ldcin = 0);
// C (L x L) = A (L x L upper) * B (L x L upper)
hipError_t launch_trmm_upper(const double* A, const double* B, int L, double* C, hipStream_t st);

// Step 4 eigensolver (small_eig.hip): M (L x L) = W diag(lam) W^T; lam_desc all L
// eigenvalues descending, sig_desc = sqrt(max(lam, 0)), W[:, 0:kk] the leading eigenvectors
size_t syev_small_work(int L, int kk);
hipError_t launch_syev_small(const double* M, int L, int kk, double* work, double* lam_desc, double* sig_desc,
                             double* W, int ldw, size_t max_lds, hipStream_t st);
// V[:, j] /= ||V[:, j]|| and sign so the largest |entry| is positive; sig[j] = norm; sgn[j] = sign
hipError_t launch_normalize_sign(double* V, int64_t rows, int k, int64_t ldv, double* sig, double* sgn,
                                 hipStream_t st);
// out32[r][j] = (float) (X[r][j] * colscale[j])
hipError_t launch_to_f32(const double* X, int64_t rows, int cols, int64_t ldx, const double* colscale,
                         float* out, int64_t ldo, hipStream_t st);

// ---------------------------------------------------------------- backward (backward.hip)
// out (na x nb) = (X^T Y) * colscale (columns), X rows x na, Y rows x nb, split over rows
hipError_t launch_xty(bool x64, const void* X, int64_t ldx, int na, bool y64, const void* Y, int64_t ldy, int nb,
                      int64_t rows, int64_t rows_per_split, int nsplit, const double* colscale, double* part,
                      double* out, hipStream_t st);
hipError_t launch_svdadj_prep(const double* W, const double* sig, const double* sgn, int L, int k, double* WT,
                              double* Wsc, double* Ck, double* Bp, hipStream_t st);
hipError_t launch_svdadj_mid(const double* XV, const double* YW, const double* sig, const float* gS, int L, int k,
                             double* N, hipStream_t st);
hipError_t launch_copyltu_neg(const double* M2, int L, double* S, hipStream_t st);
hipError_t launch_transpose_sq(const double* in, int L, bool upper_only, double* out, hipStream_t st);
hipError_t launch_transpose_out(const double* X, int64_t ldx, int64_t rows, int cols, float* out32, double* out64,
                                int64_t ldo, hipStream_t st);
hipError_t launch_widen(const float* X, int64_t ldx, int nrows, int64_t ncols, double* Y, int64_t ldy,
                        hipStream_t st);
hipError_t launch_add_f32(const float* Z, int64_t ldz, int64_t rows, int cols, double* C, int64_t ldc,
                          bool accumulate, hipStream_t st);
hipError_t launch_combine(const double* Hb, int64_t ldh, const float* Zf, int64_t ldz, int64_t rows, int cols,
                          const double* alpha, double* out64, int64_t ld64, float* out32, int64_t ld32,
                          hipStream_t st);
hipError_t launch_copy_cols(bool x64, const void* X, int64_t ldx, int64_t rows, int cols, double* out, int64_t ldo,
                            hipStream_t st);
hipError_t launch_center_f64(double* X, int64_t ldx, int64_t rows, int cols, int64_t rows_per_split, int nsplit,
                             double* part, hipStream_t st);
// residual estimator helpers
hipError_t launch_gen_normal64(uint64_t seed, uint32_t stream, int64_t rows, int cols, double* out, int64_t ldo,
                               hipStream_t st);
hipError_t launch_neg_rowscale(double* C, const float* s, int k, int q, hipStream_t st);
hipError_t launch_sqrt_max(const double* v, int q, double* out, hipStream_t st);

// ---------------------------------------------------------------- quantiser entry points (plan.cpp)
// split rule and scratch bytes; argument checks; the kernels on a caller-provided scratch
size_t quantize_scratch(int64_t m, int64_t n, int* ns, int64_t* rps);
int quantize_check(int32_t storage, int64_t m, int64_t n, const float* A, int64_t lda, const void* out, int64_t ldo,
                   const float* col_scale, const float* shift, int32_t shift_mode);
hipError_t quantize_run(int32_t storage, int64_t m, int64_t n, const float* A, int64_t lda, void* out, int64_t ldo,
                        float* col_scale, float* shift, int32_t shift_mode, void* scratch, int ns, int64_t rps,
                        hipStream_t st);

}  // namespace rpca
