// Internal launch interface of the rSVD kernels (not part of the C ABI).
#pragma once

#include "common.hpp"

namespace rsvd {

// ---- FP64 matrix-core GEMM (gemm.hip) --------------------------------------
struct GemmShape {
  int nt = 1, tiles_m = 1, tiles_n = 1, splits = 1;
  int64_t kchunk = 0;
  size_t part_doubles = 0;
};
GemmShape dgemm_shape(int64_t M, int64_t N, int64_t K, int max_splits = 64);
// select the LDS-DMA streaming kernel where eligible, with 4 or 8 waves per workgroup
void dgemm_set_dma(bool on, int waves = 4);
// whether an untransposed product of inner size K with N columns, A and B as
// given, streams through the LDS-DMA kernel
// whether A^T B with A (K x M) in its stored orientation streams through the
// LDS-DMA kernel's transposed variant
bool dgemm_dma_eligible_t(int64_t M, int64_t K, int64_t N, const double* A, int64_t lda,
                          const double* B, int64_t ldb);
bool dgemm_dma_eligible(int64_t K, int64_t N, const double* A, int64_t lda, const double* B,
                        int64_t ldb);
// Bf (FP32 schedule only): the FP32 panel of B (ldbf floats per row, 16-byte
// aligned, ldbf a multiple of 4) that the streaming kernel reads instead of B
// where it applies; B must still be given. Bp (A B only): a copy of B with an
// even leading dimension ldbp >= N + (N & 1), 16-byte aligned, that the
// streaming kernel stages when B itself does not fit it (odd N or ldb); its
// padding column is read but never reaches C. B must still be given.
rsvd_status dgemm(bool ta, int64_t M, int64_t N, int64_t K, double alpha, const double* A,
                  int64_t lda, const double* B, int64_t ldb, double beta, double* C, int64_t ldc,
                  double* part, size_t part_doubles, hipStream_t st, int max_splits = 64,
                  const uint32_t* pred = nullptr, int prec = kPrecF64, const float* Bf = nullptr,
                  int64_t ldbf = 0, const double* Bp = nullptr, int64_t ldbp = 0);
// Error-free sliced product C = A X (sliced.hip): A (M x K, lda) and X
// (K x N, ldx) FP64, cut into 7 INT8 slices per entry with one power-of-two
// scale per row of A and per column of X, the slice products exact in INT32
// on the integer matrix cores, summed in FP64 (about 1e-14 relative to
// K max_k |a_ik| max_k |x_kj|). work: sliced_work_bytes(M, N, K) bytes,
// 256-byte aligned. sliced_prepare_a slices A into work once; sliced_gemm
// then slices X and forms C (ldc >= N) from both; both on stream s.
size_t sliced_work_bytes(int64_t M, int64_t N, int64_t K);
rsvd_status sliced_prepare_a(int64_t M, int64_t N, int64_t K, const double* A, int64_t lda,
                             void* work, hipStream_t s);
rsvd_status sliced_gemm(int64_t M, int64_t N, int64_t K, const double* X, int64_t ldx, double* C,
                        int64_t ldc, void* work, hipStream_t s);
// FP32 panel Xf (rows x f32_panel_ld(cols)) of X, rounded to nearest, zero padded
int64_t f32_panel_ld(int64_t cols);
rsvd_status f32_panel(int64_t rows, int64_t cols, const double* X, int64_t ldx, float* Xf,
                      hipStream_t s);
// ||A - US * Vt||_F^2 and ||A||_F^2 accumulated into st->resid2 / st->fro2
// (US: M x K, Vt: K x N, A: M x N). partial: >= resid_partials(M, N) doubles.
size_t resid_partials(int64_t M, int64_t N);
rsvd_status resid(int64_t M, int64_t N, int64_t K, const double* US, int64_t ldus,
                  const double* Vt, int64_t ldvt, const double* A, int64_t lda,
                  double* partial, DevState* st, hipStream_t s);

// ---- BF16 early products from BF16 planes (bf16gemm.hip) ------------------
// Plane layout: row-major uint16 BF16 bits, leading dimension a multiple of
// 64, zero padded. Split schedule: a lo plane beside each hi plane.
struct Bf16Shape {
  int nt = 1, rw = 1, tiles_m = 1, tiles_n = 1, splits = 1;
  int64_t Kp = 0, kchunk = 0, xt_rows = 0;
  size_t part_floats = 0;
};
int64_t bf16_pad(int64_t k);
// largest split count bf16_shape uses for M x N, and the partials it needs
int bf16_split_cap(int64_t M, int64_t N);
size_t bf16_part_floats_max(int64_t M, int64_t N);
// rw: 16-row fragments per wave (1 or 2; 0 picks), splits: K ranges (0
// picks, at most 16), groups: column groups (0 picks the fewest; at most
// twice the fewest)
Bf16Shape bf16_shape(int64_t M, int64_t N, int64_t K, bool split, int rw = 0, int splits = 0,
                     int groups = 0);
// the tuned shape of this product if the autotuner has one, else bf16_shape's
Bf16Shape bf16_tuned_shape(int64_t M, int64_t N, int64_t K, bool split);
// rows of XT any shape for N columns may use
int64_t bf16_xt_rows_max(int64_t N);
// Planes of X (R x C, FP64): same orientation into n_hi / n_lo (R x ld_n)
// and / or transposed into t_hi / t_lo (rows_t x ld_t, t(c, r) = X(r, c)),
// zero padded. Null hi pointers skip an orientation, null lo pointers the lo plane.
rsvd_status bf16_planes(int64_t R, int64_t C, const double* X, int64_t ldx, uint16_t* n_hi,
                        uint16_t* n_lo, int64_t ld_n, uint16_t* t_hi, uint16_t* t_lo, int64_t ld_t,
                        int64_t rows_t, hipStream_t s);
// C (M x N) = P X with P the A planes (M x sh.Kp, lda) and X given as XT
// planes (sh.xt_rows x sh.Kp); split: hi*lo + lo*hi + hi*hi per term.
// part: >= sh.part_floats floats when sh.splits > 1.
rsvd_status bf16_gemm(const Bf16Shape& sh, int64_t M, int64_t N, const uint16_t* A_hi,
                      const uint16_t* A_lo, int64_t lda, const uint16_t* XT_hi,
                      const uint16_t* XT_lo, double* C, int64_t ldc, float* part,
                      size_t part_floats, bool split, hipStream_t st);

// ---- random projection (omega.hip) -----------------------------------------
rsvd_status gaussian_omega(int64_t n, int64_t l, int64_t col0, uint64_t seed, uint64_t channel,
                           double* out, int64_t ldo, hipStream_t st);

// ---- small dense l x l kernels (smalldense.hip) -----------------------------
// Cholesky of the Gram G (l x l; overwritten, used as scratch) into R (upper,
// R^T R = G [+ shift I]) and Rinv = R^{-1} (full_inverse), or only the
// inverses of R's 16 x 16 diagonal tiles in Rinv (what trsm_upper uses).
// pass 0 may switch to the shifted factorization (sets st->qr_shifted); a
// pass with only_if_shifted != 0 does nothing unless st->qr_shifted is set.
// m = rows of the panel (sizes the shift). Without the full inverse and for
// l <= 272 one workgroup factors with the tiles in registers; otherwise a
// grid of workgroups (at most 1/share of the device's co-resident capacity,
// for runs on concurrent streams) with the current 32-row block row in
// scratch: chol_panel_doubles(l) doubles of global memory (required).
size_t chol_panel_doubles(int64_t l);
rsvd_status chol_inv(int64_t l, double* G, double* R, double* Rinv, double* scratch, int64_t m,
                     int pass, int only_if_shifted, DevState* st, hipStream_t s, int share = 1,
                     bool full_inverse = true);
// Q = Y R^{-1} (rows x l) by block forward substitution with R upper
// triangular and Xd holding the inverses of R's 16 x 16 diagonal tiles (as
// chol_inv writes them, with or without the full inverse), both with leading
// dimension ldr; skipped when pred is non-null and *pred == 0. Y and Q may be
// the same panel. Supported for l <= 608 (trsm_supported); wider factors are
// solved by column blocks (orth).
bool trsm_supported(int64_t l);
// G = Y^T Y (l x l, both triangles) of a rows x l panel by slabs of rows on
// the matrix cores (upper tiles, per-slab partials in part, summed in a fixed
// order) for l <= 272; the general product for wider panels or when part has
// too little room; skipped when pred is non-null and *pred == 0.
rsvd_status gram(int64_t rows, int64_t l, const double* Y, int64_t ldy, double* G, double* part,
                 size_t part_doubles, const uint32_t* pred, hipStream_t s);
rsvd_status trsm_upper(int64_t rows, int64_t l, const double* Y, int64_t ldy, const double* R,
                       int64_t ldr, const double* Xd, double* Q, int64_t ldq,
                       const uint32_t* pred, hipStream_t s);
// Householder QR of the rows x l panel Yorig into Y (= Q) and R, run only
// when st->qr_householder is set (tau: 2 l doubles of scratch; scratch: l x l
// doubles for the grid variant of large panels, may be null; share: runs on
// concurrent streams, as for chol_inv).
rsvd_status householder_fallback(int64_t rows, int64_t l, const double* Yorig, double* Y,
                                 double* R, double* tau, double* scratch, DevState* st,
                                 hipStream_t s, int share = 1);
// Copy src -> dst (rows x cols, row-major): always (cond 0), only when
// st->qr_shifted is set (cond 1), only when it is clear (cond 2).
rsvd_status copy_panel(int64_t rows, int64_t cols, const double* src, int64_t lds, double* dst,
                       int64_t ldd, int cond_shifted, DevState* st, hipStream_t s);
// Block one-sided Jacobi (bjacobi.hip): M, P are Lp x Lp (Lp = jacobi_padded(l))
// workspace buffers; M <- R zero padded, P <- I, then the rows of M are
// orthogonalized and the rotations accumulated in P (P null: not
// accumulated, for runs that want the values only).
int64_t jacobi_padded(int64_t l);
// Batched small SVDs: one channel of the table, byte offsets into the batch
// workspace of its Jacobi matrix (Lp x Lp, prepared by jacobi_prepare), of
// its device state and of its rotations P (or -1).
struct JacChan {
  int64_t M_off, st_off, P_off;  // P_off < 0: no rotations kept
  int l, Lp, max_sweeps, pad;
};
// M <- R zero padded (Lp x Lp), P <- I when given, the state's sweep
// counters cleared and its sweep count unset
rsvd_status jacobi_prepare(int64_t l, const double* R, double* M, double* P, DevState* st,
                           hipStream_t s);
size_t jacobi_batch_max_channels();
// the sweeps of every channel of the (device) table in one launch, all
// channels in lockstep rounds separated by the grid barrier bar (in device
// memory, reset here); first_round_pairs: the pairs of all channels in the
// first round (the grid is at most that and what the device holds at once)
rsvd_status jacobi_batch(const JacChan* table, int nch, int64_t first_round_pairs, char* work,
                         GridBar* bar, hipStream_t s);
// a channel whose batched sweeps never finished is flagged SYNC_TIMEOUT
rsvd_status jacobi_check_done(DevState* st, hipStream_t s);
// share > 1: at most 1/share of the device's co-resident workgroups (for
// runs on concurrent streams, whose cooperative grids must fit together).
rsvd_status block_jacobi(int64_t l, const double* R, double* M, double* P, int max_sweeps,
                         int inner_sweeps, DevState* st, hipStream_t s, int share = 1);
// From converged M, P: s (decreasing), Us (l x kc), W (l x kc); scratch:
// 2 l doubles. kc = 0: the values only (P may then be null).
rsvd_status svd_finish(int64_t l, int64_t kc, const double* M, const double* P, int64_t ld,
                       double* s, double* Us, double* W, double* scratch, DevState* st,
                       hipStream_t st_);
rsvd_status select_rank(int64_t l, int64_t p, int64_t kc, int mode, double param,
                        const double* s, DevState* st, hipStream_t hs);
// Sign rule on the first kc columns of U (m x kc) and V (n x kc, may be null);
// scratch: 2 kc doubles.
rsvd_status sign_fix(int64_t m, int64_t n, int64_t kc, double* U, int64_t ldu, double* V,
                     int64_t ldv, double* scratch, hipStream_t s);
// US = U diag(s) (m x kcp), Vt = V^T (kcp x n); columns / rows >= rank are zero
rsvd_status resid_prep(int64_t m, int64_t n, int64_t kc, int64_t kcp, const double* U,
                       int64_t ldu, const double* s_vals, const double* V, int64_t ldv, double* US,
                       double* Vt, const DevState* st, hipStream_t s);
rsvd_status check_finite(int64_t rows, int64_t cols, const double* Y, int64_t ldy, DevState* st,
                         hipStream_t s);
rsvd_status sumsq(int64_t m, int64_t n, const double* A, int64_t lda, double* partial,
                  DevState* st, hipStream_t s);
// dev_est: err_est = kPosteriorFactor sqrt(st->est2) instead of the argument
rsvd_status finalize(int64_t m, int64_t n, int64_t l, int want_residual, double err_est,
                     int blocks, const DevState* st, rsvd_result* res, hipStream_t s,
                     bool dev_est = false);
// UNCONVERGED / POSTERIOR_FAIL flags of a judged fixed-l run (after the rank rule)
rsvd_status judge(int64_t l, int64_t mn, int q, int mode, double tau, const double* sv,
                  DevState* st, hipStream_t s);
// st->flags = (st->flags & ~clear) | set
rsvd_status clear_flags(DevState* st, uint32_t clear, uint32_t set, hipStream_t s);
// Column sums of squares of X (rows x cols <= 256, row-major): mode 0 sets
// st->est2 to their maximum; mode 1 raises st->s1lb2 to their maximum and
// adds their sum to st->froY2. partial: scratch of partial_doubles >= cols.
rsvd_status colsumsq(int64_t rows, int cols, const double* X, int64_t ld, double* partial,
                     size_t partial_doubles, int mode, DevState* st, hipStream_t s);
rsvd_status init_state(DevState* st, uint32_t flags, hipStream_t s);
rsvd_status clear_shift(DevState* st, hipStream_t s);
rsvd_status sum_partials_into(int64_t cnt, const double* p, double* out, hipStream_t s);
rsvd_status set_identity(int64_t l, double* P, hipStream_t s);
// B <- (B + B^T) / 2 (l x l, in place)
rsvd_status symmetrize(int64_t l, double* B, int64_t ldb, hipStream_t s);
rsvd_status transpose(int64_t rows, int64_t cols, const double* src, int64_t lds, double* dst,
                      int64_t ldd, hipStream_t s);

// ---- learned (k, p, q) predictor (mlp.hip) ---------------------------------
rsvd_status mlp_init(float* p, uint64_t seed, hipStream_t s);
rsvd_status mlp_forward(const float* p, const float* X, int64_t B, float* Y, hipStream_t s);
// One batch (B <= 128): loss into *loss (may be null); adam: Adam step
// number `step` (>= 1) applied to p, m, v; else the gradient into G.
rsvd_status mlp_grad(float* p, const float* X, const float* T, int64_t B, bool adam, float* m,
                     float* v, int64_t step, float lr, float* G, float* loss, hipStream_t s);
// sizing (k, p, q) per sample from the network (rsvd_mlp_predict)
rsvd_status mlp_predict(const float* p, const float* stats, const float* X, int64_t B,
                        const int64_t* n_cap, int64_t* kpq, hipStream_t s);
// standardized training targets and their stats (rsvd_mlp_targets)
rsvd_status mlp_targets(const int64_t* labels, int64_t B, float* stats, float* T, hipStream_t s);
// label of one channel from a computed spectrum (rsvd_size_label)
rsvd_status size_label(const double* sv, int64_t count, int64_t k, int64_t n, int64_t l_min,
                       int64_t* kpq, hipStream_t s);
// f_i = max(log10(sig_i / sig_0), -16) for i < 16 (sig: l decreasing values)
rsvd_status pilot_features(int l, const double* sig, float* feat, hipStream_t s);

}  // namespace rsvd
