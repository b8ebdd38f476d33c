/*
 * rsvd.h - C ABI of the MI355X randomized truncated SVD library (librsvd.so).
 *
 * The library computes the randomized SVD described in arXiv:2307.15572,
 * section "Randomized matrix decompositions" (Fig. 1, Eq. 1, Eq. 2): for a
 * dense real matrix V (here called A, m x n) it draws a Gaussian random
 * projection P (n x l), forms Z = A P, an orthonormal basis Q of Z (thin
 * QR, step 1), projects Y = Q^T A, takes the thin SVD Y = L_Y Sigma R^T
 * (step 2) and lifts L = Q L_Y (step 3). l = R_SVD + p with oversampling p.
 * The singular values come back sorted decreasingly (Eq. 1) and the result
 * is truncated to a rank R_SVD chosen by one of the rank rules below.
 * Optional q power iterations (Halko et al.'s randomized subspace iteration,
 * a QR after every product) sit between step 1 and step 2; q = 0 is the
 * paper's method.
 *
 * Conventions shared by every entry point:
 *  - All matrices are row-major FP64 (C / torch-contiguous order). A has
 *    leading dimension lda >= n. Device pointers unless stated otherwise.
 *  - The caller owns every buffer (inputs, outputs, result record and
 *    workspace). The library never allocates device memory in rsvd_run and
 *    never writes A.
 *  - All work is enqueued on the caller's stream (a hipStream_t passed as
 *    void*, NULL = the null stream). Nothing synchronizes the host.
 *  - Errors are reported by return code only; no exception crosses the ABI.
 *    Data-dependent outcomes (non-finite input, capped rank, QR fallback,
 *    Jacobi not converged) are flags in the device-side result record.
 */
#ifndef RSVD_H
#define RSVD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum rsvd_status {
  RSVD_OK = 0,
  RSVD_EINVAL = 1,        /* invalid argument (sizes, modes, pointers)            */
  RSVD_ENOMEM = 2,        /* workspace smaller than rsvd_plan reported            */
  RSVD_EHIP = 3,          /* a HIP runtime call or kernel launch failed           */
  RSVD_EUNSUPPORTED = 4   /* valid request this build does not implement          */
} rsvd_status;

/* Rank rules (section "Randomized matrix decompositions": R_SVD is the number
 * of singular values kept, R% = 100 R_SVD / N). */
enum {
  RSVD_RANK_FIXED = 0,         /* R_SVD = k                                        */
  RSVD_RANK_PERCENT = 1,       /* R_SVD = ceil(R% min(m,n) / 100), rank_param = R% */
  RSVD_RANK_REL_THRESHOLD = 2, /* R_SVD = #{j : s_j >= tau s_1}, capped at l - p
                                  unless l = min(m, n) (exact SVD)                 */
  RSVD_RANK_FROB_TAIL = 3      /* smallest R_SVD with discarded energy <= tau ||A||_F */
};

/* Arithmetic of the products with A (the 2q+2 streaming passes). */
enum {
  RSVD_PREC_FP64 = 0,          /* every product in FP64 (MFMA f64)                  */
  RSVD_PREC_MIXED_FP32 = 1,    /* early passes FP32 MFMA, trailing passes FP64       */
  RSVD_PREC_MIXED_BF16 = 2,    /* early passes BF16 MFMA (FP32 accumulate)           */
  RSVD_PREC_MIXED_BF16_SPLIT = 3, /* early passes on BF16 matrix cores with each operand
                                    split x = hi + lo (hi = bf16(x), lo = bf16(x - hi)):
                                    hi*lo + lo*hi + hi*hi, FP32 accumulation          */
  RSVD_PREC_MIXED_FP32_SLICED = 4 /* early passes as RSVD_PREC_MIXED_FP32; the trailing
                                    passes and the projection (products A X; A^T X of a
                                    non-symmetric A stays FP64) as error-free sliced
                                    products: 7 INT8 slices per entry (one power-of-two
                                    scale per row of A, per column of the panel), slice
                                    products exact in INT32 on the integer matrix
                                    cores, summed in FP64 (rsvd_gemm, mode 4)         */
};

/* How step 2 projects A (rsvd_problem.form). */
enum {
  RSVD_FORM_SVD = 0,           /* the paper's form: Y = Q^T A (l x n), thin SVD of Y   */
  RSVD_FORM_SYMMETRIC = 1      /* symmetric channels (section "Low-rank interactions":
                                  the interaction is Hermitian, each channel block
                                  symmetric): A ~ Q B Q^T with B = Q^T A Q (l x l),
                                  B symmetrized, SVD of B = L_B Sigma R_B^T, then
                                  L = Q L_B and R = Q R_B (Halko, Martinsson and
                                  Tropp 2011, section 5.3). Needs symmetric = 1;
                                  fixed-l runs only (not adaptive)                   */
};

/* Flags in rsvd_result.flags */
enum {
  RSVD_FLAG_FULL_SVD = 1u << 0,        /* l = min(m, n): the result is an exact SVD  */
  RSVD_FLAG_RANK_CAPPED = 1u << 1,     /* rank rule wanted more than l - p or k_cap  */
  RSVD_FLAG_QR_FALLBACK = 1u << 2,     /* Cholesky QR broke down (rank-deficient panel): Householder QR used */
  RSVD_FLAG_JACOBI_MAXSWEEP = 1u << 3, /* small SVD stopped at max_sweeps            */
  RSVD_FLAG_NONFINITE_INPUT = 1u << 4, /* A holds NaN or Inf                         */
  RSVD_FLAG_ZERO_SIGMA = 1u << 5,      /* a singular value is exactly zero           */
  RSVD_FLAG_ADAPT_LIMIT = 1u << 6,     /* adaptive growth stopped at l_max           */
  RSVD_FLAG_SYNC_TIMEOUT = 1u << 7,    /* a grid-wide barrier (multi-workgroup Cholesky,
                                          Householder fallback or small SVD) gave up
                                          waiting (bounded wait): results invalid     */
  /* set only by runs with posterior > 0 (the a-posteriori judge, below):       */
  RSVD_FLAG_POSTERIOR_FAIL = 1u << 8,  /* REL_THRESHOLD: the posterior estimate of
                                          ||(I - QQ^T) A||_2 exceeds tau s_1: the basis
                                          may miss values above the threshold        */
  RSVD_FLAG_UNCONVERGED = 1u << 9      /* threshold rules: (s_l / s_k)^(4q + 2) > 1e-8
                                          for the kept rank k (Halko et al.'s subspace-
                                          iteration factor): kept values not converged */
};

typedef struct rsvd_problem {
  int64_t m, n;          /* A is m x n                                             */
  int64_t k;             /* target rank; l = min(k + oversample, m, n)             */
  int64_t k_cap;         /* columns of U, V and entries of S the caller provides;
                            0 = l                                                  */
  int32_t symmetric;     /* caller asserts A == A^T; A is then used for A^T        */
  int32_t rank_mode;     /* RSVD_RANK_*                                            */
  double rank_param;     /* R% for PERCENT, tau for the threshold rules            */
  int32_t oversample;    /* p >= 0 (the paper uses p = 5)                          */
  int32_t power_iters;   /* q >= 0 (0 = the paper's method)                        */
  int32_t precision;     /* RSVD_PREC_*                                            */
  int32_t trailing_hp;   /* mixed modes: how many of the last products before the
                            projection stay FP64 (the projection always does)      */
  uint64_t seed;         /* key word 0 of the Philox stream that draws P           */
  uint64_t channel;      /* key word 1 (symmetry channel index)                    */
  int32_t want_u;        /* write U (m x rank)                                     */
  int32_t want_v;        /* write V (n x rank)                                     */
  int32_t want_residual; /* stream A once more for ||A - U S V^T||_F / ||A||_F     */
  int32_t max_sweeps;    /* Jacobi sweep limit for the small SVD; 0 = 30           */
  int32_t adaptive;      /* 1: grow l block by block (adaptive range finder, below);
                            threshold rules only, FP64 only, k is ignored          */
  int32_t block;         /* adaptive: columns added per growth step (1..256; 0 = 64) */
  int64_t l_max;         /* adaptive: largest l (0 = min(m, n, 4096))              */
  int32_t form;          /* RSVD_FORM_* (0 = the paper's one-sided projection)     */
  int32_t posterior;     /* fixed-l runs: r probe columns (0 = none, 1..64) for the
                            a-posteriori judge: columns l .. l+r-1 of the same
                            Philox stream, W = (I - QQ^T) A P_r on the final basis
                            Q (one more FP64 stream of A with r columns), err_est =
                            10 sqrt(2/pi) max_j ||W_j|| (Halko et al. 2011, section
                            4.3: bounds ||(I - QQ^T) A||_2 except with probability
                            10^-r); threshold rules then also set POSTERIOR_FAIL /
                            UNCONVERGED. Adaptive runs: must be 0 (they judge
                            every block themselves)                              */
} rsvd_problem;

/* Result record, written to DEVICE memory by rsvd_run (so runs stay
 * capturable in a graph); copy it back after synchronizing the stream. */
typedef struct rsvd_result {
  int64_t rank;          /* R_SVD: number of valid entries of S / columns of U, V  */
  int64_t l_used;        /* sketch width l                                         */
  double residual;       /* ||A - U_k S_k V_k^T||_F / ||A||_F (NaN if not asked)   */
  double rel_percent;    /* R% = 100 rank / min(m, n)                              */
  double c_eq2;          /* Eq. 2 as printed: m n / ((m + n) rank + rank)          */
  double c_sym;          /* one stored factor: m n / (max(m, n) rank + rank)       */
  double fro2;           /* ||A||_F^2                                              */
  int32_t sweeps;        /* Jacobi sweeps used by the small SVD                    */
  uint32_t flags;        /* RSVD_FLAG_*                                            */
  double err_est;        /* adaptive: last error estimate of the basis (posterior
                            estimate of ||(I - QQ^T) A||_2 for REL_THRESHOLD, the
                            Frobenius indicator sqrt(||A||_F^2 - ||Q^T A||_F^2) for
                            FROB_TAIL); fixed-l run: the posterior estimate when
                            posterior > 0, else NaN                                */
  int32_t blocks;        /* adaptive: growth steps taken (0 for a fixed-l run)     */
  int32_t reserved;
} rsvd_result;

typedef struct rsvd_plan_s* rsvd_plan_t;

/*
 * rsvd_plan - validate a problem and size its workspace.
 *   prob            host pointer, read only.
 *   out             receives an immutable plan (host object); free it with
 *                   rsvd_destroy. Concurrent runs of one plan need distinct
 *                   workspaces.
 * Concurrency: the multi-workgroup Cholesky, Householder and Jacobi kernels
 * synchronize their workgroups with grid-wide barriers and size their grids
 * to what the whole device holds at once. Two rsvd_run calls whose kernels
 * overlap on one device (different streams) may therefore not all be
 * co-resident: their barriers then time out and the results carry
 * RSVD_FLAG_SYNC_TIMEOUT. Independent decompositions that should run side
 * by side go through rsvd_batch_run, which divides the device among its
 * lanes; rsvd_run calls on one device are meant to be ordered (one stream,
 * or streams joined by events).
 *   workspace_bytes receives the device workspace size rsvd_run needs.
 *                   For m n >= 2^18 it includes, when n is odd, room for a
 *                   copy of A with an even leading dimension (made by runs
 *                   whose lda is odd or whose A is not 16-byte aligned) and,
 *                   when l is odd, for a copy of the streamed panel with an
 *                   even leading dimension: the streaming products read
 *                   16-byte rows.
 * Returns RSVD_EINVAL for m, n < 1, k < 1 (fixed rule), p < 0, q < 0,
 * R% outside (0, 100], tau outside (0, 1), an unknown mode, trailing_hp < 0,
 * or k_cap < the fixed rank, an unknown form, the symmetric form without
 * symmetric = 1, posterior outside 0..64 (or != 0 when adaptive), and for
 * an adaptive problem with a fixed or
 * percent rule, block outside 0..256 or l_max < 0; RSVD_EUNSUPPORTED for
 * an adaptive problem in a mixed mode or in the symmetric form, or l > 4096.
 * Mixed modes: of the 2q + 1 products before the projection (sketch and
 * power products), all but the last trailing_hp run on FP32 or BF16 (plain
 * or split) matrix cores with FP32 accumulation; the projection, every QR,
 * the small SVD and the residual stay FP64.
 */
rsvd_status rsvd_plan(const rsvd_problem* prob, rsvd_plan_t* out, size_t* workspace_bytes);

/*
 * Adaptive range finder (problem.adaptive = 1). The paper fixes l before the
 * projection; with a threshold rule the rank, and so l, is not known in
 * advance. The basis Q then grows by blocks of b columns of the same
 * projection stream (columns l .. l+b-1, so P never depends on l), following
 * the blocked adaptive range finder of Halko, Martinsson and Tropp (SIAM
 * Rev. 2011, section 4.4) with the power scheme and Frobenius indicator of
 * blocked randQB (Martinsson and Voronin 2016; Yu, Gu and Li 2018):
 *   W = (I - QQ^T) A P_blk; est = 10 sqrt(2/pi) max_j ||W_j|| bounds
 *   ||(I - QQ^T) A||_2 except with probability 10^-b (section 4.3 there).
 *   REL_THRESHOLD: stop when est <= tau * (largest row norm of Q^T A) and the
 *     small SVD of the current projection keeps at most l - p values.
 *   otherwise Q_b = orth(W) (re-orthonormalized against Q), q power steps on
 *     (I - QQ^T) A, Y_b = Q_b^T A, Q = [Q Q_b], l += b.
 *   FROB_TAIL: stop when ||A||_F^2 - ||Q^T A||_F^2 <= tau^2 ||A||_F^2 and the
 *     rule keeps at most l - p values.
 * Steps 2 and 3 then run on the final basis. The growth decisions are taken
 * on the host: an adaptive rsvd_run synchronizes its stream once or twice per
 * block and cannot be captured in a graph. omega must be NULL. U, V, S
 * receive min(k_cap, l_used) columns / values; the workspace is sized for
 * l_max.
 */

/* Sketch width l of a plan (host query; l_max for an adaptive plan). */
int64_t rsvd_plan_l(rsvd_plan_t plan);

/*
 * rsvd_run - one randomized SVD of A (Fig. 1 steps 1-3 plus truncation).
 *   A, lda        m x n input (device, read only), lda >= n.
 *   omega, ldo    optional caller-provided projection P (n x l, device, ldo >= l);
 *                 NULL draws P from the Philox4x64-10 / Box-Muller stream keyed
 *                 by (seed, channel): entry (i, j) uses counter (i, j/4, 0, 0).
 *   S             k_cap singular values (device), decreasing; first rank valid.
 *   U, ldu        m x k_cap left vectors (device, ldu >= k_cap) or NULL if !want_u.
 *   V, ldv        n x k_cap right vectors (device, ldv >= k_cap) or NULL if !want_v.
 *   res_dev       device rsvd_result record.
 *   work          device workspace of at least the planned size (256-B aligned).
 *   stream        hipStream_t.
 * Signs: each pair (U_j, V_j) is flipped so the largest-magnitude entry of
 * U_j is positive (lowest index on ties).
 */
rsvd_status rsvd_run(rsvd_plan_t plan, const double* A, int64_t lda,
                     const double* omega, int64_t ldo,
                     double* S, double* U, int64_t ldu, double* V, int64_t ldv,
                     rsvd_result* res_dev, void* work, size_t work_bytes, void* stream);

/*
 * rsvd_run_noalloc - rsvd_run for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc). Arguments as rsvd_run, without work / work_bytes: the workspace
 * is a static device array of RSVD_NOALLOC_MAX_BYTES (64 MiB) inside the
 * library, one copy per device, held until the process ends. Its device
 * address is looked up on the first call on each device (with that device
 * current; the call runs on the device current at the call). Nothing is
 * allocated, and the run clears what must start at zero itself.
 * Returns RSVD_ENOMEM, before enqueueing anything, when the plan's workspace
 * (rsvd_plan's workspace_bytes) exceeds RSVD_NOALLOC_MAX_BYTES; otherwise
 * what rsvd_run returns. Calls that overlap on one device (other streams,
 * other host threads) share the array and race: order them.
 */
#define RSVD_NOALLOC_MAX_BYTES ((size_t)64 << 20)
size_t rsvd_noalloc_max_bytes(void);
rsvd_status rsvd_run_noalloc(rsvd_plan_t plan, const double* A, int64_t lda,
                             const double* omega, int64_t ldo,
                             double* S, double* U, int64_t ldu, double* V, int64_t ldv,
                             rsvd_result* res_dev, void* stream);

/* Free a plan (NULL is ignored). */
void rsvd_destroy(rsvd_plan_t plan);

/* Static description of a status code. */
const char* rsvd_strerror(rsvd_status s);

/*
 * Batched decompositions (independent symmetry channels, section "Low-rank
 * interactions": every partial-wave channel's matrix is decomposed on its
 * own). A batch plan holds one plan per channel and runs them together:
 *  - channels are ordered by cost m n l (2q + 2) (longest first) and dealt
 *    to `lanes` HIP streams, each to the least-loaded lane (LPT schedule);
 *  - the channels of one lane run one after another in one workspace slice
 *    sized for the largest of them; the lanes run concurrently and join the
 *    caller's stream at the end;
 *  - with count > 1 every channel stops after the QR of its projection;
 *    once the lanes have joined, one launch runs the Jacobi sweeps of all
 *    of them (channels in lockstep rounds, widest first, their pairs dealt
 *    over the whole device, one rotation counter per channel and sweep
 *    deciding its convergence), then each channel is finished: values-only
 *    channels (no vectors, no residual) on the caller's stream from compact
 *    slots (about 8 Lp^2 bytes each, Lp = l rounded up to an even multiple
 *    of 16), the others on their lanes in a workspace slice of their own
 *    (lift, signs, residual). Channels with vectors beyond 64 GiB of such
 *    slices run whole in their lane's slice;
 *  - with use_graph != 0 the whole fork / run / join sequence is captured
 *    into a hipGraph on the first call and replayed by later calls with the
 *    same pointers and leading dimensions (a call with other pointers
 *    captures again). If the runtime refuses the capture, the batch runs
 *    eagerly from then on (rsvd_batch_info reports it).
 * Each channel computes exactly what rsvd_run computes for its problem
 * (bitwise: the same kernels on the same data; the grouped sweeps apply each
 * channel's pair steps with the single run's pair kernel in its order).
 */
typedef struct rsvd_batch_s* rsvd_batch_t;

/*
 * rsvd_batch_plan - plan count >= 1 problems (host array, read only). Every
 * problem is validated as by rsvd_plan; adaptive problems are rejected with
 * RSVD_EINVAL (they synchronize). lanes: 1..16 concurrent streams (0 = 4).
 * workspace_bytes receives the device workspace rsvd_batch_run needs.
 * Streams, events and graphs are created on the device that is current at
 * the first rsvd_batch_run and released by rsvd_batch_destroy.
 */
rsvd_status rsvd_batch_plan(const rsvd_problem* probs, int64_t count, int32_t lanes,
                            int32_t use_graph, rsvd_batch_t* out, size_t* workspace_bytes);

/*
 * rsvd_batch_run - run every channel. All pointer arrays are HOST arrays of
 * count entries holding DEVICE pointers (A[c], S[c], U[c], V[c]) and the
 * leading dimensions lda[c], ldu[c], ldv[c], with the meaning of rsvd_run
 * (U / V entries may be NULL where the problem does not want them; ldu / ldv
 * may then be NULL too). res_dev: count device result records. work: device
 * workspace of the planned size, 256-B aligned. Ordered on `stream`: the
 * lanes wait for the work enqueued before and the stream waits for them.
 */
rsvd_status rsvd_batch_run(rsvd_batch_t plan, const double* const* A, const int64_t* lda,
                           double* const* S, double* const* U, const int64_t* ldu,
                           double* const* V, const int64_t* ldv, rsvd_result* res_dev,
                           void* work, size_t work_bytes, void* stream);

/* rsvd_batch_info - host query: lane of channel c (lane_of, count entries,
 * may be NULL), and whether the last run replayed a captured graph. */
rsvd_status rsvd_batch_info(rsvd_batch_t plan, int32_t* lane_of, int32_t* graph_replayed);

/* Free a batch plan with its streams, events and graph (NULL is ignored).
 * Synchronizes the lanes first. */
void rsvd_batch_destroy(rsvd_batch_t plan);

/*
 * rsvd_residual - one decomposition truncated at rank k (section "Randomized
 * matrix decompositions": R_SVD is the number of kept singular values, R%
 * = 100 R_SVD / N, Eq. 2 the compression ratio; the results sweep R% and a
 * decomposition computed at the largest R% serves every smaller one).
 *   A, lda        m x n input (device, read only, lda >= n).
 *   S             at least k singular values (device), U (m x >= k, ldu) and
 *                 V (n x >= k, ldv): a decomposition of A, e.g. rsvd_run's.
 *   k             1 <= k <= min(m, n): the leading k triplets are kept.
 *   res_dev       device rsvd_result: rank = l_used = k, residual =
 *                 ||A - U_k diag(S_k) V_k^T||_F / ||A||_F (one FP64 stream of
 *                 A), rel_percent, c_eq2, c_sym and fro2 as rsvd_run reports
 *                 them for rank k; sweeps, flags and blocks 0, err_est NaN.
 *   work          device workspace of rsvd_residual_work_bytes(m, n, k)
 *                 bytes, 256-byte aligned (RSVD_ENOMEM if smaller).
 * RSVD_EINVAL for k outside 1..min(m, n), lda < n, ldu or ldv < k, null
 * pointers. Enqueued on stream; no host synchronization.
 */
size_t rsvd_residual_work_bytes(int64_t m, int64_t n, int64_t k);
rsvd_status rsvd_residual(int64_t m, int64_t n, int64_t k, const double* A, int64_t lda,
                          const double* S, const double* U, int64_t ldu, const double* V,
                          int64_t ldv, rsvd_result* res_dev, void* work, size_t work_bytes,
                          void* stream);

/*
 * rsvd_factor_transform - basis transformation of a decomposed matrix on its
 * thin factors (section "Low-rank interactions": Vbar = U^dagger V U acts on
 * the thin L and R^dagger alone). For real U: Vbar = (U^T L) Sigma (U^T R)^T,
 * so Lout = U^T L and Rout = U^T R; Sigma is unchanged. Both factors are
 * multiplied in one stream of U (side by side as one N x 2k panel).
 *   Ub, ldub      the basis, N x Nb (device, row-major, ldub >= Nb, Nb <= N);
 *                 orthonormal columns keep Lout, Rout orthonormal (not checked).
 *   L, ldl        N x k (device, ldl >= k); R, ldr N x k or R = NULL (then
 *                 only L is transformed and Rout is not written).
 *   Lout, ldlo    Nb x k output (device, ldlo >= k); Rout, ldro likewise.
 *   work          device workspace of rsvd_factor_transform_work_bytes(N, Nb,
 *                 k, R != NULL) bytes, 256-byte aligned (RSVD_ENOMEM if less).
 * RSVD_EINVAL for N, Nb, k < 1, Nb > N, bad leading dimensions or null
 * pointers. FP64 on the matrix cores; enqueued on stream.
 */
size_t rsvd_factor_transform_work_bytes(int64_t N, int64_t Nb, int64_t k, int32_t with_r);
rsvd_status rsvd_factor_transform(int64_t N, int64_t Nb, int64_t k, const double* Ub, int64_t ldub,
                                  const double* L, int64_t ldl, const double* R, int64_t ldr,
                                  double* Lout, int64_t ldlo, double* Rout, int64_t ldro,
                                  void* work, size_t work_bytes, void* stream);

/*
 * Learned (k, p, q) predictor. The paper fixes R_SVD and the oversampling by
 * hand; here a small MLP maps 16 features of a cheap pilot sketch of a
 * channel to (log10 k, p, q) in standardized units, so the decomposition can
 * be sized without adaptive growth (the caller checks the result and falls
 * back to the adaptive range finder where it fails).
 *
 * Features (rsvd_pilot_features): Y0 = A P0 with P0 the first 32 columns of
 * the Philox / Box-Muller projection keyed by (seed, channel), computed on
 * FP32 matrix cores (operands rounded to FP32, FP32 accumulation); s_i the
 * singular values of Y0 (FP64 QR + Jacobi); f_i = max(log10(s_i / s_1), -16)
 * for i = 1..16 (-16 beyond min(32, m, n) values).
 *
 * Model: h1 = relu(W1 f + b1), h2 = relu(W2 h1 + b2), y = W3 h2 + b3 with
 * W1 64 x 16, W2 64 x 64, W3 3 x 64; parameters are one flat FP32 device
 * array of RSVD_MLP_PARAMS values in the order W1 (row-major), b1, W2, b2,
 * W3, b3, owned by the caller (save / load it as plain floats). Training
 * minimizes the mean of (y - t)^2 over the batch and the 3 outputs with Adam
 * (Kingma and Ba 2015; beta1 0.9, beta2 0.999, eps 1e-8).
 * All arrays are device FP32, row-major: X is B x 16, T and Y are B x 3.
 */
#define RSVD_MLP_PARAMS 5443
#define RSVD_MLP_IN 16
#define RSVD_MLP_OUT 3
#define RSVD_MLP_MAX_BATCH 128
#define RSVD_PILOT_COLS 32

/* He-normal initialization: W ~ N(0, 2 / fan_in) with entry (i, j) of layer
 * L (0, 1, 2) the Philox / Box-Muller draw at counter (i, j / 4, 0, 0), key
 * (seed, L); biases 0. */
rsvd_status rsvd_mlp_init(float* params, uint64_t seed, void* stream);
/* Y = MLP(X) for B >= 0 samples. */
rsvd_status rsvd_mlp_forward(const float* params, const float* X, int64_t B, float* Y,
                             void* stream);
/* Loss (device float, may be NULL) and its gradient (RSVD_MLP_PARAMS device
 * floats, same layout as params) for one batch, 1 <= B <= 128. */
rsvd_status rsvd_mlp_grad(const float* params, const float* X, const float* T, int64_t B,
                          float* grad, float* loss, void* stream);
/* One Adam step (step >= 1 counts the steps taken, for the bias corrections)
 * on one batch, 1 <= B <= 128: params, adam_m and adam_v (RSVD_MLP_PARAMS
 * device floats each, zero before the first step) are updated in place; loss
 * (device float, may be NULL) receives the batch loss before the step. */
rsvd_status rsvd_mlp_train_step(float* params, float* adam_m, float* adam_v, int64_t step,
                                const float* X, const float* T, int64_t B, float lr,
                                float* loss, void* stream);
/* Training targets: labels (B x 3 device int64: k, p, q per sample, k >= 1)
 * -> raw targets (log10 k, p, q) -> per-column mean and standard deviation
 * (population; a zero deviation counts as 1) into stats (6 device floats:
 * mean[3], sd[3]) -> standardized targets T (B x 3 device floats). B >= 1. */
rsvd_status rsvd_mlp_targets(const int64_t* labels, int64_t B, float* stats, float* T,
                             void* stream);
/* Sizing from the network: y = MLP(X) (B x 16 features), raw = y sd + mean
 * (stats as rsvd_mlp_targets writes them), then per sample
 *   k = min(max(ceil(1.05 * 10^raw0), 1), n_cap[b])  (5 % rank margin)
 *   p = the smallest of {8, 16, 32, 48, 64, 96, 128, 160, 192, 256, 320, 384,
 *       448, 512} >= raw1 (else 512)
 *   q = min(max(floor(raw2 + 1/2), 0), 4)    (nearest; a q too small shows in
 *       the judge's UNCONVERGED flag)
 * into kpq (B x 3 device int64). n_cap: B device int64 (min(m, n) of each
 * channel). B >= 0. */
rsvd_status rsvd_mlp_predict(const float* params, const float* stats, const float* X, int64_t B,
                             const int64_t* n_cap, int64_t* kpq, void* stream);
/* Label of one channel from a spectrum the method computed (e.g. the
 * adaptive finder's singular values s, count of them, decreasing, device)
 * with threshold rank k (>= 1) of an n x n channel: the cheapest (p, q) on
 * the grid p in {8, 16, 32, 48, 64, 96, 128, 160, 192, 256, 320, 384, 448,
 * 512}, q in 0..4 whose l = k + p reaches
 * n (an exact SVD), or whose l is at least l_min (the width at which the
 * adaptive finder's posterior estimate passed: the basis covers the tail)
 * and whose kept values are converged, (s[k+p-1] / s[k-1])^(4q+2) <= 1e-8
 * (for k + p > count the last computed value stands in: the ratio only
 * falls beyond it). Cost of a decomposition of width l, in seconds fitted to
 * this library's measured times on MI355X: (2q + 2) (2 n^2 l / 60e12 +
 * 0.44e-3 (l / 272)^1.6) for the products with A and the panel QRs (2q + 1
 * in the power iteration and the QR of the projection) plus
 * 3.2e-3 (l / 272)^1.6 for the small SVD (both latency-bound at these widths).
 * kpq (3 device int64) = (k, p, q); p = q = -1 when no grid point
 * qualifies. */
rsvd_status rsvd_size_label(const double* s, int64_t count, int64_t k, int64_t n, int64_t l_min,
                            int64_t* kpq, void* stream);
/* Save / load the network: a binary file holding the 8-byte tag
 * "RSVDMLP1", the counts 5443 and 6 (uint32 each), the parameters and the
 * stats (FP32). Both synchronize the stream; RSVD_EINVAL for a file that
 * cannot be opened or holds anything else. */
rsvd_status rsvd_mlp_save(const char* path, const float* params, const float* stats,
                          void* stream);
rsvd_status rsvd_mlp_load(const char* path, float* params, float* stats, void* stream);
/* Pilot features of A (m x n, lda, device): feat = 16 device floats. work:
 * device workspace of rsvd_pilot_work_bytes(m, n) bytes, 256-B aligned. */
size_t rsvd_pilot_work_bytes(int64_t m, int64_t n);
rsvd_status rsvd_pilot_features(const double* A, int64_t lda, int64_t m, int64_t n, uint64_t seed,
                                uint64_t channel, float* feat, void* work, size_t work_bytes,
                                void* stream);

/*
 * Component entry points (each one step of the path, for testing and reuse).
 */

/* rsvd_gaussian_omega - the projection P: out (n x l, ldo >= l, device) gets
 * columns col0 .. col0+l-1 of the Philox/Box-Muller stream keyed by
 * (seed, channel) (section "Randomized matrix decompositions": a random
 * projection matrix P drawn once per decomposition). */
rsvd_status rsvd_gaussian_omega(int64_t n, int64_t l, int64_t col0, uint64_t seed,
                                uint64_t channel, double* out, int64_t ldo, void* stream);

/* rsvd_dgemm - C = alpha op(A) B + beta C in FP64 on the matrix cores; the
 * kernel behind the sketch Z = A P, the power products and the projection
 * Q^T A. op(A) = A (m x k, lda) when trans_a == 0, A^T with A stored k x m
 * (lda) when trans_a != 0. B is k x n (ldb), C is m x n (ldc); all device.
 * work (device, may be NULL when work_bytes is 0) holds split-K partial
 * sums; rsvd_dgemm_work_bytes gives the size it wants. */
size_t rsvd_dgemm_work_bytes(int64_t m, int64_t n, int64_t k, int32_t trans_a);
rsvd_status rsvd_dgemm(int32_t trans_a, int64_t m, int64_t n, int64_t k, double alpha,
                       const double* A, int64_t lda, const double* B, int64_t ldb,
                       double beta, double* C, int64_t ldc, void* work, size_t work_bytes,
                       void* stream);

/* rsvd_gemm - the same product with the arithmetic of a precision mode:
 * RSVD_PREC_FP64 (= rsvd_dgemm), RSVD_PREC_MIXED_FP32 (operands rounded to
 * FP32, FP32 matrix cores, FP32 accumulation) or RSVD_PREC_MIXED_BF16
 * (operands rounded to BF16, BF16 matrix cores, FP32 accumulation) or
 * RSVD_PREC_MIXED_BF16_SPLIT (operands split into BF16 hi + lo, three BF16
 * products, FP32 accumulation). Inputs
 * and output stay FP64 in memory; work as for rsvd_dgemm. These are the
 * early products of the precision schedule of the mixed modes.
 * RSVD_PREC_MIXED_FP32_SLICED: the error-free sliced product of that
 * schedule's FP64-accurate passes (the splitting of Ozaki, Ogita, Oishi and
 * Rump with 8-bit integer slices): A and B cut into 7 signed 7-bit slices
 * per entry with one power-of-two scale per row of A and per column of B,
 * the 28 slice products of weight >= 2^-56 computed exactly (INT32, flushed
 * to FP64 every 16384 terms of k) and summed in FP64; each entry of C within
 * about 1e-14 k max_k |a_ik| max_k |b_kj| of the exact product, integer
 * inputs of at most 7 bits reproduced exactly. Only trans_a = 0, alpha = 1,
 * beta = 0 (RSVD_EINVAL otherwise); work: at least
 * rsvd_sliced_gemm_work_bytes(m, n, k) bytes, 256-byte aligned
 * (RSVD_ENOMEM otherwise). */
size_t rsvd_sliced_gemm_work_bytes(int64_t m, int64_t n, int64_t k);
rsvd_status rsvd_gemm(int32_t precision, int32_t trans_a, int64_t m, int64_t n, int64_t k,
                      double alpha, const double* A, int64_t lda, const double* B, int64_t ldb,
                      double beta, double* C, int64_t ldc, void* work, size_t work_bytes,
                      void* stream);

/* rsvd_bf16_gemm - C = op(A) B (m x n, FP64, overwritten) as rsvd_run
 * computes the early products of the BF16 schedules: op(A) (m x k) and B
 * (k x n) are rounded into BF16 planes in the workspace (split != 0: hi =
 * bf16(x) and lo = bf16(x - hi), three products hi*lo + lo*hi + hi*hi per
 * term), multiplied on the BF16 matrix cores with FP32 accumulation, and
 * split-K partial sums are added in FP64. A is m x k (lda), or k x m when
 * trans_a != 0; B is k x n (ldb); C is m x n (ldc); all device, row-major.
 * work: device, 256-byte aligned, at least rsvd_bf16_gemm_work_bytes bytes
 * (RSVD_ENOMEM otherwise). Same error bounds as rsvd_gemm's BF16 modes. */
size_t rsvd_bf16_gemm_work_bytes(int64_t m, int64_t n, int64_t k, int32_t split);
rsvd_status rsvd_bf16_gemm(int32_t split, int32_t trans_a, int64_t m, int64_t n, int64_t k,
                           const double* A, int64_t lda, const double* B, int64_t ldb, double* C,
                           int64_t ldc, void* work, size_t work_bytes, void* stream);

/* rsvd_orth - thin QR of a tall panel Y (m x l, ldy, device, m >= l), step 1's
 * "QR decomposition Z = Q X": Y is overwritten by Q (orthonormal columns,
 * diag(X) > 0); X (l x l upper triangular, row-major, device) receives the
 * R factor when non-NULL. Shifted Cholesky QR (Gram, Cholesky, triangular
 * solve, repeated). flags (device uint32) gets RSVD_FLAG_QR_FALLBACK when
 * the unshifted factorization broke down. */
size_t rsvd_orth_work_bytes(int64_t m, int64_t l);
rsvd_status rsvd_orth(int64_t m, int64_t l, double* Y, int64_t ldy, double* X,
                      uint32_t* flags, void* work, size_t work_bytes, void* stream);

/* rsvd_small_svd - SVD of a square upper-triangular R (l x l, row-major,
 * device), step 2's thin SVD applied to the triangular factor of Y^T:
 * R^T = Us diag(s) W^T. s (l, device) decreasing; Us and W (l x l row-major,
 * device) hold the singular vectors as columns. One-sided Jacobi on the rows
 * of R. sweeps (device int32) receives the sweep count; flags as above. */
size_t rsvd_small_svd_work_bytes(int64_t l);
rsvd_status rsvd_small_svd(int64_t l, const double* R, double* s, double* Us, double* W,
                           int32_t max_sweeps, int32_t* sweeps, uint32_t* flags,
                           void* work, size_t work_bytes, void* stream);

/*
 * Autotuning of the tile shapes of the matrix-core products (the
 * "autotuned tiles" of the batched mode; the paper fixes no tiling).
 *
 * Every product launch (FP64 streaming and small products, the residual
 * pass, the BF16 plane products) picks its tiling from a process-wide table
 * keyed by kernel kind, arithmetic, transposition and (M, N, K), and falls
 * back to a built-in heuristic for keys not in the table. rsvd_tune fills
 * the table for the products of one decomposition: it runs the decomposition
 * once (arguments exactly as rsvd_run) while each launch records itself,
 * replays every recorded key not yet in the table once per candidate tiling
 * (FP64 kernel: 4 or 8 waves per workgroup x K-split counts whose partial
 * sums fit the plan's workspace; residual pass: U diag(s) held in
 * registers (inner size at most 272) or the streaming kernel with 4 or 8
 * waves and narrower column tiles; BF16 plane
 * kernel: 16 or 32 rows per wave x one or two times the fewest column
 * groups x K-split counts), timed with HIP events over `reps` (1..100)
 * launches after one warm-up, keeps the fastest, and runs the
 * decomposition once more, so that S, U, V and *res_dev hold the result of
 * the tuned shapes. Synchronizes `stream`; device-predicated launches (the
 * third Cholesky QR pass) are not timed. Tuned shapes change summation
 * orders only: results stay within the same error bounds. n_tuned (host,
 * may be NULL) receives the number of keys added. One tuning caller at a
 * time; runs on other host threads during tuning see the forced candidate
 * of the key being timed.
 *
 * rsvd_batch_tune does the same for every channel of a batch (arguments as
 * rsvd_batch_run), channel by channel on `stream` in the channel's lane
 * workspace (shapes timed with the device to themselves); the next
 * rsvd_batch_run captures a new graph with the tuned shapes.
 *
 * rsvd_tune_entries copies up to `max` entries of the table (kind[i] =
 * 100 kind + 10 arithmetic + transposed; mnk[3i..3i+2] = M, N, K; cfg[3i..]
 * = the tiling: waves / rows per wave, K splits (residual: column tiles per
 * workgroup, 0 for the widest), column groups (residual: 1 for U diag(s)
 * held in registers, 0 for the streaming kernel)) into host arrays (each
 * may be NULL) and returns the number of entries;
 * rsvd_tune_clear empties the table. rsvd_tune_set pins the tiling of one
 * key (kind 0 FP64 streaming, 1 register-staged, 2 residual, 3 BF16 plane
 * product; arith 0 FP64, 1 FP32, 2 BF16, 3 split BF16; a, b, c as in
 * rsvd_tune_entries): RSVD_EINVAL for values out of range; a launch falls
 * back to its heuristic when the pinned tiling does not fit its scratch.
 */
rsvd_status rsvd_tune(rsvd_plan_t plan, const double* A, int64_t lda, const double* omega,
                      int64_t ldo, double* S, double* U, int64_t ldu, double* V, int64_t ldv,
                      rsvd_result* res_dev, void* work, size_t work_bytes, int32_t reps,
                      int32_t* n_tuned, void* stream);
rsvd_status rsvd_batch_tune(rsvd_batch_t plan, const double* const* A, const int64_t* lda,
                            double* const* S, double* const* U, const int64_t* ldu,
                            double* const* V, const int64_t* ldv, rsvd_result* res_dev,
                            void* work, size_t work_bytes, int32_t reps, int32_t* n_tuned,
                            void* stream);
int64_t rsvd_tune_entries(int64_t max, int32_t* kind, int64_t* mnk, int32_t* cfg);
void rsvd_tune_clear(void);
rsvd_status rsvd_tune_set(int32_t kind, int32_t arith, int32_t trans, int64_t M, int64_t N,
                          int64_t K, int32_t a, int32_t b, int32_t c);

/*
 * Phase trace (measurement aid). When enabled, rsvd_run records a HIP event
 * pair on its stream around every launch group of a phase; the events are
 * kept on the host until collected. Not thread-safe: one tracing caller at a
 * time. Phases:
 *   0 streaming products with A in FP64 (sketch, power iterations, projection)
 *   1 QR of the panels    2 small SVD (Jacobi + ordering)   3 lift + signs
 *   4 residual pass       5 projection P                    6 everything else
 *   7 rounding A into the BF16 planes of the BF16 schedules
 *   8 the BF16 products of those schedules (panel planes, product, partial sums)
 *   9 the FP32 products of the FP32 schedule (operands rounded in registers)
 */
#define RSVD_TRACE_PHASES 10
void rsvd_trace_enable(int32_t on);
/* Synchronize on the recorded events, add their durations per phase into
 * ms[RSVD_TRACE_PHASES] and counts[RSVD_TRACE_PHASES] (host arrays), and
 * clear the record. Returns RSVD_EHIP if an event query fails. */
rsvd_status rsvd_trace_collect(double* ms, int64_t* counts);

#ifdef __cplusplus
}
#endif

#endif /* RSVD_H */
