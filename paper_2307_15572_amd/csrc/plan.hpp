// Plan object behind rsvd_plan_t (internal; shared by the single and
// batched entry points).
#pragma once

#include <stddef.h>
#include <stdint.h>

#include "../../include/rsvd.h"
#include "kernels.hpp"

struct rsvd_plan_s {
  rsvd_problem p;
  int64_t l = 0;        // sketch width
  int64_t kc = 0;       // columns produced: min(k_cap, l)
  int64_t k_fixed = 0;  // resolved fixed rank (fixed / percent rules)
  int mode = 0;
  double param = 0.0;
  // workspace layout (byte offsets, 256-B aligned)
  size_t off_state = 0, off_Y = 0, off_Z = 0, off_T = 0, off_part = 0, off_G = 0;
  size_t off_R1 = 0, off_R1i = 0, off_R2 = 0, off_R2i = 0, off_R3 = 0, off_R3i = 0;
  size_t off_Rt = 0, off_Rtmp = 0, off_M = 0, off_P = 0, off_sig = 0, off_Us = 0, off_W = 0;
  size_t off_Ub = 0, off_Vb = 0, off_US = 0, off_Vt = 0, off_rpart = 0;
  size_t off_Yorig = 0, off_tau = 0;
  // symmetric form: the l x l core B = Q^T A Q (then Q_B of its QR)
  int form = 0;
  // singular vectors (or the residual, which needs them) requested: without
  // them the small SVD does not accumulate its right rotations and the lift,
  // the sign rule and the vector products are skipped
  bool vectors = true;
  size_t off_Bs = 0;
  // grouped small SVD (a batch's values-only channels): with defer_M set, a
  // run stops after the QR of its projection, leaving the padded Jacobi
  // matrix in defer_M and its device state in defer_st and returning
  // kStatusDeferred; the batch runs the sweeps of all such channels in one
  // launch (jacobi_batch) and then finish_deferred
  double* defer_M = nullptr;
  rsvd::DevState* defer_st = nullptr;
  // the same for a channel with its own workspace (vectors wanted): the run
  // stops with the Jacobi matrix (and P) prepared in place and is resumed
  // by resume_deferred in that workspace after the grouped sweeps
  bool defer_inplace = false;
  // a-posteriori judge: r probe columns (P_r, A P_r deflated, Q^T A P_r)
  int post_r = 0;
  size_t off_Op = 0, off_Wp = 0, off_Cp = 0;
  // adaptive range finder: l above is l_max; blocks of blk columns
  bool adaptive = false;
  int64_t blk = 0;
  size_t off_Wb = 0, off_Zb = 0, off_Ob = 0, off_Cb = 0, off_Zc = 0;
  // the small SVD's cooperative grid is capped at 1/coop_share of what the
  // device holds at once (runs sharing the device concurrently set it to
  // their number, so their grids are co-resident together)
  int coop_share = 1;
  // BF16 schedules: planes of A (m x ld_an) and, for a non-symmetric A with
  // a low-precision A^T product, of A^T (n x ld_at); XT planes of the panel
  // (xt_rows x xt_ld); FP32 split-K partials of the BF16 products
  bool bf16 = false, bf16_t = false, bf16_split = false;
  int64_t ld_an = 0, ld_at = 0, xt_rows = 0, xt_ld = 0;
  rsvd::Bf16Shape sh_n, sh_t;
  size_t off_Ah = 0, off_Al = 0, off_Ath = 0, off_Atl = 0, off_XTh = 0, off_XTl = 0;
  size_t off_fpart = 0, fpart_floats = 0;
  // FP32 schedule: the FP32 panel of each low-precision product's operand
  size_t off_Xf = 0;
  // odd sizes: a copy of A with an even leading dimension (odd n; made at
  // the start of a run whose A has odd rows) and of each streamed FP64 panel
  // (odd l), so that the products stream through the LDS-DMA kernel
  size_t off_Apad = 0, off_Xp = 0;
  int64_t ld_apad = 0, ld_xp = 0;
  // error-free sliced schedule: the slices of A (made once per run) and of
  // the panel of each sliced product
  size_t off_sl = 0;
  size_t part_doubles = 0;
  size_t total = 0;
};

// internal status of a run that deferred its small SVD to the batch (never
// returned through the C ABI; within the range of the enumeration's values)
constexpr rsvd_status kStatusDeferred = static_cast<rsvd_status>(7);

// The rest of a deferred run once its sweeps are done: ordering of the
// values (svd_finish on M), rank rule, values to S, the judge and the result
// record, all on st; sig: l doubles, scratch: 2 l doubles.
// The rest of a run deferred in place, in its own workspace, once its sweeps
// are done: ordering, rank rule, the symmetric form's W, lift, signs,
// residual and result record (arguments as for rsvd_run).
rsvd_status resume_deferred(const rsvd_plan_s& pl, const double* A, int64_t lda, double* S,
                            double* U, int64_t ldu, double* V, int64_t ldv, rsvd_result* res_dev,
                            void* work, hipStream_t s);
rsvd_status finish_deferred(const rsvd_plan_s& pl, double* M, rsvd::DevState* st, double* sig,
                            double* scratch, double* S, rsvd_result* res_dev, hipStream_t s);
