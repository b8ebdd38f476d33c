// Host runtime and C ABI of the randomized SVD library (include/rsvd.h).
//
// rsvd_run enqueues, on the caller's stream and without host synchronization,
// the steps of the method (arXiv:2307.15572, section "Randomized matrix
// decompositions", Fig. 1):
//   P          Gaussian projection (Philox4x64-10 + Box-Muller), unless given
//   step 1     Z = A P; thin QR Z = Q X
//   (q times)  Z' = A^T Q -> QR -> Z = A Q' -> QR   (Halko et al. subspace
//              iteration; q = 0 is the paper's method)
//   step 2     Y^T = A^T Q (= Q^T A transposed); Y^T = Q_B X_B (QR);
//              SVD of X_B^T by one-sided Jacobi: X_B^T = L_Y Sigma W^T, so
//              Y = L_Y Sigma (Q_B W)^T and R = Q_B W
//   step 3     L = Q L_Y
//   then       rank rule (R_SVD, R%, Eq. 2), sign rule, optional residual.
// Every decision that depends on data (QR shift, rank) is taken on the
// device, so a run is a fixed sequence of launches.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"
#include "plan.hpp"

using namespace rsvd;

namespace {

// ---- phase trace ------------------------------------------------------------
struct TraceMark {
  int phase;
  hipEvent_t a, b;
};
bool g_trace_on = false;
std::vector<TraceMark> g_marks;
std::vector<hipEvent_t> g_event_pool;

hipEvent_t trace_event() {
  if (!g_event_pool.empty()) {
    hipEvent_t e = g_event_pool.back();
    g_event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// RAII scope: records an event pair around the launches of one phase.
struct PhaseScope {
  int phase;
  hipStream_t s;
  hipEvent_t a = nullptr;
  PhaseScope(int ph, hipStream_t st) : phase(ph), s(st) {
    if (!g_trace_on) return;
    a = trace_event();
    if (a) (void)hipEventRecord(a, s);
  }
  ~PhaseScope() {
    if (!a) return;
    hipEvent_t b = trace_event();
    if (!b) return;
    (void)hipEventRecord(b, s);
    g_marks.push_back({phase, a, b});
  }
};

}  // namespace

namespace {

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Carver {
  size_t at = 0;
  size_t take(size_t bytes) {
    const size_t o = at;
    at = align256(at + bytes);
    return o;
  }
};

int64_t percent_rank(double pct, int64_t m, int64_t n) {
  const double x = pct * (double)(m < n ? m : n) / 100.0;
  return (int64_t)std::ceil(x * (1.0 - 1e-12));
}

// m n from which a transposed streaming product A^T X runs as (X^T A)^T on the
// LDS-DMA kernel (below it the two extra transposes and launches do not pay)
constexpr int64_t kTransStreamMin = (int64_t)1 << 24;
// matrices from this size on get even-leading-dimension copies of A and of
// the streamed panels when their sizes are odd
constexpr int64_t kPadMin = (int64_t)1 << 18;
constexpr int kTransSplits = 8;

// Split-K scratch needed by the products of one run.
size_t gemm_part_need(int64_t m, int64_t n, int64_t l) {
  size_t need = 0;
  auto upd = [&](int64_t M, int64_t N, int64_t K) {
    GemmShape s = dgemm_shape(M, N, K);
    if (s.part_doubles > need) need = s.part_doubles;
  };
  upd(m, l, n);  // A P, A Q
  upd(n, l, m);  // A^T Q
  upd(l, l, m);  // Gram of an m x l panel
  upd(l, l, n);  // Gram of an n x l panel
  upd(m, l, l);  // panel x R^{-1}
  upd(n, l, l);
  upd(l, l, l);
  return need;
}

struct Ws {
  char* base;
  template <class T>
  T* at(size_t off) const { return reinterpret_cast<T*>(base + off); }
};

// Thin QR of the rows x l panel Y (contiguous, ld = l) in place (Y <- Q) by
// Cholesky QR (l <= the plan's l):
//   pass 0  G = Y^T Y, R1 = chol(G), T = Y R1^{-1}. When the pivots of R1
//           spread by more than 1e5 (or the factorization breaks down) the
//           shifted factorization chol(G + s I) is used instead and the
//           panel takes the three-pass route (shifted Cholesky QR3).
//   pass 1  Y = T R2^{-1} with R2 = chol(T^T T)
//   pass 2  only after a shifted pass 0: one more Cholesky QR pass.
// full == false (an intermediate panel of the power iteration, where only
// the span is used next): a well-conditioned panel stops after pass 0, whose
// orthogonality error u kappa^2 <= 1e-6 does not change the span.
// If Rout is non-null it receives the R factor (upper, l x l).
// A panel that is rank deficient even for the shifted passes is refactored
// by Householder QR from a saved copy.
rsvd_status orth(const rsvd_plan_s& pl, const Ws& w, int64_t rows, int64_t l, double* Y,
                 double* Rout, hipStream_t s, bool full = true) {
  DevState* st = w.at<DevState>(pl.off_state);
  double* G = w.at<double>(pl.off_G);
  double* T = w.at<double>(pl.off_T);
  double* part = w.at<double>(pl.off_part);
  double* R1 = w.at<double>(pl.off_R1);
  double* R1i = w.at<double>(pl.off_R1i);
  double* R2 = w.at<double>(pl.off_R2);
  double* R2i = w.at<double>(pl.off_R2i);
  double* R3 = w.at<double>(pl.off_R3);
  double* R3i = w.at<double>(pl.off_R3i);
  double* Yorig = w.at<double>(pl.off_Yorig);
  double* tau = w.at<double>(pl.off_tau);
  double* Rtmp = w.at<double>(pl.off_Rtmp);  // block-row scratch of the factorization
  const uint32_t* shifted = &st->qr_shifted;
  const uint32_t* p1 = full ? nullptr : shifted;  // pass 1 runs always, or only after a shift
  rsvd_status r;
#define RSVD_TRY(x) do { r = (x); if (r != RSVD_OK) return r; } while (0)
  RSVD_TRY(clear_shift(st, s));
  RSVD_TRY(copy_panel(rows, l, Y, l, Yorig, l, 0, st, s));
  // Q = Y R^{-1}: block forward substitution with the diagonal tiles'
  // inverses (the factorization skips the full inverse). Beyond the
  // substitution kernel's width, by column blocks B of at most that width:
  //   Q_B = (Y_B - Q_{<B} R_{<B,B}) R_BB^{-1}
  // (copy, one product with the blocks already solved, substitution in place)
  const bool tri = true;
  auto apply = [&](const double* src, const double* Rf, const double* Ri, double* dst,
                   const uint32_t* pred) -> rsvd_status {
    if (trsm_supported(l)) return trsm_upper(rows, l, src, l, Rf, l, Ri, dst, l, pred, s);
    int64_t wb = 16;
    while (trsm_supported(wb + 16)) wb += 16;  // widest supported multiple of 16
    const int64_t nblk = (l + wb - 1) / wb;
    wb = ((l + nblk - 1) / nblk + 15) / 16 * 16;  // balanced blocks
    for (int64_t cb = 0; cb < l; cb += wb) {
      const int64_t w = l - cb < wb ? l - cb : wb;
      if (cb == 0) {
        RSVD_TRY(trsm_upper(rows, w, src, l, Rf, l, Ri, dst, l, pred, s));
        continue;
      }
      // pred is either absent or the shift word (copy_panel's condition 1)
      RSVD_TRY(copy_panel(rows, w, src + cb, l, dst + cb, l, pred ? 1 : 0, st, s));
      RSVD_TRY(dgemm(false, rows, w, cb, -1.0, dst, l, Rf + cb, l, 1.0, dst + cb, l, part,
                     pl.part_doubles, s, 64, pred));
      RSVD_TRY(trsm_upper(rows, w, dst + cb, l, Rf + cb * l + cb, l, Ri + cb * l + cb, dst + cb, l,
                          pred, s));
    }
    return RSVD_OK;
  };
  // pass 0
  RSVD_TRY(gram(rows, l, Y, l, G, part, pl.part_doubles, nullptr, s));
  RSVD_TRY(chol_inv(l, G, R1, R1i, Rtmp, rows, 0, 0, st, s, pl.coop_share, !tri));
  RSVD_TRY(apply(Y, R1, R1i, T, nullptr));
  // pass 1
  RSVD_TRY(gram(rows, l, T, l, G, part, pl.part_doubles, p1, s));
  RSVD_TRY(chol_inv(l, G, R2, R2i, Rtmp, rows, 1, full ? 0 : 1, st, s, pl.coop_share, !tri));
  RSVD_TRY(apply(T, R2, R2i, Y, p1));
  if (!full) RSVD_TRY(copy_panel(rows, l, T, l, Y, l, 2, st, s));  // unshifted: Q = T
  // pass 2 (device-predicated on the shift), for the bases that must be
  // orthonormal to working accuracy; an intermediate basis after a shifted
  // pass and one unshifted pass is orthonormal to about u kappa(T)^2 with
  // kappa(T) <= 1 / sqrt(shift / ||G||) (~1e4 here), which carries its span
  // to the next product unchanged
  if (full) {
    RSVD_TRY(gram(rows, l, Y, l, G, part, pl.part_doubles, shifted, s));
    RSVD_TRY(chol_inv(l, G, R3, R3i, Rtmp, rows, 2, 1, st, s, pl.coop_share, !tri));
    RSVD_TRY(apply(Y, R3, R3i, T, shifted));
    RSVD_TRY(copy_panel(rows, l, T, l, Y, l, 1, st, s));
  }
  if (Rout && full) {
    // R = R2 R1, then R3 R when shifted
    RSVD_TRY(dgemm(false, l, l, l, 1.0, R2, l, R1, l, 0.0, Rout, l, part, pl.part_doubles, s));
    RSVD_TRY(dgemm(false, l, l, l, 1.0, R3, l, Rout, l, 0.0, Rtmp, l, part, pl.part_doubles, s, 64, shifted));
    RSVD_TRY(copy_panel(l, l, Rtmp, l, Rout, l, 1, st, s));
  }
  // rank-deficient panel: Householder QR of the saved original
  // (Rtmp is free again: its last use, the product R3 R, is done)
  RSVD_TRY(householder_fallback(rows, l, Yorig, Y, Rout, tau, Rtmp, st, s, pl.coop_share));
  return RSVD_OK;
#undef RSVD_TRY
}

}  // namespace

extern "C" {

const char* rsvd_strerror(rsvd_status s) {
  switch (s) {
    case RSVD_OK: return "ok";
    case RSVD_EINVAL: return "invalid argument";
    case RSVD_ENOMEM: return "workspace too small";
    case RSVD_EHIP: return "HIP runtime error";
    case RSVD_EUNSUPPORTED: return "unsupported request";
  }
  return "unknown status";
}

rsvd_status rsvd_plan(const rsvd_problem* prob, rsvd_plan_t* out, size_t* workspace_bytes) {
  if (!prob || !out) return RSVD_EINVAL;
  const rsvd_problem& p = *prob;
  if (p.m < 1 || p.n < 1 || p.oversample < 0 || p.power_iters < 0) return RSVD_EINVAL;
  if (p.symmetric && p.m != p.n) return RSVD_EINVAL;
  if (p.precision < RSVD_PREC_FP64 || p.precision > RSVD_PREC_MIXED_FP32_SLICED) return RSVD_EINVAL;
  if (p.trailing_hp < 0) return RSVD_EINVAL;
  if (p.posterior < 0 || p.posterior > 64) return RSVD_EINVAL;
  if (p.posterior != 0 && p.adaptive) return RSVD_EINVAL;
  if (p.form != RSVD_FORM_SVD && p.form != RSVD_FORM_SYMMETRIC) return RSVD_EINVAL;
  if (p.form == RSVD_FORM_SYMMETRIC && !p.symmetric) return RSVD_EINVAL;
  const bool adaptive = p.adaptive != 0;
  if (adaptive && p.form == RSVD_FORM_SYMMETRIC) return RSVD_EUNSUPPORTED;
  int64_t k = p.k;
  int mode = p.rank_mode;
  double param = p.rank_param;
  switch (mode) {
    case RSVD_RANK_FIXED:
      if (adaptive || k < 1) return RSVD_EINVAL;
      param = (double)k;
      break;
    case RSVD_RANK_PERCENT:
      if (adaptive) return RSVD_EINVAL;
      if (!(p.rank_param > 0.0 && p.rank_param <= 100.0)) return RSVD_EINVAL;
      k = percent_rank(p.rank_param, p.m, p.n);
      mode = RSVD_RANK_FIXED;
      param = (double)k;
      break;
    case RSVD_RANK_REL_THRESHOLD:
    case RSVD_RANK_FROB_TAIL:
      if (!(p.rank_param > 0.0 && p.rank_param < 1.0)) return RSVD_EINVAL;
      if (!adaptive && k < 1) return RSVD_EINVAL;
      break;
    default:
      return RSVD_EINVAL;
  }
  const int64_t mn = p.m < p.n ? p.m : p.n;
  int64_t l = 0, blk = 0;
  if (adaptive) {
    if (p.block < 0 || p.block > 256 || p.l_max < 0) return RSVD_EINVAL;
    if (p.precision != RSVD_PREC_FP64) return RSVD_EUNSUPPORTED;
    blk = p.block > 0 ? p.block : 64;
    l = p.l_max > 0 ? p.l_max : 4096;
    if (l > mn) l = mn;
  } else {
    l = k + p.oversample;
    if (l > mn) l = mn;
  }
  if (l > 4096) return RSVD_EUNSUPPORTED;
  int64_t kcap = p.k_cap > 0 ? p.k_cap : l;
  if (mode == RSVD_RANK_FIXED && kcap < (k < l ? k : l)) return RSVD_EINVAL;
  rsvd_plan_s* pl = new (std::nothrow) rsvd_plan_s();
  if (!pl) return RSVD_ENOMEM;
  pl->p = p;
  pl->l = l;
  pl->kc = kcap < l ? kcap : l;
  pl->k_fixed = k;
  pl->mode = mode;
  pl->param = param;
  pl->adaptive = adaptive;
  pl->blk = blk;
  pl->form = p.form;
  pl->vectors = p.want_u || p.want_v || p.want_residual;
  pl->post_r = p.posterior;
  const int64_t m = p.m, n = p.n, kc = pl->kc;
  const int64_t mx = m > n ? m : n;
  const size_t D = sizeof(double);
  Carver c;
  pl->off_state = c.take(sizeof(DevState));
  pl->off_Y = c.take((size_t)m * l * D);
  pl->off_Z = c.take((size_t)n * l * D);
  pl->off_T = c.take((size_t)mx * l * D);
  pl->off_Yorig = c.take((size_t)mx * l * D);
  pl->off_tau = c.take((size_t)2 * l * D);
  if (!adaptive && m * n >= kPadMin) {
    // 16-byte rows for the streaming kernel (copies cost one pass over A per
    // run, one over the panel per product)
    if (n & 1) {
      pl->ld_apad = n + 1;
      pl->off_Apad = c.take((size_t)m * pl->ld_apad * D);
    }
    if (l & 1) {
      pl->ld_xp = l + 1;
      pl->off_Xp = c.take((size_t)mx * pl->ld_xp * D);
    }
  }
  pl->part_doubles = gemm_part_need(m, n, l);
  if (!p.symmetric && !adaptive && m * n >= kTransStreamMin) {
    // A^T X as (X^T A)^T: its l output rows make few tiles; room for up to
    // kTransSplits K splits so that the tuner can fill the device
    const size_t need = (size_t)kTransSplits * l * n;
    if (need > pl->part_doubles) pl->part_doubles = need;
  }
  if (adaptive) {
    auto upd = [&](int64_t M, int64_t N, int64_t K) {
      const size_t need = dgemm_shape(M, N, K).part_doubles;
      if (need > pl->part_doubles) pl->part_doubles = need;
    };
    upd(m, blk, n);  // A P_blk, A Q_b
    upd(n, blk, m);  // A^T Q_b
    upd(l, blk, m);  // Q^T W
    upd(m, blk, l);  // Q (Q^T W)
    upd(blk, blk, m);
    upd(blk, blk, n);
    upd(m, blk, blk);
    upd(n, blk, blk);
    if (pl->part_doubles < (size_t)512 * 256) pl->part_doubles = (size_t)512 * 256;  // column norms
  }
  if (pl->post_r) {
    const int64_t r = pl->post_r;
    auto upd = [&](int64_t M, int64_t N, int64_t K) {
      const size_t need = dgemm_shape(M, N, K).part_doubles;
      if (need > pl->part_doubles) pl->part_doubles = need;
    };
    upd(m, r, n);  // A P_r
    upd(l, r, m);  // Q^T W
    upd(m, r, l);  // Q (Q^T W)
    pl->off_Op = c.take((size_t)n * r * D);
    pl->off_Wp = c.take((size_t)m * r * D);
    pl->off_Cp = c.take((size_t)l * r * D);
  }
  if (pl->part_doubles < 2048) pl->part_doubles = 2048;
  pl->off_part = c.take(pl->part_doubles * D);
  const size_t ll = (size_t)l * l * D;
  pl->off_G = c.take(ll);
  pl->off_R1 = c.take(ll);
  pl->off_R1i = c.take(ll);
  pl->off_R2 = c.take(ll);
  pl->off_R2i = c.take(ll);
  pl->off_R3 = c.take(ll);
  pl->off_R3i = c.take(ll);
  pl->off_Rt = c.take(ll);
  pl->off_Rtmp = c.take(ll);
  const int64_t Lp = jacobi_padded(l);
  pl->off_M = c.take((size_t)Lp * Lp * D);
  pl->off_P = c.take((size_t)Lp * Lp * D);
  pl->off_sig = c.take((size_t)l * D);
  if (p.form == RSVD_FORM_SYMMETRIC) pl->off_Bs = c.take(ll);
  pl->off_Us = c.take((size_t)l * kc * D);
  pl->off_W = c.take((size_t)l * kc * D);
  pl->off_Ub = c.take((size_t)m * kc * D);
  pl->off_Vb = c.take((size_t)n * kc * D);
  if (p.want_residual) {
    const int64_t kcp = (kc + 15) / 16 * 16;
    pl->off_US = c.take((size_t)m * kcp * D);
    pl->off_Vt = c.take((size_t)n * kcp * D);
    pl->off_rpart = c.take(resid_partials(m, n) * D);
  }
  // BF16 schedules: planes for the low-precision products
  const int n_low = 2 * p.power_iters + 1 - p.trailing_hp;
  if (!adaptive && n_low > 0 &&
      (p.precision == RSVD_PREC_MIXED_BF16 || p.precision == RSVD_PREC_MIXED_BF16_SPLIT)) {
    const size_t H = sizeof(uint16_t);
    const int planes = p.precision == RSVD_PREC_MIXED_BF16_SPLIT ? 2 : 1;
    pl->bf16 = true;
    pl->bf16_split = planes == 2;
    pl->bf16_t = !p.symmetric && n_low >= 2;  // products 1, 3, .. are A^T ones
    pl->ld_an = bf16_pad(n);
    pl->sh_n = bf16_shape(m, l, n, planes == 2);
    size_t fpart = bf16_part_floats_max(m, l);
    pl->xt_ld = pl->ld_an;
    pl->off_Ah = c.take((size_t)m * pl->ld_an * H);
    if (planes == 2) pl->off_Al = c.take((size_t)m * pl->ld_an * H);
    if (pl->bf16_t) {
      pl->ld_at = bf16_pad(m);
      pl->sh_t = bf16_shape(n, l, m, planes == 2);
      const size_t f2 = bf16_part_floats_max(n, l);
      if (f2 > fpart) fpart = f2;
      if (pl->ld_at > pl->xt_ld) pl->xt_ld = pl->ld_at;
      pl->off_Ath = c.take((size_t)n * pl->ld_at * H);
      if (planes == 2) pl->off_Atl = c.take((size_t)n * pl->ld_at * H);
    }
    pl->xt_rows = bf16_xt_rows_max(l);
    pl->off_XTh = c.take((size_t)pl->xt_rows * pl->xt_ld * H);
    if (planes == 2) pl->off_XTl = c.take((size_t)pl->xt_rows * pl->xt_ld * H);
    pl->fpart_floats = fpart;
    if (fpart) pl->off_fpart = c.take(fpart * sizeof(float));
  }
  if (!adaptive && n_low > 0 &&
      (p.precision == RSVD_PREC_MIXED_FP32 || p.precision == RSVD_PREC_MIXED_FP32_SLICED))
    pl->off_Xf = c.take((size_t)mx * f32_panel_ld(l) * sizeof(float));
  if (!adaptive && p.precision == RSVD_PREC_MIXED_FP32_SLICED)
    pl->off_sl = c.take(sliced_work_bytes(m, l, n));
  if (adaptive) {
    pl->off_Wb = c.take((size_t)m * blk * D);
    pl->off_Zb = c.take((size_t)n * blk * D);
    pl->off_Ob = c.take((size_t)n * blk * D);
    pl->off_Cb = c.take((size_t)l * blk * D);
    pl->off_Zc = c.take((size_t)n * l * D);
  }
  pl->total = c.at;
  *out = pl;
  if (workspace_bytes) *workspace_bytes = pl->total;
  return RSVD_OK;
}

int64_t rsvd_plan_l(rsvd_plan_t plan) { return plan ? plan->l : -1; }

void rsvd_destroy(rsvd_plan_t plan) { delete plan; }

}  // extern "C"

namespace {

#define RSVD_TRY(x) do { rsvd_status r_ = (x); if (r_ != RSVD_OK) return r_; } while (0)

// Output buffers of one run (caller's U / V, or workspace stand-ins).
struct Outs {
  double* S;
  double* U;
  int64_t ldu;
  double* V;
  int64_t ldv;
};

// The rest of step 2 once the Jacobi sweeps are done: the values ordered
// decreasingly (with the vectors when wanted), then the rank rule.
rsvd_status small_svd_tail(const rsvd_plan_s& pl, const Ws& w, int64_t l, hipStream_t s) {
  const rsvd_problem& p = pl.p;
  DevState* st = w.at<DevState>(pl.off_state);
  const int64_t kcl = pl.kc < l ? pl.kc : l;
  {
    PhaseScope ph(2, s);
    double* P = pl.vectors ? w.at<double>(pl.off_P) : nullptr;
    // the Householder fallback's tau (2 l doubles) is free again: ordering scratch
    RSVD_TRY(svd_finish(l, pl.vectors ? kcl : 0, w.at<double>(pl.off_M), P, jacobi_padded(l),
                        w.at<double>(pl.off_sig), w.at<double>(pl.off_Us), w.at<double>(pl.off_W),
                        w.at<double>(pl.off_tau), st, s));
  }
  // the l - p cap protects unconverged trailing values; an exact SVD
  // (l = min(m, n)) has none
  const int64_t p_cap = l == (p.m < p.n ? p.m : p.n) ? 0 : p.oversample;
  return select_rank(l, p_cap, kcl, pl.mode, pl.param, w.at<double>(pl.off_sig), st, s);
}

// Step 2 on a basis of width l whose transposed projection Y^T = A^T Q
// (n x l, contiguous) is in Zc: Y^T = Q_B X_B (Zc <- Q_B), SVD of X_B^T by
// one-sided Jacobi, singular values ordered decreasingly, then the rank rule.
// rows: the rows of the panel Zc (n, or l for the symmetric form's l x l core).
rsvd_status small_svd_and_rank(const rsvd_plan_s& pl, const Ws& w, int64_t l, double* Zc,
                               hipStream_t s, int64_t rows = -1) {
  const rsvd_problem& p = pl.p;
  DevState* st = w.at<DevState>(pl.off_state);
  double* Rt = w.at<double>(pl.off_Rt);
  const int64_t kcl = pl.kc < l ? pl.kc : l;
  {
    PhaseScope ph(1, s);
    RSVD_TRY(orth(pl, w, rows < 0 ? p.n : rows, l, Zc, Rt, s, true));
  }
  // values only: no right rotations (P) and no vectors gathered
  double* P = pl.vectors ? w.at<double>(pl.off_P) : nullptr;
  if (pl.defer_inplace) {
    // grouped small SVD, the run resumed later in this workspace
    RSVD_TRY(jacobi_prepare(l, Rt, w.at<double>(pl.off_M), P, st, s));
    return kStatusDeferred;
  }
  if (pl.defer_M) {
    // grouped small SVD: the Jacobi matrix and the state go to the batch
    RSVD_TRY(jacobi_prepare(l, Rt, pl.defer_M, nullptr, st, s));
    if (hipMemcpyAsync(pl.defer_st, st, sizeof(DevState), hipMemcpyDeviceToDevice, s) !=
        hipSuccess)
      return RSVD_EHIP;
    return kStatusDeferred;
  }
  {
    PhaseScope ph(2, s);
    RSVD_TRY(block_jacobi(l, Rt, w.at<double>(pl.off_M), P, p.max_sweeps > 0 ? p.max_sweeps : 30,
                          1, st, s, pl.coop_share));
  }
  return small_svd_tail(pl, w, l, s);
}

// Step 3 and the outputs: L = Q L_Y (Q: m x l, ldq), R = Q_B W (Q_B = Zc),
// sign rule, S, optional residual pass, result record.
rsvd_status lift_and_finish(const rsvd_plan_s& pl, const Ws& w, const double* A, int64_t lda,
                            int64_t l, const double* Q, int64_t ldq, const double* Zc,
                            const Outs& o, double err_est, int blocks, rsvd_result* res_dev,
                            hipStream_t s) {
  const rsvd_problem& p = pl.p;
  const int64_t m = p.m, n = p.n;
  const int64_t kcl = pl.kc < l ? pl.kc : l;
  DevState* st = w.at<DevState>(pl.off_state);
  double* part = w.at<double>(pl.off_part);
  const double* sig = w.at<double>(pl.off_sig);
  if (pl.vectors) {
    PhaseScope ph(3, s);
    RSVD_TRY(dgemm(false, m, kcl, l, 1.0, Q, ldq, w.at<double>(pl.off_Us), kcl, 0.0, o.U, o.ldu,
                   part, pl.part_doubles, s));
    RSVD_TRY(dgemm(false, n, kcl, l, 1.0, Zc, l, w.at<double>(pl.off_W), kcl, 0.0, o.V, o.ldv,
                   part, pl.part_doubles, s));
    // the Householder fallback's tau (2 l doubles) is free by now
    RSVD_TRY(sign_fix(m, n, kcl, o.U, o.ldu, o.V, o.ldv, w.at<double>(pl.off_tau), s));
  }
  if (hipMemcpyAsync(o.S, sig, (size_t)kcl * sizeof(double), hipMemcpyDeviceToDevice, s) !=
      hipSuccess)
    return RSVD_EHIP;
  if (p.want_residual) {
    PhaseScope ph(4, s);
    double* US = w.at<double>(pl.off_US);
    double* Vt = w.at<double>(pl.off_Vt);
    // inner size: the rank, padded to 16 with zero columns / rows (under the
    // fixed rule the rank is known here: k within [1, kcl]; otherwise up to kcl)
    int64_t kres = kcl;
    if (pl.mode == RSVD_RANK_FIXED) kres = pl.k_fixed < 1 ? 1 : (pl.k_fixed < kcl ? pl.k_fixed : kcl);
    const int64_t kcp = (kres + 15) / 16 * 16;
    RSVD_TRY(resid_prep(m, n, kcl, kcp, o.U, o.ldu, sig, o.V, o.ldv, US, Vt, st, s));
    RSVD_TRY(resid(m, n, kcp, US, kcp, Vt, n, A, lda, w.at<double>(pl.off_rpart), st, s));
  }
  if (pl.post_r) {
    RSVD_TRY(judge(l, m < n ? m : n, p.power_iters, pl.mode, pl.param, sig, st, s));
    return finalize(m, n, l, p.want_residual, err_est, blocks, st, res_dev, s, true);
  }
  return finalize(m, n, l, p.want_residual, err_est, blocks, st, res_dev, s);
}

// Step 3 of a fixed-width run after its small SVD: for the symmetric form
// first R_small = Q_b W; then L = Q L_Y, R = Q_B W and the outputs.
rsvd_status run_tail(const rsvd_plan_s& pl, const Ws& w, const double* A, int64_t lda,
                     const Outs& o, rsvd_result* res_dev, hipStream_t s) {
  const int64_t l = pl.l;
  double* Y = w.at<double>(pl.off_Y);
  if (pl.form == RSVD_FORM_SYMMETRIC) {
    const int64_t kcl = pl.kc < l ? pl.kc : l;
    double* Wv = w.at<double>(pl.off_W);
    double* Rtmp = w.at<double>(pl.off_Rtmp);
    if (pl.vectors) {
      PhaseScope ph(3, s);
      RSVD_TRY(dgemm(false, l, kcl, l, 1.0, w.at<double>(pl.off_Bs), l, Wv, kcl, 0.0, Rtmp, kcl,
                     w.at<double>(pl.off_part), pl.part_doubles, s));
      RSVD_TRY(copy_panel(l, kcl, Rtmp, kcl, Wv, kcl, 0, w.at<DevState>(pl.off_state), s));
    }
    return lift_and_finish(pl, w, A, lda, l, Y, l, Y, o, __builtin_nan(""), 0, res_dev, s);
  }
  return lift_and_finish(pl, w, A, lda, l, Y, l, w.at<double>(pl.off_Z), o, __builtin_nan(""), 0,
                         res_dev, s);
}

// Output buffers of a run: the caller's U / V, or workspace stand-ins.
Outs make_outs(const rsvd_plan_s& pl, const Ws& w, double* S, double* U, int64_t ldu, double* V,
               int64_t ldv) {
  const rsvd_problem& p = pl.p;
  Outs o;
  o.S = S;
  o.U = p.want_u ? U : w.at<double>(pl.off_Ub);
  o.ldu = p.want_u ? ldu : pl.kc;
  o.V = p.want_v ? V : w.at<double>(pl.off_Vb);
  o.ldv = p.want_v ? ldv : pl.kc;
  return o;
}

}  // namespace

rsvd_status resume_deferred(const rsvd_plan_s& pl, const double* A, int64_t lda, double* S,
                            double* U, int64_t ldu, double* V, int64_t ldv, rsvd_result* res_dev,
                            void* work, hipStream_t s) {
  Ws w{(char*)work};
  const Outs o = make_outs(pl, w, S, U, ldu, V, ldv);
  RSVD_TRY(jacobi_check_done(w.at<DevState>(pl.off_state), s));
  RSVD_TRY(small_svd_tail(pl, w, pl.l, s));
  return run_tail(pl, w, A, lda, o, res_dev, s);
}

rsvd_status finish_deferred(const rsvd_plan_s& pl, double* M, DevState* st, double* sig,
                            double* scratch, double* S, rsvd_result* res_dev, hipStream_t s) {
  const rsvd_problem& p = pl.p;
  const int64_t m = p.m, n = p.n, l = pl.l;
  const int64_t kcl = pl.kc < l ? pl.kc : l;
  RSVD_TRY(jacobi_check_done(st, s));
  RSVD_TRY(svd_finish(l, 0, M, nullptr, jacobi_padded(l), sig, nullptr, nullptr, scratch, st, s));
  const int64_t p_cap = l == (m < n ? m : n) ? 0 : p.oversample;
  RSVD_TRY(select_rank(l, p_cap, kcl, pl.mode, pl.param, sig, st, s));
  if (hipMemcpyAsync(S, sig, (size_t)kcl * sizeof(double), hipMemcpyDeviceToDevice, s) !=
      hipSuccess)
    return RSVD_EHIP;
  if (pl.post_r) {
    RSVD_TRY(judge(l, m < n ? m : n, p.power_iters, pl.mode, pl.param, sig, st, s));
    return finalize(m, n, l, 0, __builtin_nan(""), 0, st, res_dev, s, true);
  }
  return finalize(m, n, l, 0, __builtin_nan(""), 0, st, res_dev, s);
}

namespace {

// The adaptive range finder (header: "Adaptive range finder").
rsvd_status run_adaptive(const rsvd_plan_s& pl, const Ws& w, const double* A, int64_t lda,
                         const Outs& o, rsvd_result* res_dev, hipStream_t s) {
  const rsvd_problem& p = pl.p;
  const int64_t m = p.m, n = p.n, lmax = pl.l, b = pl.blk, mn = m < n ? m : n;
  const int64_t over = p.oversample;
  const double tau = pl.param;
  const bool frob = pl.mode == RSVD_RANK_FROB_TAIL;
  DevState* st = w.at<DevState>(pl.off_state);
  double* Q = w.at<double>(pl.off_Y);    // m x lmax, ld lmax
  double* Bt = w.at<double>(pl.off_Z);   // n x lmax, ld lmax: (Q^T A)^T
  double* Wb = w.at<double>(pl.off_Wb);  // m x b
  double* Zb = w.at<double>(pl.off_Zb);  // n x b
  double* Ob = w.at<double>(pl.off_Ob);  // n x b
  double* Cb = w.at<double>(pl.off_Cb);  // lmax x b
  double* Zc = w.at<double>(pl.off_Zc);  // n x lmax contiguous
  double* part = w.at<double>(pl.off_part);
  const size_t pd = pl.part_doubles;
  DevState hs;
  auto sync_state = [&]() -> rsvd_status {
    if (hipMemcpyAsync(&hs, st, sizeof(DevState), hipMemcpyDeviceToHost, s) != hipSuccess)
      return RSVD_EHIP;
    if (hipStreamSynchronize(s) != hipSuccess) return RSVD_EHIP;
    return RSVD_OK;
  };
  int64_t l = 0;
  // X (rows m, width bi, contiguous) <- (I - Q Q^T) X
  auto deflate = [&](double* X, int64_t bi) -> rsvd_status {
    if (l == 0) return RSVD_OK;
    RSVD_TRY(dgemm(true, l, bi, m, 1.0, Q, lmax, X, bi, 0.0, Cb, bi, part, pd, s));
    return dgemm(false, m, bi, l, -1.0, Q, lmax, Cb, bi, 1.0, X, bi, part, pd, s);
  };
  // X <- orthonormal basis of X, orthogonal to Q (orth, deflate, orth)
  auto orth_against = [&](double* X, int64_t bi) -> rsvd_status {
    PhaseScope ph(1, s);
    RSVD_TRY(orth(pl, w, m, bi, X, nullptr, s, true));
    RSVD_TRY(deflate(X, bi));
    return orth(pl, w, m, bi, X, nullptr, s, true);
  };
  // steps 2: small SVD of the current projection; returns whether the rule
  // keeps at most l - p values
  auto try_finish = [&](bool* ok) -> rsvd_status {
    RSVD_TRY(clear_flags(st, RSVD_FLAG_RANK_CAPPED | RSVD_FLAG_JACOBI_MAXSWEEP, 0u, s));
    RSVD_TRY(copy_panel(n, l, Bt, lmax, Zc, l, 0, st, s));
    RSVD_TRY(small_svd_and_rank(pl, w, l, Zc, s));
    RSVD_TRY(sync_state());
    *ok = hs.rank_wanted <= l - over;
    return RSVD_OK;
  };

  RSVD_TRY(init_state(st, 0u, s));
  if (frob) {
    PhaseScope ph(6, s);
    RSVD_TRY(sumsq(m, n, A, lda, part, st, s));
  }
  double est = __builtin_nan("");
  int blocks = 0;
  bool done = false;
  while (!done) {
    const int64_t bi = b < lmax - l ? b : lmax - l;
    if (bi <= 0) {
      RSVD_TRY(clear_flags(st, 0u, RSVD_FLAG_ADAPT_LIMIT, s));
      bool ok = false;
      RSVD_TRY(try_finish(&ok));
      break;
    }
    {
      PhaseScope ph(5, s);
      RSVD_TRY(gaussian_omega(n, bi, l, p.seed, p.channel, Ob, bi, s));
    }
    {
      PhaseScope ph(0, s);
      RSVD_TRY(dgemm(false, m, bi, n, 1.0, A, lda, Ob, bi, 0.0, Wb, bi, part, pd, s));
    }
    if (l == 0) {
      RSVD_TRY(check_finite(m, bi, Wb, bi, st, s));
      RSVD_TRY(sync_state());
      if (hs.flags & RSVD_FLAG_NONFINITE_INPUT) {
        // nothing meaningful to grow: report the flag with an empty result
        return finalize(m, n, 0, p.want_residual, est, blocks, st, res_dev, s);
      }
    }
    RSVD_TRY(deflate(Wb, bi));
    if (!frob && l > 0) {
      RSVD_TRY(colsumsq(m, (int)bi, Wb, bi, part, pd, 0, st, s));
      RSVD_TRY(sync_state());
      est = kPosteriorFactor * std::sqrt(hs.est2);
      if (est <= tau * std::sqrt(hs.s1lb2)) {
        bool ok = false;
        RSVD_TRY(try_finish(&ok));
        if (ok) break;
      }
    }
    RSVD_TRY(orth_against(Wb, bi));
    for (int t = 0; t < p.power_iters; t++) {
      {
        PhaseScope ph(0, s);
        RSVD_TRY(dgemm(!p.symmetric, n, bi, m, 1.0, A, lda, Wb, bi, 0.0, Zb, bi, part, pd, s));
      }
      {
        PhaseScope ph(1, s);
        RSVD_TRY(orth(pl, w, n, bi, Zb, nullptr, s, false));
      }
      {
        PhaseScope ph(0, s);
        RSVD_TRY(dgemm(false, m, bi, n, 1.0, A, lda, Zb, bi, 0.0, Wb, bi, part, pd, s));
      }
      RSVD_TRY(deflate(Wb, bi));
      RSVD_TRY(orth_against(Wb, bi));
    }
    {
      PhaseScope ph(0, s);
      RSVD_TRY(dgemm(!p.symmetric, n, bi, m, 1.0, A, lda, Wb, bi, 0.0, Bt + l, lmax, part, pd, s));
    }
    RSVD_TRY(copy_panel(m, bi, Wb, bi, Q + l, lmax, 0, st, s));
    RSVD_TRY(colsumsq(n, (int)bi, Bt + l, lmax, part, pd, 1, st, s));
    l += bi;
    blocks++;
    if (frob) {
      RSVD_TRY(sync_state());
      const double miss = hs.fro2 - hs.froY2;
      est = std::sqrt(miss > 0.0 ? miss : 0.0);
      if (est <= tau * std::sqrt(hs.fro2)) {
        bool ok = false;
        RSVD_TRY(try_finish(&ok));
        if (ok) break;
      }
    }
  }
  if (l == mn) RSVD_TRY(clear_flags(st, 0u, RSVD_FLAG_FULL_SVD, s));
  return lift_and_finish(pl, w, A, lda, l, Q, lmax, Zc, o, est, blocks, res_dev, s);
}

}  // namespace

extern "C" {

rsvd_status rsvd_run(rsvd_plan_t plan, const double* A, int64_t lda, const double* omega,
                     int64_t ldo, double* S, double* U, int64_t ldu, double* V, int64_t ldv,
                     rsvd_result* res_dev, void* work, size_t work_bytes, void* stream) {
  if (!plan || !A || !S || !res_dev || !work) return RSVD_EINVAL;
  const rsvd_plan_s& pl = *plan;
  const rsvd_problem& p = pl.p;
  const int64_t m = p.m, n = p.n, l = pl.l, kc = pl.kc;
  if (lda < n) return RSVD_EINVAL;
  if (omega && (pl.adaptive || ldo < l)) return RSVD_EINVAL;
  if (p.want_u && (!U || ldu < kc)) return RSVD_EINVAL;
  if (p.want_v && (!V || ldv < kc)) return RSVD_EINVAL;
  if (work_bytes < pl.total) return RSVD_ENOMEM;
  if (((uintptr_t)work & 255) != 0) return RSVD_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  Ws w{(char*)work};
  const Outs o = make_outs(pl, w, S, U, ldu, V, ldv);
  if (pl.adaptive) return run_adaptive(pl, w, A, lda, o, res_dev, s);

  DevState* st = w.at<DevState>(pl.off_state);
  double* Y = w.at<double>(pl.off_Y);
  double* Z = w.at<double>(pl.off_Z);
  double* part = w.at<double>(pl.off_part);
  const int64_t mn = m < n ? m : n;
  RSVD_TRY(init_state(st, l == mn ? RSVD_FLAG_FULL_SVD : 0u, s));
  if (pl.off_Apad && (lda % 2 != 0 || ((uintptr_t)A & 15) != 0)) {
    // rows of A that the streaming kernel cannot copy whole: the run reads a
    // copy with an even leading dimension instead
    double* Ap = w.at<double>(pl.off_Apad);
    RSVD_TRY(copy_panel(m, n, A, lda, Ap, pl.ld_apad, 0, st, s));
    A = Ap;
    lda = pl.ld_apad;
  }
  if (pl.mode == RSVD_RANK_FROB_TAIL) {
    PhaseScope ph(6, s);
    RSVD_TRY(sumsq(m, n, A, lda, part, st, s));
  }

  // step 1: Z = A P and its orthonormal basis
  const double* Om = omega;
  int64_t ldom = ldo;
  if (!Om) {
    PhaseScope ph(5, s);
    RSVD_TRY(gaussian_omega(n, l, 0, p.seed, p.channel, Z, l, s));
    Om = Z;
    ldom = l;
  }
  // precision schedule: of the 2q + 1 products before the projection, all but
  // the last trailing_hp use the low-precision matrix cores in mixed modes;
  // the projection, QR, small SVD and residual are always FP64
  const int n_early = 2 * p.power_iters + 1;
  const int lowp = p.precision == RSVD_PREC_MIXED_FP32 ||
                           p.precision == RSVD_PREC_MIXED_FP32_SLICED
                       ? kPrecF32
                   : p.precision == RSVD_PREC_MIXED_BF16       ? kPrecBF16
                   : p.precision == RSVD_PREC_MIXED_BF16_SPLIT ? kPrecBF16S
                                                               : kPrecF64;
  bool a_sliced = false;  // the slices of A, made by the first sliced product
  int product = 0;
  uint16_t* Ah = pl.bf16 ? w.at<uint16_t>(pl.off_Ah) : nullptr;
  uint16_t* Al = pl.bf16_split ? w.at<uint16_t>(pl.off_Al) : nullptr;
  uint16_t* Ath = pl.bf16_t ? w.at<uint16_t>(pl.off_Ath) : nullptr;
  uint16_t* Atl = pl.bf16_t && pl.bf16_split ? w.at<uint16_t>(pl.off_Atl) : nullptr;
  uint16_t* XTh = pl.bf16 ? w.at<uint16_t>(pl.off_XTh) : nullptr;
  uint16_t* XTl = pl.bf16_split ? w.at<uint16_t>(pl.off_XTl) : nullptr;
  float* fpart = pl.fpart_floats ? w.at<float>(pl.off_fpart) : nullptr;
  if (pl.bf16) {
    // BF16 schedules: A rounded once into the planes its low-precision
    // products stream (A for A X, and A^T for A^T X when A is not symmetric)
    PhaseScope ph(7, s);
    RSVD_TRY(bf16_planes(m, n, A, lda, Ah, Al, pl.ld_an, Ath, Atl, pl.ld_at, n, s));
  }
  auto stream_pass = [&](bool trans, const double* X, int64_t ldx, double* out, int64_t rows_out,
                         int64_t inner) -> rsvd_status {
    int prec = product < n_early - p.trailing_hp ? lowp : kPrecF64;
    product++;
    if (prec == kPrecF64 && pl.off_sl && !trans) {
      // the FP64-accurate passes of the sliced schedule (A X; A^T X of a
      // non-symmetric A stays FP64)
      PhaseScope ph(0, s);
      void* ws = w.at<char>(pl.off_sl);
      if (!a_sliced) {
        RSVD_TRY(sliced_prepare_a(m, l, n, A, lda, ws, s));
        a_sliced = true;
      }
      return sliced_gemm(rows_out, l, inner, X, ldx, out, l, ws, s);
    }
    const bool f32_panel_path = prec == kPrecF32 && !trans && pl.off_Xf;
    if (f32_panel_path) {
      // the panel rounded to FP32 once: the streaming kernel stages half the
      // bytes of it and feeds the matrix cores without conversions
      PhaseScope ph6(6, s);
      RSVD_TRY(f32_panel(inner, l, X, ldx, w.at<float>(pl.off_Xf), s));
    }
    PhaseScope ph(pl.bf16 && prec != kPrecF64 ? 8 : (prec == kPrecF32 ? 9 : 0), s);
    if (pl.bf16 && prec != kPrecF64) {
      // X (inner x l) -> XT planes, then the product from the planes
      const Bf16Shape sh = bf16_tuned_shape(rows_out, l, inner, pl.bf16_split);
      RSVD_TRY(bf16_planes(inner, l, X, ldx, nullptr, nullptr, 0, XTh, XTl, sh.Kp, sh.xt_rows, s));
      return bf16_gemm(sh, rows_out, l, trans ? Ath : Ah, trans ? Atl : Al,
                       trans ? pl.ld_at : pl.ld_an, XTh, XTl, out, l, fpart, pl.fpart_floats,
                       pl.bf16_split, s);
    }
    if (trans && dgemm_dma_eligible_t(rows_out, inner - inner % 16, l, A, lda, X, ldx)) {
      // A^T X on the streaming kernel's transposed variant (A in its stored
      // orientation, no transposes of the panels)
      return dgemm(true, rows_out, l, inner, 1.0, A, lda, X, ldx, 0.0, out, l, part,
                   pl.part_doubles, s, 64, nullptr, prec);
    }
    if (trans && rows_out * inner >= kTransStreamMin && l >= 16) {
      // A^T X = (X^T A)^T: the LDS-DMA streaming kernel takes X^T A with A
      // in its stored orientation, between two transposes of the skinny
      // panels (X^T into T, the l x n product into Yorig; both are free
      // between QRs)
      double* Xt = w.at<double>(pl.off_T);
      double* Ct = w.at<double>(pl.off_Yorig);
      if (dgemm_dma_eligible(inner, rows_out, Xt, inner, A, lda)) {
        RSVD_TRY(transpose(inner, l, X, ldx, Xt, inner, s));
        RSVD_TRY(dgemm(false, l, rows_out, inner, 1.0, Xt, inner, A, lda, 0.0, Ct, rows_out, part,
                       pl.part_doubles, s, 64, nullptr, prec));
        return transpose(l, rows_out, Ct, rows_out, out, l, s);
      }
    }
    if (f32_panel_path)
      return dgemm(false, rows_out, l, inner, 1.0, A, lda, X, ldx, 0.0, out, l, part,
                   pl.part_doubles, s, 64, nullptr, prec, w.at<float>(pl.off_Xf), f32_panel_ld(l));
    if (!trans && prec == kPrecF64 && pl.off_Xp && (ldx % 2 != 0 || ((uintptr_t)X & 15) != 0)) {
      // an odd-width panel staged through its copy with an even leading
      // dimension (the padding column reaches no output)
      double* Xp = w.at<double>(pl.off_Xp);
      RSVD_TRY(copy_panel(inner, l, X, ldx, Xp, pl.ld_xp, 0, st, s));
      return dgemm(false, rows_out, l, inner, 1.0, A, lda, X, ldx, 0.0, out, l, part,
                   pl.part_doubles, s, 64, nullptr, prec, nullptr, 0, Xp, pl.ld_xp);
    }
    return dgemm(trans, rows_out, l, inner, 1.0, A, lda, X, ldx, 0.0, out, l, part,
                 pl.part_doubles, s, 64, nullptr, prec);
  };
  auto qr = [&](int64_t rows, double* panel, bool full) -> rsvd_status {
    PhaseScope ph(1, s);
    return orth(pl, w, rows, l, panel, nullptr, s, full);
  };
  RSVD_TRY(stream_pass(false, Om, ldom, Y, m, n));
  RSVD_TRY(check_finite(m, l, Y, l, st, s));
  // the basis that B = Q^T A is taken against must be orthonormal to working
  // accuracy; bases inside the power iteration only carry the span forward
  RSVD_TRY(qr(m, Y, p.power_iters == 0));
  // power iterations
  for (int t = 0; t < p.power_iters; t++) {
    RSVD_TRY(stream_pass(!p.symmetric, Y, l, Z, n, m));
    RSVD_TRY(qr(n, Z, false));
    RSVD_TRY(stream_pass(false, Z, l, Y, m, n));
    RSVD_TRY(qr(m, Y, t + 1 == p.power_iters));
  }
  if (pl.post_r) {
    // a-posteriori judge: r fresh columns of the same stream (l .. l + r - 1),
    // W = (I - QQ^T) A P_r in FP64, est2 = max_j ||W_j||^2
    const int64_t r = pl.post_r;
    double* Op = w.at<double>(pl.off_Op);
    double* Wp = w.at<double>(pl.off_Wp);
    double* Cp = w.at<double>(pl.off_Cp);
    PhaseScope ph(6, s);
    RSVD_TRY(gaussian_omega(n, r, l, p.seed, p.channel, Op, r, s));
    RSVD_TRY(dgemm(false, m, r, n, 1.0, A, lda, Op, r, 0.0, Wp, r, part, pl.part_doubles, s));
    RSVD_TRY(dgemm(true, l, r, m, 1.0, Y, l, Wp, r, 0.0, Cp, r, part, pl.part_doubles, s));
    RSVD_TRY(dgemm(false, m, r, l, -1.0, Y, l, Cp, r, 1.0, Wp, r, part, pl.part_doubles, s));
    RSVD_TRY(colsumsq(m, (int)r, Wp, r, part, pl.part_doubles, 0, st, s));
  }
  if (pl.form == RSVD_FORM_SYMMETRIC) {
    // symmetric form: C = A Q (the projection's stream of A), B = Q^T C
    // (l x l) symmetrized; B = Q_b X_b (QR of B = B^T), SVD of X_b^T =
    // L_b Sigma W^T by Jacobi, so B = L_b Sigma (Q_b W)^T; then L = Q L_b and
    // R = Q (Q_b W)
    RSVD_TRY(stream_pass(false, Y, l, Z, n, m));
    double* Bs = w.at<double>(pl.off_Bs);
    {
      PhaseScope ph(2, s);
      RSVD_TRY(dgemm(true, l, l, m, 1.0, Y, l, Z, l, 0.0, Bs, l, part, pl.part_doubles, s));
      RSVD_TRY(symmetrize(l, Bs, l, s));
    }
    RSVD_TRY(small_svd_and_rank(pl, w, l, Bs, s, l));
    return run_tail(pl, w, A, lda, o, res_dev, s);
  }
  // step 2: Y^T = A^T Q = Q_B X_B, small SVD of X_B^T, rank rule
  RSVD_TRY(stream_pass(!p.symmetric, Y, l, Z, n, m));
  RSVD_TRY(small_svd_and_rank(pl, w, l, Z, s));
  return run_tail(pl, w, A, lda, o, res_dev, s);
}

#undef RSVD_TRY

rsvd_status rsvd_gaussian_omega(int64_t n, int64_t l, int64_t col0, uint64_t seed,
                                uint64_t channel, double* out, int64_t ldo, void* stream) {
  if (n < 0 || l < 0 || col0 < 0 || (n > 0 && l > 0 && (!out || ldo < l))) return RSVD_EINVAL;
  return gaussian_omega(n, l, col0, seed, channel, out, ldo, (hipStream_t)stream);
}

rsvd_status rsvd_gemm(int32_t precision, int32_t trans_a, int64_t m, int64_t n, int64_t k,
                      double alpha, const double* A, int64_t lda, const double* B, int64_t ldb,
                      double beta, double* C, int64_t ldc, void* work, size_t work_bytes,
                      void* stream) {
  if (precision < RSVD_PREC_FP64 || precision > RSVD_PREC_MIXED_FP32_SLICED) return RSVD_EINVAL;
  if (m < 0 || n < 0 || k < 0) return RSVD_EINVAL;
  if (m == 0 || n == 0) return RSVD_OK;
  if (!C || ldc < n) return RSVD_EINVAL;
  if (k > 0) {
    if (!A || !B || ldb < n) return RSVD_EINVAL;
    if (trans_a ? lda < m : lda < k) return RSVD_EINVAL;
  }
  if (precision == RSVD_PREC_MIXED_FP32_SLICED) {
    if (trans_a || alpha != 1.0 || beta != 0.0 || k == 0) return RSVD_EINVAL;
    if (!work || ((uintptr_t)work & 255) != 0) return RSVD_EINVAL;
    if (work_bytes < sliced_work_bytes(m, n, k)) return RSVD_ENOMEM;
    hipStream_t s = (hipStream_t)stream;
    rsvd_status r = sliced_prepare_a(m, n, k, A, lda, work, s);
    if (r != RSVD_OK) return r;
    return sliced_gemm(m, n, k, B, ldb, C, ldc, work, s);
  }
  const int prec = precision == RSVD_PREC_MIXED_FP32         ? kPrecF32
                   : precision == RSVD_PREC_MIXED_BF16       ? kPrecBF16
                   : precision == RSVD_PREC_MIXED_BF16_SPLIT ? kPrecBF16S
                                                             : kPrecF64;
  return dgemm(trans_a != 0, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, (double*)work,
               work_bytes / sizeof(double), (hipStream_t)stream, 64, nullptr, prec);
}

size_t rsvd_sliced_gemm_work_bytes(int64_t m, int64_t n, int64_t k) {
  return sliced_work_bytes(m, n, k);
}

namespace {
// workspace of rsvd_bf16_gemm: A planes (m x Kp), XT planes, FP32 partials
struct Bf16GemmLayout {
  size_t off_a = 0, off_al = 0, off_x = 0, off_xl = 0, off_part = 0, total = 0;
  int64_t Kp = 0, xt_rows = 0;
  size_t part_floats = 0;
  Bf16GemmLayout(int64_t m, int64_t n, int64_t k, bool split) {
    Carver c;
    Kp = bf16_pad(k);
    xt_rows = bf16_xt_rows_max(n);
    part_floats = bf16_part_floats_max(m, n);
    const size_t H = sizeof(uint16_t);
    off_a = c.take((size_t)m * Kp * H);
    if (split) off_al = c.take((size_t)m * Kp * H);
    off_x = c.take((size_t)xt_rows * Kp * H);
    if (split) off_xl = c.take((size_t)xt_rows * Kp * H);
    if (part_floats) off_part = c.take(part_floats * sizeof(float));
    total = c.at;
  }
};
}  // namespace

size_t rsvd_bf16_gemm_work_bytes(int64_t m, int64_t n, int64_t k, int32_t split) {
  if (m <= 0 || n <= 0 || k <= 0) return 0;
  return Bf16GemmLayout(m, n, k, split != 0).total;
}

rsvd_status rsvd_bf16_gemm(int32_t split, int32_t trans_a, int64_t m, int64_t n, int64_t k,
                           const double* A, int64_t lda, const double* B, int64_t ldb, double* C,
                           int64_t ldc, void* work, size_t work_bytes, void* stream) {
  if (m < 0 || n < 0 || k < 0) return RSVD_EINVAL;
  if (m == 0 || n == 0) return RSVD_OK;
  if (!C || ldc < n) return RSVD_EINVAL;
  if (k == 0) return dgemm(false, m, n, 0, 1.0, nullptr, 1, nullptr, n, 0.0, C, ldc, nullptr, 0,
                           (hipStream_t)stream);
  if (!A || !B || ldb < n || (trans_a ? lda < m : lda < k)) return RSVD_EINVAL;
  const Bf16GemmLayout lay(m, n, k, split != 0);
  if (!work || work_bytes < lay.total) return RSVD_ENOMEM;
  if (((uintptr_t)work & 255) != 0) return RSVD_EINVAL;
  char* wb = (char*)work;
  uint16_t* ah = (uint16_t*)(wb + lay.off_a);
  uint16_t* al = split ? (uint16_t*)(wb + lay.off_al) : nullptr;
  uint16_t* xh = (uint16_t*)(wb + lay.off_x);
  uint16_t* xl = split ? (uint16_t*)(wb + lay.off_xl) : nullptr;
  float* part = lay.part_floats ? (float*)(wb + lay.off_part) : nullptr;
  hipStream_t s = (hipStream_t)stream;
  const Bf16Shape sh = bf16_tuned_shape(m, n, k, split != 0);
  rsvd_status r;
  // op(A) planes (m x Kp): A itself, or the transpose of the k x m A
  if (trans_a)
    r = bf16_planes(k, m, A, lda, nullptr, nullptr, 0, ah, al, lay.Kp, m, s);
  else
    r = bf16_planes(m, k, A, lda, ah, al, lay.Kp, nullptr, nullptr, 0, 0, s);
  if (r != RSVD_OK) return r;
  if ((r = bf16_planes(k, n, B, ldb, nullptr, nullptr, 0, xh, xl, lay.Kp, sh.xt_rows, s)) != RSVD_OK)
    return r;
  return bf16_gemm(sh, m, n, ah, al, lay.Kp, xh, xl, C, ldc, part, lay.part_floats, split != 0, s);
}

size_t rsvd_dgemm_work_bytes(int64_t m, int64_t n, int64_t k, int32_t trans_a) {
  (void)trans_a;
  if (m <= 0 || n <= 0 || k <= 0) return 0;
  return dgemm_shape(m, n, k).part_doubles * sizeof(double);
}

rsvd_status rsvd_dgemm(int32_t trans_a, int64_t m, int64_t n, int64_t k, double alpha,
                       const double* A, int64_t lda, const double* B, int64_t ldb, double beta,
                       double* C, int64_t ldc, void* work, size_t work_bytes, void* stream) {
  if (m < 0 || n < 0 || k < 0) return RSVD_EINVAL;
  if (m == 0 || n == 0) return RSVD_OK;
  if (!C || ldc < n) return RSVD_EINVAL;
  if (k > 0) {
    if (!A || !B || ldb < n) return RSVD_EINVAL;
    if (trans_a ? lda < m : lda < k) return RSVD_EINVAL;
  }
  return dgemm(trans_a != 0, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, (double*)work,
               work_bytes / sizeof(double), (hipStream_t)stream);
}

size_t rsvd_orth_work_bytes(int64_t m, int64_t l) {
  rsvd_plan_s pl;
  pl.l = l;
  Carver c;
  pl.off_state = c.take(sizeof(DevState));
  pl.off_T = c.take((size_t)m * l * sizeof(double));
  pl.off_Yorig = c.take((size_t)m * l * sizeof(double));
  pl.off_tau = c.take((size_t)2 * l * sizeof(double));
  pl.part_doubles = gemm_part_need(m, m, l);
  pl.off_part = c.take(pl.part_doubles * sizeof(double));
  const size_t ll = (size_t)l * l * sizeof(double);
  for (int i = 0; i < 9; i++) c.take(ll);
  return c.at;
}

rsvd_status rsvd_orth(int64_t m, int64_t l, double* Y, int64_t ldy, double* X, uint32_t* flags,
                      void* work, size_t work_bytes, void* stream) {
  if (m < 1 || l < 1 || l > m || !Y || ldy != l || !work) return RSVD_EINVAL;
  if (work_bytes < rsvd_orth_work_bytes(m, l)) return RSVD_ENOMEM;
  if (((uintptr_t)work & 255) != 0) return RSVD_EINVAL;
  rsvd_plan_s pl;
  pl.l = l;
  Carver c;
  pl.off_state = c.take(sizeof(DevState));
  pl.off_T = c.take((size_t)m * l * sizeof(double));
  pl.off_Yorig = c.take((size_t)m * l * sizeof(double));
  pl.off_tau = c.take((size_t)2 * l * sizeof(double));
  pl.part_doubles = gemm_part_need(m, m, l);
  pl.off_part = c.take(pl.part_doubles * sizeof(double));
  const size_t ll = (size_t)l * l * sizeof(double);
  pl.off_G = c.take(ll);
  pl.off_R1 = c.take(ll);
  pl.off_R1i = c.take(ll);
  pl.off_R2 = c.take(ll);
  pl.off_R2i = c.take(ll);
  pl.off_R3 = c.take(ll);
  pl.off_R3i = c.take(ll);
  pl.off_Rtmp = c.take(ll);
  c.take(ll);
  hipStream_t s = (hipStream_t)stream;
  Ws w{(char*)work};
  DevState* st = w.at<DevState>(pl.off_state);
  rsvd_status r = init_state(st, 0, s);
  if (r != RSVD_OK) return r;
  r = orth(pl, w, m, l, Y, X, s);
  if (r != RSVD_OK) return r;
  if (flags) {
    if (hipMemcpyAsync(flags, &st->flags, sizeof(uint32_t), hipMemcpyDeviceToDevice, s) != hipSuccess)
      return RSVD_EHIP;
  }
  return RSVD_OK;
}

size_t rsvd_small_svd_work_bytes(int64_t l) {
  const int64_t Lp = jacobi_padded(l);
  Carver c;
  c.take(sizeof(DevState));
  c.take((size_t)Lp * Lp * sizeof(double));
  c.take((size_t)Lp * Lp * sizeof(double));
  c.take((size_t)2 * l * sizeof(double));
  return c.at;
}

rsvd_status rsvd_small_svd(int64_t l, const double* R, double* sv, double* Us, double* W,
                           int32_t max_sweeps, int32_t* sweeps, uint32_t* flags, void* work,
                           size_t work_bytes, void* stream) {
  if (l < 1 || !R || !sv || !Us || !W || !work) return RSVD_EINVAL;
  if (work_bytes < rsvd_small_svd_work_bytes(l)) return RSVD_ENOMEM;
  if (((uintptr_t)work & 255) != 0) return RSVD_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  const int64_t Lp = jacobi_padded(l);
  Carver c;
  const size_t off_state = c.take(sizeof(DevState));
  const size_t off_M = c.take((size_t)Lp * Lp * sizeof(double));
  const size_t off_P = c.take((size_t)Lp * Lp * sizeof(double));
  const size_t off_scr = c.take((size_t)2 * l * sizeof(double));
  Ws w{(char*)work};
  DevState* st = w.at<DevState>(off_state);
  double* Mj = w.at<double>(off_M);
  double* Pj = w.at<double>(off_P);
  rsvd_status r;
#define RSVD_TRY(x) do { r = (x); if (r != RSVD_OK) return r; } while (0)
  RSVD_TRY(init_state(st, 0, s));
  RSVD_TRY(block_jacobi(l, R, Mj, Pj, max_sweeps > 0 ? max_sweeps : 30, 1, st, s));
  RSVD_TRY(svd_finish(l, l, Mj, Pj, Lp, sv, Us, W, w.at<double>(off_scr), st, s));
  if (sweeps && hipMemcpyAsync(sweeps, &st->sweeps, sizeof(int32_t), hipMemcpyDeviceToDevice, s) != hipSuccess)
    return RSVD_EHIP;
  if (flags && hipMemcpyAsync(flags, &st->flags, sizeof(uint32_t), hipMemcpyDeviceToDevice, s) != hipSuccess)
    return RSVD_EHIP;
  return RSVD_OK;
#undef RSVD_TRY
}

// ---- truncation of a computed decomposition ---------------------------------

#define RSVD_TRY(x) do { rsvd_status r_ = (x); if (r_ != RSVD_OK) return r_; } while (0)

namespace {
struct ResidualLayout {
  size_t off_state = 0, off_US = 0, off_Vt = 0, off_part = 0, total = 0;
  int64_t kcp = 0;
  ResidualLayout(int64_t m, int64_t n, int64_t k) {
    kcp = (k + 15) / 16 * 16;
    Carver c;
    off_state = c.take(sizeof(DevState));
    off_US = c.take((size_t)m * kcp * sizeof(double));
    off_Vt = c.take((size_t)kcp * n * sizeof(double));
    off_part = c.take(resid_partials(m, n) * sizeof(double));
    total = c.at;
  }
};
}  // namespace

size_t rsvd_residual_work_bytes(int64_t m, int64_t n, int64_t k) {
  if (m < 1 || n < 1 || k < 1) return 0;
  return ResidualLayout(m, n, k).total;
}

rsvd_status rsvd_residual(int64_t m, int64_t n, int64_t k, const double* A, int64_t lda,
                          const double* S, const double* U, int64_t ldu, const double* V,
                          int64_t ldv, rsvd_result* res_dev, void* work, size_t work_bytes,
                          void* stream) {
  if (m < 1 || n < 1 || k < 1 || k > (m < n ? m : n)) return RSVD_EINVAL;
  if (!A || !S || !U || !V || !res_dev || !work || lda < n || ldu < k || ldv < k)
    return RSVD_EINVAL;
  const ResidualLayout lay(m, n, k);
  if (work_bytes < lay.total) return RSVD_ENOMEM;
  if (((uintptr_t)work & 255) != 0) return RSVD_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  Ws w{(char*)work};
  DevState* st = w.at<DevState>(lay.off_state);
  double* US = w.at<double>(lay.off_US);
  double* Vt = w.at<double>(lay.off_Vt);
  RSVD_TRY(init_state(st, 0u, s));
  // the fixed rule at k sets the rank the padded factors keep
  RSVD_TRY(select_rank(k, 0, k, RSVD_RANK_FIXED, (double)k, S, st, s));
  RSVD_TRY(resid_prep(m, n, k, lay.kcp, U, ldu, S, V, ldv, US, Vt, st, s));
  RSVD_TRY(resid(m, n, lay.kcp, US, lay.kcp, Vt, n, A, lda, w.at<double>(lay.off_part), st, s));
  return finalize(m, n, k, 1, __builtin_nan(""), 0, st, res_dev, s);
}

// ---- basis transformation on thin factors -------------------------------------

namespace {
struct TransformLayout {
  size_t off_X = 0, off_Xt = 0, off_Ct = 0, off_O = 0, off_part = 0, total = 0;
  int64_t K2 = 0;
  size_t part_doubles = 0;
  TransformLayout(int64_t N, int64_t Nb, int64_t k, bool with_r) {
    K2 = with_r ? 2 * k : k;
    part_doubles = dgemm_shape(Nb, K2, N).part_doubles;
    const size_t t1 = dgemm_shape(K2, Nb, N).part_doubles;
    if (t1 > part_doubles) part_doubles = t1;
    const size_t t2 = (size_t)kTransSplits * K2 * Nb;
    if (t2 > part_doubles) part_doubles = t2;
    if (part_doubles < 2048) part_doubles = 2048;
    const size_t D = sizeof(double);
    Carver c;
    off_X = c.take((size_t)N * K2 * D);
    off_Xt = c.take((size_t)K2 * N * D);
    off_Ct = c.take((size_t)K2 * Nb * D);
    off_O = c.take((size_t)Nb * K2 * D);
    off_part = c.take(part_doubles * D);
    total = c.at;
  }
};
}  // namespace

size_t rsvd_factor_transform_work_bytes(int64_t N, int64_t Nb, int64_t k, int32_t with_r) {
  if (N < 1 || Nb < 1 || k < 1 || Nb > N) return 0;
  return TransformLayout(N, Nb, k, with_r != 0).total;
}

rsvd_status rsvd_factor_transform(int64_t N, int64_t Nb, int64_t k, const double* Ub, int64_t ldub,
                                  const double* L, int64_t ldl, const double* R, int64_t ldr,
                                  double* Lout, int64_t ldlo, double* Rout, int64_t ldro,
                                  void* work, size_t work_bytes, void* stream) {
  if (N < 1 || Nb < 1 || k < 1 || Nb > N) return RSVD_EINVAL;
  if (!Ub || !L || !Lout || !work || ldub < Nb || ldl < k || ldlo < k) return RSVD_EINVAL;
  if (R && (!Rout || ldr < k || ldro < k)) return RSVD_EINVAL;
  const TransformLayout lay(N, Nb, k, R != nullptr);
  if (work_bytes < lay.total) return RSVD_ENOMEM;
  if (((uintptr_t)work & 255) != 0) return RSVD_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  Ws w{(char*)work};
  const int64_t K2 = lay.K2;
  double* X = w.at<double>(lay.off_X);
  double* O = w.at<double>(lay.off_O);
  double* part = w.at<double>(lay.off_part);
  // [L R] side by side: one stream of U serves both factors
  RSVD_TRY(copy_panel(N, k, L, ldl, X, K2, 0, nullptr, s));
  if (R) RSVD_TRY(copy_panel(N, k, R, ldr, X + k, K2, 0, nullptr, s));
  double* Xt = w.at<double>(lay.off_Xt);
  double* Ct = w.at<double>(lay.off_Ct);
  if (dgemm_dma_eligible_t(Nb, N - N % 16, K2, Ub, ldub, X, K2)) {
    // U^T X on the streaming kernel's transposed variant (U in its stored
    // orientation)
    RSVD_TRY(dgemm(true, Nb, K2, N, 1.0, Ub, ldub, X, K2, 0.0, O, K2, part, lay.part_doubles, s));
  } else if (N * Nb >= kTransStreamMin && K2 >= 16 && dgemm_dma_eligible(N, Nb, Xt, N, Ub, ldub)) {
    // U^T X = (X^T U)^T: U streams in its stored orientation through the
    // LDS-DMA kernel between two transposes of the skinny panels
    RSVD_TRY(transpose(N, K2, X, K2, Xt, N, s));
    RSVD_TRY(dgemm(false, K2, Nb, N, 1.0, Xt, N, Ub, ldub, 0.0, Ct, Nb, part, lay.part_doubles, s));
    RSVD_TRY(transpose(K2, Nb, Ct, Nb, O, K2, s));
  } else {
    RSVD_TRY(dgemm(true, Nb, K2, N, 1.0, Ub, ldub, X, K2, 0.0, O, K2, part, lay.part_doubles, s));
  }
  RSVD_TRY(copy_panel(Nb, k, O, K2, Lout, ldlo, 0, nullptr, s));
  if (R) RSVD_TRY(copy_panel(Nb, k, O + k, K2, Rout, ldro, 0, nullptr, s));
  return RSVD_OK;
}

#undef RSVD_TRY

// ---- learned (k, p, q) predictor ---------------------------------------------

rsvd_status rsvd_mlp_init(float* params, uint64_t seed, void* stream) {
  if (!params) return RSVD_EINVAL;
  return mlp_init(params, seed, (hipStream_t)stream);
}

rsvd_status rsvd_mlp_forward(const float* params, const float* X, int64_t B, float* Y,
                             void* stream) {
  if (B < 0 || (B > 0 && (!params || !X || !Y))) return RSVD_EINVAL;
  return mlp_forward(params, X, B, Y, (hipStream_t)stream);
}

rsvd_status rsvd_mlp_grad(const float* params, const float* X, const float* T, int64_t B,
                          float* grad, float* loss, void* stream) {
  if (!params || !X || !T || !grad || B < 1 || B > RSVD_MLP_MAX_BATCH) return RSVD_EINVAL;
  return mlp_grad(const_cast<float*>(params), X, T, B, false, nullptr, nullptr, 1, 0.0f, grad,
                  loss, (hipStream_t)stream);
}

rsvd_status rsvd_mlp_train_step(float* params, float* adam_m, float* adam_v, int64_t step,
                                const float* X, const float* T, int64_t B, float lr,
                                float* loss, void* stream) {
  if (!params || !adam_m || !adam_v || !X || !T || step < 1 || B < 1 ||
      B > RSVD_MLP_MAX_BATCH || !(lr > 0.0f))
    return RSVD_EINVAL;
  return mlp_grad(params, X, T, B, true, adam_m, adam_v, step, lr, nullptr, loss,
                  (hipStream_t)stream);
}

rsvd_status rsvd_mlp_targets(const int64_t* labels, int64_t B, float* stats, float* T,
                             void* stream) {
  if (!labels || !stats || !T || B < 1) return RSVD_EINVAL;
  return mlp_targets(labels, B, stats, T, (hipStream_t)stream);
}

rsvd_status rsvd_mlp_predict(const float* params, const float* stats, const float* X, int64_t B,
                             const int64_t* n_cap, int64_t* kpq, void* stream) {
  if (B < 0 || (B > 0 && (!params || !stats || !X || !n_cap || !kpq))) return RSVD_EINVAL;
  return mlp_predict(params, stats, X, B, n_cap, kpq, (hipStream_t)stream);
}

rsvd_status rsvd_size_label(const double* sv, int64_t count, int64_t k, int64_t n, int64_t l_min,
                            int64_t* kpq, void* stream) {
  if (!sv || !kpq || k < 1 || count < k || n < k || l_min < 0) return RSVD_EINVAL;
  return size_label(sv, count, k, n, l_min, kpq, (hipStream_t)stream);
}

namespace {
constexpr char kMlpTag[8] = {'R', 'S', 'V', 'D', 'M', 'L', 'P', '1'};
constexpr uint32_t kMlpStats = 6;
}  // namespace

rsvd_status rsvd_mlp_save(const char* path, const float* params, const float* stats,
                          void* stream) {
  if (!path || !params || !stats) return RSVD_EINVAL;
  std::vector<float> buf(RSVD_MLP_PARAMS + kMlpStats);
  hipStream_t s = (hipStream_t)stream;
  if (hipMemcpyAsync(buf.data(), params, RSVD_MLP_PARAMS * sizeof(float), hipMemcpyDeviceToHost,
                     s) != hipSuccess ||
      hipMemcpyAsync(buf.data() + RSVD_MLP_PARAMS, stats, kMlpStats * sizeof(float),
                     hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return RSVD_EHIP;
  FILE* f = std::fopen(path, "wb");
  if (!f) return RSVD_EINVAL;
  const uint32_t counts[2] = {RSVD_MLP_PARAMS, kMlpStats};
  const bool ok = std::fwrite(kMlpTag, 1, 8, f) == 8 && std::fwrite(counts, 4, 2, f) == 2 &&
                  std::fwrite(buf.data(), sizeof(float), buf.size(), f) == buf.size();
  const bool closed = std::fclose(f) == 0;
  return ok && closed ? RSVD_OK : RSVD_EINVAL;
}

rsvd_status rsvd_mlp_load(const char* path, float* params, float* stats, void* stream) {
  if (!path || !params || !stats) return RSVD_EINVAL;
  FILE* f = std::fopen(path, "rb");
  if (!f) return RSVD_EINVAL;
  char tag[8];
  uint32_t counts[2];
  std::vector<float> buf(RSVD_MLP_PARAMS + kMlpStats);
  bool ok = std::fread(tag, 1, 8, f) == 8 && std::memcmp(tag, kMlpTag, 8) == 0 &&
            std::fread(counts, 4, 2, f) == 2 && counts[0] == RSVD_MLP_PARAMS &&
            counts[1] == kMlpStats &&
            std::fread(buf.data(), sizeof(float), buf.size(), f) == buf.size();
  char extra;
  ok = ok && std::fread(&extra, 1, 1, f) == 0;  // nothing after the stats
  std::fclose(f);
  if (!ok) return RSVD_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  if (hipMemcpyAsync(params, buf.data(), RSVD_MLP_PARAMS * sizeof(float), hipMemcpyHostToDevice,
                     s) != hipSuccess ||
      hipMemcpyAsync(stats, buf.data() + RSVD_MLP_PARAMS, kMlpStats * sizeof(float),
                     hipMemcpyHostToDevice, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return RSVD_EHIP;
  return RSVD_OK;
}

namespace {
// Layout of the pilot: a plan for l = min(32, m, n) columns in the FP32
// schedule with no power step (the sketch is the only product with A).
rsvd_status pilot_plan(int64_t m, int64_t n, rsvd_plan_t* pl, size_t* bytes) {
  rsvd_problem p{};
  p.m = m;
  p.n = n;
  p.k = RSVD_PILOT_COLS;
  p.rank_mode = RSVD_RANK_FIXED;
  p.precision = RSVD_PREC_MIXED_FP32;
  return rsvd_plan(&p, pl, bytes);
}
}  // namespace

size_t rsvd_pilot_work_bytes(int64_t m, int64_t n) {
  rsvd_plan_t pl = nullptr;
  size_t bytes = 0;
  if (m < 1 || n < 1 || pilot_plan(m, n, &pl, &bytes) != RSVD_OK) return 0;
  rsvd_destroy(pl);
  return bytes;
}

rsvd_status rsvd_pilot_features(const double* A, int64_t lda, int64_t m, int64_t n, uint64_t seed,
                                uint64_t channel, float* feat, void* work, size_t work_bytes,
                                void* stream) {
  if (!A || !feat || !work || m < 1 || n < 1 || lda < n) return RSVD_EINVAL;
  if (((uintptr_t)work & 255) != 0) return RSVD_EINVAL;
  rsvd_plan_t plh = nullptr;
  size_t need = 0;
  rsvd_status r = pilot_plan(m, n, &plh, &need);
  if (r != RSVD_OK) return r;
  struct Guard {
    rsvd_plan_t p;
    ~Guard() { rsvd_destroy(p); }
  } guard{plh};
  if (work_bytes < need) return RSVD_ENOMEM;
  const rsvd_plan_s& pl = *plh;
  const int64_t l = pl.l;
  hipStream_t s = (hipStream_t)stream;
  Ws w{(char*)work};
  DevState* st = w.at<DevState>(pl.off_state);
  double* Y = w.at<double>(pl.off_Y);
  double* P0 = w.at<double>(pl.off_Z);
  double* Rt = w.at<double>(pl.off_Rt);
  double* part = w.at<double>(pl.off_part);
  if ((r = init_state(st, 0u, s)) != RSVD_OK) return r;
  if ((r = gaussian_omega(n, l, 0, seed, channel, P0, l, s)) != RSVD_OK) return r;
  // Y0 = A P0 on the FP32 matrix cores
  if ((r = dgemm(false, m, l, n, 1.0, A, lda, P0, l, 0.0, Y, l, part, pl.part_doubles, s, 64,
                 nullptr, kPrecF32)) != RSVD_OK)
    return r;
  // singular values of Y0 = those of its triangular factor
  if ((r = orth(pl, w, m, l, Y, Rt, s, true)) != RSVD_OK) return r;
  if ((r = block_jacobi(l, Rt, w.at<double>(pl.off_M), w.at<double>(pl.off_P), 30, 1, st, s)) !=
      RSVD_OK)
    return r;
  if ((r = svd_finish(l, pl.kc, w.at<double>(pl.off_M), w.at<double>(pl.off_P), jacobi_padded(l),
                      w.at<double>(pl.off_sig), w.at<double>(pl.off_Us), w.at<double>(pl.off_W),
                      w.at<double>(pl.off_tau), st, s)) != RSVD_OK)
    return r;
  return pilot_features((int)l, w.at<double>(pl.off_sig), feat, s);
}

void rsvd_trace_enable(int32_t on) { g_trace_on = on != 0; }

rsvd_status rsvd_trace_collect(double* ms, int64_t* counts) {
  rsvd_status st = RSVD_OK;
  for (auto& mk : g_marks) {
    float t = 0.0f;
    if (hipEventSynchronize(mk.b) != hipSuccess || hipEventElapsedTime(&t, mk.a, mk.b) != hipSuccess) {
      st = RSVD_EHIP;
    } else if (mk.phase >= 0 && mk.phase < RSVD_TRACE_PHASES) {
      if (ms) ms[mk.phase] += t;
      if (counts) counts[mk.phase] += 1;
    }
    g_event_pool.push_back(mk.a);
    g_event_pool.push_back(mk.b);
  }
  g_marks.clear();
  return st;
}

}  // extern "C"
