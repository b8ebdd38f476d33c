// Small dense kernels of the randomized SVD: the l x l work between the
// streaming products (Cholesky QR factors, Householder fallback, ordering of
// the small SVD, rank rule, signs, residual bookkeeping). The Jacobi sweeps
// of the small SVD are in bjacobi.hip.
//
// Paper mapping (section "Randomized matrix decompositions", Fig. 1):
//   chol_inv      thin QR Z = Q X of step 1 (Cholesky QR: X^T X = Z^T Z)
//   svd_finish    singular values ordered decreasingly (Eq. 1)
//   select_rank   R_SVD, R% and the compression ratio of Eq. 2
#include <utility>

#include "common.hpp"
#include "kernels.hpp"

#include <math.h>

namespace rsvd {

namespace {

constexpr double kUnitRoundoff = 1.1102230246251565e-16;  // 2^-53
constexpr int kBig = 1024;                                // threads of the l x l kernels
constexpr int64_t kHouseGridMin = 1 << 16;  // rows x l from which the Householder fallback runs on a grid

__device__ __forceinline__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  const int nw = (blockDim.x + 63) >> 6;
  for (int i = 0; i < nw; i++) s += red[i];
  return s;
}

// ---------------------------------------------------------------------------
// Householder QR of a rows x l panel (rows >= l), one workgroup: the fallback
// for panels whose Cholesky QR broke down (numerically rank deficient). Y is
// overwritten by the explicit Q (diag(R) >= 0), R (l x l upper) if non-null.
// Runs only when st->qr_householder is set. Y holds a copy of the original
// panel on entry (restored from Yorig).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBig) householder_kernel(int64_t rows, int l,
                                                           const double* __restrict__ Yorig,
                                                           double* __restrict__ Y,
                                                           double* __restrict__ R,
                                                           double* __restrict__ tau_buf,
                                                           DevState* st) {
  if (st->qr_householder == 0) return;
  __shared__ double red[kBig / 64];
  __shared__ double sh[4];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int nw = blockDim.x >> 6;
  const int64_t tot = rows * l;
  double* W = Y;  // factor in place
  for (int64_t e = threadIdx.x; e < tot; e += blockDim.x) W[e] = Yorig[e];
  __syncthreads();
  for (int j = 0; j < l; j++) {
    // sigma2 = sum_{i > j} W[i][j]^2
    double s2 = 0.0;
    for (int64_t i = j + 1 + threadIdx.x; i < rows; i += blockDim.x) {
      const double x = W[i * l + j];
      s2 += x * x;
    }
    s2 = block_sum(s2, red);
    if (threadIdx.x == 0) {
      const double alpha = W[(int64_t)j * l + j];
      const double nrm = sqrt(alpha * alpha + s2);
      double beta, tau, scale;
      if (s2 == 0.0) {
        beta = alpha;
        tau = 0.0;
        scale = 0.0;
      } else {
        beta = alpha >= 0.0 ? -nrm : nrm;
        tau = (beta - alpha) / beta;
        scale = 1.0 / (alpha - beta);
      }
      sh[0] = beta;
      sh[1] = tau;
      sh[2] = scale;
      tau_buf[j] = tau;
    }
    __syncthreads();
    const double beta = sh[0], tau = sh[1], scale = sh[2];
    for (int64_t i = j + 1 + threadIdx.x; i < rows; i += blockDim.x) W[i * l + j] *= scale;
    __syncthreads();
    if (threadIdx.x == 0) W[(int64_t)j * l + j] = beta;
    // apply H = I - tau v v^T (v_j = 1) to columns c > j, one wave per column
    if (tau != 0.0) {
      for (int c = j + 1 + wave; c < l; c += nw) {
        double d = (lane == 0) ? W[(int64_t)j * l + c] : 0.0;
        for (int64_t i = j + 1 + lane; i < rows; i += 64) d += W[i * l + j] * W[i * l + c];
        d = wave_sum(d) * tau;
        if (lane == 0) W[(int64_t)j * l + c] -= d;
        for (int64_t i = j + 1 + lane; i < rows; i += 64) W[i * l + c] -= d * W[i * l + j];
      }
    }
    __syncthreads();
  }
  // R = upper(W), sign-fixed so diag(R) >= 0 (rows of R and columns of Q flip together)
  if (R) {
    for (int64_t e = threadIdx.x; e < (int64_t)l * l; e += blockDim.x) {
      const int i = (int)(e / l), c = (int)(e % l);
      const double d = W[(int64_t)i * l + i];
      R[e] = (c >= i) ? (d < 0.0 ? -W[(int64_t)i * l + c] : W[(int64_t)i * l + c]) : 0.0;
    }
  }
  // keep the diagonal signs in tau_buf[l + j]
  for (int j = threadIdx.x; j < l; j += blockDim.x) tau_buf[l + j] = W[(int64_t)j * l + j] < 0.0 ? -1.0 : 1.0;
  __syncthreads();
  // Q = H_0 ... H_{l-1} [I; 0], accumulated backwards in place. Before
  // column j is rebuilt, rows > j of column j still hold v_j.
  for (int j = l - 1; j >= 0; j--) {
    const double tau = tau_buf[j];
    // columns c > j: Q[j:, c] -= tau v (v^T Q[j:, c]); Q[j][c] is 0 for c > j before H_j
    for (int c = j + 1 + wave; c < l; c += nw) {
      double d = 0.0;
      for (int64_t i = j + 1 + lane; i < rows; i += 64) d += W[i * l + j] * W[i * l + c];
      d = wave_sum(d) * tau;
      if (lane == 0) W[(int64_t)j * l + c] = -d;
      for (int64_t i = j + 1 + lane; i < rows; i += 64) W[i * l + c] -= d * W[i * l + j];
    }
    __syncthreads();
    // column j: H_j e_j = e_j - tau v
    for (int64_t i = j + 1 + threadIdx.x; i < rows; i += blockDim.x) W[i * l + j] = -tau * W[i * l + j];
    if (threadIdx.x == 0) {
      W[(int64_t)j * l + j] = 1.0 - tau;
      for (int i = 0; i < j; i++) W[(int64_t)i * l + j] = 0.0;
    }
    __syncthreads();
  }
  for (int64_t e = threadIdx.x; e < tot; e += blockDim.x) W[e] *= tau_buf[l + (int)(e % l)];
  if (threadIdx.x == 0) atomicOr(&st->flags, (uint32_t)RSVD_FLAG_QR_FALLBACK);
}
// ---------------------------------------------------------------------------
// Blocked Cholesky + triangular inverse on 16 x 16 tiles with the FP64 matrix
// cores, one workgroup of 16 waves. Upper form: G (+ shift I) = R^T R.
// Right-looking over block rows k:
//   R_kk  = chol(G_kk)            one wave, in registers (cross-lane shuffles)
//   R_kJ  = R_kk^{-T} G_kJ        MFMA, tiles of block row k (J > k)
//   G_IJ -= R_kI^T R_kJ           MFMA, trailing tiles (k < I <= J)
// then X = R^{-1} by block back substitution: X_IJ = -X_II sum_{K>I} R_IK X_KJ.
// Tiles live in global memory (L2-resident at these sizes); the current block
// row of R is staged in LDS. Padding rows/columns beyond l act as identity.
// Register layout of a 16 x 16 tile (the MFMA accumulator layout): lane
// (r = lane % 16, g = lane / 16), item t holds entry (g + 4 t, r).
// ---------------------------------------------------------------------------
struct TileCtx {
  int l, nb, ps;
  __device__ __forceinline__ bool in(int i, int c) const { return i < l && c < l; }
};

__device__ __forceinline__ void load_tile(const TileCtx& cx, const double* W, int I, int J,
                                          double t[4]) {
  const int lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
#pragma unroll
  for (int it = 0; it < 4; it++) {
    const int i = 16 * I + g + 4 * it, c = 16 * J + r;
    t[it] = cx.in(i, c) ? W[(int64_t)i * cx.l + c] : (i == c ? 1.0 : 0.0);
  }
}

__device__ __forceinline__ void store_tile(const TileCtx& cx, double* W, int I, int J,
                                           const double t[4]) {
  const int lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
#pragma unroll
  for (int it = 0; it < 4; it++) {
    const int i = 16 * I + g + 4 * it, c = 16 * J + r;
    if (cx.in(i, c)) W[(int64_t)i * cx.l + c] = t[it];
  }
}

__device__ __forceinline__ double bcast_lane(double v, int src) {
  const long long bits = __double_as_longlong(v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(bits >> 32), src);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)bits, src);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Pivot of one Cholesky step: clamped (pivots at most clampv raised to it,
// when clamping), replaced by 1 with ok cleared when non-positive or
// non-finite; inv = 1 / sqrt(piv), rjj = sqrt(piv).
__device__ __forceinline__ void chol_pivot(double piv, bool clamp, double clampv, bool& ok,
                                           double& inv, double& rjj) {
  if (clamp && !(piv > clampv)) piv = clampv;
  if (!(piv > 0.0) || !isfinite(piv)) {
    ok = false;
    piv = 1.0;
  }
  if (piv >= 1e-290) {
    inv = rsq_nr(piv);
    rjj = piv * inv;
  } else {
    rjj = sqrt(piv);
    inv = 1.0 / rjj;
  }
}

// Upper Cholesky of one tile held by a wave together with Z = R^{-T} (lower,
// same layout): the row operations of the factorization (row j scaled by
// 1 / r_jj, then row i > j less r_ji times row j) are L^{-1} for G = L L^T,
// L = R^T, so applied to the identity beside G they leave L^{-1} = R^{-T}.
// Row j of Z is final after step j, so the inverse costs a few more FMAs per
// step instead of a second 16-step substitution. Row j of R and Z goes
// through the wave's own 32 doubles of LDS (rowbuf), which every lane then
// reads by broadcast (LDS operations of one wave complete in order, so no
// barrier is needed). The next pivot, (j+1, j+1) less the square of the
// scaled (j, j+1), is formed from two lanes' values read into scalar
// registers and its inverse square root taken while row j is in flight
// through LDS; it is the same FMA on the same operands that the row update
// applies to that entry, so the result does not depend on this order.
// Returns false on a non-positive or non-finite pivot (unless clamping:
// pivots at most clampv are raised to it); tracks the range of the diagonal
// of R over rows below lmax.
__device__ bool tile_chol_inv(d4& t, d4& z, double* rowbuf, bool clamp, double clampv, int row0,
                              int lmax, double& dmax, double& dmin) {
  // an opaque lane index: the lane masks below are formed here, not hoisted
  // into the caller's loops (where they would stay live beside its tiles)
  int lane = threadIdx.x & 63;
  asm volatile("" : "+v"(lane));
  const int r = lane & 15, g = lane >> 4;
  bool ok = true;
#pragma unroll
  for (int it = 0; it < 4; it++) z[it] = (g + 4 * it == r) ? 1.0 : 0.0;
  // entry (i, c) is item i / 4 of lane c + 16 (i % 4)
  double inv, rjj;
  chol_pivot(bcast_lane(t[0], 0), clamp, clampv, ok, inv, rjj);
#pragma unroll
  for (int j = 0; j < 16; j++) {
    const int jg = j & 3, jt = j >> 2;
    if (row0 + j < lmax) {
      dmax = fmax(dmax, rjj);
      dmin = fmin(dmin, rjj);
    }
    // (j, j+1) and (j+1, j+1) before this step's update
    double a = 0.0, b = 0.0;
    if (j < 15) {
      const int j1 = j + 1;
      a = bcast_lane(t[jt], j1 + 16 * jg);
      b = bcast_lane(t[j1 >> 2], j1 + 16 * (j1 & 3));
    }
    if (g == jg) {
      if (r > j) t[jt] *= inv;
      else if (r == j) t[jt] = rjj;
      z[jt] *= inv;
      rowbuf[r] = t[jt];       // r_j,r
      rowbuf[16 + r] = z[jt];  // z_j,r
    }
    __builtin_amdgcn_wave_barrier();
    const double colv = rowbuf[r];
    const double colz = rowbuf[16 + r];
    double rowv[4];
#pragma unroll
    for (int it = 0; it < 4; it++) rowv[it] = rowbuf[g + 4 * it];  // r_j,i
    double inv_n = 1.0, rjj_n = 1.0;
    if (j < 15) {
      const double as = a * inv;
      chol_pivot(fma(-as, as, b), clamp, clampv, ok, inv_n, rjj_n);
    }
#pragma unroll
    for (int it = 0; it < 4; it++) {
      const int i = g + 4 * it;
      const double tn = fma(-rowv[it], colv, t[it]);
      const double zn = fma(-rowv[it], colz, z[it]);
      t[it] = (i > j && r >= i) ? tn : t[it];
      z[it] = i > j ? zn : z[it];
    }
    __builtin_amdgcn_wave_barrier();
    inv = inv_n;
    rjj = rjj_n;
  }
#pragma unroll
  for (int it = 0; it < 4; it++) {
    if (g + 4 * it > r) t[it] = 0.0;
    if (g + 4 * it < r) z[it] = 0.0;
  }
  return ok;
}

// x mod m in [0, m) for any int x (m > 0)
__device__ __forceinline__ int mod_pos(int x, int m) {
  const int q = x % m;
  return q < 0 ? q + m : q;
}

__device__ __forceinline__ void trailing_coords(int t, int n, int& I, int& J) {
  // t-th tile of the upper triangle (row-major) of an n x n tile grid
  int row = 0, cnt = n;
  while (t >= cnt) {
    t -= cnt;
    row++;
    cnt--;
  }
  I = row;
  J = row + t;
}

// Tile in the MFMA A-operand layout: lane (r, g), item t holds entry (r, g + 4 t).
__device__ __forceinline__ void load_tile_a(const TileCtx& cx, const double* W, int I, int J,
                                            double t[4]) {
  const int lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
#pragma unroll
  for (int it = 0; it < 4; it++) {
    const int i = 16 * I + r, c = 16 * J + g + 4 * it;
    t[it] = cx.in(i, c) ? W[(int64_t)i * cx.l + c] : (i == c ? 1.0 : 0.0);
  }
}

// X = R^{-1} by recursive doubling on tile blocks: with the inverses X11, X22
// of two adjacent diagonal blocks known, the off-diagonal block of the inverse
// of [[R11, R12], [0, R22]] is -X11 R12 X22. Block sizes 1, 2, 4, ... tiles;
// every level runs T = R12 X22 into the scratch S, then X12 = -X11 T.
// Diagonal tiles of X are already in Xg.
// Team: the waves that share the work (id in [0, size)) and their barrier
// (a workgroup's __syncthreads, or a grid barrier across workgroups).
struct GridTeam {
  DevState* st;
  int* s_ok;
  __device__ int id() const { return blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); }
  __device__ int size() const { return gridDim.x * (blockDim.x >> 6); }
  __device__ bool sync() const {
    if (grid_barrier(&st->bar, s_ok)) return true;
    if (threadIdx.x == 0)
      __hip_atomic_fetch_or(&st->flags, (uint32_t)RSVD_FLAG_SYNC_TIMEOUT, __ATOMIC_RELAXED,
                            __HIP_MEMORY_SCOPE_AGENT);
    return false;
  }
};

template <class Team>
__device__ bool tiled_inverse(const Team& tm, const TileCtx& cx, const double* W, double* Xg,
                              double* S) {
  const int wave = tm.id();
  const int nw = tm.size();
  const int nb = cx.nb;
  constexpr int KB = 4;
  for (int bs = 1; bs < nb; bs *= 2) {
    for (int phase = 0; phase < 2; phase++) {
      // enumerate the output tiles (i, j) of all block pairs of this level
      int count = 0;
      for (int a = 0; a + bs < nb; a += 2 * bs) {
        const int b1 = a + bs, b2 = min(a + 2 * bs, nb);
        count += bs * (b2 - b1);
      }
      for (int t = wave; t < count; t += nw) {
        int a = 0, rem = t, b1 = 0, b2 = 0;
        for (;; a += 2 * bs) {
          b1 = a + bs;
          b2 = min(a + 2 * bs, nb);
          const int c = bs * (b2 - b1);
          if (rem < c) break;
          rem -= c;
        }
        const int i = a + rem / (b2 - b1), j = b1 + rem % (b2 - b1);
        d4 acc = {0.0, 0.0, 0.0, 0.0};
        // phase 0: T_ij = sum_{k in [b1, j]} R_ik X_kj ; phase 1: X_ij = -sum_{k in [i, b1)} X_ik T_kj
        const int k0 = phase == 0 ? b1 : i;
        const int k1 = phase == 0 ? j + 1 : b1;
        for (int kb = k0; kb < k1; kb += KB) {
          double ta[KB][4], tb[KB][4];
#pragma unroll
          for (int q = 0; q < KB; q++) {
            if (kb + q < k1) {
              load_tile_a(cx, phase == 0 ? W : Xg, i, kb + q, ta[q]);
              load_tile(cx, phase == 0 ? Xg : S, kb + q, j, tb[q]);
            }
          }
#pragma unroll
          for (int q = 0; q < KB; q++) {
            if (kb + q < k1) {
#pragma unroll
              for (int s = 0; s < 4; s++) acc = mfma_f64_16x16x4(ta[q][s], tb[q][s], acc);
            }
          }
        }
        double o[4];
#pragma unroll
        for (int it = 0; it < 4; it++) o[it] = phase == 0 ? acc[it] : -acc[it];
        store_tile(cx, phase == 0 ? S : Xg, i, j, o);
      }
      if (!tm.sync()) return false;
    }
  }
  return true;
}

// ---------------------------------------------------------------------------
// The Cholesky for l <= 272 by one workgroup with the off-diagonal tiles of
// the upper triangle resident in registers (tile t of the row-major strict
// upper triangle in slot t / 8 of wave t % 8) and the diagonal tiles in LDS.
// Block row k:
//   every wave factors the (updated) diagonal tile k itself: R_kk and
//     Z_kk = R_kk^{-T} together (tile_chol_inv), Z_kk through a private LDS
//     tile into the operand layout
//   its tiles of row k: R_kJ = Z_kk G_kJ, into the LDS panel and to R
//   barrier
//   its tiles with I > k: G_IJ -= R_kI^T R_kJ; diagonal tiles d > k (d mod 8
//     = wave): G_dd -= R_kd^T R_kd in LDS
//   barrier
// The factorization is computed redundantly by every wave (identical inputs
// and instructions, so identical results and decisions), which avoids a
// third barrier and a broadcast per block row; its 16-column chain is the
// only serial part. Only the diagonal tiles of Rinv are formed (what the
// triangular solve of the QR uses); the strictly lower tiles of R and Rinv
// are cleared. Pivot checks, shift and retries as in chol_grid_kernel.
// ---------------------------------------------------------------------------
// max(e, d) for d >= 0 that turns a NaN d into infinity (fmax would drop it)
__device__ __forceinline__ double dev_max(double e, double d) {
  return d <= e ? e : (d == d ? d : INFINITY);
}

// First-order factor of a near-identity Gram on the grid path (the rule of
// chol_reg_kernel; the neglected terms are at most l 2^-66 <= 5.6e-17 for
// l <= 4096, below the unit roundoff): st->gram_dev is cleared (or set to infinity
// when the pass is skipped), raised to max |G - I| by every workgroup, and
// read by the writer and by chol_grid_kernel, which returns at once when the
// first-order factor stands.
constexpr double kNearIdentity = 0x1p-33;

__global__ void gram_dev_clear_kernel(int only_if_shifted, DevState* st) {
  if (threadIdx.x == 0 && blockIdx.x == 0)
    st->gram_dev = (only_if_shifted && st->qr_shifted == 0) ? INFINITY : 0.0;
}

__global__ void __launch_bounds__(256) gram_dev_kernel(int l, const double* __restrict__ G,
                                                       DevState* st) {
  __shared__ double red[4];
  if (st->gram_dev == INFINITY) return;
  const int64_t tot = (int64_t)l * l;
  double e = 0.0;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < tot;
       x += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = x / l, c = x - i * l;
    e = dev_max(e, fabs(G[x] - (i == c ? 1.0 : 0.0)));
  }
  e = wave_max(e);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = e;
  __syncthreads();
  if (threadIdx.x == 0) {
    e = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    // non-negative doubles order as their bit patterns
    atomicMax(reinterpret_cast<unsigned long long*>(&st->gram_dev),
              (unsigned long long)__double_as_longlong(e));
  }
}

// R = I + X and R^-1 = I - X (the full upper triangle) when the Gram is
// within kNearIdentity of the identity; nothing otherwise
__global__ void __launch_bounds__(256) gram_first_order_kernel(int l, const double* __restrict__ G,
                                                               double* __restrict__ R,
                                                               double* __restrict__ Rinv,
                                                               const DevState* st) {
  if (!(st->gram_dev <= kNearIdentity)) return;
  const int64_t tot = (int64_t)l * l;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < tot;
       x += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = x / l, c = x - i * l;
    const double v = G[x];
    R[x] = i < c ? v : (i == c ? 0.5 * (1.0 + v) : 0.0);
    Rinv[x] = i < c ? -v : (i == c ? 0.5 * (3.0 - v) : 0.0);
  }
}

constexpr int kCholRegMaxNB = 17;
constexpr int kCholRegWaves = 8;
constexpr int kCholRegSlots =
    (kCholRegMaxNB * (kCholRegMaxNB - 1) / 2 + kCholRegWaves - 1) / kCholRegWaves;  // 17

__global__ void __launch_bounds__(64 * kCholRegWaves) chol_reg_kernel(
    int l, const double* __restrict__ G, double* __restrict__ R, double* __restrict__ Rinv,
    int64_t m, int pass, int only_if_shifted, DevState* st) {
  constexpr int kPs = 16 * kCholRegMaxNB + 1;
  __shared__ double panel[16 * kPs];
  // diagonal tiles: item it of lane x of tile d at [256 d + 64 it + x]
  __shared__ double diag[kCholRegMaxNB * 256];
  __shared__ double zl[4][16 * 17];  // Z_kk of waves 0..3, row-major
  __shared__ double rowbuf[4][32];  // current row of R_kk and Z_kk, waves 0..3
  __shared__ double red[kCholRegWaves];
  __shared__ int s_flag;
  __shared__ double s_range[2];
  if (only_if_shifted && st->qr_shifted == 0) return;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
  if (pass > 0) {
    // a re-orthogonalization pass whose Gram is within eps = 2^-33 of the
    // identity (G = I + E, |E_ij| <= eps): R = I + X with X the strict upper
    // triangle of E plus half its diagonal, and R^-1 = I - X, both to first
    // order; the neglected terms (X^T X, X^2) are at most l eps^2 <= 4e-18
    // for l <= 272, below the rounding of the exact factorization. Only the
    // diagonal tiles of R^-1 are formed, as below.
    double e = 0.0;
    for (int i = wave; i < l; i += kCholRegWaves)
      for (int c = lane; c < l; c += 64)
        e = dev_max(e, fabs(G[(int64_t)i * l + c] - (i == c ? 1.0 : 0.0)));
    e = wave_max(e);
    if (lane == 0) red[wave] = e;
    __syncthreads();
    double emax = 0.0;
#pragma unroll
    for (int w = 0; w < kCholRegWaves; w++) emax = fmax(emax, red[w]);
    if (emax <= kNearIdentity) {
      for (int i = wave; i < l; i += kCholRegWaves) {
        for (int c = lane; c < l; c += 64) {
          const int64_t x = (int64_t)i * l + c;
          const double v = G[x];
          R[x] = i < c ? v : (i == c ? 0.5 * (1.0 + v) : 0.0);
          if (i / 16 == c / 16)
            Rinv[x] = i < c ? -v : (i == c ? 0.5 * (3.0 - v) : 0.0);
          else if (i > c)
            Rinv[x] = 0.0;
        }
      }
      return;
    }
    __syncthreads();  // red is reused by the trace sum below
  }
  TileCtx cx;
  cx.l = l;
  cx.nb = (l + 15) / 16;
  cx.ps = kPs;
  const int nb = cx.nb;
  const int noff = nb * (nb - 1) / 2;

  // slot coordinates (I << 8 | J), -1 for an empty slot; wave-uniform
  int crd[kCholRegSlots];
  {
    int t = wave, I = 0, J = 1, cur = 0;  // (I, J): tile `cur` of the strict upper triangle
#pragma unroll
    for (int s = 0; s < kCholRegSlots; s++) {
      if (t < noff) {
        while (cur < t) {
          cur++;
          if (++J >= nb) {
            I++;
            J = I + 1;
          }
        }
        crd[s] = I << 8 | J;
      } else {
        crd[s] = -1;
      }
      t += kCholRegWaves;
    }
  }

  double tr = 0.0;
  for (int i = threadIdx.x; i < l; i += blockDim.x) tr += G[(int64_t)i * l + i];
  tr = block_sum(tr, red);
  const double shift = 11.0 * ((double)m * l + (double)l * (l + 1)) * kUnitRoundoff * tr;
  const double clampv = fmax(shift, 1e-300);

  bool use_shift = pass == 0 && st->prefer_shift != 0u, clamp = false;
  if (use_shift && threadIdx.x == 0) st->qr_shifted = 1;
  d4 tl[kCholRegSlots];  // one MFMA accumulator per slot
  // barrier for LDS traffic only: the stores of R and Rinv are not read in
  // this kernel, so the waves do not wait for them at every block row
  auto lds_barrier = [] {
    asm volatile("" ::: "memory");
    wait_vm_lgkm<63, 0>();
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
  };
  for (int attempt = 0; attempt < 3; attempt++) {
    double dmax = 0.0, dmin = INFINITY;
    if (threadIdx.x == 0) s_flag = 0;
    // off-diagonal tiles of G (zero beyond l): a uniform base per tile and
    // one lane offset for all
#pragma unroll
    for (int s = 0; s < kCholRegSlots; s++) {
      crd[s] = __builtin_amdgcn_readfirstlane(crd[s]);
      asm volatile("" : "+s"(crd[s]));
      if (crd[s] >= 0) {
        const int I = crd[s] >> 8, J = crd[s] & 255;
        const double* base = G + (int64_t)16 * I * l + 16 * J;
        if (16 * I + 16 <= l && 16 * J + 16 <= l) {
#pragma unroll
          for (int it = 0; it < 4; it++) tl[s][it] = base[(g + 4 * it) * l + r];
        } else {
#pragma unroll
          for (int it = 0; it < 4; it++) {
            const int i = 16 * I + g + 4 * it, c = 16 * J + r;
            tl[s][it] = cx.in(i, c) ? base[(g + 4 * it) * l + r] : 0.0;
          }
        }
      }
    }
    // diagonal tiles of G (+ shift; identity beyond l)
    for (int d = wave; d < nb; d += kCholRegWaves) {
#pragma unroll
      for (int it = 0; it < 4; it++) {
        const int i = 16 * d + g + 4 * it, c = 16 * d + r;
        double v = cx.in(i, c) ? G[(int64_t)i * l + c] : (i == c ? 1.0 : 0.0);
        if (use_shift && i == c && i < l) v += shift;
        diag[256 * d + 64 * it + lane] = v;
      }
    }
    lds_barrier();
    bool failed = false;
    for (int k = 0; k < nb; k++) {
      // opaque per-step copies of the slot coordinates, the lane and l: keeps
      // the compiler from hoisting per-slot addresses and lane masks out of
      // this loop (hundreds of them would stay live beside the tiles)
      int ln = lane, lk = l;
      asm volatile("" : "+v"(ln));
      asm volatile("" : "+s"(lk));
      const int rr = ln & 15, gg = ln >> 4;
      TileCtx ck = cx;
      ck.l = lk;
#pragma unroll
      for (int s = 0; s < kCholRegSlots; s++) {
        crd[s] = __builtin_amdgcn_readfirstlane(crd[s]);
        asm volatile("" : "+s"(crd[s]));
      }
      // ---- diagonal tile k: waves 0..3 (one per SIMD) factor it, each into
      // its own LDS copy of Z_kk (identical), which the waves sharing its
      // SIMD read after the barrier
      if (wave < 4) {
        d4 t, z;
#pragma unroll
        for (int it = 0; it < 4; it++) t[it] = diag[256 * k + 64 * it + ln];
        const bool ok = tile_chol_inv(t, z, rowbuf[wave], clamp, clampv, 16 * k, lk, dmax, dmin);
        if (wave == 0) {
          double o[4] = {t[0], t[1], t[2], t[3]};
          store_tile(ck, R, k, k, o);
#pragma unroll
          for (int it = 0; it < 4; it++) {
            // X = Z^T: lane (r, g) item it holds x_{r, g + 4 it}
            const int i = 16 * k + rr, c = 16 * k + gg + 4 * it;
            if (ck.in(i, c)) Rinv[(int64_t)i * lk + c] = z[it];
          }
          if (!ok && ln == 0) s_flag = 1;
        }
        // Z_kk into the operand layout through this wave's LDS tile
#pragma unroll
        for (int it = 0; it < 4; it++) zl[wave][(gg + 4 * it) * 17 + rr] = z[it];
      }
      lds_barrier();
      // ---- this wave's tiles of block row k: R_kJ = Z_kk G_kJ
#pragma unroll
      for (int s = 0; s < kCholRegSlots; s++) {
        if (crd[s] >= 0 && (crd[s] >> 8) == k) {
          const int J = crd[s] & 255;
          d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
          for (int s4 = 0; s4 < 4; s4++)
            acc = mfma_f64_16x16x4(zl[wave & 3][rr * 17 + 4 * s4 + gg], tl[s][s4], acc);
          tl[s] = acc;
          double o[4];
#pragma unroll
          for (int it = 0; it < 4; it++) {
            o[it] = acc[it];
            panel[(gg + 4 * it) * kPs + 16 * J + rr] = acc[it];
          }
          store_tile(ck, R, k, J, o);
        }
      }
      lds_barrier();
      failed = s_flag != 0;
      if (failed) break;
      // ---- trailing tiles
#pragma unroll
      for (int s = 0; s < kCholRegSlots; s++) {
        if (crd[s] >= 0 && (crd[s] >> 8) > k) {
          const int I = crd[s] >> 8, J = crd[s] & 255;
#pragma unroll
          for (int s4 = 0; s4 < 4; s4++) {
            const double a = -panel[(4 * s4 + gg) * kPs + 16 * I + rr];
            const double b = panel[(4 * s4 + gg) * kPs + 16 * J + rr];
            tl[s] = mfma_f64_16x16x4(a, b, tl[s]);
          }
        }
      }
      for (int d = k + 1 + mod_pos(wave - k - 1, kCholRegWaves); d < nb; d += kCholRegWaves) {
        d4 acc;
#pragma unroll
        for (int it = 0; it < 4; it++) acc[it] = diag[256 * d + 64 * it + ln];
#pragma unroll
        for (int s4 = 0; s4 < 4; s4++) {
          const double b = panel[(4 * s4 + gg) * kPs + 16 * d + rr];
          acc = mfma_f64_16x16x4(-b, b, acc);
        }
#pragma unroll
        for (int it = 0; it < 4; it++) diag[256 * d + 64 * it + ln] = acc[it];
      }
      // strictly lower tiles of tile row k of R and Rinv (16 rows, 16 k columns)
      const int rows = min(16, lk - 16 * k), cols = 16 * k;
      for (int i = wave; i < rows; i += kCholRegWaves) {
        double* rR = R + (int64_t)(16 * k + i) * lk;
        double* rX = Rinv + (int64_t)(16 * k + i) * lk;
        for (int c = ln; c < cols; c += 64) {
          rR[c] = 0.0;
          rX[c] = 0.0;
        }
      }
      lds_barrier();
    }
    if (wave == 0 && lane == 0) {
      s_range[0] = dmax;
      s_range[1] = dmin;
    }
    __syncthreads();
    if (clamp) break;
    bool ok = !failed;
    if (ok && pass == 0 && !use_shift && s_range[0] > 1e5 * s_range[1]) ok = false;
    if (ok) break;
    if (use_shift || pass == 2) {
      if (threadIdx.x == 0) st->qr_householder = 1;
      clamp = true;
      use_shift = true;
    } else {
      use_shift = true;
      if (threadIdx.x == 0) st->qr_shifted = 1;
    }
    __syncthreads();
  }
  if (pass == 0 && threadIdx.x == 0) st->prefer_shift = use_shift ? 1u : 0u;
}

// ---------------------------------------------------------------------------
// The same Cholesky and inverse spread over a grid of workgroups (large l),
// in super-steps of 32 rows (two tile rows, 2K and 2K+1):
//   row      R_{2K,J} = X_00^T G_{2K,J};  R_{2K+1,J} = X_11^T (G_{2K+1,J} -
//            R_01^T R_{2K,J}) for every tile column J beyond the block
//            (forward substitution with the diagonal block [R_00 R_01; 0 R_11]
//            and the inverses X_00, X_11 of its diagonal tiles)
//   trailing G_IJ -= R_{2K,I}^T R_{2K,J} + R_{2K+1,I}^T R_{2K+1,J}
// with the next diagonal block updated and factored by one wave as soon as
// its three tiles are done (look-ahead), so a super-step has two grid
// barriers. Every wave of the grid takes tiles; the 32-row panel lives in
// global scratch. A tile count that is odd is padded with an identity tile.
// Decisions (breakdown, pivot spread, retries) are uniform across the grid.
// ---------------------------------------------------------------------------

// Pivot bookkeeping of one factored diagonal tile (lane 0 of the wave; one
// writer per super-step).
__device__ __forceinline__ void note_pivots(bool ok, double dmax, double dmin, DevState* st) {
  if ((threadIdx.x & 63) == 0) {
    if (!ok) st->chol_fail = 1u;
    if (dmax > st->piv_max) st->piv_max = dmax;
    if (dmin < st->piv_min) st->piv_min = dmin;
  }
}

// Factor the updated 32 x 32 diagonal block of super-step K held by one wave
// (t00, t01, t11 in the accumulator layout): R_00, R_01, R_11 to W and the
// inverses X_00, X_11 to Xg. Each diagonal tile is factored together with
// Z = R^{-T} (tile_chol_inv: the inverse costs a few FMAs per pivot instead
// of a second 16-step substitution); Z holds X^T in the accumulator layout,
// so X is stored transposed and turned into the operand layout of
//   R_01 = X_00^T t01 (the accumulator layout of x00 is the operand it needs)
// through the wave's 16 x 17 LDS tile zl (rowbuf: 32 doubles, the factor's
// row broadcast). Then t11 -= R_01^T R_01 and R_11 = chol(t11).
struct Tiles3 {
  double t00[4], t01[4], t11[4];
};

// X (entry (g + 4 it, r) of the accumulator layout) from Z = X^T held in
// the same layout, through the wave's LDS tile.
__device__ __forceinline__ void tile_transpose(const d4& z, double x[4], double* zl) {
  const int lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
#pragma unroll
  for (int it = 0; it < 4; it++) zl[(g + 4 * it) * 17 + r] = z[it];
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int it = 0; it < 4; it++) x[it] = zl[r * 17 + g + 4 * it];
  __builtin_amdgcn_wave_barrier();
}

// Store Z = X^T of diagonal tile k as X (entries beyond l are not stored).
__device__ __forceinline__ void store_tile_t(const TileCtx& cx, double* W, int k, const d4& z) {
  const int lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
#pragma unroll
  for (int it = 0; it < 4; it++) {
    const int i = 16 * k + r, c = 16 * k + g + 4 * it;
    if (cx.in(i, c)) W[(int64_t)i * cx.l + c] = z[it];
  }
}

// Not inlined: its unrolled chains would otherwise share the register
// budget of the grid kernel's trailing loop (and spill it).
__device__ __noinline__ void grid_block_factor(TileCtx cx, Tiles3 tb, int K, double* W, double* Xg,
                                               bool clamp, double clampv, DevState* st,
                                               double* lds) {
  double* zl = lds;             // 16 x 17
  double* rowbuf = lds + 272;   // 32
  const int i0 = 2 * K, i1 = 2 * K + 1;
  double dmax = 0.0, dmin = INFINITY, x00[4];
  d4 t0 = {tb.t00[0], tb.t00[1], tb.t00[2], tb.t00[3]}, z0;
  bool ok = tile_chol_inv(t0, z0, rowbuf, clamp, clampv, 16 * i0, cx.l, dmax, dmin);
  tile_transpose(z0, x00, zl);
  d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int s4 = 0; s4 < 4; s4++) acc = mfma_f64_16x16x4(x00[s4], tb.t01[s4], acc);
  double r01[4] = {acc[0], acc[1], acc[2], acc[3]};
  d4 upd = {tb.t11[0], tb.t11[1], tb.t11[2], tb.t11[3]};
#pragma unroll
  for (int s4 = 0; s4 < 4; s4++) upd = mfma_f64_16x16x4(-r01[s4], r01[s4], upd);
  d4 z1;
  ok = tile_chol_inv(upd, z1, rowbuf, clamp, clampv, 16 * i1, cx.l, dmax, dmin) && ok;
  const double r00[4] = {t0[0], t0[1], t0[2], t0[3]};
  const double r11[4] = {upd[0], upd[1], upd[2], upd[3]};
  store_tile(cx, W, i0, i0, r00);
  store_tile(cx, W, i0, i1, r01);
  store_tile(cx, W, i1, i1, r11);
  store_tile_t(cx, Xg, i0, z0);
  store_tile_t(cx, Xg, i1, z1);
  note_pivots(ok, dmax, dmin, st);
}

// Entry (row, col) of the inverse diagonal tile k (identity beyond l).
__device__ __forceinline__ double xdiag(const TileCtx& cx, const double* Xg, int k, int row,
                                        int col) {
  const int i = 16 * k + row, c = 16 * k + col;
  return cx.in(i, c) ? Xg[(int64_t)i * cx.l + c] : (row == col ? 1.0 : 0.0);
}

// Scratch (doubles) of the grid Cholesky's 32-row panel.
__host__ __device__ __forceinline__ int64_t grid_panel_ld(int64_t l) {
  const int64_t nb = (l + 15) / 16;
  return 16 * (nb + (nb & 1)) + 1;
}

// 256 threads: one wave per SIMD, so each wave may use the whole register
// file (the 32-row trailing batch needs ~330 registers; at 512 threads a
// wave is limited to 256 and the kernel spills).
__global__ void __launch_bounds__(256) chol_grid_kernel(int l, double* __restrict__ G,
                                                         double* __restrict__ R,
                                                         double* __restrict__ Rinv,
                                                         double* __restrict__ panel, int64_t m,
                                                         int pass, int only_if_shifted,
                                                         int full_inverse, DevState* st) {
  __shared__ double red[256 / 64];
  __shared__ double flds[272 + 32];  // the factor wave's transpose tile and row buffer
  __shared__ int s_ok;
  if (only_if_shifted && st->qr_shifted == 0) return;
  // a re-orthogonalization pass already factored to first order
  if (pass > 0 && st->gram_dev <= kNearIdentity) return;
  const GridTeam tm{st, &s_ok};
  const int gw = tm.id(), TW = tm.size();
  const int lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
  TileCtx cx;
  cx.l = l;
  cx.nb = (l + 15) / 16;
  cx.ps = (int)grid_panel_ld(l);
  const int nbe = cx.nb + (cx.nb & 1);  // tiles, padded to an even count
  const int nsup = nbe / 2;
  const int ps = cx.ps;
  const int64_t ll = (int64_t)l * l;
  const int64_t gthreads = (int64_t)gridDim.x * blockDim.x;
  const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;

  // every workgroup forms the same trace (same entries, same order)
  double tr = 0.0;
  for (int i = threadIdx.x; i < l; i += blockDim.x) tr += G[(int64_t)i * l + i];
  tr = block_sum(tr, red);
  const double shift = 11.0 * ((double)m * l + (double)l * (l + 1)) * kUnitRoundoff * tr;
  const double clampv = fmax(shift, 1e-300);

  // a panel of the same run already needed the shift: start shifted
  bool use_shift = pass == 0 && st->prefer_shift != 0u, clamp = false;
  if (use_shift && gw == 0 && lane == 0) st->qr_shifted = 1;
  for (int attempt = 0; attempt < 3; attempt++) {
    if (gw == 0 && lane == 0) {
      st->chol_fail = 0u;
      st->piv_max = 0.0;
      st->piv_min = INFINITY;
    }
    for (int64_t e = gtid; e < ll; e += gthreads) {
      double v = G[e];
      if (use_shift && (e / l) == (e % l)) v += shift;
      R[e] = v;
    }
    if (!tm.sync()) return;
    if (gw == 0) {
      Tiles3 tb;
      load_tile(cx, R, 0, 0, tb.t00);
      load_tile(cx, R, 0, 1, tb.t01);
      load_tile(cx, R, 1, 1, tb.t11);
      grid_block_factor(cx, tb, 0, R, Rinv, clamp, clampv, st, flds);
    }
    if (!tm.sync()) return;
    bool failed = __hip_atomic_load(&st->chol_fail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u;
    for (int K = 0; K < nsup && !failed; K++) {
      const int i0 = 2 * K, i1 = 2 * K + 1;
      // block row: the two tile rows of the block against every later column
      for (int J = i1 + 1 + gw; J < nbe; J += TW) {
        double g0[4], g1[4], w01[4];
        load_tile(cx, R, i0, J, g0);
        load_tile(cx, R, i1, J, g1);
        load_tile(cx, R, i0, i1, w01);
        d4 a0 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s4 = 0; s4 < 4; s4++) a0 = mfma_f64_16x16x4(xdiag(cx, Rinv, i0, 4 * s4 + g, r), g0[s4], a0);
        double r0[4] = {a0[0], a0[1], a0[2], a0[3]};
        d4 a1 = {g1[0], g1[1], g1[2], g1[3]};
#pragma unroll
        for (int s4 = 0; s4 < 4; s4++) a1 = mfma_f64_16x16x4(-w01[s4], r0[s4], a1);
        double h1[4] = {a1[0], a1[1], a1[2], a1[3]};
        d4 a2 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s4 = 0; s4 < 4; s4++) a2 = mfma_f64_16x16x4(xdiag(cx, Rinv, i1, 4 * s4 + g, r), h1[s4], a2);
        double r1[4] = {a2[0], a2[1], a2[2], a2[3]};
        store_tile(cx, R, i0, J, r0);
        store_tile(cx, R, i1, J, r1);
#pragma unroll
        for (int it = 0; it < 4; it++) {
          panel[(g + 4 * it) * ps + 16 * J + r] = r0[it];
          panel[(16 + g + 4 * it) * ps + 16 * J + r] = r1[it];
        }
      }
      if (!tm.sync()) return;
      // trailing update of the tiles beyond the block (upper triangle)
      const int n = nbe - i1 - 1;
      if (n > 0) {
        const int first = i1 + 1;
        // wave 0 of the grid: the next diagonal block, then its factorization
        if (gw == 0) {
          Tiles3 tb;
          double* dst[3] = {tb.t00, tb.t01, tb.t11};
          const int bi[3] = {first, first, first + 1}, bj[3] = {first, first + 1, first + 1};
#pragma unroll
          for (int q = 0; q < 3; q++) {
            double t[4];
            load_tile(cx, R, bi[q], bj[q], t);
            d4 acc = {t[0], t[1], t[2], t[3]};
#pragma unroll
            for (int h = 0; h < 2; h++)
#pragma unroll
              for (int s4 = 0; s4 < 4; s4++) {
                const double a = -panel[(16 * h + 4 * s4 + g) * ps + 16 * bi[q] + r];
                const double bb = panel[(16 * h + 4 * s4 + g) * ps + 16 * bj[q] + r];
                acc = mfma_f64_16x16x4(a, bb, acc);
              }
#pragma unroll
            for (int it = 0; it < 4; it++) dst[q][it] = acc[it];
          }
          grid_block_factor(cx, tb, K + 1, R, Rinv, clamp, clampv, st, flds);
        }
        // every other wave: the remaining tiles, TB at a time so their L2
        // round trips overlap
        const int T = n * (n + 1) / 2;
        constexpr int TB = 4;
        if (gw > 0) {
          for (int t0 = (gw - 1) * TB; t0 < T; t0 += (TW - 1) * TB) {
            int Is[TB], Js[TB];
            double tl[TB][4];
            int I, J;
            trailing_coords(t0, n, I, J);
#pragma unroll
            for (int q = 0; q < TB; q++) {
              Is[q] = I + first;
              Js[q] = J + first;
              if (++J >= n) {
                I++;
                J = I;
              }
            }
#pragma unroll
            for (int q = 0; q < TB; q++) {
              // the next diagonal block belongs to wave 0
              const bool mine = t0 + q < T && !(Is[q] <= first + 1 && Js[q] <= first + 1);
              if (mine) load_tile(cx, R, Is[q], Js[q], tl[q]);
            }
#pragma unroll
            for (int q = 0; q < TB; q++) {
              const bool mine = t0 + q < T && !(Is[q] <= first + 1 && Js[q] <= first + 1);
              if (mine) {
                d4 acc = {tl[q][0], tl[q][1], tl[q][2], tl[q][3]};
#pragma unroll
                for (int h = 0; h < 2; h++)
#pragma unroll
                  for (int s4 = 0; s4 < 4; s4++) {
                    const double a = -panel[(16 * h + 4 * s4 + g) * ps + 16 * Is[q] + r];
                    const double bb = panel[(16 * h + 4 * s4 + g) * ps + 16 * Js[q] + r];
                    acc = mfma_f64_16x16x4(a, bb, acc);
                  }
                double o[4] = {acc[0], acc[1], acc[2], acc[3]};
                store_tile(cx, R, Is[q], Js[q], o);
              }
            }
          }
        }
      }
      if (!tm.sync()) return;
      failed = __hip_atomic_load(&st->chol_fail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u;
    }
    if (clamp) break;
    bool ok = !failed;
    if (ok && pass == 0 && !use_shift && st->piv_max > 1e5 * st->piv_min) ok = false;
    if (ok) break;
    if (use_shift || pass == 2) {
      // breakdown even with the shift (or in the last pass): numerically
      // rank-deficient panel
      if (gw == 0 && lane == 0) st->qr_householder = 1;
      clamp = true;
      use_shift = true;
    } else {
      use_shift = true;
      if (gw == 0 && lane == 0) st->qr_shifted = 1;
    }
    // every workgroup has read this attempt's outcome before the next resets it
    if (!tm.sync()) return;
  }
  if (pass == 0 && gw == 0 && lane == 0) st->prefer_shift = use_shift ? 1u : 0u;
  // G is no longer read: it serves as scratch for the inverse (without
  // full_inverse only the diagonal tiles of Rinv are valid)
  if (full_inverse && !tiled_inverse(tm, cx, R, Rinv, G)) return;
  for (int64_t e = gtid; e < ll; e += gthreads) {
    if (e / l > e % l) {
      R[e] = 0.0;
      Rinv[e] = 0.0;
    }
  }
}

// ---------------------------------------------------------------------------
// The Householder fallback spread over a grid of workgroups (panels too large
// for one workgroup). Workgroup w owns a contiguous range of rows. Column j of
// the factorization:
//   partial  part[w][c] = sum over its rows i > j of W[i][j] W[i][c], c >= j
//            (c = j: the squared norm below the diagonal)
//   reduce   every workgroup forms the same reflector (beta, tau, scale) from
//            the same sum; workgroup c mod G finishes column c > j:
//            d_c = tau (W[j][c] + scale u_c) into dfin[c], W[j][c] -= d_c
//   update   its rows i > j: W[i][c] -= d_c scale W[i][j], then v_i = scale W[i][j]
// with a grid barrier after the partial and after the reduce; the explicit Q
// is accumulated backwards the same way. The arithmetic is that of
// householder_kernel with the row sums split by workgroup. part: G l + l
// doubles of scratch; tau_buf[j] = tau_j, tau_buf[l + j] = beta_j.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) householder_grid_kernel(int64_t rows, int l,
                                                                const double* __restrict__ Yorig,
                                                                double* __restrict__ Y,
                                                                double* __restrict__ R,
                                                                double* __restrict__ tau_buf,
                                                                double* __restrict__ part,
                                                                DevState* st) {
  __shared__ int s_ok;
  if (st->qr_householder == 0) return;
  const GridTeam tm{st, &s_ok};
  const int G = (int)gridDim.x, w = (int)blockIdx.x;
  const int64_t per = (rows + G - 1) / G;
  const int64_t r0 = min(rows, (int64_t)w * per), r1 = min(rows, r0 + per);
  double* dfin = part + (int64_t)G * l;
  double* W = Y;
  const int64_t tot = rows * l;
  const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t gthreads = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = gtid; e < tot; e += gthreads) W[e] = Yorig[e];
  if (!tm.sync()) return;
  for (int j = 0; j < l; j++) {
    const int64_t i0 = max(r0, (int64_t)j + 1);
    for (int c = j + threadIdx.x; c < l; c += blockDim.x) {
      double acc = 0.0;
      for (int64_t i = i0; i < r1; i++) acc += W[i * l + j] * W[i * l + c];
      part[(int64_t)w * l + c] = acc;
    }
    if (!tm.sync()) return;
    double s2 = 0.0;
    for (int v = 0; v < G; v++) s2 += part[(int64_t)v * l + j];
    const double alpha = W[(int64_t)j * l + j];
    double beta, tau, scale;
    if (s2 == 0.0) {
      beta = alpha;
      tau = 0.0;
      scale = 0.0;
    } else {
      const double nrm = sqrt(alpha * alpha + s2);
      beta = alpha >= 0.0 ? -nrm : nrm;
      tau = (beta - alpha) / beta;
      scale = 1.0 / (alpha - beta);
    }
    {
      const int first = j + 1 + ((w - (j + 1)) % G + G) % G;  // smallest c > j with c = w (mod G)
      for (int c = first + G * (int)threadIdx.x; c < l; c += G * (int)blockDim.x) {
        double u = 0.0;
        for (int v = 0; v < G; v++) u += part[(int64_t)v * l + c];
        const double d = tau * (W[(int64_t)j * l + c] + scale * u);
        dfin[c] = d;
        W[(int64_t)j * l + c] -= d;
      }
    }
    if (w == j % G && threadIdx.x == 0) {
      tau_buf[j] = tau;
      tau_buf[l + j] = beta;
    }
    if (!tm.sync()) return;
    for (int c = j + 1 + threadIdx.x; c < l; c += blockDim.x) {
      const double d = dfin[c] * scale;
      for (int64_t i = i0; i < r1; i++) W[i * l + c] -= d * W[i * l + j];
    }
    __syncthreads();
    for (int64_t i = i0 + threadIdx.x; i < r1; i += blockDim.x) W[i * l + j] *= scale;
    if (threadIdx.x == 0 && j >= r0 && j < r1) W[(int64_t)j * l + j] = beta;
    __syncthreads();
  }
  if (!tm.sync()) return;
  // R = upper(W) with diag(R) >= 0 (rows of R and columns of Q flip together)
  if (R) {
    for (int64_t e = gtid; e < (int64_t)l * l; e += gthreads) {
      const int i = (int)(e / l), c = (int)(e % l);
      const double v = W[(int64_t)i * l + c];
      R[e] = (c >= i) ? (tau_buf[l + i] < 0.0 ? -v : v) : 0.0;
    }
  }
  if (!tm.sync()) return;
  // Q = H_0 ... H_{l-1} [I; 0], backwards; rows > j of column j hold v_j
  for (int j = l - 1; j >= 0; j--) {
    const double tau = tau_buf[j];
    const int64_t i0 = max(r0, (int64_t)j + 1);
    for (int c = j + 1 + threadIdx.x; c < l; c += blockDim.x) {
      double acc = 0.0;
      for (int64_t i = i0; i < r1; i++) acc += W[i * l + j] * W[i * l + c];
      part[(int64_t)w * l + c] = acc;
    }
    if (!tm.sync()) return;
    {
      const int first = j + 1 + ((w - (j + 1)) % G + G) % G;
      for (int c = first + G * (int)threadIdx.x; c < l; c += G * (int)blockDim.x) {
        double u = 0.0;
        for (int v = 0; v < G; v++) u += part[(int64_t)v * l + c];
        const double d = tau * u;
        dfin[c] = d;
        W[(int64_t)j * l + c] = -d;  // Q[j][c] is 0 before H_j
      }
    }
    if (!tm.sync()) return;
    for (int c = j + 1 + threadIdx.x; c < l; c += blockDim.x) {
      const double d = dfin[c];
      for (int64_t i = i0; i < r1; i++) W[i * l + c] -= d * W[i * l + j];
    }
    __syncthreads();
    // column j: H_j e_j = e_j - tau v
    for (int64_t i = r0 + threadIdx.x; i < r1; i += blockDim.x) {
      const double x = W[i * l + j];
      W[i * l + j] = i > j ? -tau * x : (i == j ? 1.0 - tau : 0.0);
    }
    __syncthreads();
  }
  if (!tm.sync()) return;
  for (int64_t e = gtid; e < tot; e += gthreads)
    if (tau_buf[l + (int)(e % l)] < 0.0) W[e] = -W[e];
  if (gtid == 0) atomicOr(&st->flags, (uint32_t)RSVD_FLAG_QR_FALLBACK);
}

// ---------------------------------------------------------------------------
// Q = Y R^{-1} for the upper-triangular factor R (l x l, row-major) by block
// forward substitution over 16-column tiles, in transposed form
//   Q_J^T = X_JJ^T (Y_J^T - sum_{K<J} R_KJ^T Q_K^T),   X_JJ = R_JJ^{-1}
// (X_JJ: the diagonal tiles of Xd, written by the factorization). In this
// form the FP64 accumulator layout of a result tile (lane (r, g), item t:
// entry (g + 4 t, r)) is the B-operand layout the later tiles read, so a wave
// keeps the Q^T tiles of its 16 rows in registers (l <= 16 kTrsmMaxNB). The
// workgroup stages R's column block J (rows 0 .. 16 J - 1, 16 columns) in
// LDS, double buffered. Rows past `rows` read as zero and are not stored;
// columns past l act as identity.
// ---------------------------------------------------------------------------
constexpr int kTrsmMaxNB = 20;      // l <= 320: the register budget of the common widths
constexpr int kTrsmMaxNBWide = 38;  // l <= 608: R's two column blocks fill the LDS
constexpr int kTrsmWaves = 4;

struct TrsmCtx {
  int64_t rows, ldy, ldq, ldr, row;
  int l, nb, r, g;
  bool row_ok;
  const double* Y;
  const double* R;
  const double* Xd;
  double* Q;
  double* lds;
};

// Column tile J of the substitution (J a constant, so the register arrays
// are indexed statically).
template <int J, int MAXNB>
__device__ __forceinline__ void trsm_tile(const TrsmCtx& c, double (&qt)[MAXNB][4]) {
  constexpr int kT = 64 * kTrsmWaves;
  constexpr int kU = (256 * (J + 1) + kT - 1) / kT;
  if (J >= c.nb) return;
  const int r = c.r, g = c.g, l = c.l;
  // this thread's share of block J + 1 (rows 0 .. 16 J + 15 of columns
  // 16 (J + 1) ..), loaded now and written to LDS after this block's
  // products, so the loads overlap them
  const bool more = J + 1 < c.nb;
  double nxt[kU];
#pragma unroll
  for (int u = 0; u < kU; u++) {
    const int e = (int)threadIdx.x + kT * u;
    const int i = e >> 4, cc = 16 * (J + 1) + (e & 15);
    nxt[u] = (more && e < 256 * (J + 1) && cc < l) ? c.R[(int64_t)i * c.ldr + cc] : 0.0;
  }
  d4 acc;
  double xa[4];
#pragma unroll
  for (int t = 0; t < 4; t++) {
    const int cc = 16 * J + g + 4 * t;
    acc[t] = (c.row_ok && cc < l) ? c.Y[c.row * c.ldy + cc] : 0.0;
    const int i = 16 * J + g + 4 * t, cd = 16 * J + r;
    xa[t] = (i < l && cd < l) ? c.Xd[(int64_t)i * c.ldr + cd] : (i == cd ? 1.0 : 0.0);
  }
  if constexpr (J > 0) {
    __syncthreads();  // block J written, block J - 1 no longer read
    const double* Rb = c.lds + (size_t)(J & 1) * c.nb * 256;
#pragma unroll
    for (int K = 0; K < J; K++) {
#pragma unroll
      for (int s4 = 0; s4 < 4; s4++)
        acc = mfma_f64_16x16x4(-Rb[(16 * K + g + 4 * s4) * 16 + r], qt[K][s4], acc);
    }
    // LDS reads of the R fragments run six products ahead of their use
    // (masks: 0x100 LDS reads, 0x008 matrix ops)
    constexpr int kPF = 6, kN = 4 * J;
#pragma unroll
    for (int u = 0; u < kPF && u < kN; u++) __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
#pragma unroll
    for (int u = 0; u < kN; u++) {
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
      if (u + kPF < kN) __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
    }
  }
  d4 out = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int s4 = 0; s4 < 4; s4++) out = mfma_f64_16x16x4(xa[s4], acc[s4], out);
#pragma unroll
  for (int t = 0; t < 4; t++) {
    qt[J][t] = out[t];
    const int cc = 16 * J + g + 4 * t;
    if (c.row_ok && cc < l) c.Q[c.row * c.ldq + cc] = out[t];
  }
  // block J + 1 into the other buffer (its last reader, block J - 1,
  // finished before this block's barrier)
  if (more) {
    double* dst = c.lds + (size_t)((J + 1) & 1) * c.nb * 256;
#pragma unroll
    for (int u = 0; u < kU; u++) {
      const int e = (int)threadIdx.x + kT * u;
      if (e < 256 * (J + 1)) dst[e] = nxt[u];
    }
  }
}

template <int MAXNB, int... Js>
__device__ __forceinline__ void trsm_tiles(const TrsmCtx& c, double (&qt)[MAXNB][4],
                                           std::integer_sequence<int, Js...>) {
  (trsm_tile<Js, MAXNB>(c, qt), ...);
}

template <int MAXNB>
__global__ void __launch_bounds__(64 * kTrsmWaves) trsm_upper_kernel(
    int64_t rows, int l, const double* __restrict__ Y, int64_t ldy, const double* __restrict__ R,
    int64_t ldr, const double* __restrict__ Xd, double* __restrict__ Q, int64_t ldq,
    const uint32_t* pred) {
  extern __shared__ double lds[];
  if (pred != nullptr && *pred == 0) return;
  TrsmCtx c;
  c.rows = rows;
  c.ldy = ldy;
  c.ldq = ldq;
  c.l = l;
  c.ldr = ldr;
  c.nb = (l + 15) / 16;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  c.r = lane & 15;
  c.g = lane >> 4;
  c.row = (int64_t)blockIdx.x * (16 * kTrsmWaves) + wave * 16 + c.r;
  c.row_ok = c.row < rows;
  c.Y = Y;
  c.R = R;
  c.Xd = Xd;
  c.Q = Q;
  c.lds = lds;
  double qt[MAXNB][4];
  trsm_tiles<MAXNB>(c, qt, std::make_integer_sequence<int, MAXNB>{});
}

// ---------------------------------------------------------------------------
// Gram matrix G = Y^T Y of a rows x l panel on the FP64 matrix cores, upper
// 16 x 16 tiles only. Workgroup (slab, group) sums the rows of its slab for
// up to kGramWaves x kGramSlots upper tiles (tile t of the upper triangle,
// row-major, goes to wave t mod kGramWaves, slot t / kGramWaves of its
// group). Both MFMA operands of tile (I, J) are 4-row fragments of the same
// rows (lane (r, g): Y[k + g][16 I + r] and Y[k + g][16 J + r]), read from
// 32-row chunks staged in LDS (double buffered, the next chunk's loads in
// registers while the current one is consumed). Each slab writes its tiles
// to part[slab][t][256]; gram_reduce_kernel sums the slabs in order and
// mirrors the lower triangle.
// ---------------------------------------------------------------------------
constexpr int kGramWaves = 16;
constexpr int kGramSlots = 5;
constexpr int kGramRows = 32;  // rows per LDS chunk (eight 4-row k-steps)
constexpr int kGramMaxNB = 17;  // column tiles (l <= 272): chunk and prefetch sizes

__global__ void __launch_bounds__(64 * kGramWaves) gram_kernel(int64_t rows, int l,
                                                                const double* __restrict__ Y,
                                                                int64_t ldy, int64_t per_slab,
                                                                double* __restrict__ part,
                                                                const uint32_t* pred) {
  extern __shared__ double lds[];
  if (pred != nullptr && *pred == 0) return;
  constexpr int kT = 64 * kGramWaves;
  const int nb = (l + 15) / 16, lp = 16 * nb;
  const int ntiles = nb * (nb + 1) / 2;
  const int slab = blockIdx.x;
  // the wave index as a wave-uniform value: the tile coordinates below stay in scalar registers
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
  const int64_t r0 = (int64_t)slab * per_slab;
  const int64_t r1 = min(rows, r0 + per_slab);
  const int nch = r1 > r0 ? (int)((r1 - r0 + kGramRows - 1) / kGramRows) : 0;
  // this wave's tiles: the LDS column offsets of tile (I, J), 16 I and 16 J,
  // packed in one word (0xffffffff: no tile)
  uint32_t toff[kGramSlots];
  const int t0 = (int)blockIdx.y * kGramWaves * kGramSlots + wave;
#pragma unroll
  for (int q = 0; q < kGramSlots; q++) {
    const int t = t0 + q * kGramWaves;
    int I = 0, J = 0;
    if (t < ntiles) trailing_coords(t, nb, I, J);
    toff[q] = t < ntiles ? (uint32_t)(16 * I) | ((uint32_t)(16 * J) << 16) : 0xffffffffu;
  }
  d4 acc[kGramSlots];
#pragma unroll
  for (int q = 0; q < kGramSlots; q++) acc[q] = d4{0.0, 0.0, 0.0, 0.0};
  // a chunk is kGramRows x lp doubles: nu <= kMaxU per thread (registers)
  constexpr int kMaxU = (kGramRows * 16 * kGramMaxNB + kT - 1) / kT;
  const int nu = (kGramRows * lp + kT - 1) / kT;
  double nxt[kMaxU];
  auto load_chunk = [&](int c) {
#pragma unroll
    for (int u = 0; u < kMaxU; u++) {
      if (u < nu) {
        const int e = (int)threadIdx.x + kT * u;
        const int i = e / lp, col = e % lp;
        const int64_t row = r0 + (int64_t)kGramRows * c + i;
        nxt[u] = (e < kGramRows * lp && row < r1 && col < l) ? Y[row * ldy + col] : 0.0;
      }
    }
  };
  auto store_chunk = [&](int b) {
    double* dst = lds + (size_t)b * kGramRows * lp;
#pragma unroll
    for (int u = 0; u < kMaxU; u++) {
      const int e = (int)threadIdx.x + kT * u;
      if (u < nu && e < kGramRows * lp) dst[e] = nxt[u];
    }
  };
  if (nch > 0) {
    load_chunk(0);
    store_chunk(0);
  }
  for (int c = 0; c < nch; c++) {
    if (c + 1 < nch) load_chunk(c + 1);
    __syncthreads();  // chunk c stored, chunk c - 1 no longer read
    const double* buf = lds + (size_t)(c & 1) * kGramRows * lp;
#pragma unroll
    for (int s4 = 0; s4 < kGramRows / 4; s4++) {
      const double* rowp = buf + (4 * s4 + g) * lp + r;
#pragma unroll
      for (int q = 0; q < kGramSlots; q++) {
        if (toff[q] != 0xffffffffu)
          acc[q] = mfma_f64_16x16x4(rowp[toff[q] & 0xffffu], rowp[toff[q] >> 16], acc[q]);
      }
    }
    if (c + 1 < nch) store_chunk((c + 1) & 1);
  }
#pragma unroll
  for (int q = 0; q < kGramSlots; q++) {
    if (toff[q] != 0xffffffffu) {
      double* dst = part + ((int64_t)slab * ntiles + (t0 + q * kGramWaves)) * 256;
#pragma unroll
      for (int t = 0; t < 4; t++) dst[(g + 4 * t) * 16 + r] = acc[q][t];
    }
  }
}

// G (l x l) = sum over the slabs of part, in slab order; the lower triangle
// mirrored from the upper tiles.
__global__ void __launch_bounds__(256) gram_reduce_kernel(int l, int slabs,
                                                          const double* __restrict__ part,
                                                          double* __restrict__ G,
                                                          const uint32_t* pred) {
  if (pred != nullptr && *pred == 0) return;
  const int nb = (l + 15) / 16;
  const int ntiles = nb * (nb + 1) / 2;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)ntiles * 256) return;
  const int t = (int)(idx / 256), e = (int)(idx % 256);
  // eight independent running sums (loads in flight together), combined in a
  // fixed order: deterministic
  const double* p = part + (int64_t)t * 256 + e;
  const int64_t stride = (int64_t)ntiles * 256;
  double v8[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  int sl = 0;
  for (; sl + 8 <= slabs; sl += 8) {
#pragma unroll
    for (int u = 0; u < 8; u++) v8[u] += p[(int64_t)(sl + u) * stride];
  }
  for (int u = 0; sl < slabs; sl++, u++) v8[u] += p[(int64_t)sl * stride];
  const double v = ((v8[0] + v8[1]) + (v8[2] + v8[3])) + ((v8[4] + v8[5]) + (v8[6] + v8[7]));
  int I, J;
  trailing_coords(t, nb, I, J);
  const int i = 16 * I + e / 16, j = 16 * J + e % 16;
  if (i < l && j < l) {
    G[(int64_t)i * l + j] = v;
    if (I != J) G[(int64_t)j * l + i] = v;
  }
}

__global__ void __launch_bounds__(256) copy_panel_kernel(int64_t rows, int64_t cols,
                                                         const double* __restrict__ src, int64_t lds,
                                                         double* __restrict__ dst, int64_t ldd,
                                                         int cond, const DevState* st) {
  // cond 1: copy only after a shifted pass 0; cond 2: only when unshifted
  if (cond == 1 && st->qr_shifted == 0) return;
  if (cond == 2 && st->qr_shifted != 0) return;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * cols) return;
  const int64_t r = idx / cols, c = idx % cols;
  dst[r * ldd + c] = src[r * lds + c];
}

// B <- (B + B^T) / 2 in place (l x l): the thread of each pair i < j reads
// both entries and writes their average to both, so no entry is read after
// another thread wrote it.
__global__ void __launch_bounds__(256) symmetrize_kernel(int64_t l, double* __restrict__ B,
                                                         int64_t ldb) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= l * l) return;
  const int64_t i = idx / l, j = idx % l;
  if (i >= j) return;
  const double a = 0.5 * (B[i * ldb + j] + B[j * ldb + i]);
  B[i * ldb + j] = a;
  B[j * ldb + i] = a;
}

__global__ void __launch_bounds__(256) identity_kernel(int64_t l, double* P) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= l * l) return;
  P[idx] = (idx / l == idx % l) ? 1.0 : 0.0;
}

// s_i = |row i of M|, sorted decreasingly (ties keep the lower row first);
// Us[:, i] = row pi(i) of M / s_i, W[:, i] = row pi(i) of P.
// Ordering and extraction of the small SVD from converged M (rows mutually
// orthogonal: row i = s_i u_i^T) and P (rotations), in three launches:
//   norms  one wave per row of M (coalesced), summed in a fixed lane order
//   rank   one workgroup ranks the norms by (norm, index), NaN below every
//          norm, so the positions always form a permutation; s sorted
//   gather Us[r][i] = M[perm i][r] / s_i and W[r][i] = P[perm i][r] through
//          32 x 32 LDS tiles (rows of M and P read along r, Us and W written
//          along i)
// scratch: 2 l doubles (the norms, then the permutation as integers).
__global__ void __launch_bounds__(256) svd_norms_kernel(int l, const double* __restrict__ M,
                                                        int64_t ld, double* __restrict__ nrm) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (row >= l) return;
  double a = 0.0;
  for (int c = lane; c < l; c += 64) {
    const double x = M[(int64_t)row * ld + c];
    a += x * x;
  }
  a = wave_sum(a);
  if (lane == 0) nrm[row] = sqrt(a);
}

__global__ void __launch_bounds__(kBig) svd_rank_kernel(int l, const double* __restrict__ nrm,
                                                        int* __restrict__ perm,
                                                        double* __restrict__ s, DevState* st) {
  __shared__ int s_zero;
  if (threadIdx.x == 0) s_zero = 0;
  __syncthreads();
  for (int i = threadIdx.x; i < l; i += blockDim.x) {
    const double v = isnan(nrm[i]) ? -1.0 : nrm[i];
    int pos = 0;
    for (int j = 0; j < l; j++) {
      const double u = isnan(nrm[j]) ? -1.0 : nrm[j];
      pos += (u > v) || (u == v && j < i);
    }
    perm[pos] = i;
    s[pos] = nrm[i];
    if (!(nrm[i] > 0.0)) s_zero = 1;
  }
  __syncthreads();
  if (threadIdx.x == 0 && s_zero) atomicOr(&st->flags, (uint32_t)RSVD_FLAG_ZERO_SIGMA);
}

__global__ void __launch_bounds__(256) svd_gather_kernel(int l, int kc,
                                                         const double* __restrict__ M,
                                                         const double* __restrict__ P, int64_t ld,
                                                         const int* __restrict__ perm,
                                                         const double* __restrict__ s,
                                                         double* __restrict__ Us,
                                                         double* __restrict__ W) {
  __shared__ double tm[32][33], tp[32][33];
  const int r0 = blockIdx.x * 32, i0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 8 rows of threads
  for (int y = ty; y < 32; y += 8) {
    const int i = i0 + y, r = r0 + tx;
    double vm = 0.0, vp = 0.0;
    if (i < kc && i < l && r < l) {
      const int src = min(max(perm[i], 0), l - 1);
      vm = M[(int64_t)src * ld + r];
      vp = P[(int64_t)src * ld + r];
    }
    tm[y][tx] = vm;
    tp[y][tx] = vp;
  }
  __syncthreads();
  for (int y = ty; y < 32; y += 8) {
    const int r = r0 + y, i = i0 + tx;
    if (r < l && i < kc) {
      const double sv = i < l ? s[i] : 0.0;
      Us[(int64_t)r * kc + i] = sv > 0.0 ? tm[tx][y] / sv : 0.0;
      W[(int64_t)r * kc + i] = tp[tx][y];
    }
  }
}

// Rank rule (a single thread; l is small).
__global__ void select_rank_kernel(int64_t l, int64_t p, int64_t kc, int mode, double param,
                                   const double* __restrict__ s, DevState* st) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int64_t k = 0;
  uint32_t f = 0;
  const int64_t cap = (l - p) > 1 ? (l - p) : 1;
  if (mode == RSVD_RANK_FIXED) {
    k = (int64_t)param;
    st->rank_wanted = (int32_t)k;
  } else if (mode == RSVD_RANK_REL_THRESHOLD) {
    // an all-zero projection has no value above the threshold (k = 1 below)
    if (s[0] > 0.0)
      for (int64_t j = 0; j < l; j++) k += (s[j] >= param * s[0]) ? 1 : 0;
    st->rank_wanted = (int32_t)k;
    if (k > cap) { k = cap; f |= RSVD_FLAG_RANK_CAPPED; }
  } else if (mode == RSVD_RANK_FROB_TAIL) {
    double tot = 0.0;
    for (int64_t j = 0; j < l; j++) tot += s[j] * s[j];
    double missed = st->fro2 - tot;
    if (missed < 0.0) missed = 0.0;
    const double lim = param * sqrt(st->fro2);
    // tail[k] = sum_{j >= k} s_j^2, accumulated from the small end
    k = l;
    double tail = 0.0;
    int64_t best = l;
    for (int64_t kk = l; kk >= 0; kk--) {
      if (kk < l) tail += s[kk] * s[kk];
      if (sqrt(tail + missed) <= lim) best = kk;
    }
    k = best;
    st->rank_wanted = (int32_t)k;
    if (k > cap) { k = cap; f |= RSVD_FLAG_RANK_CAPPED; }
  }
  if (k < 1) k = 1;
  if (k > l) k = l;
  if (k > kc) { k = kc; f |= RSVD_FLAG_RANK_CAPPED; }
  st->rank = (int32_t)k;
  st->flags |= f;
}

// Sign rule: flip (U_j, V_j) so the largest-magnitude entry of U_j is positive
// (lowest row on ties; NaN entries never win). Four coalesced passes over the
// row-major factors, threads along the columns of a row:
//   colmax  key_j = max_i |U_ij| as the bit pattern of a non-negative double
//           (ordered like the value), a workgroup per block of rows, one
//           atomic max per column and workgroup;
//   colarg  idx_j = the lowest row whose |U_ij| has that pattern (atomic min);
//   colsign sign_j = -1 where U[idx_j][j] < 0, else +1 (into key_j);
//   flip    U_ij, V_ij negated in the columns with sign_j = -1.
constexpr int64_t kSignRows = 64;  // rows per workgroup of colmax / colarg

__global__ void __launch_bounds__(256) colmax_init_kernel(int64_t kc, unsigned long long* key,
                                                          unsigned long long* idx) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < kc) {
    key[j] = 0ull;
    idx[j] = ~0ull;
  }
}

__global__ void __launch_bounds__(256) colmax_kernel(int64_t m, int64_t kc,
                                                     const double* __restrict__ U, int64_t ldu,
                                                     unsigned long long* key) {
  const int64_t j = (int64_t)blockIdx.y * blockDim.x + threadIdx.x;
  if (j >= kc) return;
  const int64_t r0 = (int64_t)blockIdx.x * kSignRows;
  const int64_t r1 = r0 + kSignRows < m ? r0 + kSignRows : m;
  double best = 0.0;
  for (int64_t i = r0; i < r1; i++) {
    const double a = fabs(U[i * ldu + j]);
    if (a > best) best = a;
  }
  if (best > 0.0) atomicMax(&key[j], (unsigned long long)__double_as_longlong(best));
}

__global__ void __launch_bounds__(256) colarg_kernel(int64_t m, int64_t kc,
                                                     const double* __restrict__ U, int64_t ldu,
                                                     const unsigned long long* key,
                                                     unsigned long long* idx) {
  const int64_t j = (int64_t)blockIdx.y * blockDim.x + threadIdx.x;
  if (j >= kc) return;
  const int64_t r0 = (int64_t)blockIdx.x * kSignRows;
  const int64_t r1 = r0 + kSignRows < m ? r0 + kSignRows : m;
  const unsigned long long k = key[j];
  for (int64_t i = r0; i < r1; i++) {
    if ((unsigned long long)__double_as_longlong(fabs(U[i * ldu + j])) == k) {
      atomicMin(&idx[j], (unsigned long long)i);
      break;
    }
  }
}

__global__ void __launch_bounds__(256) colsign_kernel(int64_t m, int64_t kc,
                                                      const double* __restrict__ U, int64_t ldu,
                                                      const unsigned long long* idx,
                                                      double* sign) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= kc) return;
  const unsigned long long i = idx[j];
  sign[j] = (i < (unsigned long long)m && U[(int64_t)i * ldu + j] < 0.0) ? -1.0 : 1.0;
}

__global__ void __launch_bounds__(256) flip_kernel(int64_t m, int64_t n, int64_t kc,
                                                   double* __restrict__ U, int64_t ldu,
                                                   double* __restrict__ V, int64_t ldv,
                                                   const double* __restrict__ sign) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t rows = m + (V ? n : 0);
  if (e >= rows * kc) return;
  const int64_t i = e / kc, j = e % kc;
  if (sign[j] < 0.0) {
    double* p = i < m ? &U[i * ldu + j] : &V[(i - m) * ldv + j];
    *p = -*p;
  }
}

// US = U diag(s) (columns >= rank zeroed), Vt = V^T (rows >= rank zeroed).
__global__ void __launch_bounds__(256) resid_prep_kernel(int64_t m, int64_t n, int64_t kc,
                                                         int64_t kcp,
                                                         const double* __restrict__ U, int64_t ldu,
                                                         const double* __restrict__ s,
                                                         const double* __restrict__ V, int64_t ldv,
                                                         double* __restrict__ US,
                                                         double* __restrict__ Vt,
                                                         const DevState* st) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t rank = st->rank < kc ? st->rank : kc;
  if (idx < m * kcp) {
    const int64_t i = idx / kcp, j = idx % kcp;  // US is m x kcp
    US[idx] = j < rank ? U[i * ldu + j] * s[j] : 0.0;
  }
  if (idx < n * kcp) {
    const int64_t j = idx / n, i = idx % n;  // Vt is kcp x n
    Vt[idx] = j < rank ? V[i * ldv + j] : 0.0;
  }
}

__global__ void __launch_bounds__(256) check_finite_kernel(int64_t rows, int64_t cols,
                                                           const double* __restrict__ Y, int64_t ldy,
                                                           DevState* st) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool bad = false;
  if (idx < rows * cols) bad = !isfinite(Y[(idx / cols) * ldy + idx % cols]);
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(&st->flags, (uint32_t)RSVD_FLAG_NONFINITE_INPUT);
}

__global__ void __launch_bounds__(256) sumsq_kernel(int64_t m, int64_t n,
                                                    const double* __restrict__ A, int64_t lda,
                                                    double* __restrict__ partial) {
  __shared__ double red[4];
  double s = 0.0;
  for (int64_t r = blockIdx.x; r < m; r += gridDim.x) {
    for (int64_t c = threadIdx.x; c < n; c += blockDim.x) {
      const double x = A[r * lda + c];
      s += x * x;
    }
  }
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ void __launch_bounds__(256) sum_partials_kernel(int64_t cnt, const double* __restrict__ p,
                                                           double* __restrict__ out) {
  __shared__ double red[4];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < cnt; i += blockDim.x) s += p[i];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) *out = red[0] + red[1] + red[2] + red[3];
}

// The a-posteriori judge of a fixed-l run (posterior > 0), after the rank
// rule: UNCONVERGED when (s_l / s_k)^(4q + 2) > 1e-8 for the kept rank k
// (threshold rules), POSTERIOR_FAIL when the posterior estimate exceeds
// tau s_1 (relative threshold). An exact decomposition (l = min(m, n)) passes.
__global__ void judge_kernel(int64_t l, int64_t mn, int q, int mode, double tau,
                             const double* __restrict__ s, DevState* st) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (l >= mn || (mode != RSVD_RANK_REL_THRESHOLD && mode != RSVD_RANK_FROB_TAIL)) return;
  const int64_t k = st->rank;
  uint32_t f = 0;
  if (k >= 1 && k < l && s[k - 1] > 0.0) {
    const double r = s[l - 1] / s[k - 1];
    if (!(pow(r, (double)(4 * q + 2)) <= kConvergedRatio)) f |= RSVD_FLAG_UNCONVERGED;
  }
  if (mode == RSVD_RANK_REL_THRESHOLD) {
    const double est = kPosteriorFactor * sqrt(st->est2);
    if (!(est <= tau * s[0])) f |= RSVD_FLAG_POSTERIOR_FAIL;
  }
  st->flags |= f;
}

__global__ void finalize_kernel(int64_t m, int64_t n, int64_t l, int want_residual,
                                double err_est, int blocks, int dev_est, const DevState* st,
                                rsvd_result* res) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int64_t k = st->rank;
  const double N = (double)(m < n ? m : n);
  res->rank = k;
  res->l_used = l;
  res->residual = want_residual ? sqrt(st->resid2) / sqrt(st->fro2) : __builtin_nan("");
  res->rel_percent = 100.0 * (double)k / N;
  res->c_eq2 = (double)m * (double)n / ((double)(m + n) * k + k);
  res->c_sym = (double)m * (double)n / ((double)(m > n ? m : n) * k + k);
  res->fro2 = st->fro2;
  res->sweeps = st->sweeps;
  res->flags = st->flags;
  res->err_est = dev_est ? kPosteriorFactor * sqrt(st->est2) : err_est;
  res->blocks = blocks;
  res->reserved = 0;
}

__global__ void init_state_kernel(DevState* st, uint32_t flags) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    st->flags = flags;
    st->qr_shifted = 0;
    st->qr_householder = 0;
    st->sweeps = 0;
    st->rank = 0;
    st->fro2 = 0.0;
    st->resid2 = 0.0;
    st->rank_wanted = 0;
    st->pad_ = 0;
    st->est2 = 0.0;
    st->s1lb2 = 0.0;
    st->froY2 = 0.0;
    st->prefer_shift = 0u;
    st->gram_dev = INFINITY;
  }
  if (blockIdx.x == 0) {
    if (threadIdx.x < 64) st->rot_count[threadIdx.x] = 0;
    grid_barrier_reset(&st->bar);
  }
}

__global__ void clear_flags_kernel(DevState* st, uint32_t clear, uint32_t set) {
  if (threadIdx.x == 0 && blockIdx.x == 0) st->flags = (st->flags & ~clear) | set;
}

// Column sums of squares of a rows x cols row-major panel (cols <= 256):
// partial[b * cols + c] = sum over the rows of row block b of X[r][c]^2.
// Wave w of block b takes rows 4 b + w, 4 b + w + 4 gridDim, ...; lane c
// reads column c (+ 64 g), so each wave reads whole rows contiguously.
__global__ void __launch_bounds__(256) colsumsq_kernel(int64_t rows, int cols,
                                                       const double* __restrict__ X, int64_t ld,
                                                       double* __restrict__ partial) {
  __shared__ double red[4][256];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t r = (int64_t)blockIdx.x * 4 + w; r < rows; r += (int64_t)gridDim.x * 4) {
    const double* row = X + r * ld;
#pragma unroll
    for (int g = 0; g < 4; g++) {
      const int c = lane + 64 * g;
      if (c < cols) {
        const double x = row[c];
        acc[g] += x * x;
      }
    }
  }
#pragma unroll
  for (int g = 0; g < 4; g++) red[w][lane + 64 * g] = acc[g];
  __syncthreads();
  for (int c = threadIdx.x; c < cols; c += 256)
    partial[(int64_t)blockIdx.x * cols + c] = (red[0][c] + red[1][c]) + (red[2][c] + red[3][c]);
}

// Reduce the partials of colsumsq_kernel over the row blocks, then
//   mode 0: st->est2 = max_c colsum
//   mode 1: st->s1lb2 = max(st->s1lb2, max_c colsum); st->froY2 += sum_c colsum
__global__ void __launch_bounds__(256) colsumsq_finish_kernel(int nblk, int cols,
                                                              const double* __restrict__ partial,
                                                              int mode, DevState* st) {
  __shared__ double smax[4], ssum[4];
  const int c = threadIdx.x;
  double v = 0.0;
  if (c < cols)
    for (int b = 0; b < nblk; b++) v += partial[(int64_t)b * cols + c];
  // a NaN column must not vanish in fmax: carry it explicitly
  const double vm = v != v ? __builtin_inf() : v;
  const double mx = wave_max(vm), sm = wave_sum(v);
  if ((threadIdx.x & 63) == 0) {
    smax[threadIdx.x >> 6] = mx;
    ssum[threadIdx.x >> 6] = sm;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double M = fmax(fmax(smax[0], smax[1]), fmax(smax[2], smax[3]));
    const double S = (ssum[0] + ssum[1]) + (ssum[2] + ssum[3]);
    if (mode == 0) {
      st->est2 = M;
    } else {
      if (M > st->s1lb2) st->s1lb2 = M;
      st->froY2 += S;
    }
  }
}

__global__ void clear_shift_kernel(DevState* st) {
  if (blockIdx.x != 0) return;
  if (threadIdx.x == 0) {
    st->qr_shifted = 0;
    st->qr_householder = 0;
  }
  grid_barrier_reset(&st->bar);
}

__global__ void __launch_bounds__(256) transpose_kernel(int64_t rows, int64_t cols,
                                                        const double* __restrict__ src, int64_t lds,
                                                        double* __restrict__ dst, int64_t ldd) {
  __shared__ double tile[32][33];
  const int64_t r0 = (int64_t)blockIdx.y * 32, c0 = (int64_t)blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int k = 0; k < 32; k += 8) {
    const int64_t r = r0 + ty + k, c = c0 + tx;
    if (r < rows && c < cols) tile[ty + k][tx] = src[r * lds + c];
  }
  __syncthreads();
  for (int k = 0; k < 32; k += 8) {
    const int64_t c = c0 + ty + k, r = r0 + tx;  // dst[c][r] = src[r][c]
    if (r < rows && c < cols) dst[c * ldd + r] = tile[tx][ty + k];
  }
}

inline unsigned blocks_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

size_t chol_panel_doubles(int64_t l) {
  // the grid kernel's 32-row panel
  return (size_t)32 * (size_t)grid_panel_ld(l);
}

rsvd_status chol_inv(int64_t l, double* G, double* R, double* Rinv, double* scratch, int64_t m,
                     int pass, int only_if_shifted, DevState* st, hipStream_t s, int share,
                     bool full_inverse) {
  if (!full_inverse && l <= 16 * kCholRegMaxNB) {
    hipLaunchKernelGGL(chol_reg_kernel, dim3(1), dim3(64 * kCholRegWaves), 0, s, (int)l, G, R,
                       Rinv, m, pass, only_if_shifted, st);
    RSVD_LAUNCH_CHECK();
    return RSVD_OK;
  }
  if (!scratch) return RSVD_EINVAL;
  {
    // one 4-wave workgroup per ~48 tiles of the first trailing update, at
    // most 64 (measured at l = 528 .. 1541: more workgroups cost more in the
    // two grid barriers per super-step than they save in the updates), and
    // capped so the grids of concurrent runs fit on the device together
    static int cap_all = 0;
    if (cap_all == 0) {
      int dev = 0, ncu = 0, per_cu = 0;
      if (hipGetDevice(&dev) != hipSuccess ||
          hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
          hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)chol_grid_kernel, 256,
                                                       0) != hipSuccess)
        return RSVD_EHIP;
      cap_all = ncu * (per_cu > 0 ? per_cu : 1);
    }
    const int64_t nb = (l + 15) / 16;
    int grid = (int)((nb * (nb - 1) / 2 + 47) / 48);
    // concurrent runs: half of a fair share, so that grids of different
    // kernels (different per-CU footprints) also fit together
    int cap = cap_all / (share > 1 ? 2 * share : 1);
    if (cap > 64) cap = 64;
    if (grid > cap) grid = cap;
    if (grid < 1) grid = 1;
    if (pass > 0) {
      // a Gram within 2^-33 of the identity: the first-order factor instead
      const unsigned gb = (unsigned)((l * l + 4095) / 4096 < 256 ? (l * l + 4095) / 4096 : 256);
      hipLaunchKernelGGL(gram_dev_clear_kernel, dim3(1), dim3(64), 0, s, only_if_shifted, st);
      hipLaunchKernelGGL(gram_dev_kernel, dim3(gb), dim3(256), 0, s, (int)l, (const double*)G, st);
      hipLaunchKernelGGL(gram_first_order_kernel, dim3(gb), dim3(256), 0, s, (int)l,
                         (const double*)G, R, Rinv, (const DevState*)st);
      RSVD_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(chol_grid_kernel, dim3(grid), dim3(256), 0, s, (int)l, G, R, Rinv, scratch,
                       m, pass, only_if_shifted, full_inverse ? 1 : 0, st);
    RSVD_LAUNCH_CHECK();
    return RSVD_OK;
  }
}

rsvd_status gram(int64_t rows, int64_t l, const double* Y, int64_t ldy, double* G, double* part,
                 size_t part_doubles, const uint32_t* pred, hipStream_t s) {
  if (rows <= 0 || l <= 0) return RSVD_OK;
  const int64_t nb = (l + 15) / 16;
  const int64_t ntiles = nb * (nb + 1) / 2;
  // enough (slab, tile group) workgroups for the device: slabs of at least
  // 64 rows, as many as the partials' room allows
  const int64_t groups = (ntiles + kGramWaves * kGramSlots - 1) / (kGramWaves * kGramSlots);
  int64_t slabs = (rows + 63) / 64;
  if (slabs > 256 / groups) slabs = 256 / groups;
  const int64_t room = part ? (int64_t)(part_doubles / ((size_t)ntiles * 256)) : 0;
  if (slabs > room) slabs = room;
  if (nb > kGramMaxNB || slabs < 16 || ldy < l) {
    // too little room or too wide: the general product
    return dgemm(true, l, l, rows, 1.0, Y, ldy, Y, ldy, 0.0, G, l, part, part_doubles, s, 64, pred);
  }
  static bool attr = false;
  if (!attr) {
    attr = true;
    (void)hipFuncSetAttribute((const void*)gram_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                              2 * kGramRows * 16 * kGramMaxNB * (int)sizeof(double));
  }
  const int64_t per = ((rows + slabs - 1) / slabs + kGramRows - 1) / kGramRows * kGramRows;
  slabs = (rows + per - 1) / per;
  const size_t lds = (size_t)2 * kGramRows * 16 * nb * sizeof(double);
  hipLaunchKernelGGL(gram_kernel, dim3((unsigned)slabs, (unsigned)groups), dim3(64 * kGramWaves),
                     lds, s, rows, (int)l, Y, ldy, per, part, pred);
  RSVD_LAUNCH_CHECK();
  hipLaunchKernelGGL(gram_reduce_kernel, dim3((unsigned)((ntiles * 256 + 255) / 256)), dim3(256),
                     0, s, (int)l, (int)slabs, (const double*)part, G, pred);
  RSVD_LAUNCH_CHECK();
  return RSVD_OK;
}

bool trsm_supported(int64_t l) { return l >= 1 && (l + 15) / 16 <= kTrsmMaxNBWide; }

rsvd_status trsm_upper(int64_t rows, int64_t l, const double* Y, int64_t ldy, const double* R,
                       int64_t ldr, const double* Xd, double* Q, int64_t ldq,
                       const uint32_t* pred, hipStream_t s) {
  if (rows <= 0 || l <= 0) return RSVD_OK;
  if (!trsm_supported(l) || ldy < l || ldq < l || ldr < l) return RSVD_EINVAL;
  static bool attr = false;
  if (!attr) {
    attr = true;
    (void)hipFuncSetAttribute((const void*)trsm_upper_kernel<kTrsmMaxNB>,
                              hipFuncAttributeMaxDynamicSharedMemorySize,
                              2 * kTrsmMaxNB * 256 * (int)sizeof(double));
    (void)hipFuncSetAttribute((const void*)trsm_upper_kernel<kTrsmMaxNBWide>,
                              hipFuncAttributeMaxDynamicSharedMemorySize,
                              2 * kTrsmMaxNBWide * 256 * (int)sizeof(double));
  }
  const int nb = (int)((l + 15) / 16);
  const size_t lds = (size_t)2 * nb * 256 * sizeof(double);
  const int64_t per = 16 * kTrsmWaves;
  const dim3 grid((unsigned)((rows + per - 1) / per));
  if (nb <= kTrsmMaxNB)
    hipLaunchKernelGGL(trsm_upper_kernel<kTrsmMaxNB>, grid, dim3(64 * kTrsmWaves), lds, s, rows,
                       (int)l, Y, ldy, R, ldr, Xd, Q, ldq, pred);
  else
    hipLaunchKernelGGL(trsm_upper_kernel<kTrsmMaxNBWide>, grid, dim3(64 * kTrsmWaves), lds, s,
                       rows, (int)l, Y, ldy, R, ldr, Xd, Q, ldq, pred);
  RSVD_LAUNCH_CHECK();
  return RSVD_OK;
}

rsvd_status householder_fallback(int64_t rows, int64_t l, const double* Yorig, double* Y,
                                 double* R, double* tau, double* scratch, DevState* st,
                                 hipStream_t s, int share) {
  // a grid of workgroups (64 rows or more each) for panels that would keep one
  // workgroup busy for long; its scratch (G l + l doubles) fits in l x l
  int grid = (int)((rows + 63) / 64);
  if (grid > (int)l - 1) grid = (int)l - 1;
  if (grid > 128) grid = 128;
  if (scratch && rows * l >= kHouseGridMin && grid >= 2) {
    static int cap_all = 0;
    if (cap_all == 0) {
      int dev = 0, ncu = 0, per_cu = 0;
      if (hipGetDevice(&dev) != hipSuccess ||
          hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
          hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)householder_grid_kernel,
                                                       256, 0) != hipSuccess)
        return RSVD_EHIP;
      cap_all = ncu * (per_cu > 0 ? per_cu : 1);
    }
    // concurrent runs: half of a fair share (as the other grid kernels)
    const int cap = cap_all / (share > 1 ? 2 * share : 1);
    if (grid > cap) grid = cap;
    if (grid >= 2) {
      hipLaunchKernelGGL(householder_grid_kernel, dim3(grid), dim3(256), 0, s, rows, (int)l, Yorig,
                         Y, R, tau, scratch, st);
      RSVD_LAUNCH_CHECK();
      return RSVD_OK;
    }
  }
  hipLaunchKernelGGL(householder_kernel, dim3(1), dim3(kBig), 0, s, rows, (int)l, Yorig, Y, R,
                     tau, st);
  RSVD_LAUNCH_CHECK();
  return RSVD_OK;
}

rsvd_status copy_panel(int64_t rows, int64_t cols, const double* src, int64_t lds, double* dst,
                       int64_t ldd, int cond_shifted, DevState* st, hipStream_t s) {
  if (rows * cols == 0) return RSVD_OK;
  hipLaunchKernelGGL(copy_panel_kernel, dim3(blocks_for(rows * cols, 256)), dim3(256), 0, s, rows,
                     cols, src, lds, dst, ldd, cond_shifted, (const DevState*)st);
  RSVD_LAUNCH_CHECK();
  return RSVD_OK;
}

rsvd_status symmetrize(int64_t l, double* B, int64_t ldb, hipStream_t s) {
  if (l <= 1) return RSVD_OK;
  hipLaunchKernelGGL(symmetrize_kernel, dim3(blocks_for(l * l, 256)), dim3(256), 0, s, l, B, ldb);
  RSVD_LAUNCH_CHECK();
  return RSVD_OK;
}

rsvd_status set_identity(int64_t l, double* P, hipStream_t s) {
  hipLaunchKernelGGL(identity_kernel, dim3(blocks_for(l * l, 256)), dim3(256), 0, s, l, P);
  RSVD_LAUNCH_CHECK();
  return RSVD_OK;
}

rsvd_status svd_finish(int64_t l, int64_t kc, const double* M, const double* P, int64_t ld,
                       double* sv, double* Us, double* W, double* scratch, DevState* st,
                       hipStream_t s) {
  double* nrm = scratch;
  int* perm = reinterpret_cast<int*>(scratch + l);
  hipLaunchKernelGGL(svd_norms_kernel, dim3((unsigned)((l + 3) / 4)), dim3(256), 0, s, (int)l, M,
                     ld, nrm);
  RSVD_LAUNCH_CHECK();
  hipLaunchKernelGGL(svd_rank_kernel, dim3(1), dim3(kBig), 0, s, (int)l, nrm, perm, sv, st);
  RSVD_LAUNCH_CHECK();
  if (kc > 0) {
    hipLaunchKernelGGL(svd_gather_kernel, dim3((unsigned)((l + 31) / 32), (unsigned)((kc + 31) / 32)),
                       dim3(256), 0, s, (int)l, (int)kc, M, P, ld, perm, sv, Us, W);
    RSVD_LAUNCH_CHECK();
  }
  return RSVD_OK;
}

rsvd_status select_rank(int64_t l, int64_t p, int64_t kc, int mode, double param,
                        const double* sv, DevState* st, hipStream_t s) {
  hipLaunchKernelGGL(select_rank_kernel, dim3(1), dim3(64), 0, s, l, p, kc, mode, param, sv, st);
  RSVD_LAUNCH_CHECK();
  return RSVD_OK;
}

rsvd_status sign_fix(int64_t m, int64_t n, int64_t kc, double* U, int64_t ldu, double* V,
                     int64_t ldv, double* scratch, hipStream_t s) {
  if (kc == 0 || m == 0) return RSVD_OK;
  unsigned long long* key = reinterpret_cast<unsigned long long*>(scratch);
  unsigned long long* idx = key + kc;
  const unsigned cb = blocks_for(kc, 256);
  const dim3 grid(blocks_for(m, kSignRows), cb);
  if (grid.y > 65535) return RSVD_EUNSUPPORTED;
  hipLaunchKernelGGL(colmax_init_kernel, dim3(cb), dim3(256), 0, s, kc, key, idx);
  RSVD_LAUNCH_CHECK();
  hipLaunchKernelGGL(colmax_kernel, grid, dim3(256), 0, s, m, kc, U, ldu, key);
  RSVD_LAUNCH_CHECK();
  hipLaunchKernelGGL(colarg_kernel, grid, dim3(256), 0, s, m, kc, U, ldu, key, idx);
  RSVD_LAUNCH_CHECK();
  // the sign overwrites the key of its column (read by this thread only)
  hipLaunchKernelGGL(colsign_kernel, dim3(cb), dim3(256), 0, s, m, kc, U, ldu, idx, scratch);
  RSVD_LAUNCH_CHECK();
  const int64_t tot = (m + (V ? n : 0)) * kc;
  hipLaunchKernelGGL(flip_kernel, dim3(blocks_for(tot, 256)), dim3(256), 0, s, m, n, kc, U, ldu,
                     V, ldv, scratch);
  RSVD_LAUNCH_CHECK();
  return RSVD_OK;
}

rsvd_status resid_prep(int64_t m, int64_t n, int64_t kc, int64_t kcp, const double* U,
                       int64_t ldu, const double* sv, const double* V, int64_t ldv, double* US,
                       double* Vt, const DevState* st, hipStream_t s) {
  const int64_t tot = (m > n ? m : n) * kcp;
  hipLaunchKernelGGL(resid_prep_kernel, dim3(blocks_for(tot, 256)), dim3(256), 0, s, m, n, kc, kcp,
                     U, ldu, sv, V, ldv, US, Vt, st);
  RSVD_LAUNCH_CHECK();
  return RSVD_OK;
}

rsvd_status check_finite(int64_t rows, int64_t cols, const double* Y, int64_t ldy, DevState* st,
                         hipStream_t s) {
  hipLaunchKernelGGL(check_finite_kernel, dim3(blocks_for(rows * cols, 256)), dim3(256), 0, s,
                     rows, cols, Y, ldy, st);
  RSVD_LAUNCH_CHECK();
  return RSVD_OK;
}

rsvd_status sumsq(int64_t m, int64_t n, const double* A, int64_t lda, double* partial,
                  DevState* st, hipStream_t s) {
  const int nb = 2048;
  hipLaunchKernelGGL(sumsq_kernel, dim3(nb), dim3(256), 0, s, m, n, A, lda, partial);
  RSVD_LAUNCH_CHECK();
  hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(256), 0, s, (int64_t)nb,
                     (const double*)partial, &st->fro2);
  RSVD_LAUNCH_CHECK();
  return RSVD_OK;
}

rsvd_status sum_partials_into(int64_t cnt, const double* p, double* out, hipStream_t s) {
  hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(256), 0, s, cnt, p, out);
  RSVD_LAUNCH_CHECK();
  return RSVD_OK;
}

rsvd_status finalize(int64_t m, int64_t n, int64_t l, int want_residual, double err_est,
                     int blocks, const DevState* st, rsvd_result* res, hipStream_t s,
                     bool dev_est) {
  hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(64), 0, s, m, n, l, want_residual, err_est,
                     blocks, (int)dev_est, st, res);
  RSVD_LAUNCH_CHECK();
  return RSVD_OK;
}

rsvd_status judge(int64_t l, int64_t mn, int q, int mode, double tau, const double* sv,
                  DevState* st, hipStream_t s) {
  hipLaunchKernelGGL(judge_kernel, dim3(1), dim3(64), 0, s, l, mn, q, mode, tau, sv, st);
  RSVD_LAUNCH_CHECK();
  return RSVD_OK;
}

rsvd_status init_state(DevState* st, uint32_t flags, hipStream_t s) {
  hipLaunchKernelGGL(init_state_kernel, dim3(1), dim3(64), 0, s, st, flags);
  RSVD_LAUNCH_CHECK();
  return RSVD_OK;
}

rsvd_status clear_flags(DevState* st, uint32_t clear, uint32_t set, hipStream_t s) {
  hipLaunchKernelGGL(clear_flags_kernel, dim3(1), dim3(64), 0, s, st, clear, set);
  RSVD_LAUNCH_CHECK();
  return RSVD_OK;
}

int colsumsq_blocks(int64_t rows, int cols, size_t partial_doubles) {
  int64_t nb = (rows + 15) / 16;
  if (nb > 512) nb = 512;
  const int64_t cap = (int64_t)(partial_doubles / (size_t)(cols > 0 ? cols : 1));
  if (nb > cap) nb = cap;
  return nb < 1 ? 1 : (int)nb;
}

rsvd_status colsumsq(int64_t rows, int cols, const double* X, int64_t ld, double* partial,
                     size_t partial_doubles, int mode, DevState* st, hipStream_t s) {
  if (cols < 1 || cols > 256 || partial_doubles < (size_t)cols) return RSVD_EINVAL;
  const int nb = colsumsq_blocks(rows, cols, partial_doubles);
  hipLaunchKernelGGL(colsumsq_kernel, dim3(nb), dim3(256), 0, s, rows, cols, X, ld, partial);
  RSVD_LAUNCH_CHECK();
  hipLaunchKernelGGL(colsumsq_finish_kernel, dim3(1), dim3(256), 0, s, nb, cols,
                     (const double*)partial, mode, st);
  RSVD_LAUNCH_CHECK();
  return RSVD_OK;
}

rsvd_status clear_shift(DevState* st, hipStream_t s) {
  hipLaunchKernelGGL(clear_shift_kernel, dim3(1), dim3(64), 0, s, st);
  RSVD_LAUNCH_CHECK();
  return RSVD_OK;
}

rsvd_status transpose(int64_t rows, int64_t cols, const double* src, int64_t lds, double* dst,
                      int64_t ldd, hipStream_t s) {
  if (rows == 0 || cols == 0) return RSVD_OK;
  dim3 grid(blocks_for(cols, 32), blocks_for(rows, 32));
  hipLaunchKernelGGL(transpose_kernel, grid, dim3(256), 0, s, rows, cols, src, lds, dst, ldd);
  RSVD_LAUNCH_CHECK();
  return RSVD_OK;
}

}  // namespace rsvd
