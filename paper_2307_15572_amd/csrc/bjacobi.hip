// Small SVD of step 2 (section "Randomized matrix decompositions": thin SVD
// of the projected matrix) by block one-sided Jacobi on the rows of the
// l x l factor M. Rows are grouped in blocks of 16; blocks are paired by a
// round-robin (circle) tournament, nb - 1 steps per sweep, one workgroup per
// pair, a grid-wide barrier between steps. The grid is capped at what the
// device holds at once (divided among runs on concurrent streams), and the
// barrier lives in the run's workspace, so the launch is an ordinary one:
// it can run beside other streams' work and be captured in a graph. Every
// wait at the barrier is bounded (RSVD_FLAG_SYNC_TIMEOUT instead of a hang).
// For a pair of blocks (32 rows):
//   H = rows rows^T                   32 x 32 Gram, FP64 matrix cores
//   V^T H V ~ diagonal                two-sided Jacobi on H in LDS (cyclic,
//                                     parallel ordering, Rutishauser rotations)
//   rows <- V^T rows, P_rows <- V^T P_rows   FP64 matrix cores
// A pair whose scaled off-diagonal |H_ij| / sqrt(H_ii H_jj) is at most tol
// is left alone; a sweep with no rotated pair ends the iteration.
#include "common.hpp"
#include "kernels.hpp"

namespace rsvd {

namespace {

constexpr double kU = 1.1102230246251565e-16;

__device__ __forceinline__ void rr_pair_blk(int L, int step, int i, int& a, int& b) {
  if (i == 0) {
    a = L - 1;
    b = step;
  } else {
    a = (step + i) % (L - 1);
    b = (step - i + (L - 1)) % (L - 1);
  }
}

struct JacArgs {
  int l, Lp, max_sweeps, inner_sweeps;
  double* M;
  double* P;
  DevState* st;
};

// returns true if the pair needed rotating
__device__ bool process_pair(const JacArgs& a, int I, int J, double tol, double (*H)[33],
                             double (*Vm)[33], double* red, double* rot_c, double* rot_s,
                             int* rot_p, int* rot_q, int* s_any) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
  const int Lp = a.Lp;
  const int nct = Lp / 16;
  const double* rI = a.M + (int64_t)16 * I * Lp;
  const double* rJ = a.M + (int64_t)16 * J * Lp;

  // ---- Gram of the 32 rows (tiles 00, 01, 11), K split over the 4 waves
  d4 h00 = {0, 0, 0, 0}, h01 = {0, 0, 0, 0}, h11 = {0, 0, 0, 0};
  for (int ct = wave; ct < nct; ct += 4) {
    const int c0 = 16 * ct + 4 * g;
    double xi[4], xj[4];
#pragma unroll
    for (int s = 0; s < 4; s++) {
      xi[s] = rI[(int64_t)r * Lp + c0 + s];
      xj[s] = rJ[(int64_t)r * Lp + c0 + s];
    }
#pragma unroll
    for (int s = 0; s < 4; s++) {
      h00 = mfma_f64_16x16x4(xi[s], xi[s], h00);
      h01 = mfma_f64_16x16x4(xi[s], xj[s], h01);
      h11 = mfma_f64_16x16x4(xj[s], xj[s], h11);
    }
  }
#pragma unroll
  for (int it = 0; it < 4; it++) {
    const int e = (g + 4 * it) * 16 + r;
    red[(wave * 3 + 0) * 256 + e] = h00[it];
    red[(wave * 3 + 1) * 256 + e] = h01[it];
    red[(wave * 3 + 2) * 256 + e] = h11[it];
  }
  if (threadIdx.x == 0) *s_any = 0;
  __syncthreads();
  for (int e = threadIdx.x; e < 256; e += blockDim.x) {
    double v0 = 0, v1 = 0, v2 = 0;
    for (int w = 0; w < 4; w++) {
      v0 += red[(w * 3 + 0) * 256 + e];
      v1 += red[(w * 3 + 1) * 256 + e];
      v2 += red[(w * 3 + 2) * 256 + e];
    }
    const int i = e / 16, j = e % 16;
    H[i][j] = v0;
    H[i][16 + j] = v1;
    H[16 + j][i] = v1;
    H[16 + i][16 + j] = v2;
  }
  __syncthreads();
  // ---- any pair above tolerance?
  for (int e = threadIdx.x; e < 32 * 32; e += blockDim.x) {
    const int i = e / 32, j = e % 32;
    if (i < j) {
      const double hij = H[i][j];
      if (fabs(hij) > tol * sqrt(H[i][i]) * sqrt(H[j][j]) && hij != 0.0) *s_any = 1;
    }
  }
  __syncthreads();
  if (*s_any == 0) return false;

  // ---- two-sided Jacobi on H, V accumulates the rotations
  for (int e = threadIdx.x; e < 32 * 32; e += blockDim.x) Vm[e / 32][e % 32] = (e / 32 == e % 32) ? 1.0 : 0.0;
  __syncthreads();
  for (int isw = 0; isw < a.inner_sweeps; isw++) {
    for (int round = 0; round < 31; round++) {
      if (threadIdx.x < 16) {
        int p, q;
        rr_pair_blk(32, round, threadIdx.x, p, q);
        if (p > q) { const int t = p; p = q; q = t; }
        const double hpp = H[p][p], hqq = H[q][q], hpq = H[p][q];
        double c = 1.0, s = 0.0;
        if (fabs(hpq) > tol * sqrt(hpp) * sqrt(hqq) && hpq != 0.0) {
          const double zeta = (hqq - hpp) / (2.0 * hpq);
          const double t = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          c = 1.0 / sqrt(1.0 + t * t);
          s = c * t;
        }
        rot_c[threadIdx.x] = c;
        rot_s[threadIdx.x] = s;
        rot_p[threadIdx.x] = p;
        rot_q[threadIdx.x] = q;
      }
      __syncthreads();
      // rows: H <- J^T H
      for (int e = threadIdx.x; e < 16 * 32; e += blockDim.x) {
        const int k = e / 32, x = e % 32;
        const double c = rot_c[k], s = rot_s[k];
        if (s != 0.0) {
          const int p = rot_p[k], q = rot_q[k];
          const double hp = H[p][x], hq = H[q][x];
          H[p][x] = c * hp - s * hq;
          H[q][x] = s * hp + c * hq;
        }
      }
      __syncthreads();
      // columns: H <- H J, V <- V J
      for (int e = threadIdx.x; e < 16 * 32; e += blockDim.x) {
        const int k = e / 32, x = e % 32;
        const double c = rot_c[k], s = rot_s[k];
        if (s != 0.0) {
          const int p = rot_p[k], q = rot_q[k];
          const double hp = H[x][p], hq = H[x][q];
          H[x][p] = c * hp - s * hq;
          H[x][q] = s * hp + c * hq;
          const double vp = Vm[x][p], vq = Vm[x][q];
          Vm[x][p] = c * vp - s * vq;
          Vm[x][q] = s * vp + c * vq;
        }
      }
      __syncthreads();
    }
  }

  // ---- apply: rows <- V^T rows for M and P; each wave owns whole column tiles
  for (int mat = 0; mat < 2; mat++) {
    double* base = mat == 0 ? a.M : a.P;
    double* bI = base + (int64_t)16 * I * Lp;
    double* bJ = base + (int64_t)16 * J * Lp;
    for (int ct = wave; ct < nct; ct += 4) {
      double b[8];
#pragma unroll
      for (int s = 0; s < 8; s++) {
        const int row = 4 * s + g;  // 0..31
        const double* src = row < 16 ? bI : bJ;
        b[s] = src[(int64_t)(row & 15) * Lp + 16 * ct + r];
      }
      d4 o0 = {0, 0, 0, 0}, o1 = {0, 0, 0, 0};
#pragma unroll
      for (int s = 0; s < 8; s++) {
        o0 = mfma_f64_16x16x4(Vm[4 * s + g][r], b[s], o0);
        o1 = mfma_f64_16x16x4(Vm[4 * s + g][16 + r], b[s], o1);
      }
#pragma unroll
      for (int it = 0; it < 4; it++) {
        bI[(int64_t)(g + 4 * it) * Lp + 16 * ct + r] = o0[it];
        bJ[(int64_t)(g + 4 * it) * Lp + 16 * ct + r] = o1[it];
      }
    }
  }
  __syncthreads();
  return true;
}

__global__ void __launch_bounds__(256) bjacobi_kernel(JacArgs a) {
  __shared__ int s_bar_ok;
  __shared__ double H[32][33];
  __shared__ double Vm[32][33];
  __shared__ double red[4 * 3 * 256];
  __shared__ double rot_c[16], rot_s[16];
  __shared__ int rot_p[16], rot_q[16];
  __shared__ int s_any;
  const int nb = a.Lp / 16;  // even
  const int npairs = nb / 2;
  const double tol = (double)a.l * kU;
  uint32_t* counters = a.st->rot_count;
  int sweep = 0;
  bool converged = false;
  bool timed_out = false;
  for (; sweep < a.max_sweeps && !timed_out; sweep++) {
    for (int step = 0; step < nb - 1; step++) {
      for (int pr = blockIdx.x; pr < npairs; pr += gridDim.x) {
        int I, J;
        rr_pair_blk(nb, step, pr, I, J);
        const bool rot = process_pair(a, I, J, tol, H, Vm, red, rot_c, rot_s, rot_p, rot_q, &s_any);
        if (rot && threadIdx.x == 0)
          __hip_atomic_fetch_add(&counters[sweep], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      if (!grid_barrier(&a.st->bar, &s_bar_ok)) {
        timed_out = true;
        break;
      }
    }
    if (timed_out) break;
    const uint32_t cnt = __hip_atomic_load(&counters[sweep], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (cnt == 0) {
      converged = true;
      sweep++;
      break;
    }
  }
  if (timed_out && threadIdx.x == 0)
    __hip_atomic_fetch_or(&a.st->flags, (uint32_t)RSVD_FLAG_SYNC_TIMEOUT, __ATOMIC_RELAXED,
                          __HIP_MEMORY_SCOPE_AGENT);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    a.st->sweeps = sweep;
    if (!converged)
      __hip_atomic_fetch_or(&a.st->flags, (uint32_t)RSVD_FLAG_JACOBI_MAXSWEEP, __ATOMIC_RELAXED,
                            __HIP_MEMORY_SCOPE_AGENT);
  }
}

// M (Lp x Lp) <- R (l x l) zero padded; P <- identity on the leading l x l;
// sweep counters and the grid barrier cleared.
__global__ void __launch_bounds__(256) jac_init_kernel(int l, int Lp, const double* __restrict__ R,
                                                       double* __restrict__ M, double* __restrict__ P,
                                                       DevState* st) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (blockIdx.x == 0) {
    if (threadIdx.x < 64) st->rot_count[threadIdx.x] = 0u;
    grid_barrier_reset(&st->bar);
  }
  if (idx >= (int64_t)Lp * Lp) return;
  const int i = (int)(idx / Lp), c = (int)(idx % Lp);
  M[idx] = (i < l && c < l) ? R[(int64_t)i * l + c] : 0.0;
  P[idx] = (i == c && i < l) ? 1.0 : 0.0;
}

}  // namespace

int64_t jacobi_padded(int64_t l) {
  int64_t nb = (l + 15) / 16;
  if (nb & 1) nb++;
  if (nb < 2) nb = 2;
  return nb * 16;
}

rsvd_status block_jacobi(int64_t l, const double* R, double* M, double* P, int max_sweeps,
                         int inner_sweeps, DevState* st, hipStream_t s, int share) {
  const int Lp = (int)jacobi_padded(l);
  const int64_t tot = (int64_t)Lp * Lp;
  hipLaunchKernelGGL(jac_init_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, (int)l,
                     Lp, R, M, P, st);
  RSVD_LAUNCH_CHECK();
  JacArgs a;
  a.l = (int)l;
  a.Lp = Lp;
  a.max_sweeps = max_sweeps > 64 ? 64 : max_sweeps;
  a.inner_sweeps = inner_sweeps;
  a.M = M;
  a.P = P;
  a.st = st;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return RSVD_EHIP;
  int ncu = 0, per_cu = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return RSVD_EHIP;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)bjacobi_kernel, 256, 0) !=
      hipSuccess)
    return RSVD_EHIP;
  int grid = (Lp / 16) / 2;
  // grids of concurrent runs (share of them) must fit on the device together:
  // half of a fair share, so that grids of different kernels also fit
  int cap = ncu * (per_cu > 0 ? per_cu : 1) / (share > 1 ? 2 * share : 1);
  if (cap < 1) cap = 1;
  if (grid > cap) grid = cap;
  hipLaunchKernelGGL(bjacobi_kernel, dim3(grid), dim3(256), 0, s, a);
  RSVD_LAUNCH_CHECK();
  return RSVD_OK;
}

}  // namespace rsvd
