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
// Waves per workgroup (template W, 4 or 8): all of them load and multiply in
// the Gram and the apply; the first four (256 threads, one per 2 x 2 block of
// the 32 x 32 rotation problem) run the inner rounds while the others wait at
// its barriers. Eight waves halve a pair's load time but fit one workgroup
// per CU; four fit two, which matters when pairs outnumber the grid.

// x mod m for 0 <= x < 2 m
__device__ __forceinline__ int mod_once(int x, int m) { return x >= m ? x - m : x; }

// Pair i of step `step` (0 <= step, i < L - 1) of the circle tournament on L
// players: player L - 1 is fixed, the others rotate.
__device__ __forceinline__ void rr_pair_blk(int L, int step, int i, int& a, int& b) {
  a = i == 0 ? L - 1 : mod_once(step + i, L - 1);
  b = i == 0 ? step : mod_once(step - i + (L - 1), L - 1);
}



struct JacArgs {
  int l, Lp, max_sweeps, inner_sweeps;
  double* M;
  double* P;
  DevState* st;
};

// Rotation that annihilates h_pq of the symmetric 2 x 2 [h_pp h_pq; h_pq h_qq]:
// with d = h_qq - h_pp and e = 2 h_pq, Rutishauser's t = sign(zeta) / (|zeta| +
// sqrt(1 + zeta^2)), zeta = d / e, is t = sign(d) e / D with D = |d| +
// sqrt(d^2 + e^2), and c = 1 / sqrt(1 + t^2) = D / sqrt(D^2 + e^2), s = c t =
// sign(d) e / sqrt(D^2 + e^2). d and e are first scaled by the same power of
// two (exact) to a largest magnitude in [0.5, 1), so no square over- or
// underflows; c and s come from one inverse square root (rsq_nr, to about an
// ulp), so c^2 + s^2 = 1 to a few ulps. Identity when |h_pq| <= tol
// sqrt(h_pp h_qq). Two refined inverse square roots in sequence, no
// reciprocal and no special cases.
__device__ __forceinline__ void jac_rot(double hpp, double hqq, double hpq, double tol, double& c,
                                        double& s) {
  const bool rot = fabs(hpq) > tol * sqrt(hpp) * sqrt(hqq) && hpq != 0.0;
  const double e = 2.0 * hpq, d = hqq - hpp;
  const int ex = __builtin_amdgcn_frexp_exp(fmax(fabs(d), fabs(e)));
  const double ds = __builtin_amdgcn_ldexp(d, -ex), es = __builtin_amdgcn_ldexp(e, -ex);
  const double q = fma(ds, ds, es * es);          // [0.25, 2)
  const double D = fabs(ds) + q * rsq_nr(q);      // [0.5, 1 + sqrt 2)
  const double rho = rsq_nr(fma(D, D, es * es));  // 1 / sqrt(D^2 + e^2)
  c = rot ? D * rho : 1.0;
  s = rot ? copysign(1.0, d) * es * rho : 0.0;
}

// Returns true if the pair needed rotating. dsq: 32 doubles of LDS.
// jl: kJacLds doubles of LDS holding the Gram's partial sums, and after them
// (the same memory) the double-buffered 32 x 32 H and the rotations V.
constexpr int kJacLds = 8 * 3 * 256;
template <int kJacWaves>
__device__ bool process_pair(const JacArgs& a, int I, int J, double tol, double* jl, double* dsq,
                             int* s_any) {
  double (*Hb)[32][33] = reinterpret_cast<double (*)[32][33]>(jl);
  double* red = jl;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
  double (*H)[33] = Hb[0];
  const int Lp = a.Lp;
  const int nct = Lp / 16;
  const double* rI = a.M + (int64_t)16 * I * Lp;
  const double* rJ = a.M + (int64_t)16 * J * Lp;

  // ---- Gram of the 32 rows (tiles 00, 01, 11), the column tiles split into
  // kGramParts partial sums by their index mod kGramParts, whatever the
  // number of waves (a wave takes parts wave, wave + W, ...): every part is
  // summed in increasing tile order and the parts in increasing order, so
  // the Gram is bitwise the same for 4 and 8 waves. GB column tiles of a
  // part in flight together.
  constexpr int kGramParts = 8;
  constexpr int PW = kGramParts / kJacWaves;  // parts per wave
  constexpr int GB = kJacWaves == 8 ? 3 : 2;
  d4 h00[PW], h01[PW], h11[PW];
#pragma unroll
  for (int pw = 0; pw < PW; pw++) h00[pw] = h01[pw] = h11[pw] = d4{0, 0, 0, 0};
#pragma unroll
  for (int pw = 0; pw < PW; pw++) {
    const int part = wave + kJacWaves * pw;
    for (int ct0 = part; ct0 < nct; ct0 += kGramParts * GB) {
      double xi[GB][4], xj[GB][4];
#pragma unroll
      for (int u = 0; u < GB; u++) {
        const int c0 = 16 * (ct0 + kGramParts * u) + 4 * g;
        if (ct0 + kGramParts * u < nct) {
#pragma unroll
          for (int s = 0; s < 4; s++) {
            xi[u][s] = rI[(int64_t)r * Lp + c0 + s];
            xj[u][s] = rJ[(int64_t)r * Lp + c0 + s];
          }
        }
      }
#pragma unroll
      for (int u = 0; u < GB; u++) {
        if (ct0 + kGramParts * u < nct) {
#pragma unroll
          for (int s = 0; s < 4; s++) {
            h00[pw] = mfma_f64_16x16x4(xi[u][s], xi[u][s], h00[pw]);
            h01[pw] = mfma_f64_16x16x4(xi[u][s], xj[u][s], h01[pw]);
            h11[pw] = mfma_f64_16x16x4(xj[u][s], xj[u][s], h11[pw]);
          }
        }
      }
    }
  }
#pragma unroll
  for (int pw = 0; pw < PW; pw++) {
    const int part = wave + kJacWaves * pw;
#pragma unroll
    for (int it = 0; it < 4; it++) {
      const int e = (g + 4 * it) * 16 + r;
      red[(part * 3 + 0) * 256 + e] = h00[pw][it];
      red[(part * 3 + 1) * 256 + e] = h01[pw][it];
      red[(part * 3 + 2) * 256 + e] = h11[pw][it];
    }
  }
  if (threadIdx.x == 0) *s_any = 0;
  __syncthreads();
  // the parts summed into registers first: H lives in the same memory
  const int e = threadIdx.x;
  double v0 = 0, v1 = 0, v2 = 0;
  if (e < 256) {
    for (int w = 0; w < kGramParts; w++) {
      v0 += red[(w * 3 + 0) * 256 + e];
      v1 += red[(w * 3 + 1) * 256 + e];
      v2 += red[(w * 3 + 2) * 256 + e];
    }
  }
  __syncthreads();
  if (e < 256) {
    const int i = e / 16, j = e % 16;
    H[i][j] = v0;
    H[i][16 + j] = v1;
    H[16 + j][i] = v1;
    H[16 + i][16 + j] = v2;
    if (i == j) {
      dsq[i] = sqrt(v0);
      dsq[16 + i] = sqrt(v2);
    }
  }
  __syncthreads();
  // ---- any pair above tolerance? (|h_ij| > tol sqrt(h_ii) sqrt(h_jj))
  for (int e = threadIdx.x; e < 32 * 32; e += blockDim.x) {
    const int i = e / 32, j = e % 32;
    if (i < j) {
      const double hij = H[i][j];
      if (fabs(hij) > tol * dsq[i] * dsq[j] && hij != 0.0) *s_any = 1;
    }
  }
  __syncthreads();
  if (*s_any == 0) return false;

  // ---- two-sided Jacobi on H, V accumulates the rotations. A round applies
  // 16 disjoint plane rotations J_k on both sides, H <- J^T H J, V <- V J:
  // thread (k, m) applies J_k^T and J_m to the 2 x 2 block of H at rows
  // {p_k, q_k} and columns {p_m, q_m} (the arithmetic, in the same order, of
  // a row pass followed by a column pass) and J_m to the same entries of V.
  // Every lane forms the rotation of its column pair m itself (each wave
  // holds all 16) and takes J_k from lane k of its wave by a shuffle, so a
  // round needs no exchange through LDS; H is double buffered (a round reads
  // one buffer and writes the other, since other threads read the diagonal
  // entries of a block its owner rewrites), which leaves one barrier per
  // round. The blocks partition V, so V is updated in place.
  double (*V)[33] = reinterpret_cast<double (*)[33]>(jl + 2 * 32 * 33);
  for (int e = threadIdx.x; e < 32 * 32; e += blockDim.x)
    V[e / 32][e % 32] = (e / 32 == e % 32) ? 1.0 : 0.0;
  __syncthreads();
  {
    const int k = threadIdx.x >> 4, mm = threadIdx.x & 15;
    const bool rounds = threadIdx.x < 256;
    int cur = 0;
    for (int isw = 0; isw < a.inner_sweeps; isw++) {
      for (int round = 0; round < 31; round++) {
        if (!rounds) {
          __syncthreads();
          continue;
        }
        double (*Hc)[33] = Hb[cur];
        double (*Hn)[33] = Hb[cur ^ 1];
        int pk, qk, pm, qm;
        rr_pair_blk(32, round, k, pk, qk);
        if (pk > qk) { const int t = pk; pk = qk; qk = t; }
        rr_pair_blk(32, round, mm, pm, qm);
        if (pm > qm) { const int t = pm; pm = qm; qm = t; }
        // all reads of the round first: the rotation's three entries and
        // this thread's blocks of H and V
        const double dpp = Hc[pm][pm], dqq = Hc[qm][qm], dpq = Hc[pm][qm];
        double hpp = Hc[pk][pm], hpq = Hc[pk][qm], hqp = Hc[qk][pm], hqq = Hc[qk][qm];
        double vpp = V[pk][pm], vpq = V[pk][qm], vqp = V[qk][pm], vqq = V[qk][qm];
        double cm, sm;
        jac_rot(dpp, dqq, dpq, tol, cm, sm);
        const double ck = __shfl(cm, k & 15, 64), sk = __shfl(sm, k & 15, 64);
        // rows: J_k^T, then columns: J_m (an identity rotation, c = 1 and
        // s = 0, leaves finite entries exactly as they are)
        {
          const double a0 = ck * hpp - sk * hqp, a1 = sk * hpp + ck * hqp;
          const double b0 = ck * hpq - sk * hqq, b1 = sk * hpq + ck * hqq;
          hpp = a0; hqp = a1; hpq = b0; hqq = b1;
        }
        {
          const double a0 = cm * hpp - sm * hpq, a1 = sm * hpp + cm * hpq;
          const double b0 = cm * hqp - sm * hqq, b1 = sm * hqp + cm * hqq;
          hpp = a0; hpq = a1; hqp = b0; hqq = b1;
        }
        Hn[pk][pm] = hpp;
        Hn[pk][qm] = hpq;
        Hn[qk][pm] = hqp;
        Hn[qk][qm] = hqq;
        {
          const double a0 = cm * vpp - sm * vpq, a1 = sm * vpp + cm * vpq;
          const double b0 = cm * vqp - sm * vqq, b1 = sm * vqp + cm * vqq;
          vpp = a0; vpq = a1; vqp = b0; vqq = b1;
        }
        V[pk][pm] = vpp;
        V[pk][qm] = vpq;
        V[qk][pm] = vqp;
        V[qk][qm] = vqq;
        cur ^= 1;
        __syncthreads();
      }
    }
  }
  double (*Vm)[33] = V;

  // ---- apply: rows <- V^T rows for M and P (P absent: values only); each
  // wave owns whole column tiles
  const int nmat = a.P ? 2 : 1;
  for (int mat = 0; mat < nmat; mat++) {
    double* base = mat == 0 ? a.M : a.P;
    double* bI = base + (int64_t)16 * I * Lp;
    double* bJ = base + (int64_t)16 * J * Lp;
    // AB column tiles per iteration (their loads in flight together)
    constexpr int AB = kJacWaves == 8 ? 3 : 5;
    for (int ct = wave; ct < nct; ct += kJacWaves * AB) {
      double b[AB][8];
#pragma unroll
      for (int u = 0; u < AB; u++)
#pragma unroll
        for (int s = 0; s < 8; s++) {
          const int row = 4 * s + g;  // 0..31
          const double* src = row < 16 ? bI : bJ;
          b[u][s] = ct + kJacWaves * u < nct
                        ? src[(int64_t)(row & 15) * Lp + 16 * (ct + kJacWaves * u) + r]
                        : 0.0;
        }
#pragma unroll
      for (int u = 0; u < AB; u++) {
        if (ct + kJacWaves * u >= nct) break;
        const int c = 16 * (ct + kJacWaves * u) + r;
        d4 o0 = {0, 0, 0, 0}, o1 = {0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < 8; s++) {
          o0 = mfma_f64_16x16x4(Vm[4 * s + g][r], b[u][s], o0);
          o1 = mfma_f64_16x16x4(Vm[4 * s + g][16 + r], b[u][s], o1);
        }
#pragma unroll
        for (int it = 0; it < 4; it++) {
          bI[(int64_t)(g + 4 * it) * Lp + c] = o0[it];
          bJ[(int64_t)(g + 4 * it) * Lp + c] = o1[it];
        }
      }
    }
  }
  __syncthreads();
  return true;
}

template <int kJacWaves>
__global__ void __launch_bounds__(64 * kJacWaves, kJacWaves == 4 ? 2 : 1) bjacobi_kernel(JacArgs a) {
  __shared__ int s_bar_ok;
  __shared__ double jl[kJacLds];
  __shared__ double dsq[32];
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
        const bool rot = process_pair<kJacWaves>(a, I, J, tol, jl, dsq, &s_any);
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

// M (Lp x Lp) <- R (l x l) zero padded; P (if present) <- identity on the
// leading l x l; sweep counters and the grid barrier cleared.
__global__ void __launch_bounds__(256) jac_init_kernel(int l, int Lp, const double* __restrict__ R,
                                                       double* __restrict__ M, double* __restrict__ P,
                                                       DevState* st) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (blockIdx.x == 0) {
    if (threadIdx.x < 64) st->rot_count[threadIdx.x] = 0u;
    if (threadIdx.x == 0) st->sweeps = -1;  // set when the sweeps end
    grid_barrier_reset(&st->bar);
  }
  if (idx >= (int64_t)Lp * Lp) return;
  const int i = (int)(idx / Lp), c = (int)(idx % Lp);
  M[idx] = (i < l && c < l) ? R[(int64_t)i * l + c] : 0.0;
  if (P) P[idx] = (i == c && i < l) ? 1.0 : 0.0;
}

// ---------------------------------------------------------------------------
// The small SVDs of many independent channels in one launch. Every channel
// sweeps with its own tournament (nb_c - 1 steps of nb_c / 2 pairs), and all
// channels advance in lockstep global rounds: in round r channel c runs
// step r mod (nb_c - 1) of its sweep r / (nb_c - 1), unless it has finished.
// The pairs of all active channels form one task list, dealt to the
// workgroups round-robin (the channel table is ordered by cost, longest
// first), and one grid barrier separates the rounds. Per channel, the
// rotation counter of each sweep (its phase counter) decides at the sweep's
// end, identically in every workgroup, whether it has converged; workgroup 0
// then records its sweep count and flags. process_pair is the single-run
// kernel's pair step, so each channel's rows see exactly the rotations of
// its single run. A channel left unfinished (barrier timed out) keeps
// sweeps = -1 for the caller to flag.
constexpr int kBatchJacMaxChannels = 4096;

template <int kJacWaves>
__global__ void __launch_bounds__(64 * kJacWaves, kJacWaves == 4 ? 2 : 1)
    bjacobi_batch_kernel(const JacChan* __restrict__ ch, int nch, char* __restrict__ work,
                         GridBar* bar) {
  __shared__ int s_bar_ok;
  __shared__ double jl[kJacLds];
  __shared__ double dsq[32];
  __shared__ int s_any;
  __shared__ uint32_t done[kBatchJacMaxChannels / 32];
  for (int i = threadIdx.x; i < kBatchJacMaxChannels / 32; i += blockDim.x) done[i] = 0u;
  __syncthreads();
  int remaining = nch;
  for (int r = 0; remaining > 0; r++) {
    // sweep ends: channels whose previous round closed a sweep
    for (int c = 0; c < nch; c++) {
      if (done[c >> 5] & (1u << (c & 31))) continue;
      const int steps = ch[c].Lp / 16 - 1;
      if (r == 0 || r % steps != 0) continue;
      const int sw = r / steps;  // sweeps completed
      DevState* st = reinterpret_cast<DevState*>(work + ch[c].st_off);
      const uint32_t cnt =
          __hip_atomic_load(&st->rot_count[sw - 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const bool conv = cnt == 0u;
      if (conv || sw >= ch[c].max_sweeps) {
        __syncthreads();
        if (threadIdx.x == 0) done[c >> 5] |= 1u << (c & 31);
        if (blockIdx.x == 0 && threadIdx.x == 0) {
          st->sweeps = sw;
          if (!conv)
            __hip_atomic_fetch_or(&st->flags, (uint32_t)RSVD_FLAG_JACOBI_MAXSWEEP,
                                  __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
        remaining--;
      }
    }
    if (remaining == 0) break;
    // this round's tasks: pair pr of every active channel, dealt round-robin
    int64_t base = 0;
    for (int c = 0; c < nch; c++) {
      if (done[c >> 5] & (1u << (c & 31))) continue;
      const int Lp = ch[c].Lp, nb = Lp / 16, npairs = nb / 2, steps = nb - 1;
      const int step = r % steps, sw = r / steps;
      int64_t t0 = base + (((int64_t)blockIdx.x - base) % gridDim.x + gridDim.x) % gridDim.x;
      for (int64_t t = t0; t < base + npairs; t += gridDim.x) {
        const int pr = (int)(t - base);
        int I, J;
        rr_pair_blk(nb, step, pr, I, J);
        JacArgs a;
        a.l = ch[c].l;
        a.Lp = Lp;
        a.max_sweeps = ch[c].max_sweeps;
        a.inner_sweeps = 1;
        a.M = reinterpret_cast<double*>(work + ch[c].M_off);
        a.P = ch[c].P_off >= 0 ? reinterpret_cast<double*>(work + ch[c].P_off) : nullptr;
        a.st = reinterpret_cast<DevState*>(work + ch[c].st_off);
        const double tol = (double)a.l * kU;
        const bool rot = process_pair<kJacWaves>(a, I, J, tol, jl, dsq, &s_any);
        if (rot && threadIdx.x == 0)
          __hip_atomic_fetch_add(&a.st->rot_count[sw], 1u, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
      }
      base += npairs;
    }
    if (!grid_barrier(bar, &s_bar_ok)) return;
  }
}

__global__ void jac_batch_reset_kernel(GridBar* bar) { grid_barrier_reset(bar); }

// sweeps < 0: the batched sweeps never finished this channel
__global__ void jac_check_done_kernel(DevState* st) {
  if (threadIdx.x == 0 && st->sweeps < 0)
    __hip_atomic_fetch_or(&st->flags, (uint32_t)RSVD_FLAG_SYNC_TIMEOUT, __ATOMIC_RELAXED,
                          __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace

int64_t jacobi_padded(int64_t l) {
  int64_t nb = (l + 15) / 16;
  if (nb & 1) nb++;
  if (nb < 2) nb = 2;
  return nb * 16;
}

rsvd_status jacobi_prepare(int64_t l, const double* R, double* M, double* P, DevState* st,
                           hipStream_t s) {
  const int Lp = (int)jacobi_padded(l);
  const int64_t tot = (int64_t)Lp * Lp;
  hipLaunchKernelGGL(jac_init_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, (int)l,
                     Lp, R, M, P, st);
  RSVD_LAUNCH_CHECK();
  return RSVD_OK;
}

size_t jacobi_batch_max_channels() { return kBatchJacMaxChannels; }

rsvd_status jacobi_batch(const JacChan* table, int nch, int64_t first_round_pairs, char* work,
                         GridBar* bar, hipStream_t s) {
  if (nch < 1) return RSVD_OK;
  if (nch > kBatchJacMaxChannels) return RSVD_EINVAL;
  // pairs outnumbering the CUs: 4-wave workgroups, two per CU (the pair
  // step's arithmetic, and so every channel's result, is the same for 4 and
  // 8 waves); otherwise 8 waves per pair
  int dev = 0, ncu = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return RSVD_EHIP;
  const bool four = first_round_pairs > ncu;
  const void* fn = four ? (const void*)bjacobi_batch_kernel<4> : (const void*)bjacobi_batch_kernel<8>;
  const int threads = four ? 256 : 512;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, threads, 0) != hipSuccess)
    return RSVD_EHIP;
  const int64_t cap = (int64_t)ncu * (per > 0 ? per : 1);
  int64_t grid = first_round_pairs < cap ? first_round_pairs : cap;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(jac_batch_reset_kernel, dim3(1), dim3(256), 0, s, bar);
  RSVD_LAUNCH_CHECK();
  if (four)
    hipLaunchKernelGGL(bjacobi_batch_kernel<4>, dim3((unsigned)grid), dim3(256), 0, s, table, nch,
                       work, bar);
  else
    hipLaunchKernelGGL(bjacobi_batch_kernel<8>, dim3((unsigned)grid), dim3(512), 0, s, table, nch,
                       work, bar);
  RSVD_LAUNCH_CHECK();
  return RSVD_OK;
}

rsvd_status jacobi_check_done(DevState* st, hipStream_t s) {
  hipLaunchKernelGGL(jac_check_done_kernel, dim3(1), dim3(64), 0, s, st);
  RSVD_LAUNCH_CHECK();
  return RSVD_OK;
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
  int ncu = 0, per8 = 0, per4 = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return RSVD_EHIP;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per8, (const void*)bjacobi_kernel<8>, 512, 0) !=
          hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per4, (const void*)bjacobi_kernel<4>, 256, 0) !=
          hipSuccess)
    return RSVD_EHIP;
  const int npairs = (Lp / 16) / 2;
  // grids of concurrent runs (share of them) must fit on the device together:
  // half of a fair share, so that grids of different kernels also fit
  auto cap_of = [&](int per_cu) {
    int c = ncu * (per_cu > 0 ? per_cu : 1) / (share > 1 ? 2 * share : 1);
    return c < 1 ? 1 : c;
  };
  const int cap8 = cap_of(per8), cap4 = cap_of(per4);
  if (npairs <= cap8) {
    hipLaunchKernelGGL(bjacobi_kernel<8>, dim3(npairs), dim3(512), 0, s, a);
  } else {
    hipLaunchKernelGGL(bjacobi_kernel<4>, dim3(npairs < cap4 ? npairs : cap4), dim3(256), 0, s, a);
  }
  RSVD_LAUNCH_CHECK();
  return RSVD_OK;
}

}  // namespace rsvd
