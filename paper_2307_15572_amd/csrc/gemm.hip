// FP64 matrix-core GEMM for the streaming products of the randomized SVD:
// the sketch Z = A P (section "Randomized matrix decompositions", step 1),
// the power-iteration products A^T Q and A Q, the projection Q^T A (step 2,
// computed as its transpose A^T Q), Gram matrices of the QR and the lifts
// (step 3).
//
//   C (M x N) = alpha * op(A) (M x K) * B (K x N) + beta * C, all row-major.
//   op(A) = A (M x K, lda) or A^T with A stored K x M (lda).
//
// Design (gfx950): one workgroup = 4 waves; each wave owns 16 rows of C and
// NT 16-wide column tiles, so a workgroup tile is 64 x 16*NT. The big operand
// op(A) is streamed straight from HBM into registers (each lane reads the
// elements it feeds to v_mfma_f64_16x16x4f64; 16 lanes cover one 128-byte
// line); the small operand B goes through double-buffered LDS chunks of 16
// rows and is shared by the 4 waves. Every element of A is read once per
// column block, so with N <= 272 (NT = 17) A is streamed exactly once.
// Workgroups are numbered so each XCD (8 of them, dispatched round-robin)
// owns a contiguous range of (split, row block, column block) items: column
// blocks of one row strip and row strips of one K range share that XCD's L2.
// Split-K writes FP64 partial tiles that a second kernel sums in a fixed
// order (deterministic; no floating-point atomics).
#include "common.hpp"
#include "kernels.hpp"

namespace rsvd {

namespace {

constexpr int kWM = 4;      // waves per workgroup, stacked along rows
constexpr int kBK = 16;     // K chunk per LDS stage
constexpr int kThreads = 64 * kWM;
constexpr int kMaxNT = 17;  // 17 x 16 = 272 columns per workgroup

struct GemmArgs {
  int64_t M, N, K, kchunk;
  double alpha, beta;
  const double* A; int64_t lda;
  const double* B; int64_t ldb;
  double* C; int64_t ldc;
  double* part;            // split-K partials [S][M][N] or nullptr
  int tiles_m, tiles_n, splits;
  const uint32_t* pred;    // if non-null and *pred == 0 the launch does nothing
  const double* Aref;      // residual mode: the matrix the product approximates
  int64_t ldref;
  double* rpart;           // residual mode: per-workgroup partial sums [2][items]
};

template <bool TA, int NT, bool RES>
__global__ void __launch_bounds__(kThreads) dgemm_kernel(GemmArgs g) {
  constexpr int BN = NT * 16;
  constexpr int BEL = kBK * BN;
  constexpr int BPER = (BEL + kThreads - 1) / kThreads;
  __shared__ double Bs[2][BEL];
  if (g.pred != nullptr && *g.pred == 0) return;

  // XCD-aware item order: item = (z * tiles_m + tm) * tiles_n + tn
  const int total = g.tiles_m * g.tiles_n * g.splits;
  const int full = total & ~7;
  int b = blockIdx.x;
  int item = b;
  if (b < full) item = (b & 7) * (full >> 3) + (b >> 3);
  const int tn = item % g.tiles_n;
  const int tm = (item / g.tiles_n) % g.tiles_m;
  const int z = item / (g.tiles_n * g.tiles_m);

  const int64_t kb = (int64_t)z * g.kchunk;
  const int64_t ke = min(g.K, kb + g.kchunk);
  const int nk = (int)((ke - kb + kBK - 1) / kBK);

  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int r = lane & 15;
  const int gq = lane >> 4;
  const int64_t row0 = (int64_t)tm * (16 * kWM) + wave * 16;
  const int64_t col0 = (int64_t)tn * BN;
  const int64_t arow = row0 + r;
  const bool arow_ok = arow < g.M;

  const double* __restrict__ A = g.A;
  const double* __restrict__ B = g.B;

  d4 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; t++) acc[t] = (d4){0.0, 0.0, 0.0, 0.0};

  double a_cur[4], a_nxt[4];
  double b_stage[BPER];

  // lane (r, gq) feeds k = k0 + 4 s + gq at MFMA step s
  auto load_a = [&](int64_t k0, double* a) {
#pragma unroll
    for (int s = 0; s < 4; s++) {
      const int64_t k = k0 + 4 * s + gq;
      double v = 0.0;
      if (arow_ok && k < ke) v = TA ? A[k * g.lda + arow] : A[arow * g.lda + k];
      a[s] = v;
    }
  };
  auto load_b = [&](int64_t k0) {
#pragma unroll
    for (int i = 0; i < BPER; i++) {
      const int idx = threadIdx.x + i * kThreads;
      double v = 0.0;
      if (idx < BEL) {
        const int kk = idx / BN, cc = idx % BN;
        const int64_t k = k0 + kk, c = col0 + cc;
        if (k < ke && c < g.N) v = B[k * g.ldb + c];
      }
      b_stage[i] = v;
    }
  };
  auto store_b = [&](int buf) {
#pragma unroll
    for (int i = 0; i < BPER; i++) {
      const int idx = threadIdx.x + i * kThreads;
      if (idx < BEL) Bs[buf][idx] = b_stage[i];
    }
  };

  if (nk > 0) {
    load_a(kb, a_cur);
    load_b(kb);
    store_b(0);
  }
  __syncthreads();
  for (int c = 0; c < nk; c++) {
    const int buf = c & 1;
    const bool more = c + 1 < nk;
    if (more) {
      load_a(kb + (int64_t)(c + 1) * kBK, a_nxt);
      load_b(kb + (int64_t)(c + 1) * kBK);
    }
    const double* bs = Bs[buf];
#pragma unroll
    for (int s = 0; s < 4; s++) {
#pragma unroll
      for (int t = 0; t < NT; t++) {
        const double bv = bs[(4 * s + gq) * BN + 16 * t + r];
        acc[t] = mfma_f64_16x16x4(a_cur[s], bv, acc[t]);
      }
    }
    if (more) {
      store_b(buf ^ 1);
#pragma unroll
      for (int s = 0; s < 4; s++) a_cur[s] = a_nxt[s];
    }
    __syncthreads();
  }

  // D layout: lane (r, gq), item it -> row gq + 4 it, column r of the 16x16 tile
  if constexpr (RES) {
    // residual epilogue: sum (Aref - C)^2 and Aref^2 over the tile
    double sd = 0.0, sa = 0.0;
#pragma unroll
    for (int t = 0; t < NT; t++) {
#pragma unroll
      for (int it = 0; it < 4; it++) {
        const int64_t row = row0 + gq + 4 * it;
        const int64_t col = col0 + 16 * t + r;
        if (row < g.M && col < g.N) {
          const double a = g.Aref[row * g.ldref + col];
          const double d = a - acc[t][it];
          sd += d * d;
          sa += a * a;
        }
      }
    }
    sd = wave_sum(sd);
    sa = wave_sum(sa);
    __shared__ double red[2][kWM];
    if (lane == 0) {
      red[0][wave] = sd;
      red[1][wave] = sa;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double a0 = 0.0, a1 = 0.0;
      for (int w = 0; w < kWM; w++) {
        a0 += red[0][w];
        a1 += red[1][w];
      }
      g.rpart[item] = a0;
      g.rpart[total + item] = a1;
    }
    return;
  }
#pragma unroll
  for (int t = 0; t < NT; t++) {
#pragma unroll
    for (int it = 0; it < 4; it++) {
      const int64_t row = row0 + gq + 4 * it;
      const int64_t col = col0 + 16 * t + r;
      if (row < g.M && col < g.N) {
        const double v = acc[t][it];
        if (g.part) {
          g.part[((int64_t)z * g.M + row) * g.N + col] = v;
        } else {
          double o = g.alpha * v;
          if (g.beta != 0.0) o += g.beta * g.C[row * g.ldc + col];
          g.C[row * g.ldc + col] = o;
        }
      }
    }
  }
}

// C = alpha * sum_z part[z] + beta * C, summed in split order.
__global__ void __launch_bounds__(256) splitk_reduce_kernel(int64_t M, int64_t N, int S,
                                                            const double* __restrict__ part,
                                                            double alpha, double beta,
                                                            double* __restrict__ C, int64_t ldc,
                                                            const uint32_t* pred) {
  if (pred != nullptr && *pred == 0) return;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= M * N) return;
  const int64_t row = idx / N, col = idx % N;
  double s = 0.0;
  for (int z = 0; z < S; z++) s += part[(int64_t)z * M * N + idx];
  double o = alpha * s;
  if (beta != 0.0) o += beta * C[row * ldc + col];
  C[row * ldc + col] = o;
}

template <bool TA, bool RES>
hipError_t launch_nt(int nt, dim3 grid, hipStream_t st, const GemmArgs& a) {
  switch (nt) {
#define RSVD_CASE(X) case X: hipLaunchKernelGGL((dgemm_kernel<TA, X, RES>), grid, dim3(kThreads), 0, st, a); break;
    RSVD_CASE(1) RSVD_CASE(2) RSVD_CASE(3) RSVD_CASE(4) RSVD_CASE(5) RSVD_CASE(6)
    RSVD_CASE(7) RSVD_CASE(8) RSVD_CASE(9) RSVD_CASE(10) RSVD_CASE(11) RSVD_CASE(12)
    RSVD_CASE(13) RSVD_CASE(14) RSVD_CASE(15) RSVD_CASE(16) RSVD_CASE(17)
#undef RSVD_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

GemmShape dgemm_shape(int64_t M, int64_t N, int64_t K, int max_splits) {
  GemmShape s;
  const int64_t ntiles = (N + 15) / 16;
  const int64_t nblk = (ntiles + kMaxNT - 1) / kMaxNT;
  s.nt = (int)((ntiles + nblk - 1) / nblk);
  s.tiles_n = (int)nblk;
  s.tiles_m = (int)((M + 16 * kWM - 1) / (16 * kWM));
  const int64_t T = (int64_t)s.tiles_m * s.tiles_n;
  int S = 1;
  // aim for >= 512 workgroups (two per CU) with at least 128 of K per split
  while (S < max_splits && T * S < 512 && K / (2 * S) >= 128) S *= 2;
  int64_t kchunk = ((K + S - 1) / S + kBK - 1) / kBK * kBK;
  if (kchunk < kBK) kchunk = kBK;
  S = (int)((K + kchunk - 1) / kchunk);
  if (S < 1) S = 1;
  s.splits = S;
  s.kchunk = kchunk;
  s.part_doubles = S > 1 ? (size_t)S * M * N : 0;
  return s;
}

rsvd_status dgemm(bool ta, int64_t M, int64_t N, int64_t K, double alpha, const double* A,
                  int64_t lda, const double* B, int64_t ldb, double beta, double* C, int64_t ldc,
                  double* part, size_t part_doubles, hipStream_t st, int max_splits,
                  const uint32_t* pred) {
  if (M <= 0 || N <= 0) return RSVD_OK;
  if (K <= 0) {
    // C = beta * C
    GemmArgs a{};
    (void)a;
    const int64_t tot = M * N;
    hipLaunchKernelGGL(splitk_reduce_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st,
                       M, N, 0, (const double*)nullptr, alpha, beta, C, ldc, pred);
    RSVD_LAUNCH_CHECK();
    return RSVD_OK;
  }
  GemmShape s = dgemm_shape(M, N, K, max_splits);
  if (s.splits > 1 && (part == nullptr || part_doubles < s.part_doubles)) {
    // not enough scratch for split-K: run unsplit
    s.splits = 1;
    s.kchunk = K;
    s.part_doubles = 0;
  }
  GemmArgs a;
  a.M = M; a.N = N; a.K = K; a.kchunk = s.kchunk;
  a.alpha = alpha; a.beta = beta;
  a.A = A; a.lda = lda; a.B = B; a.ldb = ldb; a.C = C; a.ldc = ldc;
  a.part = s.splits > 1 ? part : nullptr;
  a.tiles_m = s.tiles_m; a.tiles_n = s.tiles_n; a.splits = s.splits;
  a.pred = pred; a.Aref = nullptr; a.ldref = 0; a.rpart = nullptr;
  const int64_t total = (int64_t)s.tiles_m * s.tiles_n * s.splits;
  dim3 grid((unsigned)total);
  hipError_t e = ta ? launch_nt<true, false>(s.nt, grid, st, a)
                    : launch_nt<false, false>(s.nt, grid, st, a);
  if (e != hipSuccess) return RSVD_EHIP;
  if (s.splits > 1) {
    const int64_t tot = M * N;
    hipLaunchKernelGGL(splitk_reduce_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st,
                       M, N, s.splits, (const double*)part, alpha, beta, C, ldc, pred);
    RSVD_LAUNCH_CHECK();
  }
  return RSVD_OK;
}

size_t resid_partials(int64_t M, int64_t N) {
  GemmShape s = dgemm_shape(M, N, 1, 1);
  return (size_t)2 * s.tiles_m * s.tiles_n;
}

rsvd_status resid(int64_t M, int64_t N, int64_t K, const double* US, int64_t ldus,
                  const double* Vt, int64_t ldvt, const double* A, int64_t lda, double* partial,
                  DevState* st, hipStream_t s) {
  GemmShape sh = dgemm_shape(M, N, K, 1);
  GemmArgs a;
  a.M = M; a.N = N; a.K = K; a.kchunk = ((K + kBK - 1) / kBK) * kBK;
  a.alpha = 1.0; a.beta = 0.0;
  a.A = US; a.lda = ldus; a.B = Vt; a.ldb = ldvt; a.C = nullptr; a.ldc = 0;
  a.part = nullptr;
  a.tiles_m = sh.tiles_m; a.tiles_n = sh.tiles_n; a.splits = 1;
  a.pred = nullptr; a.Aref = A; a.ldref = lda; a.rpart = partial;
  const int64_t total = (int64_t)sh.tiles_m * sh.tiles_n;
  hipError_t e = launch_nt<false, true>(sh.nt, dim3((unsigned)total), s, a);
  if (e != hipSuccess) return RSVD_EHIP;
  rsvd_status r = sum_partials_into(total, partial, &st->resid2, s);
  if (r != RSVD_OK) return r;
  return sum_partials_into(total, partial + total, &st->fro2, s);
}

}  // namespace rsvd
