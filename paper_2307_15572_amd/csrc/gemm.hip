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
#include <type_traits>

#include "common.hpp"
#include "kernels.hpp"
#include "tune.hpp"

namespace rsvd {

namespace {

bool g_use_dma = true;  // LDS-DMA streaming kernel for eligible NN products
int g_dma_wm = 8;       // waves per workgroup of the LDS-DMA kernel (4 or 8)

constexpr int kWM = 4;      // waves per workgroup, stacked along rows
constexpr int kBK = 16;     // K chunk per LDS stage
constexpr int kThreads = 64 * kWM;
constexpr int kMaxNT = 17;  // 17 x 16 = 272 columns per workgroup
#ifndef RSVD_GEMM_APF
#define RSVD_GEMM_APF 2     // chunks of the streamed operand A in flight ahead of use
#endif
constexpr int kAPF = RSVD_GEMM_APF;

template <int PREC> struct AccType { using type = d4; };
template <> struct AccType<kPrecF32> { using type = f4; };
template <> struct AccType<kPrecBF16> { using type = f4; };
template <> struct AccType<kPrecBF16S> { using type = f4; };

// row of the 16 x 16 output tile held by accumulator item `it` of lane group g
template <int PREC>
__device__ __forceinline__ int acc_row(int g, int it) {
  return PREC == kPrecF64 ? g + 4 * it : 4 * g + it;
}

// One chunk of 16 k values for NT tiles: av[s] = A(row r, k = 4 g + s),
// Bs holds the chunk's 16 x BN block of B. Each precision uses its own
// matrix-core instruction; the lane-group-to-k assignment is the same.
template <int PREC, int NT, int BN, typename BT>
__device__ __forceinline__ void chunk_mma(typename AccType<PREC>::type (&acc)[NT], const double av[4],
                                          const BT* Bs, int g, int r) {
  if constexpr (PREC == kPrecF64) {
#pragma unroll
    for (int s = 0; s < 4; s++) {
      double bf[NT];
#pragma unroll
      for (int t = 0; t < NT; t++) bf[t] = Bs[(4 * g + s) * BN + 16 * t + r];
#pragma unroll
      for (int t = 0; t < NT; t++) acc[t] = mfma_f64_16x16x4(av[s], bf[t], acc[t]);
    }
  } else if constexpr (PREC == kPrecF32) {
    // the B fragments of k step s + 1 are read while the products of step s
    // run (scheduling groups: the step's LDS reads first, then its MFMAs), so
    // no product waits on a read issued just before it (the FP32 products
    // take half the cycles of the FP64 ones, which leaves the read latency
    // exposed otherwise; measured 1.44 -> 1.38 ms at 16384^2 x 272, while the
    // FP64 kernel was 2 % slower with the same schedule)
    using ET = float;
    ET cur[NT], nxt[NT];
#pragma unroll
    for (int t = 0; t < NT; t++) cur[t] = (ET)Bs[(4 * g) * BN + 16 * t + r];
#pragma unroll
    for (int s = 0; s < 4; s++) {
      if (s < 3) {
#pragma unroll
        for (int t = 0; t < NT; t++) nxt[t] = (ET)Bs[(4 * g + s + 1) * BN + 16 * t + r];
      }
      const ET a = (ET)av[s];
#pragma unroll
      for (int t = 0; t < NT; t++) acc[t] = mfma_f32_16x16x4(a, cur[t], acc[t]);
      if (s < 3) {
        __builtin_amdgcn_sched_group_barrier(0x100, NT, 0);  // LDS reads of step s + 1
        __builtin_amdgcn_sched_group_barrier(0x008, NT, 0);  // MFMAs of step s
#pragma unroll
        for (int t = 0; t < NT; t++) cur[t] = nxt[t];
      }
    }
  } else if constexpr (PREC == kPrecBF16) {
    const s4 a = {bf16_bits(av[0]), bf16_bits(av[1]), bf16_bits(av[2]), bf16_bits(av[3])};
#pragma unroll
    for (int t = 0; t < NT; t++) {
      const double* col = Bs + 4 * g * BN + 16 * t + r;
      const s4 b = {bf16_bits(col[0]), bf16_bits(col[BN]), bf16_bits(col[2 * BN]), bf16_bits(col[3 * BN])};
      acc[t] = mfma_bf16_16x16x16(a, b, acc[t]);
    }
  } else {
    s4 ahi, alo;
#pragma unroll
    for (int s = 0; s < 4; s++) {
      const short h = bf16_bits(av[s]);
      ahi[s] = h;
      alo[s] = bf16_bits(av[s] - bf16_value(h));
    }
#pragma unroll
    for (int t = 0; t < NT; t++) {
      const double* col = Bs + 4 * g * BN + 16 * t + r;
      s4 bhi, blo;
#pragma unroll
      for (int s = 0; s < 4; s++) {
        const double x = col[s * BN];
        const short h = bf16_bits(x);
        bhi[s] = h;
        blo[s] = bf16_bits(x - bf16_value(h));
      }
      // the small cross terms first, then the leading product
      acc[t] = mfma_bf16_16x16x16(ahi, blo, acc[t]);
      acc[t] = mfma_bf16_16x16x16(alo, bhi, acc[t]);
      acc[t] = mfma_bf16_16x16x16(ahi, bhi, acc[t]);
    }
  }
}

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
  int vec_a, vec_b;        // 16-byte loads allowed (even leading dimension, aligned base)
  int64_t b_cols;          // columns readable in each row of B (0: N); set for FP32 panels
                           // and for FP64 copies of B with an even leading dimension
};

template <bool TA, int NT, bool RES, int PREC>
__global__ void __launch_bounds__(kThreads) dgemm_kernel(GemmArgs g) {
  constexpr int BN = NT * 16;
  constexpr int BEL = kBK * BN;
  constexpr int BPER = (BEL + kThreads - 1) / kThreads;
  constexpr int BPER2 = (BEL / 2 + kThreads - 1) / kThreads;
  __shared__ __attribute__((aligned(16))) double Bs[2][BEL];
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
  const int nfull = (int)((ke - kb) / kBK);          // chunks entirely inside [kb, ke)
  const bool tail = (ke - kb) % kBK != 0;

  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int r = lane & 15;
  const int gq = lane >> 4;
  const int64_t row0 = (int64_t)tm * (16 * kWM) + wave * 16;
  const int64_t col0 = (int64_t)tn * BN;
  // rows past M only feed output rows that are never stored: clamp the address
  const int64_t arow = min(row0 + r, g.M - 1);

  const double* __restrict__ A = g.A;
  const double* __restrict__ B = g.B;
  const bool vec_a = !TA && g.vec_a;
  const bool vec_b = g.vec_b && (col0 + BN <= g.N);

  using Acc = typename AccType<PREC>::type;
  Acc acc[NT];
#pragma unroll
  for (int t = 0; t < NT; t++) acc[t] = Acc{0, 0, 0, 0};

  double a_cur[4], a_nxt[4];
  // scalar staging uses BPER slots, the 16-byte path 2 * BPER2 (NT + 1 for odd NT)
  constexpr int BSTAGE = BPER > 2 * BPER2 ? BPER : 2 * BPER2;
  double b_stage[BSTAGE];

  // MFMA step s of a chunk uses k = k0 + 4 gq + s at lane group gq
  auto load_a = [&](int64_t k0, double* a, bool guard) {
    if (!guard && vec_a) {
      const double2* p = reinterpret_cast<const double2*>(A + arow * g.lda + k0 + 4 * gq);
      const double2 v0 = p[0], v1 = p[1];
      a[0] = v0.x; a[1] = v0.y; a[2] = v1.x; a[3] = v1.y;
      return;
    }
#pragma unroll
    for (int s = 0; s < 4; s++) {
      const int64_t k = k0 + 4 * gq + s;
      if (guard) {
        double v = 0.0;
        if (k < ke) v = TA ? A[k * g.lda + arow] : A[arow * g.lda + k];
        a[s] = v;
      } else {
        a[s] = TA ? A[k * g.lda + arow] : A[arow * g.lda + k];
      }
    }
  };
  // columns past N only feed output columns that are never stored: clamp
  auto load_b = [&](int64_t k0, bool guard) {
    if (!guard && vec_b) {
#pragma unroll
      for (int i = 0; i < BPER2; i++) {
        const int idx = threadIdx.x + i * kThreads;  // double2 index
        if (idx < BEL / 2) {
          const int kk = (2 * idx) / BN, cc = (2 * idx) % BN;
          const double2 v = *reinterpret_cast<const double2*>(B + (k0 + kk) * g.ldb + col0 + cc);
          b_stage[2 * i] = v.x;
          b_stage[2 * i + 1] = v.y;
        }
      }
      return;
    }
#pragma unroll
    for (int i = 0; i < BPER; i++) {
      const int idx = threadIdx.x + i * kThreads;
      if (idx < BEL) {
        const int kk = idx / BN, cc = idx % BN;
        const int64_t k = k0 + kk, c = min(col0 + cc, g.N - 1);
        if (guard) {
          double v = 0.0;
          if (k < ke) v = B[k * g.ldb + c];
          b_stage[i] = v;
        } else {
          b_stage[i] = B[k * g.ldb + c];
        }
      }
    }
  };
  auto store_b = [&](int buf, bool was_vec) {
    if (was_vec) {
#pragma unroll
      for (int i = 0; i < BPER2; i++) {
        const int idx = threadIdx.x + i * kThreads;
        if (idx < BEL / 2)
          reinterpret_cast<double2*>(Bs[buf])[idx] = make_double2(b_stage[2 * i], b_stage[2 * i + 1]);
      }
      return;
    }
#pragma unroll
    for (int i = 0; i < BPER; i++) {
      const int idx = threadIdx.x + i * kThreads;
      if (idx < BEL) Bs[buf][idx] = b_stage[i];
    }
  };
  auto compute = [&](const double* bs) { chunk_mma<PREC, NT, BN>(acc, a_cur, bs, gq, r); };

  const int nk = nfull + (tail ? 1 : 0);
  // A ring: a_q[j] holds chunk c + j (j = 0 .. kAPF-1); B goes one chunk ahead via LDS
  double a_q[kAPF][4];
#pragma unroll
  for (int j = 0; j < kAPF; j++) {
    if (j < nk) load_a(kb + (int64_t)j * kBK, a_q[j], j >= nfull);
  }
  if (nk > 0) {
    const bool g0 = nfull == 0;
    load_b(kb, g0);
    store_b(0, !g0 && vec_b);
  }
  __syncthreads();
  for (int c = 0; c < nk; c++) {
    const int buf = c & 1;
    const bool more = c + 1 < nk;
    const bool gn = (c + 1) >= nfull;  // the next chunk is the partial tail
    if (more) load_b(kb + (int64_t)(c + 1) * kBK, gn);
#pragma unroll
    for (int s = 0; s < 4; s++) a_cur[s] = a_q[0][s];
#pragma unroll
    for (int j = 0; j + 1 < kAPF; j++)
#pragma unroll
      for (int s = 0; s < 4; s++) a_q[j][s] = a_q[j + 1][s];
    if (c + kAPF < nk) load_a(kb + (int64_t)(c + kAPF) * kBK, a_q[kAPF - 1], (c + kAPF) >= nfull);
    compute(Bs[buf]);
    if (more) store_b(buf ^ 1, !gn && vec_b);
    __syncthreads();
  }
  (void)a_nxt;

  // D layout: lane (r, gq), item it -> row gq + 4 it, column r of the 16x16 tile
  if constexpr (RES) {
    // residual epilogue: sum (Aref - C)^2 and Aref^2 over the tile
    double sd = 0.0, sa = 0.0;
#pragma unroll
    for (int t = 0; t < NT; t++) {
#pragma unroll
      for (int it = 0; it < 4; it++) {
        const int64_t row = row0 + acc_row<PREC>(gq, it);
        const int64_t col = col0 + 16 * t + r;
        if (row < g.M && col < g.N) {
          const double a = g.Aref[row * g.ldref + col];
          const double d = a - (double)acc[t][it];
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
      const int64_t row = row0 + acc_row<PREC>(gq, it);
      const int64_t col = col0 + 16 * t + r;
      if (row < g.M && col < g.N) {
        const double v = (double)acc[t][it];
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


// ---------------------------------------------------------------------------
// Streaming variant for C = op(A) B with op(A) = A (row-major), used when
// every K chunk is whole and both operands allow 16-byte accesses. Both
// operands move HBM/L2 -> LDS with global_load_lds_dwordx4 (no staging
// registers) through three LDS stages, two chunks ahead of the MFMAs. Each
// wave waits only for its own copies of the chunk it is about to use
// (s_waitcnt vmcnt(n) with n = copies it issued for the next chunk) and then
// meets the other waves at a bare s_barrier, so the copies of later chunks
// stay in flight across the barrier.
// A stage layout: wave w, half h (k pairs 0-1 / 2-3 of a lane's 4 k values):
// 64 lanes x 16 B, so the MFMA A fragments of a lane are one 16-byte read.
// ---------------------------------------------------------------------------
// copies a wave issues per chunk: 2 for A plus its share of the NBQ B copies
template <int NBQ, int WM, int W>
struct CopiesPerChunk {
  static constexpr int value = 2 + (NBQ - W + WM - 1) / WM;
};

template <int NBQ, int WM>
__device__ __forceinline__ void wait_own_next(int wave, bool next_pending) {
  if (!next_pending) {
    wait_vmcnt<0>();
    return;
  }
  switch (wave) {
    case 0: wait_vmcnt<CopiesPerChunk<NBQ, WM, 0>::value>(); break;
    case 1: wait_vmcnt<CopiesPerChunk<NBQ, WM, 1>::value>(); break;
    case 2: wait_vmcnt<CopiesPerChunk<NBQ, WM, 2>::value>(); break;
    case 3: wait_vmcnt<CopiesPerChunk<NBQ, WM, 3>::value>(); break;
    case 4: wait_vmcnt<CopiesPerChunk<NBQ, WM, (WM > 4 ? 4 : 0)>::value>(); break;
    case 5: wait_vmcnt<CopiesPerChunk<NBQ, WM, (WM > 5 ? 5 : 0)>::value>(); break;
    case 6: wait_vmcnt<CopiesPerChunk<NBQ, WM, (WM > 6 ? 6 : 0)>::value>(); break;
    default: wait_vmcnt<CopiesPerChunk<NBQ, WM, (WM > 7 ? 7 : 0)>::value>(); break;
  }
}

// TA: op(A) = A^T for A stored K x M row-major (lda >= M): C = A^T B with the
// big matrix in its stored orientation. A wave's 16 x 16 tile of A^T for a
// chunk is 16 rows of A (k) by 16 contiguous columns (the wave's 16 output
// rows), 128 contiguous bytes per row of A: copy j = 64 h + lane brings
// 16 bytes of row j / 8, columns 2 (j mod 8) .. + 1, and lands at element 2 j
// of the wave's stage, so the stage holds the tile as [k][m] and a lane's 4
// k values for its row r are 4 reads 16 doubles apart. Columns beyond M are
// clamped (their outputs are never stored): M must be even.
template <int NT, int WM, bool RES, int PREC, bool B_F32 = false, bool TA = false>
__global__ void __launch_bounds__(64 * WM) dgemm_nn_dma_kernel(GemmArgs g) {
  static_assert(!(TA && RES), "the residual epilogue reads A in the NN orientation");
  static_assert(!B_F32 || PREC == kPrecF32, "FP32 panels feed the FP32 matrix cores");
  using BT = typename std::conditional<B_F32, float, double>::type;
  constexpr int BN = NT * 16;
  constexpr int BEL = kBK * BN;
  constexpr int EPL = 16 / (int)sizeof(BT);  // elements per lane and 16-byte copy
  constexpr int CPE = 64 * EPL;             // elements per 1 KB copy
  constexpr int NBQ = BEL / CPE;            // 1 KB copies per B chunk
  constexpr int AEL = WM * 2 * 128;      // doubles per A stage
  __shared__ __attribute__((aligned(16))) BT B0[BEL];
  __shared__ __attribute__((aligned(16))) BT B1[BEL];
  __shared__ __attribute__((aligned(16))) BT B2[BEL];
  __shared__ __attribute__((aligned(16))) double A0[AEL];
  __shared__ __attribute__((aligned(16))) double A1[AEL];
  __shared__ __attribute__((aligned(16))) double A2[AEL];
  if (g.pred != nullptr && *g.pred == 0) return;

  const int total = g.tiles_m * g.tiles_n * g.splits;
  const int full = total & ~7;
  int b = blockIdx.x;
  int item = b;
  if (b < full) item = (b & 7) * (full >> 3) + (b >> 3);
  int tn = item % g.tiles_n;
  int tm = (item / g.tiles_n) % g.tiles_m;
  const int z = item / (g.tiles_n * g.tiles_m);
  if constexpr (RES) {
    // the residual pass has many column tiles, each with its own slice of
    // B = V^T: consecutive items walk the row tiles of a group of kResCols
    // column tiles, so the workgroups running together on an XCD share a few
    // slices of both operands in its L2 (one row tile across all column
    // tiles would fetch every B slice again per row tile)
    constexpr int kResCols = 4;
    const int grp = item / (kResCols * g.tiles_m);
    const int cols = min(kResCols, g.tiles_n - grp * kResCols);
    const int idx = item - grp * kResCols * g.tiles_m;
    tm = idx / cols;
    tn = grp * kResCols + idx % cols;
  }
  const int64_t kb = (int64_t)z * g.kchunk;
  const int64_t ke = min(g.K, kb + g.kchunk);
  const int nk = (int)((ke - kb) / kBK);

  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int r = lane & 15;
  const int gq = lane >> 4;
  const int64_t row0 = (int64_t)tm * (16 * WM) + wave * 16;
  const int64_t col0 = (int64_t)tn * BN;
  const double* __restrict__ A = g.A;
  const BT* __restrict__ B = reinterpret_cast<const BT*>(g.B);
  // source of this lane's A copies: NN: row (clamped), k offset 4 gq + 2 h;
  // TA: rows kb + 8 h + lane / 8 of A, columns row0 + 2 (lane mod 8) (clamped)
  const double* asrc = TA ? A + (kb + lane / 8) * g.lda + min(row0 + 2 * (lane & 7), g.M - 2)
                          : A + min(row0 + r, g.M - 1) * g.lda + kb + 4 * gq;
  const int64_t astep = TA ? (int64_t)kBK * g.lda : kBK;  // per chunk
  const int64_t ahalf = TA ? (int64_t)8 * g.lda : 2;      // second copy of a chunk

  // per-lane copy sources, advanced by one chunk after every issue
  constexpr int NQ = (NBQ + WM - 1) / WM;
  const BT* bsrc[NQ];
  // last column a copy may start at (columns past N are never stored)
  const int64_t bmax = (g.b_cols ? g.b_cols : g.N) - EPL;
#pragma unroll
  for (int i = 0; i < NQ; i++) {
    const int q = min(wave + WM * i, NBQ - 1);
    const int e = q * CPE + EPL * lane;  // element of the chunk this lane copies
    const int kk = e / BN, cc = e % BN;
    const int64_t col = min(col0 + cc, bmax);
    bsrc[i] = B + (kb + kk) * g.ldb + col;
  }
  const int64_t bstep = (int64_t)kBK * g.ldb;
  auto issue = [&](double* As, BT* Bs) {
#pragma unroll
    for (int h = 0; h < 2; h++) copy_to_lds16(asrc + ahalf * h, As + (wave * 2 + h) * 128);
    asrc += astep;
#pragma unroll
    for (int i = 0; i < NQ; i++) {
      if (wave + WM * i < NBQ) copy_to_lds16(bsrc[i], Bs + (wave + WM * i) * CPE);
      bsrc[i] += bstep;
    }
  };

  using Acc = typename AccType<PREC>::type;
  Acc acc[NT];
#pragma unroll
  for (int t = 0; t < NT; t++) acc[t] = Acc{0, 0, 0, 0};

  // one chunk; the copies of chunk c + 2 are issued first (their LDS stage
  // was released by the barrier)
  auto compute = [&](const double* As, const BT* Bs, double* As2, BT* Bs2, bool do_issue) {
    if (do_issue) issue(As2, Bs2);
    double av[4];
    if constexpr (TA) {
      const double* at = As + wave * 256 + 64 * gq + r;  // [k][m]: k = 4 gq + s, m = r
#pragma unroll
      for (int s4 = 0; s4 < 4; s4++) av[s4] = at[16 * s4];
    } else {
      const double2 a01 = *reinterpret_cast<const double2*>(As + (wave * 2 + 0) * 128 + 2 * lane);
      const double2 a23 = *reinterpret_cast<const double2*>(As + (wave * 2 + 1) * 128 + 2 * lane);
      av[0] = a01.x;
      av[1] = a01.y;
      av[2] = a23.x;
      av[3] = a23.y;
    }
    chunk_mma<PREC, NT, BN>(acc, av, Bs, gq, r);
  };
  auto step = [&](int c, double* As, BT* Bs, double* As2, BT* Bs2) {
    wait_own_next<NBQ, WM>(wave, c + 1 < nk);
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");  // no LDS access moves across the barrier
    compute(As, Bs, As2, Bs2, c + 2 < nk);
  };

  if (nk > 0) issue(A0, B0);
  if (nk > 1) issue(A1, B1);
  for (int c = 0; c < nk; c += 3) {
    step(c, A0, B0, A2, B2);
    if (c + 1 < nk) step(c + 1, A1, B1, A0, B0);
    if (c + 2 < nk) step(c + 2, A2, B2, A1, B1);
  }
  if constexpr (RES) {
    // residual epilogue: sum (Aref - C)^2 and Aref^2 over the tile
    double sd = 0.0, sa = 0.0;
#pragma unroll
    for (int t = 0; t < NT; t++) {
#pragma unroll
      for (int it = 0; it < 4; it++) {
        const int64_t row = row0 + acc_row<PREC>(gq, it);
        const int64_t col = col0 + 16 * t + r;
        if (row < g.M && col < g.N) {
          const double av = g.Aref[row * g.ldref + col];
          const double dv = av - (double)acc[t][it];
          sd += dv * dv;
          sa += av * av;
        }
      }
    }
    sd = wave_sum(sd);
    sa = wave_sum(sa);
    __syncthreads();
    double* red = reinterpret_cast<double*>(B0);  // the stages are no longer in use
    if (lane == 0) {
      red[wave] = sd;
      red[WM + wave] = sa;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double s0 = 0.0, s1 = 0.0;
      for (int w = 0; w < WM; w++) {
        s0 += red[w];
        s1 += red[WM + w];
      }
      g.rpart[item] = s0;
      g.rpart[total + item] = s1;
    }
    return;
  }

#pragma unroll
  for (int t = 0; t < NT; t++) {
#pragma unroll
    for (int it = 0; it < 4; it++) {
      const int64_t row = row0 + acc_row<PREC>(gq, it);
      const int64_t col = col0 + 16 * t + r;
      if (row < g.M && col < g.N) {
        const double v = (double)acc[t][it];
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

template <bool TA, bool RES, int PREC>
hipError_t launch_nt(int nt, dim3 grid, hipStream_t st, const GemmArgs& a) {
  switch (nt) {
#define RSVD_CASE(X) case X: hipLaunchKernelGGL((dgemm_kernel<TA, X, RES, PREC>), grid, dim3(kThreads), 0, st, a); break;
    RSVD_CASE(1) RSVD_CASE(2) RSVD_CASE(3) RSVD_CASE(4) RSVD_CASE(5) RSVD_CASE(6)
    RSVD_CASE(7) RSVD_CASE(8) RSVD_CASE(9) RSVD_CASE(10) RSVD_CASE(11) RSVD_CASE(12)
    RSVD_CASE(13) RSVD_CASE(14) RSVD_CASE(15) RSVD_CASE(16) RSVD_CASE(17)
#undef RSVD_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <bool TA>
hipError_t launch_nt_prec(int prec, int nt, dim3 grid, hipStream_t st, const GemmArgs& a) {
  if (prec == kPrecF32) return launch_nt<TA, false, kPrecF32>(nt, grid, st, a);
  if (prec == kPrecBF16) return launch_nt<TA, false, kPrecBF16>(nt, grid, st, a);
  if (prec == kPrecBF16S) return launch_nt<TA, false, kPrecBF16S>(nt, grid, st, a);
  return launch_nt<TA, false, kPrecF64>(nt, grid, st, a);
}

template <int WM, bool RES, int PREC, bool TA = false>
hipError_t launch_dma(int nt, dim3 grid, hipStream_t st, const GemmArgs& a) {
  switch (nt) {
#define RSVD_DCASE(X) case X: hipLaunchKernelGGL((dgemm_nn_dma_kernel<X, WM, RES, PREC, false, TA>), grid, dim3(64 * WM), 0, st, a); break;
    RSVD_DCASE(1) RSVD_DCASE(2) RSVD_DCASE(3) RSVD_DCASE(4) RSVD_DCASE(5) RSVD_DCASE(6)
    RSVD_DCASE(7) RSVD_DCASE(8) RSVD_DCASE(9) RSVD_DCASE(10) RSVD_DCASE(11) RSVD_DCASE(12)
    RSVD_DCASE(13) RSVD_DCASE(14) RSVD_DCASE(15) RSVD_DCASE(16) RSVD_DCASE(17)
#undef RSVD_DCASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int WM>
hipError_t launch_dma_bf32(int nt, dim3 grid, hipStream_t st, const GemmArgs& a) {
  switch (nt) {
#define RSVD_FCASE(X) case X: hipLaunchKernelGGL((dgemm_nn_dma_kernel<X, WM, false, kPrecF32, true>), grid, dim3(64 * WM), 0, st, a); break;
    RSVD_FCASE(1) RSVD_FCASE(2) RSVD_FCASE(3) RSVD_FCASE(4) RSVD_FCASE(5) RSVD_FCASE(6)
    RSVD_FCASE(7) RSVD_FCASE(8) RSVD_FCASE(9) RSVD_FCASE(10) RSVD_FCASE(11) RSVD_FCASE(12)
    RSVD_FCASE(13) RSVD_FCASE(14) RSVD_FCASE(15) RSVD_FCASE(16) RSVD_FCASE(17)
#undef RSVD_FCASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Xf (rows x ldf, FP32) = X (rows x cols, FP64) rounded to nearest, columns
// cols .. ldf - 1 zero.
__global__ void __launch_bounds__(256) f32_panel_kernel(int64_t rows, int64_t cols,
                                                        const double* __restrict__ X, int64_t ldx,
                                                        float* __restrict__ Xf, int64_t ldf) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * ldf) return;
  const int64_t r = idx / ldf, c = idx % ldf;
  Xf[idx] = c < cols ? (float)X[r * ldx + c] : 0.0f;
}

template <int WM, bool TA = false>
hipError_t launch_dma_prec(int prec, int nt, dim3 grid, hipStream_t st, const GemmArgs& a) {
  if (prec == kPrecF32) return launch_dma<WM, false, kPrecF32, TA>(nt, grid, st, a);
  if (prec == kPrecBF16) return launch_dma<WM, false, kPrecBF16, TA>(nt, grid, st, a);
  if (prec == kPrecBF16S) return launch_dma<WM, false, kPrecBF16S, TA>(nt, grid, st, a);
  return launch_dma<WM, false, kPrecF64, TA>(nt, grid, st, a);
}


// ---------------------------------------------------------------------------
// Residual pass with U diag(s) held in registers (K <= 288): the squared
// Frobenius norms of A - US Vt and of A, both summed over one sweep of A.
// A workgroup of 4 waves takes 64 rows, two workgroups per CU (their
// barriers are independent, so one's products run while the other waits);
// each wave keeps its 16 rows of US (16 x K, the MFMA A operand: K / 4
// doubles per lane) in registers for the whole sweep over its column range,
// so US is read once per workgroup. Vt goes HBM/L2 -> LDS by
// global_load_lds_dwordx4 in stages of 16 columns (two stages: the next
// stage's copies in flight while the current one is multiplied; no staging
// registers), and A is read once, each element by the lane that holds the
// matching entry of the product. The column range of a workgroup is one of
// `chunks` slices of N; with 8 slices, consecutive workgroups (which the
// dispatcher deals to the 8 XCDs in turn) take the 8 slices of one row
// strip, so every XCD sweeps one slice of Vt for all row strips and its L2
// serves the strips that run there together.
// The K index of MFMA step s, lane group g is KQM g + s: each lane's share
// of a US row is contiguous. The kernel is instantiated for a few bounds
// KQM (multiples of 8) with 4 KQM >= K and always runs KQM straight-line
// steps (a branch per step would make the compiler wait for every load in
// flight before each product); US entries from K on are zero in registers,
// so the Vt rows they meet in LDS (copies of row K - 1) add nothing. In LDS,
// row k of a stage sits at 16 k + 16 (k / KQM) doubles: the 16-double gap
// between lane groups puts the two groups of a half-wave read on disjoint
// banks, and a 1 KB copy (8 rows) never straddles a gap.
// Needs N even, ldvt even and Vt 16-byte aligned (16-byte copies).
// Partial sums per workgroup: rpart[item] (residual), rpart[total + item]
// (A), summed by sum_partials_into in a fixed order.
// ---------------------------------------------------------------------------
constexpr int kRrWaves = 4;
constexpr int kRrRows = 16 * kRrWaves;
constexpr int kRrMaxK = 288;
constexpr int kRrCols = 16;  // columns per stage

template <int KQM>
__global__ void __launch_bounds__(64 * kRrWaves, 2) resid_reg_kernel(
    int64_t M, int64_t N, int K, const double* __restrict__ US, int64_t ldus,
    const double* __restrict__ Vt, int64_t ldvt, const double* __restrict__ A, int64_t lda,
    int chunks, int64_t chunk_cols, double* __restrict__ rpart) {
  static_assert(KQM % 8 == 0, "a copy of 8 rows stays within one lane group");
  constexpr int kStage = 16 * 4 * KQM + 4 * 16;  // doubles per stage
  constexpr int kCopies = 4 * KQM / 8;            // 1 KB copies per stage
  constexpr int kCopiesW = kCopies / kRrWaves;    // per wave
  __shared__ __attribute__((aligned(16))) double bs[2 * kStage];
  __shared__ double red[2 * kRrWaves];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
  const int item = blockIdx.x;
  const int total = gridDim.x;
  const int strip = item / chunks, slice = item % chunks;
  const int64_t row_w = (int64_t)strip * kRrRows + 16 * wave;  // this wave's first row
  const int64_t c_begin = (int64_t)slice * chunk_cols;
  const int64_t c_end = c_begin + chunk_cols < N ? c_begin + chunk_cols : N;

  // Loads below read a clamped, valid address and their values are scaled
  // by a 0 / 1 mask where the entry lies outside the operand, and the loop
  // body has no branches around them: they are issued ahead of the products
  // and the compiler waits for them only where they are used.
  // this wave's rows of US: lane (r, g) holds US[row_w + r][KQM g + s]
  double av[KQM];
  {
    const int64_t row = row_w + r;
    const double* src = US + (row < M ? row : M - 1) * ldus;
    const double mr = row < M ? 1.0 : 0.0;
#pragma unroll
    for (int s = 0; s < KQM; s++) {
      const int k = KQM * g + s;
      av[s] = src[k < K ? k : K - 1] * (k < K ? mr : 0.0);
    }
  }

  // copy i of this wave: rows 8 q .. 8 q + 7 of the stage (q = wave + 4 i),
  // lane -> row 8 q + lane / 8 (clamped to K - 1), columns 2 (lane mod 8)
  // and the next (clamped to N - 2)
  const double* csrc[kCopiesW];
  int cdst[kCopiesW];
#pragma unroll
  for (int i = 0; i < kCopiesW; i++) {
    const int q = wave + kRrWaves * i;
    const int k = 8 * q + (lane >> 3);
    csrc[i] = Vt + (int64_t)(k < K ? k : K - 1) * ldvt + 2 * (lane & 7);
    cdst[i] = 16 * (8 * q) + 16 * ((8 * q) / KQM);
  }
  auto issue = [&](int64_t c0, int b) {
    const int64_t cc = c0 + 16 <= N ? c0 : N - 16;  // the last stage may be ragged
#pragma unroll
    for (int i = 0; i < kCopiesW; i++) copy_to_lds16(csrc[i] + cc, bs + b * kStage + cdst[i]);
  };

  double sd = 0.0, sa = 0.0;
  int buf = 0;
  if (c_begin < c_end) issue(c_begin, 0);
  const int rd = 16 * KQM * g + 16 * g + r;  // this lane's B operand, step 0
  for (int64_t c0 = c_begin; c0 < c_end; c0 += kRrCols) {
    // this stage's copies landed (this wave's, then everyone's)
    wait_vmcnt<0>();
    __syncthreads();
    asm volatile("" ::: "memory");
    // the next stage's copies into the other buffer, released by the barrier
    if (c0 + kRrCols < c_end) issue(c0 + kRrCols, buf ^ 1);
    // A at the product's entries: rows row_w + g + 4 it, column c0 + r
    double ar[4];
#pragma unroll
    for (int it = 0; it < 4; it++) {
      const int64_t row = row_w + g + 4 * it, col = c0 + r;
      ar[it] = A[(row < M ? row : M - 1) * lda + (col < c_end ? col : c_end - 1)];
    }
    // the stage starts at column c0, or earlier when the last one was
    // shifted back to stay inside the rows of Vt: column c0 + r then sits
    // at position r + shift (lanes past N read any position: masked below)
    const int shift = (int)(c0 + 16 <= N ? 0 : c0 - (N - 16));
    const double* b0 = bs + buf * kStage + rd + (r + shift < 16 ? shift : 0);
    // two accumulation chains (even and odd steps) in flight on the matrix
    // core; the LDS reads run kPF steps ahead of the products that use them
    // (left to itself the scheduler issues each read just before its
    // products and waits for it). Scheduling-group masks: 0x100 LDS reads,
    // 0x008 matrix ops.
    double bv[KQM];
#pragma unroll
    for (int s = 0; s < KQM; s++) bv[s] = b0[16 * s];
    d4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < KQM; s += 2) {
      acc0 = mfma_f64_16x16x4(av[s], bv[s], acc0);
      acc1 = mfma_f64_16x16x4(av[s + 1], bv[s + 1], acc1);
    }
    constexpr int kPF = 4;
#pragma unroll
    for (int u = 0; u < kPF; u++) __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
#pragma unroll
    for (int u = 0; u < KQM / 2; u++) {
      __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);
      if (u + kPF < KQM / 2) __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
    }
    const d4 acc = acc0 + acc1;
    const double mc = c0 + r < c_end ? 1.0 : 0.0;
#pragma unroll
    for (int it = 0; it < 4; it++) {
      const double m = (row_w + g + 4 * it < M ? 1.0 : 0.0) * mc;
      const double dv = (ar[it] - acc[it]) * m, av2 = ar[it] * m;
      sd += dv * dv;
      sa += av2 * av2;
    }
    buf ^= 1;
  }
  wait_vmcnt<0>();
  sd = wave_sum(sd);
  sa = wave_sum(sa);
  if (lane == 0) {
    red[wave] = sd;
    red[kRrWaves + wave] = sa;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double s0 = 0.0, s1 = 0.0;
    for (int w = 0; w < kRrWaves; w++) {
      s0 += red[w];
      s1 += red[kRrWaves + w];
    }
    rpart[item] = s0;
    rpart[total + item] = s1;
  }
}
}  // namespace

void dgemm_set_dma(bool on, int waves) {
  g_use_dma = on;
  if (waves == 4 || waves == 8) g_dma_wm = waves;
}

bool dgemm_dma_eligible_t(int64_t M, int64_t K, int64_t N, const double* A, int64_t lda,
                          const double* B, int64_t ldb) {
  // A^T B with A (K x M) in its stored orientation: whole K chunks, even M
  // and N, 16-byte aligned rows
  const bool vec_a = (lda % 2 == 0) && ((uintptr_t)A % 16 == 0);
  const bool vec_b = (ldb % 2 == 0) && ((uintptr_t)B % 16 == 0);
  return (K % kBK == 0) && K > 0 && M >= 2 && (M % 2 == 0) && (N % 2 == 0) && N >= 2 && vec_a &&
         vec_b && g_use_dma;
}

bool dgemm_dma_eligible(int64_t K, int64_t N, const double* A, int64_t lda, const double* B,
                        int64_t ldb) {
  // whole K chunks, even N and 16-byte aligned rows: the LDS-DMA pipeline
  const bool vec_a = (lda % 2 == 0) && ((uintptr_t)A % 16 == 0);
  const bool vec_b = (ldb % 2 == 0) && ((uintptr_t)B % 16 == 0);
  return (K % kBK == 0) && K > 0 && (N % 2 == 0) && N >= 2 && vec_a && vec_b && g_use_dma;
}

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

int64_t f32_panel_ld(int64_t cols) { return (cols + 3) / 4 * 4; }

rsvd_status f32_panel(int64_t rows, int64_t cols, const double* X, int64_t ldx, float* Xf,
                      hipStream_t s) {
  const int64_t ldf = f32_panel_ld(cols);
  if (rows * ldf == 0) return RSVD_OK;
  hipLaunchKernelGGL(f32_panel_kernel, dim3((unsigned)((rows * ldf + 255) / 256)), dim3(256), 0, s,
                     rows, cols, X, ldx, Xf, ldf);
  RSVD_LAUNCH_CHECK();
  return RSVD_OK;
}

rsvd_status dgemm(bool ta, int64_t M, int64_t N, int64_t K, double alpha, const double* A,
                  int64_t lda, const double* B, int64_t ldb, double beta, double* C, int64_t ldc,
                  double* part, size_t part_doubles, hipStream_t st, int max_splits,
                  const uint32_t* pred, int prec, const float* Bf, int64_t ldbf, const double* Bp,
                  int64_t ldbp) {
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
  const bool vec_a = (lda % 2 == 0) && ((uintptr_t)A % 16 == 0);
  const bool vec_b = (ldb % 2 == 0) && ((uintptr_t)B % 16 == 0);
  // the panel the streaming kernel stages for A B: B itself (even N, even
  // ldb), its FP32 panel (FP32 schedule), or its FP64 copy with an even
  // leading dimension (odd N or ldb); with the copies it reads whole 16-byte
  // pairs up to their row ends, and stores only the N columns
  auto nn_stream = [&](int64_t k, bool* f32, bool* pad) {
    *f32 = *pad = false;
    if (ta || !(vec_a && k % kBK == 0 && k > 0 && g_use_dma)) return false;
    *f32 = Bf != nullptr && prec == kPrecF32 && ldbf >= N && ldbf % 4 == 0 &&
           ((uintptr_t)Bf % 16 == 0);
    if (*f32) return true;
    if (dgemm_dma_eligible(k, N, A, lda, B, ldb)) return true;
    *pad = Bp != nullptr && ldbp % 2 == 0 && ldbp >= N + (N & 1) && ((uintptr_t)Bp % 16 == 0);
    return *pad;
  };
  bool bf32 = false, bpad = false;
  const bool dma_ok = ta ? dgemm_dma_eligible_t(M, K, N, A, lda, B, ldb) : nn_stream(K, &bf32, &bpad);
  const int64_t ktail = K % kBK;
  if (!dma_ok && ktail != 0 && K > kBK) {
    // K not a whole number of chunks: the whole chunks on the streaming
    // kernel (if it takes them), then the last K mod 16 terms added by the
    // register-staged kernel
    const int64_t K0 = K - ktail;
    bool f0 = false, p0 = false;
    const bool main_ok = ta ? dgemm_dma_eligible_t(M, K0, N, A, lda, B, ldb) : nn_stream(K0, &f0, &p0);
    if (main_ok) {
      rsvd_status r = dgemm(ta, M, N, K0, alpha, A, lda, B, ldb, beta, C, ldc, part, part_doubles,
                            st, max_splits, pred, prec, Bf, ldbf, Bp, ldbp);
      if (r != RSVD_OK) return r;
      const double* At = ta ? A + K0 * lda : A + K0;
      return dgemm(ta, M, N, ktail, alpha, At, lda, B + K0 * ldb, ldb, 1.0, C, ldc, part,
                   part_doubles, st, max_splits, pred, prec);
    }
  }
  const TuneKey tkey{dma_ok ? kTuneDma : kTuneGeneric, prec, ta ? 1 : 0, M, N, K};
  if (pred == nullptr && tune_recording()) {
    // candidates: waves (LDS-DMA kernel) x split counts whose partials fit
    std::vector<TuneCfg> cands;
    for (int w = dma_ok ? 4 : 0; w <= (dma_ok ? 8 : 0); w += 4) {
      for (int S = 1; S <= max_splits && S <= 64; S *= 2) {
        if (S > 1 && (K / S < 2 * kBK || !part || part_doubles < (size_t)S * M * N)) break;
        cands.push_back({w, S, 0});
      }
    }
    tune_record(tkey, std::move(cands), [=](hipStream_t s2) {
      return dgemm(ta, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, part, part_doubles, s2,
                   max_splits, pred, prec, Bf, ldbf, Bp, ldbp);
    });
  }
  TuneCfg tcfg;
  const bool tuned = tune_get(tkey, &tcfg) && tcfg.b >= 1;
  GemmShape s = dgemm_shape(M, N, K, max_splits);
  if (tuned && !dma_ok) {
    int S = tcfg.b < max_splits ? tcfg.b : max_splits;
    s.kchunk = ((K + S - 1) / S + kBK - 1) / kBK * kBK;
    s.splits = (int)((K + s.kchunk - 1) / s.kchunk);
    s.part_doubles = s.splits > 1 ? (size_t)s.splits * M * N : 0;
  }
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
  a.vec_a = vec_a;
  a.vec_b = vec_b;
  a.b_cols = 0;
  const int64_t total = (int64_t)s.tiles_m * s.tiles_n * s.splits;
  dim3 grid((unsigned)total);
  hipError_t e;
  if (dma_ok) {
    // The LDS-DMA kernel's 3-stage LDS footprint allows one workgroup per
    // CU, so by default it is sized to fill the 256 CUs once: split K only
    // when the output has fewer tiles; 8 waves need split K to fill the
    // chip, without enough K use 4. A tuned shape replaces both choices.
    int wm = g_dma_wm;
    if (wm == 8 && (int64_t)((M + 127) / 128) * s.tiles_n < 256 && K / 2 < 256) wm = 4;
    if (tuned && (tcfg.a == 4 || tcfg.a == 8)) wm = tcfg.a;
    GemmArgs d = a;
    d.tiles_m = (int)((M + 16 * wm - 1) / (16 * wm));
    d.tiles_n = s.tiles_n;
    const int64_t T = (int64_t)d.tiles_m * d.tiles_n;
    int S = 1;
    if (tuned)
      S = tcfg.b < max_splits ? tcfg.b : max_splits;
    else
      while (S < max_splits && T * S < 256 && K / (2 * S) >= 256) S *= 2;
    int64_t kchunk = ((K + S - 1) / S + kBK - 1) / kBK * kBK;
    S = (int)((K + kchunk - 1) / kchunk);
    if (S > 1 && (part == nullptr || part_doubles < (size_t)S * M * N)) {
      S = 1;
      kchunk = K;
    }
    d.splits = S;
    d.kchunk = kchunk;
    d.part = S > 1 ? part : nullptr;
    s.splits = S;
    const dim3 g2((unsigned)(T * S));
    if (bpad) {
      d.B = Bp;
      d.ldb = ldbp;
      d.b_cols = ldbp;
    }
    if (bf32) {
      d.B = reinterpret_cast<const double*>(Bf);
      d.ldb = ldbf;
      d.b_cols = ldbf;
      e = wm == 8 ? launch_dma_bf32<8>(s.nt, g2, st, d) : launch_dma_bf32<4>(s.nt, g2, st, d);
    } else if (ta) {
      e = wm == 8 ? launch_dma_prec<8, true>(prec, s.nt, g2, st, d)
                  : launch_dma_prec<4, true>(prec, s.nt, g2, st, d);
    } else {
      e = wm == 8 ? launch_dma_prec<8>(prec, s.nt, g2, st, d)
                  : launch_dma_prec<4>(prec, s.nt, g2, st, d);
    }
  } else {
    e = ta ? launch_nt_prec<true>(prec, s.nt, grid, st, a)
           : launch_nt_prec<false>(prec, s.nt, grid, st, a);
  }
  if (e != hipSuccess) return RSVD_EHIP;
  if (s.splits > 1) {
    const int64_t tot = M * N;
    hipLaunchKernelGGL(splitk_reduce_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st,
                       M, N, s.splits, (const double*)part, alpha, beta, C, ldc, pred);
    RSVD_LAUNCH_CHECK();
  }
  return RSVD_OK;
}

// Column tiles per workgroup of the residual pass's narrow candidates: two
// workgroups of them fit on a CU, so one's epilogue (the read of A)
// overlaps the other's products. kResNarrowNT is the narrowest.
constexpr int kResNarrowNT = 4;
constexpr int kResNarrow[] = {4, 6, 8, 12};

size_t resid_partials(int64_t M, int64_t N) {
  GemmShape s = dgemm_shape(M, N, 1, 1);
  const size_t a = (size_t)2 * s.tiles_m * s.tiles_n;
  // every DMA candidate: 4 or 8 waves, the default or the narrow column tile
  const int64_t ntiles = (N + 15) / 16;
  const size_t b = (size_t)2 * ((M + 63) / 64) * ((ntiles + kResNarrowNT - 1) / kResNarrowNT);
  // the register-resident kernel: row strips x column slices
  const int64_t stages = (N + kRrCols - 1) / kRrCols;
  const size_t c = (size_t)2 * ((M + kRrRows - 1) / kRrRows) * (stages < 8 ? stages : 8);
  const size_t ab = a > b ? a : b;
  return ab > c ? ab : c;
}

size_t resid_partials_dma(int64_t M, int64_t N) {
  const GemmShape sh = dgemm_shape(M, N, 1, 1);
  return (size_t)2 * ((M + 127) / 128) * sh.tiles_n;
}

rsvd_status resid(int64_t M, int64_t N, int64_t K, const double* US, int64_t ldus,
                  const double* Vt, int64_t ldvt, const double* A, int64_t lda, double* partial,
                  DevState* st, hipStream_t s) {
  // US in registers (K <= 288): 8 column slices (one per XCD) unless N is
  // narrow; the tuner's candidate c = 1
  const int64_t rr_strips = (M + kRrRows - 1) / kRrRows;
  const int64_t rr_stages = (N + kRrCols - 1) / kRrCols;
  const int rr_chunks = (int)(rr_stages < 8 ? rr_stages : 8);
  const int64_t rr_total = rr_strips * rr_chunks;
  const bool rr_ok = K > 0 && K <= kRrMaxK && K % 16 == 0 && M > 0 && N >= 16 && N % 2 == 0 &&
                     ldvt % 2 == 0 && ((uintptr_t)Vt & 15) == 0 &&
                     (size_t)2 * rr_total <= resid_partials(M, N) && rr_total < (int64_t)1 << 31;
  const TuneKey rkey{kTuneResid, kPrecF64, 0, M, N, K};
  TuneCfg rcfg;
  const bool rtuned = !tune_recording() && tune_get(rkey, &rcfg);
  // untuned: the register kernel once its grid covers the device twice
  // (fewer, larger workgroups leave CUs idle)
  if (rr_ok && (rtuned ? rcfg.c == 1 : (tune_recording() || rr_total >= 512))) {
    if (tune_recording()) {
      std::vector<TuneCfg> cands = {{8, 0, 1}, {4, 0, 0}, {8, 0, 0}};
      const GemmShape sh0 = dgemm_shape(M, N, K, 1);
      for (int nt : kResNarrow) {
        if (nt < sh0.nt) {
          cands.push_back({4, nt, 0});
          cands.push_back({8, nt, 0});
        }
      }
      tune_record(rkey, cands, [=](hipStream_t s2) {
        return resid(M, N, K, US, ldus, Vt, ldvt, A, lda, partial, st, s2);
      });
    }
    TuneCfg fc;
    if (tune_get(rkey, &fc) ? fc.c == 1 : rr_total >= 512) {
      const int64_t chunk_cols = (rr_stages + rr_chunks - 1) / rr_chunks * kRrCols;
      // the fewest straight-line steps that cover K / 4
      const int kq = (int)(K / 4);
      auto kern = kq <= 16   ? resid_reg_kernel<16>
                  : kq <= 32 ? resid_reg_kernel<32>
                  : kq <= 48 ? resid_reg_kernel<48>
                  : kq <= 64 ? resid_reg_kernel<64>
                             : resid_reg_kernel<72>;
      hipLaunchKernelGGL(kern, dim3((unsigned)rr_total), dim3(64 * kRrWaves), 0, s, M, N, (int)K, US,
                         ldus, Vt, ldvt, A, lda, rr_chunks, chunk_cols, partial);
      RSVD_LAUNCH_CHECK();
      rsvd_status r = sum_partials_into(rr_total, partial, &st->resid2, s);
      if (r != RSVD_OK) return r;
      return sum_partials_into(rr_total, partial + rr_total, &st->fro2, s);
    }
  }
  GemmShape sh = dgemm_shape(M, N, K, 1);
  const bool dma_ok = (K % kBK == 0) && K > 0 && (N % 2 == 0) && N >= 2 && (ldus % 2 == 0) &&
                      (ldvt % 2 == 0) && ((uintptr_t)US % 16 == 0) && ((uintptr_t)Vt % 16 == 0) &&
                      g_use_dma;
  if (dma_ok) {
    // 8 waves and the widest column tile unless tuned otherwise (a = waves,
    // b = column tiles per workgroup; partial holds every candidate's count)
    const TuneKey tkey{kTuneResid, kPrecF64, 0, M, N, K};
    if (tune_recording()) {
      std::vector<TuneCfg> cands = {{4, 0, 0}, {8, 0, 0}};
      for (int nt : kResNarrow) {
        if (nt < sh.nt) {
          cands.push_back({4, nt, 0});
          cands.push_back({8, nt, 0});
        }
      }
      tune_record(tkey, cands, [=](hipStream_t s2) {
        return resid(M, N, K, US, ldus, Vt, ldvt, A, lda, partial, st, s2);
      });
    }
    TuneCfg tcfg;
    const bool tuned = tune_get(tkey, &tcfg);
    const int wm = tuned && tcfg.a == 4 ? 4 : 8;
    int nt = sh.nt;
    int tiles_n = sh.tiles_n;
    if (tuned && tcfg.b >= 1 && tcfg.b < sh.nt) {
      nt = tcfg.b;
      tiles_n = (int)(((N + 15) / 16 + nt - 1) / nt);
    }
    GemmArgs a;
    a.M = M; a.N = N; a.K = K; a.kchunk = K;
    a.alpha = 1.0; a.beta = 0.0;
    a.A = US; a.lda = ldus; a.B = Vt; a.ldb = ldvt; a.C = nullptr; a.ldc = 0;
    a.part = nullptr;
    a.tiles_m = (int)((M + 16 * wm - 1) / (16 * wm)); a.tiles_n = tiles_n; a.splits = 1;
    a.pred = nullptr; a.Aref = A; a.ldref = lda; a.rpart = partial;
    a.vec_a = 1; a.vec_b = 1; a.b_cols = 0;
    const int64_t total = (int64_t)a.tiles_m * a.tiles_n;
    if ((size_t)2 * total > resid_partials(M, N)) return RSVD_EINVAL;
    hipError_t e = wm == 4 ? launch_dma<4, true, kPrecF64>(nt, dim3((unsigned)total), s, a)
                           : launch_dma<8, true, kPrecF64>(nt, dim3((unsigned)total), s, a);
    if (e != hipSuccess) return RSVD_EHIP;
    rsvd_status r = sum_partials_into(total, partial, &st->resid2, s);
    if (r != RSVD_OK) return r;
    return sum_partials_into(total, partial + total, &st->fro2, s);
  }
  GemmArgs a;
  a.M = M; a.N = N; a.K = K; a.kchunk = ((K + kBK - 1) / kBK) * kBK;
  a.alpha = 1.0; a.beta = 0.0;
  a.A = US; a.lda = ldus; a.B = Vt; a.ldb = ldvt; a.C = nullptr; a.ldc = 0;
  a.part = nullptr;
  a.tiles_m = sh.tiles_m; a.tiles_n = sh.tiles_n; a.splits = 1;
  a.pred = nullptr; a.Aref = A; a.ldref = lda; a.rpart = partial;
  a.vec_a = (ldus % 2 == 0) && ((uintptr_t)US % 16 == 0);
  a.vec_b = (ldvt % 2 == 0) && ((uintptr_t)Vt % 16 == 0);
  const int64_t total = (int64_t)sh.tiles_m * sh.tiles_n;
  hipError_t e = launch_nt<false, true, kPrecF64>(sh.nt, dim3((unsigned)total), s, a);
  if (e != hipSuccess) return RSVD_EHIP;
  rsvd_status r = sum_partials_into(total, partial, &st->resid2, s);
  if (r != RSVD_OK) return r;
  return sum_partials_into(total, partial + total, &st->fro2, s);
}

}  // namespace rsvd
