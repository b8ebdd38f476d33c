// Error-free sliced product C = A X for the FP64-accurate passes of a mixed
// schedule (Ozaki, Ogita, Oishi and Rump's error-free splitting of a matrix
// product into exactly computed products of short slices, here with 8-bit
// integer slices on the integer matrix cores):
//   A's row i is scaled by 2^-e_i (|a_ik| < 2^e_i) and cut into kSlices
//   7-bit signed digits: a_ik = 2^e_i sum_s d^A_s,ik 2^-7s + (a remainder
//   below 2^(e_i - 7 kSlices)); X's column j likewise with 2^f_j.
//   Every slice product A_s X_t is exact in INT32 (|digits| <= 127); the
//   products of one weight 2^-7(s+t) share an INT32 accumulator, flushed to
//   FP64 every kSliceChunk terms of K so that no sum can overflow
//   (7 x 16384 x 127^2 < 2^31); only the products with s + t <= kSlices + 1
//   are formed (the dropped ones weigh at most 2^-63 K 127^2 relative to
//   2^(e_i + f_j)).
// The result agrees with the FP64 product to about 1e-14 relative to
// K 2^(e_i + f_j); integer inputs of at most 7 bits are reproduced exactly.
#include "common.hpp"
#include "kernels.hpp"

namespace rsvd {

namespace {

constexpr int kSlices = 7;
constexpr int kSliceChunk = 16384;  // K terms per INT32 sum

typedef int v4i __attribute__((ext_vector_type(4)));

// v_mfma_i32_16x16x64_i8 (checked on the device): lane (r, g) supplies
// A[r][16g .. 16g+15] and B[16g .. 16g+15][r] (16 bytes each, lowest k in
// the lowest byte) and receives C[4g + i][r] in item i.
__device__ __forceinline__ v4i mfma_i8_16x16x64(v4i a, v4i b, v4i c) {
  return __builtin_amdgcn_mfma_i32_16x16x64_i8(a, b, c, 0, 0, 0);
}

// The digits of x (|x| < 2^e, e the line's exponent) into kSlices planes.
__device__ __forceinline__ void digits(double x, int e, int8_t* dst, int64_t plane) {
  double r = __builtin_amdgcn_ldexp(x, -e);  // |r| < 1, exact
#pragma unroll
  for (int s = 0; s < kSlices; s++) {
    r *= 128.0;                  // exact
    const double d = trunc(r);   // |d| <= 127
    r -= d;                      // exact
    dst[s * plane] = (int8_t)(int)d;
  }
}

// Exponent of a line whose largest magnitude is m: |x| < 2^e for every entry
// (0 for an all-zero line).
__device__ __forceinline__ int line_exponent(double m) {
  return m > 0.0 ? __builtin_amdgcn_frexp_exp(m) : 0;
}

__device__ __forceinline__ double block_max(double v, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) red[w] = v;
  __syncthreads();
  double m = 0.0;
  for (int i = 0; i < (int)(blockDim.x >> 6); i++) m = fmax(m, red[i]);
  __syncthreads();
  return m;
}

// One workgroup per row of A (M x K): its exponent and its digits into the
// planes AS[s] (M x Kp, zero beyond K).
__global__ void __launch_bounds__(256) slice_rows_kernel(int64_t M, int64_t K, int64_t Kp,
                                                         const double* __restrict__ A, int64_t lda,
                                                         int8_t* __restrict__ AS,
                                                         int* __restrict__ ea) {
  __shared__ double red[4];
  const int64_t row = blockIdx.x;
  if (row >= M) return;
  const double* a = A + row * lda;
  double m = 0.0;
  for (int64_t k = threadIdx.x; k < K; k += blockDim.x) m = fmax(m, fabs(a[k]));
  const int e = line_exponent(block_max(m, red));
  if (threadIdx.x == 0) ea[row] = e;
  // 1024 entries at a time: digits of coalesced reads into LDS planes, then
  // 16-byte stores of each plane
  __shared__ __attribute__((aligned(16))) int8_t dig[kSlices][1024];
  const int64_t plane = M * Kp;
  for (int64_t c0 = 0; c0 < Kp; c0 += 1024) {
#pragma unroll
    for (int j = 0; j < 4; j++) {
      const int kk = (int)threadIdx.x + 256 * j;
      const int64_t k = c0 + kk;
      double r = __builtin_amdgcn_ldexp(k < K ? a[k] : 0.0, -e);  // |r| < 1, exact
#pragma unroll
      for (int s = 0; s < kSlices; s++) {
        r *= 128.0;                  // exact
        const double d = trunc(r);   // |d| <= 127
        r -= d;                      // exact
        dig[s][kk] = (int8_t)(int)d;
      }
    }
    __syncthreads();
    for (int q = (int)threadIdx.x; q < kSlices * 64; q += 256) {
      const int s = q / 64, off = 16 * (q % 64);
      if (c0 + off < Kp)
        *reinterpret_cast<v4i*>(AS + s * plane + row * Kp + c0 + off) =
            *reinterpret_cast<const v4i*>(&dig[s][off]);
    }
    __syncthreads();
  }
}

// One workgroup per column of X (K x N): its exponent and its digits into
// the transposed planes XS[t] (N x Kp, zero beyond K).
__global__ void __launch_bounds__(256) slice_cols_kernel(int64_t K, int64_t N, int64_t Kp,
                                                         const double* __restrict__ X, int64_t ldx,
                                                         int8_t* __restrict__ XS,
                                                         int* __restrict__ fx) {
  __shared__ double red[4];
  const int64_t col = blockIdx.x;
  if (col >= N) return;
  double m = 0.0;
  for (int64_t k = threadIdx.x; k < K; k += blockDim.x) m = fmax(m, fabs(X[k * ldx + col]));
  const int e = line_exponent(block_max(m, red));
  if (threadIdx.x == 0) fx[col] = e;
  const int64_t plane = N * Kp;
  for (int64_t k = threadIdx.x; k < Kp; k += blockDim.x)
    digits(k < K ? X[k * ldx + col] : 0.0, e, XS + col * Kp + k, plane);
}

// C (M x N) from the planes. A workgroup of 8 waves takes 128 rows (16 per
// wave) by 64 columns (4 tiles of 16). The panel slices of its columns are
// staged in LDS, kSlStage values of K at a time (double buffered, 16-byte
// copies); each wave reads its A slices from global memory, 16 bytes per
// lane and slice for 64 values of K, and keeps one INT32 tile per weight
// 2^-7(s+t) and column tile, flushed to FP64 every kSliceChunk terms. Within
// a block of 64 values of K, lane (r, g) takes k = 16 g .. 16 g + 15 of its
// row of A and of column r of the panel (one 16x16x64 product): integer
// sums are exact, so the assignment of k to lanes does not change a bit of
// the result. Tiles are ordered so that the column groups of one row block
// are consecutive and land on the same XCD (their A slices are then shared
// in its L2).
constexpr int kSlWaves = 8;
constexpr int kSlRows = 16 * kSlWaves;
constexpr int kSlCols = 64;
constexpr int kSlTiles = kSlCols / 16;
constexpr int kSlStage = 128;                 // values of K per LDS stage
constexpr int kSlRowB = kSlStage + 16;        // bytes per staged column (padded)
constexpr int kSlSliceB = kSlCols * kSlRowB;  // bytes per staged slice
constexpr int kSlStageB = kSlices * kSlSliceB;
static_assert(kSlCols * (kSlStage / 16) == 64 * kSlWaves, "one 16-byte copy per thread and slice");

typedef v4i v4i32;

__global__ void __launch_bounds__(64 * kSlWaves) sliced_gemm_kernel(
    int64_t M, int64_t N, int64_t Kp, const int8_t* __restrict__ AS, const int* __restrict__ ea,
    const int8_t* __restrict__ XS, const int* __restrict__ fx, double* __restrict__ C, int64_t ldc,
    int tiles_n, int total) {
  __shared__ __attribute__((aligned(16))) int8_t bst[2][kSlStageB];
  const int full = total & ~7;
  const int bid = blockIdx.x;
  const int item = bid < full ? (bid & 7) * (full >> 3) + (bid >> 3) : bid;
  const int tm = item / tiles_n, tn = item % tiles_n;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
  const int64_t row0 = (int64_t)tm * kSlRows + wave * 16;
  const int64_t col0 = (int64_t)tn * kSlCols;
  const int64_t arow = row0 + r;
  const bool arow_ok = arow < M;
  const int64_t pa = M * Kp, px = N * Kp;
  const int8_t* abase = AS + (arow_ok ? arow : 0) * Kp + 16 * g;
  // this thread's staging copy: column tid / 8, K bytes 16 (tid mod 8), every slice
  const int ccol = threadIdx.x >> 3, ck = 16 * (threadIdx.x & 7);
  const bool ccol_ok = col0 + ccol < N;
  const int8_t* cbase = XS + (ccol_ok ? col0 + ccol : 0) * Kp + ck;
  // staging copies in two groups of slices (0..3 during the first block of
  // 64 values of K, 4..6 during the second), stored after their block
  constexpr int kHalf = (kSlices + 1) / 2;
  v4i32 cregs[kHalf];
  auto stage_load = [&](int64_t kb, int t0, int t1) {
#pragma unroll
    for (int t = 0; t < kHalf; t++)
      if (t0 + t < t1)
        cregs[t] = ccol_ok ? *reinterpret_cast<const v4i32*>(cbase + (t0 + t) * px + kb)
                           : v4i32{0, 0, 0, 0};
  };
  auto stage_store = [&](int buf, int t0, int t1) {
#pragma unroll
    for (int t = 0; t < kHalf; t++)
      if (t0 + t < t1)
        *reinterpret_cast<v4i32*>(&bst[buf][(t0 + t) * kSlSliceB + ccol * kSlRowB + ck]) = cregs[t];
  };

  v4i acc[kSlices][kSlTiles];
#pragma unroll
  for (int ct = 0; ct < kSlTiles; ct++)
#pragma unroll
    for (int d = 0; d < kSlices; d++) acc[d][ct] = v4i{0, 0, 0, 0};
  // a chunk's sums, smallest weights first, scaled by 2^(e_i + f_j) (exact)
  // and added to C (the first chunk stores)
  bool first = true;
  auto flush = [&]() {
#pragma unroll
    for (int ct = 0; ct < kSlTiles; ct++) {
      const int64_t col = col0 + 16 * ct + r;
      const int fcol = col < N ? fx[col] : 0;
#pragma unroll
      for (int i = 0; i < 4; i++) {
        double v = 0.0;
#pragma unroll
        for (int d = kSlices - 1; d >= 0; d--)
          v += __builtin_amdgcn_ldexp((double)acc[d][ct][i], -7 * (d + 2));
        const int64_t row = row0 + 4 * g + i;
        if (row < M && col < N) {
          const double o = __builtin_amdgcn_ldexp(v, ea[row] + fcol);
          double* dst = C + row * ldc + col;
          *dst = first ? o : *dst + o;
        }
      }
#pragma unroll
      for (int d = 0; d < kSlices; d++) acc[d][ct] = v4i{0, 0, 0, 0};
    }
    first = false;
  };

  const int nst = (int)(Kp / kSlStage);
  stage_load(0, 0, kHalf);
  stage_store(0, 0, kHalf);
  stage_load(0, kHalf, kSlices);
  stage_store(0, kHalf, kSlices);
  __syncthreads();
  int in_chunk = 0;
  for (int st = 0; st < nst; st++) {
    const int buf = st & 1;
    const bool more = st + 1 < nst;
    const int64_t knext = (int64_t)(st + 1) * kSlStage;
#pragma unroll
    for (int seg = 0; seg < kSlStage / 64; seg++) {
      if (more) stage_load(knext, seg == 0 ? 0 : kHalf, seg == 0 ? kHalf : kSlices);
      const int64_t k = (int64_t)st * kSlStage + seg * 64;
      v4i32 a[kSlices];
#pragma unroll
      for (int s2 = 0; s2 < kSlices; s2++)
        a[s2] = arow_ok ? *reinterpret_cast<const v4i32*>(abase + s2 * pa + k) : v4i32{0, 0, 0, 0};
#pragma unroll
      for (int t = 0; t < kSlices; t++) {
#pragma unroll
        for (int ct = 0; ct < kSlTiles; ct++) {
          const v4i32 bv = *reinterpret_cast<const v4i32*>(
              &bst[buf][t * kSlSliceB + (16 * ct + r) * kSlRowB + seg * 64 + 16 * g]);
#pragma unroll
          for (int s2 = 0; s2 + t < kSlices; s2++)
            acc[s2 + t][ct] = mfma_i8_16x16x64(a[s2], bv, acc[s2 + t][ct]);
        }
      }
      if (more) stage_store(buf ^ 1, seg == 0 ? 0 : kHalf, seg == 0 ? kHalf : kSlices);
    }
    __syncthreads();
    in_chunk += kSlStage;
    if (in_chunk >= kSliceChunk) {
      flush();
      in_chunk = 0;
    }
  }
  if (in_chunk > 0 || first) flush();
}

struct SlicedLayout {
  int64_t Kp;
  size_t as, ea, xs, fx, total;
};

SlicedLayout sliced_layout(int64_t M, int64_t N, int64_t K) {
  auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
  SlicedLayout L;
  L.Kp = (K + kSlStage - 1) / kSlStage * kSlStage;
  size_t at = 0;
  L.as = at;
  at += up((size_t)kSlices * M * L.Kp);
  L.ea = at;
  at += up((size_t)M * sizeof(int));
  L.xs = at;
  at += up((size_t)kSlices * N * L.Kp);
  L.fx = at;
  at += up((size_t)N * sizeof(int));
  L.total = at;
  return L;
}

}  // namespace

size_t sliced_work_bytes(int64_t M, int64_t N, int64_t K) {
  if (M <= 0 || N <= 0 || K <= 0) return 0;
  return sliced_layout(M, N, K).total;
}

rsvd_status sliced_prepare_a(int64_t M, int64_t N, int64_t K, const double* A, int64_t lda,
                             void* work, hipStream_t s) {
  if (M <= 0 || N <= 0 || K <= 0) return RSVD_OK;
  if (!A || !work || lda < K || ((uintptr_t)work & 255) != 0) return RSVD_EINVAL;
  const SlicedLayout L = sliced_layout(M, N, K);
  char* w = static_cast<char*>(work);
  hipLaunchKernelGGL(slice_rows_kernel, dim3((unsigned)M), dim3(256), 0, s, M, K, L.Kp, A, lda,
                     reinterpret_cast<int8_t*>(w + L.as), reinterpret_cast<int*>(w + L.ea));
  RSVD_LAUNCH_CHECK();
  return RSVD_OK;
}

rsvd_status sliced_gemm(int64_t M, int64_t N, int64_t K, const double* X, int64_t ldx, double* C,
                        int64_t ldc, void* work, hipStream_t s) {
  if (M <= 0 || N <= 0) return RSVD_OK;
  if (K <= 0 || !X || !C || !work || ldx < N || ldc < N || ((uintptr_t)work & 255) != 0)
    return RSVD_EINVAL;
  const SlicedLayout L = sliced_layout(M, N, K);
  char* w = static_cast<char*>(work);
  hipLaunchKernelGGL(slice_cols_kernel, dim3((unsigned)N), dim3(256), 0, s, K, N, L.Kp, X, ldx,
                     reinterpret_cast<int8_t*>(w + L.xs), reinterpret_cast<int*>(w + L.fx));
  RSVD_LAUNCH_CHECK();
  const int tiles_m = (int)((M + kSlRows - 1) / kSlRows);
  const int tiles_n = (int)((N + kSlCols - 1) / kSlCols);
  const int total = tiles_m * tiles_n;
  hipLaunchKernelGGL(sliced_gemm_kernel, dim3((unsigned)total), dim3(64 * kSlWaves), 0, s, M, N,
                     L.Kp,
                     reinterpret_cast<const int8_t*>(w + L.as),
                     reinterpret_cast<const int*>(w + L.ea),
                     reinterpret_cast<const int8_t*>(w + L.xs),
                     reinterpret_cast<const int*>(w + L.fx), C, ldc, tiles_n, total);
  RSVD_LAUNCH_CHECK();
  return RSVD_OK;
}

}  // namespace rsvd
