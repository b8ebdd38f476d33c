// Early products of the BF16 precision schedules, from BF16 copies of the
// operands.
//
// Rounding the FP64 matrix on every use (the in-register path of gemm.hip)
// keeps the BF16 matrix cores idle: that kernel is bound by the conversions.
// Here A is rounded once per decomposition into BF16 planes (hi = bf16(a);
// for the split schedule also lo = bf16(a - hi)), in the orientations the
// schedule needs, so an early product streams 2 bytes (split: 4) per entry:
//
//   C (M x N, FP64) = P (M x K) X (K x N)
//     P: BF16 plane(s) of A or A^T, row-major, zero padded to Kp (mult. of 64)
//     X: rounded (split) per product into transposed planes XT (N' x Kp,
//        N' = column tiles x 16 >= N, zero padded), so a column of X is a
//        contiguous row of k values.
//
// Kernel (8 waves per workgroup, wave64): a wave owns RW fragments of 16
// rows; the workgroup covers 128 RW rows and NT column tiles of 16. K goes in
// chunks of 64, two v_mfma_f32_16x16x32_bf16 k-steps: for step h each lane
// loads A[row][k + 32 h + 8 g .. + 7] (g = lane / 16; 64 contiguous bytes of
// a row per load instruction) straight into a register ring, 1 to 3 chunks
// ahead (as registers allow); the chunk of XT for all column tiles is copied
// HBM/L2 -> LDS with global_load_lds_dwordx4 (no staging registers, two LDS
// stages, one chunk ahead) and shared by the 8 waves. XT rows are stored in LDS with the
// 16-byte pieces of row c permuted by c & 7 (conflict-free reads of 8 rows
// at a time). Accumulation in FP32; split K writes FP32
// partials (exact copies of the accumulators) that a second kernel sums in
// split order in FP64. Split schedule per term: hi*lo + lo*hi + hi*hi.
#include "common.hpp"
#include "kernels.hpp"
#include "tune.hpp"

namespace rsvd {

namespace {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

constexpr int kKC = 64;      // k per chunk (two MFMA k-steps per lane)
constexpr int kWavesB = 8;   // waves per workgroup
constexpr int kMaxNT = 17;   // column tiles per workgroup
// column tiles with two fragments per wave: beyond these the accumulators,
// the A ring and the operands exceed 256 VGPRs
constexpr int kMaxNT2 = 16;
constexpr int kMaxNTSplit2 = 10;

inline int max_nt(int rw, bool split) { return rw == 1 ? kMaxNT : (split ? kMaxNTSplit2 : kMaxNT2); }

__device__ __forceinline__ f4 mfma_bf16_32(bf8 a, bf8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ uint16_t to_bf16(double x) { return (uint16_t)bf16_bits(x); }

// Planes of X (R x C, FP64, row-major, ldx). 64 x 64 tiles through LDS.
//   n_hi/n_lo (R x ld_n): the same orientation; columns C .. ld_n - 1 zero.
//   t_hi/t_lo (rows_t x ld_t): the transpose, t(c, r) = X(r, c); rows
//   C .. rows_t - 1 and columns R .. ld_t - 1 zero.
// A null hi pointer skips that orientation; a null lo pointer skips its lo.
// ld_n and ld_t are multiples of 64.
__global__ void __launch_bounds__(256) bf16_planes_kernel(
    int64_t R, int64_t C, const double* __restrict__ X, int64_t ldx, uint16_t* __restrict__ n_hi,
    uint16_t* __restrict__ n_lo, int64_t ld_n, uint16_t* __restrict__ t_hi,
    uint16_t* __restrict__ t_lo, int64_t ld_t, int64_t rows_t) {
  __shared__ double tile[64][65];
  const int64_t r0 = (int64_t)blockIdx.y * 64, c0 = (int64_t)blockIdx.x * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;  // 64 x 4
#pragma unroll 4
  for (int i = 0; i < 16; i++) {
    const int rr = ty + 4 * i;
    const int64_t r = r0 + rr, c = c0 + tx;
    tile[rr][tx] = (r < R && c < C) ? X[r * ldx + c] : 0.0;
  }
  __syncthreads();
  // 64 rows x 8 pieces of 8 values per orientation, two pieces per thread
#pragma unroll
  for (int i = 0; i < 2; i++) {
    const int piece = threadIdx.x + 256 * i;
    const int row = piece >> 3, p8 = (piece & 7) * 8;
    if (n_hi) {
      const int64_t r = r0 + row, c = c0 + p8;
      if (r < R && c < ld_n) {
        uint16_t h[8], w[8];
#pragma unroll
        for (int j = 0; j < 8; j++) {
          const double x = tile[row][p8 + j];
          h[j] = to_bf16(x);
          w[j] = to_bf16(x - bf16_value((short)h[j]));
        }
        *reinterpret_cast<uint4*>(n_hi + r * ld_n + c) = *reinterpret_cast<const uint4*>(h);
        if (n_lo) *reinterpret_cast<uint4*>(n_lo + r * ld_n + c) = *reinterpret_cast<const uint4*>(w);
      }
    }
    if (t_hi) {
      const int64_t c = c0 + row, r = r0 + p8;  // t(c, r .. r + 7)
      if (c < rows_t && r < ld_t) {
        uint16_t h[8], w[8];
#pragma unroll
        for (int j = 0; j < 8; j++) {
          const double x = tile[p8 + j][row];
          h[j] = to_bf16(x);
          w[j] = to_bf16(x - bf16_value((short)h[j]));
        }
        *reinterpret_cast<uint4*>(t_hi + c * ld_t + r) = *reinterpret_cast<const uint4*>(h);
        if (t_lo) *reinterpret_cast<uint4*>(t_lo + c * ld_t + r) = *reinterpret_cast<const uint4*>(w);
      }
    }
  }
}

// Same-orientation planes only (no transpose): each thread rounds 8
// consecutive entries of a row, 64 bytes in (four 16-byte loads when the row
// allows) and 16 bytes out per plane.
__global__ void __launch_bounds__(256) bf16_planes_n_kernel(int64_t R, int64_t C,
                                                            const double* __restrict__ X,
                                                            int64_t ldx, bool vec,
                                                            uint16_t* __restrict__ n_hi,
                                                            uint16_t* __restrict__ n_lo,
                                                            int64_t ld_n) {
  const int64_t per_row = ld_n / 8;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= R * per_row) return;
  const int64_t r = idx / per_row, c = (idx % per_row) * 8;
  const double* src = X + r * ldx + c;
  double x[8];
  if (vec && c + 8 <= C) {
#pragma unroll
    for (int j = 0; j < 4; j++) {
      const double2 v = reinterpret_cast<const double2*>(src)[j];
      x[2 * j] = v.x;
      x[2 * j + 1] = v.y;
    }
  } else {
#pragma unroll
    for (int j = 0; j < 8; j++) x[j] = c + j < C ? src[j] : 0.0;
  }
  uint16_t h[8], w[8];
#pragma unroll
  for (int j = 0; j < 8; j++) {
    h[j] = to_bf16(x[j]);
    w[j] = to_bf16(x[j] - bf16_value((short)h[j]));
  }
  *reinterpret_cast<uint4*>(n_hi + r * ld_n + c) = *reinterpret_cast<const uint4*>(h);
  if (n_lo) *reinterpret_cast<uint4*>(n_lo + r * ld_n + c) = *reinterpret_cast<const uint4*>(w);
}

struct Bf16Args {
  int64_t M, N, Kp, kchunk;
  const uint16_t* A;   // hi plane of the left operand (M x Kp, lda)
  int64_t a_lo;        // lo plane - hi plane (elements)
  int64_t lda;
  const uint16_t* B;   // hi plane of XT (tiles_n * NT * 16 x Kp, ldb)
  int64_t b_lo;
  int64_t ldb;
  double* C;
  int64_t ldc;
  float* part;         // [splits][M][N] FP32 partials when splits > 1
  int tiles_m, tiles_n, splits;
};

template <int NT, int RW, bool SPLIT>
__global__ void __launch_bounds__(64 * kWavesB) bf16_stream_kernel(Bf16Args g) {
  constexpr int PL = SPLIT ? 2 : 1;
  constexpr int SLOTS = NT * 16 * 8;      // 16-byte slots of one plane's chunk
  constexpr int NCOPY = 2 * NT;           // 1-KB copies per plane and chunk
  constexpr int NQ = (NCOPY + kWavesB - 1) / kWavesB;
  __shared__ __attribute__((aligned(16))) bf8 Bs[2][PL][SLOTS];

  // XCD-aware order: workgroup b runs on XCD b % 8; consecutive items (the
  // column groups of one row tile, then the row tiles of one K range) go to
  // the same XCD and share its L2
  const int total = g.tiles_m * g.tiles_n * g.splits;
  const int full = total & ~7;
  int item = blockIdx.x;
  if (item < full) item = (item & 7) * (full >> 3) + (item >> 3);
  const int tn = item % g.tiles_n;
  const int tm = (item / g.tiles_n) % g.tiles_m;
  const int z = item / (g.tiles_n * g.tiles_m);
  const int64_t kb = (int64_t)z * g.kchunk;
  const int64_t ke = min(g.Kp, kb + g.kchunk);
  const int nk = (int)((ke - kb) / kKC);

  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int r = lane & 15;
  const int gq = lane >> 4;
  const int64_t row0 = (int64_t)tm * (16 * RW * kWavesB) + wave * (16 * RW);
  const int64_t col0 = (int64_t)tn * (NT * 16);

  // A: rows past M read row M - 1 (never stored)
  const uint16_t* abase[RW];
#pragma unroll
  for (int f = 0; f < RW; f++) abase[f] = g.A + min(row0 + 16 * f + r, g.M - 1) * g.lda + kb + 8 * gq;
  // XT copy q = wave + 8 i: lane -> slot 64 q + lane, i.e. row c = 8 q + lane / 8
  // (c & 7 = lane / 8), slot position lane & 7 holding piece (lane & 7) ^ (lane / 8)
  const uint16_t* bsrc = g.B + (col0 + 8 * wave + (lane >> 3)) * g.ldb + kb +
                         8 * ((lane & 7) ^ (lane >> 3));
  const int64_t bq = (int64_t)64 * g.ldb;  // 8 copies = 64 rows further

  auto issue_b = [&](int stage) {
#pragma unroll
    for (int i = 0; i < NQ; i++) {
      const int q = wave + kWavesB * i;
      if (q < NCOPY) {
#pragma unroll
        for (int pl = 0; pl < PL; pl++)
          copy_to_lds16(bsrc + i * bq + pl * g.b_lo, &Bs[stage][pl][64 * q]);
      }
    }
    bsrc += kKC;
  };
  // chunk indices past the last are clamped to it: the loads stay
  // unconditional (their count is what the wait counts below rely on)
  auto load_a = [&](bf8 (&a)[RW][PL][2], int chunk) {
    const int64_t off = (int64_t)min(chunk, nk - 1) * kKC;
#pragma unroll
    for (int f = 0; f < RW; f++) {
#pragma unroll
      for (int pl = 0; pl < PL; pl++) {
        const uint16_t* p = abase[f] + pl * g.a_lo + off;
        a[f][pl][0] = *reinterpret_cast<const bf8*>(p);
        a[f][pl][1] = *reinterpret_cast<const bf8*>(p + 32);
      }
    }
  };

  f4 acc[RW][NT];
#pragma unroll
  for (int f = 0; f < RW; f++)
#pragma unroll
    for (int t = 0; t < NT; t++) acc[f][t] = (f4){0.f, 0.f, 0.f, 0.f};

  auto compute = [&](int stage, const bf8 (&a)[RW][PL][2]) {
#pragma unroll
    for (int h = 0; h < 2; h++) {
#pragma unroll
      for (int t = 0; t < NT; t++) {
        const int slot = (16 * t + r) * 8 + ((4 * h + gq) ^ (r & 7));
        const bf8 bh = Bs[stage][0][slot];
        if constexpr (SPLIT) {
          const bf8 bl = Bs[stage][PL - 1][slot];
#pragma unroll
          for (int f = 0; f < RW; f++) {
            acc[f][t] = mfma_bf16_32(a[f][0][h], bl, acc[f][t]);
            acc[f][t] = mfma_bf16_32(a[f][PL - 1][h], bh, acc[f][t]);
            acc[f][t] = mfma_bf16_32(a[f][0][h], bh, acc[f][t]);
          }
        } else {
#pragma unroll
          for (int f = 0; f < RW; f++) acc[f][t] = mfma_bf16_32(a[f][0][h], bh, acc[f][t]);
        }
      }
    }
    // Software pipeline of the LDS reads: unit u = (h, t) is PL fragment
    // reads and MPU products; the reads run kPF units ahead of the products
    // that use them (left to itself the scheduler issues each read just
    // before its product and waits for it, so every product waits the LDS
    // latency). Scheduling-group masks: 0x100 LDS reads, 0x008 matrix ops.
    constexpr int kU = NT * 2, kMPU = RW * (SPLIT ? 3 : 1), kPF = 4;
#pragma unroll
    for (int u = 0; u < kPF && u < kU; u++) __builtin_amdgcn_sched_group_barrier(0x100, PL, 0);
#pragma unroll
    for (int u = 0; u < kU; u++) {
      __builtin_amdgcn_sched_group_barrier(0x008, kMPU, 0);
      if (u + kPF < kU) __builtin_amdgcn_sched_group_barrier(0x100, PL, 0);
    }
  };
  // A runs DA chunks ahead in a register ring, XT one chunk ahead in two LDS
  // stages. Issue order: A(0 .. DA-2), XT(0), A(DA-1), then per chunk c
  // XT(c+1), A(c+DA); so when chunk c starts only A(c+DA-1) was issued after
  // XT(c), and waiting for all but those NA loads (in-order counter) lands
  // XT(c) and A(c) (DA >= 2; with DA = 1 everything). Compiler barriers on
  // both sides of the wait keep the loads where this count assumes them; the
  // wait also drains this wave's LDS reads, so after the barrier no wave
  // still reads the stage the next copies overwrite. Whole groups of DA + 1
  // chunks run with unconditional loads; the last partial group issues no A
  // loads (they would be past the end, and dead) and waits for everything.
  constexpr int DA = RW == 1 ? (SPLIT ? 2 : 3) : (SPLIT ? 1 : 2);
  constexpr int NA = RW * PL * 2;  // A load instructions per chunk
  bf8 ring[DA + 1][RW][PL][2];
  auto begin_chunk = [&](int c, bool tail) {
    asm volatile("" ::: "memory");
    if (DA >= 2 && !tail)
      wait_vm_lgkm<NA, 0>();
    else
      wait_vm_lgkm<0, 0>();
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    if (c + 1 < nk) issue_b((c + 1) & 1);
  };
#pragma unroll
  for (int i = 0; i + 1 < DA; i++) load_a(ring[i], i);
  issue_b(0);
  load_a(ring[DA - 1], DA - 1);
  int c0 = 0;
  for (; c0 + DA + 1 <= nk; c0 += DA + 1) {
#pragma unroll
    for (int i = 0; i <= DA; i++) {
      begin_chunk(c0 + i, false);
      load_a(ring[(i + DA) % (DA + 1)], c0 + i + DA);
      compute((c0 + i) & 1, ring[i]);
    }
  }
#pragma unroll
  for (int i = 0; i < DA; i++) {
    if (c0 + i < nk) {
      begin_chunk(c0 + i, true);
      compute((c0 + i) & 1, ring[i]);
    }
  }

  // D: lane (r, gq) item it holds row 4 gq + it, column r of the 16 x 16 tile
#pragma unroll
  for (int f = 0; f < RW; f++) {
#pragma unroll
    for (int t = 0; t < NT; t++) {
      const int64_t col = col0 + 16 * t + r;
#pragma unroll
      for (int it = 0; it < 4; it++) {
        const int64_t row = row0 + 16 * f + 4 * gq + it;
        if (row < g.M && col < g.N) {
          if (g.part)
            g.part[((int64_t)z * g.M + row) * g.N + col] = acc[f][t][it];
          else
            g.C[row * g.ldc + col] = (double)acc[f][t][it];
        }
      }
    }
  }
}

// C = sum over the split partials, in split order, in FP64.
__global__ void __launch_bounds__(256) bf16_reduce_kernel(int64_t M, int64_t N, int S,
                                                          const float* __restrict__ part,
                                                          double* __restrict__ C, int64_t ldc) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= M * N) return;
  double s = 0.0;
  for (int z = 0; z < S; z++) s += (double)part[(int64_t)z * M * N + idx];
  C[(idx / N) * ldc + idx % N] = s;
}

template <int RW, bool SPLIT>
hipError_t launch_rw(int nt, dim3 grid, hipStream_t st, const Bf16Args& a) {
  switch (nt) {
#define RSVD_BCASE(X) \
  case X: hipLaunchKernelGGL((bf16_stream_kernel<X, RW, SPLIT>), grid, dim3(64 * kWavesB), 0, st, a); break;
    RSVD_BCASE(1) RSVD_BCASE(2) RSVD_BCASE(3) RSVD_BCASE(4) RSVD_BCASE(5) RSVD_BCASE(6)
    RSVD_BCASE(7) RSVD_BCASE(8) RSVD_BCASE(9) RSVD_BCASE(10) RSVD_BCASE(11) RSVD_BCASE(12)
    RSVD_BCASE(13) RSVD_BCASE(14) RSVD_BCASE(15) RSVD_BCASE(16) RSVD_BCASE(17)
#undef RSVD_BCASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

inline unsigned blocks_of(int64_t n, int64_t t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

int64_t bf16_pad(int64_t k) { return (k + 63) / 64 * 64; }

int bf16_split_cap(int64_t M, int64_t N) {
  // K ranges only while the fewest tiles (two fragments per wave, fewest
  // column groups) stay under 1024 workgroups
  const int64_t ntiles = (N + 15) / 16;
  const int64_t T = ((M + 255) / 256) * ((ntiles + kMaxNT - 1) / kMaxNT);
  int cap = 1;
  while (cap < 16 && T * cap < 1024) cap *= 2;
  return cap;
}

size_t bf16_part_floats_max(int64_t M, int64_t N) {
  const int cap = bf16_split_cap(M, N);
  return cap > 1 ? (size_t)cap * M * N : 0;
}

Bf16Shape bf16_shape(int64_t M, int64_t N, int64_t K, bool split, int rw, int splits, int groups) {
  Bf16Shape s;
  const int64_t ntiles = (N + 15) / 16;
  const int64_t tn_min = (ntiles + kMaxNT - 1) / kMaxNT;
  int64_t tn = tn_min;
  if (groups > tn && groups <= 2 * tn_min && groups <= ntiles) tn = groups;
  s.tiles_n = (int)tn;
  s.nt = (int)((ntiles + tn - 1) / tn);  // balanced column groups
  s.rw = rw == 1 || rw == 2 ? rw : (M >= 2048 ? 2 : 1);
  const int cap_nt = max_nt(s.rw, split);
  if (s.nt > cap_nt) {
    if (rw == 2) {
      // keep two fragments per wave: more column groups
      tn = (ntiles + cap_nt - 1) / cap_nt;
      s.tiles_n = (int)tn;
      s.nt = (int)((ntiles + tn - 1) / tn);
    } else {
      s.rw = 1;
    }
  }
  s.tiles_m = (int)((M + 128 * s.rw - 1) / (128 * s.rw));
  s.Kp = bf16_pad(K);
  const int64_t chunks = s.Kp / kKC;
  const int64_t T = (int64_t)s.tiles_m * s.tiles_n;
  const int cap = bf16_split_cap(M, N);
  int64_t S = 1;
  if (splits > 0) {
    S = splits < cap ? splits : cap;
  } else {
    // two workgroups per CU of 256 CUs; each split keeps at least 16 chunks
    while (T * S < 512 && chunks / (2 * S) >= 16 && S < cap) S *= 2;
  }
  if (S > chunks) S = chunks > 0 ? chunks : 1;
  const int64_t per = (chunks + S - 1) / S;
  s.kchunk = per * kKC;
  s.splits = (int)((chunks + per - 1) / per);
  if (s.splits < 1) s.splits = 1;
  s.part_floats = s.splits > 1 ? (size_t)s.splits * M * N : 0;
  s.xt_rows = (int64_t)s.tiles_n * s.nt * 16;
  return s;
}

Bf16Shape bf16_tuned_shape(int64_t M, int64_t N, int64_t K, bool split) {
  TuneCfg c;
  if (tune_get({kTuneBf16, split ? kPrecBF16S : kPrecBF16, 0, M, N, bf16_pad(K)}, &c))
    return bf16_shape(M, N, K, split, c.a, c.b, c.c);
  return bf16_shape(M, N, K, split);
}

int64_t bf16_xt_rows_max(int64_t N) {
  // g balanced groups pad the tile count by less than g, and g is at most
  // twice the fewest groups
  const int64_t ntiles = (N + 15) / 16;
  return (ntiles + 2 * ((ntiles + kMaxNT - 1) / kMaxNT)) * 16;
}

rsvd_status bf16_planes(int64_t R, int64_t C, const double* X, int64_t ldx, uint16_t* n_hi,
                        uint16_t* n_lo, int64_t ld_n, uint16_t* t_hi, uint16_t* t_lo, int64_t ld_t,
                        int64_t rows_t, hipStream_t s) {
  if (R <= 0 || C <= 0 || (!n_hi && !t_hi)) return RSVD_OK;
  if ((n_hi && (ld_n % 64 != 0 || ld_n < C)) || (t_hi && (ld_t % 64 != 0 || ld_t < R || rows_t < C)))
    return RSVD_EINVAL;
  if (!t_hi) {
    const bool vec = (ldx % 2 == 0) && ((uintptr_t)X % 16 == 0);
    hipLaunchKernelGGL(bf16_planes_n_kernel, dim3(blocks_of(R * (ld_n / 8), 256)), dim3(256), 0, s,
                       R, C, X, ldx, vec, n_hi, n_lo, ld_n);
    RSVD_LAUNCH_CHECK();
    return RSVD_OK;
  }
  const int64_t cx = n_hi ? (ld_n > rows_t ? ld_n : rows_t) : rows_t;
  const int64_t rx = t_hi ? (ld_t > R ? ld_t : R) : R;
  const dim3 grid(blocks_of(cx, 64), blocks_of(rx, 64));
  if (grid.y > 65535) return RSVD_EUNSUPPORTED;
  hipLaunchKernelGGL(bf16_planes_kernel, grid, dim3(256), 0, s, R, C, X, ldx, n_hi, n_lo, ld_n,
                     t_hi, t_lo, ld_t, rows_t);
  RSVD_LAUNCH_CHECK();
  return RSVD_OK;
}

rsvd_status bf16_gemm(const Bf16Shape& sh, int64_t M, int64_t N, const uint16_t* A_hi,
                      const uint16_t* A_lo, int64_t lda, const uint16_t* XT_hi,
                      const uint16_t* XT_lo, double* C, int64_t ldc, float* part,
                      size_t part_floats, bool split, hipStream_t st) {
  if (M <= 0 || N <= 0) return RSVD_OK;
  if (tune_recording()) {
    // candidates: fragments per wave x column groups x split counts, distinct shapes
    const TuneKey key{kTuneBf16, split ? kPrecBF16S : kPrecBF16, 0, M, N, sh.Kp};
    std::vector<TuneCfg> cands;
    std::vector<Bf16Shape> seen;
    const int64_t ntiles = (N + 15) / 16;
    const int tn_min = (int)((ntiles + kMaxNT - 1) / kMaxNT);
    for (int rw = 1; rw <= 2; rw++)
      for (int g : {tn_min, 2 * tn_min})
        for (int S = 1; S <= 16; S *= 2) {
          if (g > ntiles) continue;
          const Bf16Shape c = bf16_shape(M, N, sh.Kp, split, rw, S, g);
          bool dup = false;
          for (const Bf16Shape& o : seen)
            dup = dup || (o.rw == c.rw && o.tiles_n == c.tiles_n && o.splits == c.splits);
          if (dup) continue;
          seen.push_back(c);
          cands.push_back({c.rw, c.splits, c.tiles_n});
        }
    tune_record(key, std::move(cands), [=](hipStream_t s2) {
      return bf16_gemm(bf16_tuned_shape(M, N, sh.Kp, split), M, N, A_hi, A_lo, lda, XT_hi, XT_lo,
                       C, ldc, part, part_floats, split, s2);
    });
  }
  if (sh.nt < 1 || sh.nt > kMaxNT || (sh.rw != 1 && sh.rw != 2)) return RSVD_EINVAL;
  if (sh.nt > max_nt(sh.rw, split)) return RSVD_EINVAL;
  if (lda < sh.Kp || lda % 8 != 0 || (int64_t)sh.nt * sh.tiles_n * 16 < N) return RSVD_EINVAL;
  if (split && (!A_lo || !XT_lo)) return RSVD_EINVAL;
  if (sh.splits > 1 && (!part || part_floats < sh.part_floats)) return RSVD_EINVAL;
  Bf16Args a;
  a.M = M;
  a.N = N;
  a.Kp = sh.Kp;
  a.kchunk = sh.kchunk;
  a.A = A_hi;
  a.a_lo = split ? A_lo - A_hi : 0;
  a.lda = lda;
  a.B = XT_hi;
  a.b_lo = split ? XT_lo - XT_hi : 0;
  a.ldb = sh.Kp;
  a.C = C;
  a.ldc = ldc;
  a.part = sh.splits > 1 ? part : nullptr;
  a.tiles_m = sh.tiles_m;
  a.tiles_n = sh.tiles_n;
  a.splits = sh.splits;
  const int64_t total = (int64_t)sh.tiles_m * sh.tiles_n * sh.splits;
  if (total > 0x7fffffff) return RSVD_EUNSUPPORTED;
  const dim3 grid((unsigned)total);
  hipError_t e;
  if (split)
    e = sh.rw == 2 ? launch_rw<2, true>(sh.nt, grid, st, a) : launch_rw<1, true>(sh.nt, grid, st, a);
  else
    e = sh.rw == 2 ? launch_rw<2, false>(sh.nt, grid, st, a) : launch_rw<1, false>(sh.nt, grid, st, a);
  if (e != hipSuccess) return RSVD_EHIP;
  if (sh.splits > 1) {
    hipLaunchKernelGGL(bf16_reduce_kernel, dim3(blocks_of(M * N, 256)), dim3(256), 0, st, M, N,
                       sh.splits, (const float*)part, C, ldc);
    RSVD_LAUNCH_CHECK();
  }
  return RSVD_OK;
}

}  // namespace rsvd
