// Shared device helpers for the rSVD kernels (gfx950 / CDNA4, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/rsvd.h"

namespace rsvd {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kWave = 64;

// ---- FP64 matrix-core tile (v_mfma_f64_16x16x4f64) -------------------------
// Operand layout of one 16x16x4 product on gfx950 (checked on the device):
//   A (16 x 4): lane l holds A[l % 16][l / 16]
//   B (4 x 16): lane l holds B[l / 16][l % 16]
//   D (16 x 16): lane l, item t holds D[(l / 16) + 4 t][l % 16]
__device__ __forceinline__ d4 mfma_f64_16x16x4(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// ---- FP32 / BF16 matrix-core tiles (FP32 accumulation) ---------------------
// v_mfma_f32_16x16x4f32: A lane l holds A[l % 16][l / 16], B lane l holds
// B[l / 16][l % 16]; D lane l, item t holds D[4 (l / 16) + t][l % 16].
// v_mfma_f32_16x16x16bf16_1k: lane l holds 4 consecutive k values
// 4 (l / 16) .. 4 (l / 16) + 3 of row (A) / column (B) l % 16; D as above.
typedef short s4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ f4 mfma_f32_16x16x4(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma_bf16_16x16x16(s4 a, s4 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}
// FP64 -> BF16 bits: round to FP32 (nearest even), then to BF16 (nearest even).
__device__ __forceinline__ short bf16_bits(double x) {
  const float f = (float)x;
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (short)0x7fc0;  // NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}

// BF16 bits back to a value.
__device__ __forceinline__ double bf16_value(short b) {
  return (double)__uint_as_float(((uint32_t)(uint16_t)b) << 16);
}

// Arithmetic of a streaming product: FP64 MFMA, FP32 MFMA, BF16 MFMA, or the
// BF16 split (x = hi + lo with hi = bf16(x), lo = bf16(x - hi); the product
// as hi*lo + lo*hi + hi*hi on BF16 matrix cores). The low-precision ones
// accumulate in FP32. Operands stay FP64 in memory and are rounded (split)
// when they enter the matrix core.
enum Prec { kPrecF64 = 0, kPrecF32 = 1, kPrecBF16 = 2, kPrecBF16S = 3 };
// Schedules only (no kernel template takes it): the error-free sliced
// product (sliced.hip) in place of an FP64 one.
constexpr int kPrecSliced = 4;

// ---- LDS-DMA copies ---------------------------------------------------------
#define RSVD_LDS(p) ((__attribute__((address_space(3))) void*)(p))

// One 16-byte-per-lane copy global -> LDS (lane i lands at lds + 16 i). Issued
// through asm so the compiler's wait-count model does not treat the pending
// copy as a hazard for reads of the other LDS stages; waits are explicit
// (wait_vmcnt + barrier). No register is written by the instruction.
__device__ __forceinline__ void copy_to_lds16(const void* src, const void* lds) {
  const unsigned off = (unsigned)(uintptr_t)RSVD_LDS(lds);
  asm volatile("s_nop 0\n\tglobal_load_lds_dwordx4 %0, off" ::"v"(src), "{m0}"(off) : "memory");
}

template <int N>
__device__ __forceinline__ void wait_vmcnt() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

// s_waitcnt vmcnt(N) lgkmcnt(L)
template <int N, int L>
__device__ __forceinline__ void wait_vm_lgkm() {
  static_assert(N >= 0 && N < 64 && L >= 0 && L < 16, "counter range");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (L << 8));
}


// ---- wave reductions --------------------------------------------------------
// 1/x and 1/sqrt(x) from the hardware estimates and two Newton steps each
// (the estimates carry about half the FP64 mantissa; each step doubles it).
// For normal x of moderate range (the callers keep x >= 1e-290).
__device__ __forceinline__ double rcp_nr(double x) {
  double y = __builtin_amdgcn_rcp(x);
  double e = fma(-x, y, 1.0);
  y = fma(y, e, y);
  e = fma(-x, y, 1.0);
  return fma(y, e, y);
}
__device__ __forceinline__ double rsq_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
  double e = fma(-h * y, y, 0.5);
  y = fma(y, e, y);
  e = fma(-h * y, y, 0.5);
  return fma(y, e, y);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, kWave));
  return v;
}

// Polls of the barrier generation before a workgroup gives up (each poll is
// an agent-scope load after a short sleep: a few seconds in all).
constexpr uint32_t kSpinLimit = 1u << 21;

// Words of the grid barrier (in the run's workspace, zeroed before use).
// Arrivals are counted in two levels: workgroup b arrives at group counter
// b % 8 (each on its own 128-byte line), the last of a group at the top
// counter, the last group advances the generation. A flat counter costs
// ~0.13 us per workgroup of serialized atomics at the coherence point.
struct GridBar {
  uint32_t lo[8][32];
  uint32_t hi[32];
  uint32_t gen[32];
  uint32_t abort[32];
};

// Barrier over the gridDim.x workgroups of a launch whose whole grid fits on
// the device at once. The waiters poll the generation with relaxed loads (no
// cache invalidation while they wait) and acquire once it moves.
// Memory ordering: every wave waits until its own stores are acknowledged
// (so they sit in its XCD's L2) before the workgroup barrier; thread 0 then
// arrives with agent-scope acq_rel increments (an L2 write-back per arrival
// chain), the generation is advanced with release and read back with an
// acquire fence, and after the second workgroup barrier every wave acquires
// at agent scope (its L1 / L2 lines are refetched).
// A workgroup that has waited kSpinLimit polls raises the abort word and
// leaves; waiters see it and leave too. Returns false once the barrier has
// been abandoned: the kernel must then return.
constexpr uint32_t kFlatBarrier = 32;

__device__ inline bool grid_barrier(GridBar* gb, int* s_ok) {
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  if (threadIdx.x == 0) {
    int ok = 1;
    const uint32_t g = __hip_atomic_load(&gb->gen[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    // up to kFlatBarrier workgroups arrive on one counter (one atomic fewer
    // on the critical path); larger grids in 8 groups, then across groups
    const bool flat = gridDim.x <= kFlatBarrier;
    const uint32_t grp = flat ? 0u : (blockIdx.x & 7u);
    const uint32_t gsize = flat ? gridDim.x : ((gridDim.x - grp + 7u) >> 3);
    bool last = false;
    const uint32_t a =
        __hip_atomic_fetch_add(&gb->lo[grp][0], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) + 1u;
    if (a == gsize) {
      __hip_atomic_store(&gb->lo[grp][0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const uint32_t h =
          flat ? 1u
               : __hip_atomic_fetch_add(&gb->hi[0], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) + 1u;
      if (flat || h == 8u) {
        if (!flat) __hip_atomic_store(&gb->hi[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(&gb->gen[0], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        last = true;
      }
    }
    if (!last) {
      uint32_t spins = 0;
      while (__hip_atomic_load(&gb->gen[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g) {
        if (__hip_atomic_load(&gb->abort[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) {
          ok = 0;
          break;
        }
        if (++spins > kSpinLimit) {
          __hip_atomic_store(&gb->abort[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          ok = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(4);
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    *s_ok = ok;
  }
  __syncthreads();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return *s_ok != 0;
}

// Zero the barrier words (one workgroup, any size; run before the launch
// that uses the barrier, in stream order).
__device__ inline void grid_barrier_reset(GridBar* gb) {
  uint32_t* w = &gb->lo[0][0];
  constexpr int kWords = (int)(sizeof(GridBar) / sizeof(uint32_t));
  for (int i = threadIdx.x; i < kWords; i += blockDim.x) w[i] = 0u;
}

// Device-side scalar state of one decomposition, kept in the workspace.
// Halko, Martinsson and Tropp (2011), Eq. (4.3): ||(I - QQ^T) A||_2 <=
// 10 sqrt(2/pi) max_j ||(I - QQ^T) A w_j|| for r Gaussian w_j, except with
// probability 10^-r.
constexpr double kPosteriorFactor = 7.978845608028654;
// converged kept values: (s_l / s_k)^(4q + 2) <= kConvergedRatio
constexpr double kConvergedRatio = 1e-8;

struct DevState {
  uint32_t flags;        // RSVD_FLAG_* accumulated by the kernels
  uint32_t qr_shifted;   // the current orthonormalization needs a third pass
  uint32_t qr_householder;  // its Cholesky QR broke down: Householder fallback
  int32_t sweeps;        // Jacobi sweeps used
  int32_t rank;          // chosen rank
  double fro2;           // ||A||_F^2
  double resid2;         // ||A - U S V^T||_F^2
  int32_t rank_wanted;   // rank the rule asked for before the l - p / k_cap caps
  int32_t pad_;
  // adaptive range finder
  double est2;           // max_j ||W_j||^2 of the latest deflated sketch block
  double s1lb2;          // largest squared row norm of Q^T A so far (<= sigma_1^2)
  double froY2;          // ||Q^T A||_F^2 so far
  uint32_t rot_count[64];  // rotations per Jacobi sweep (convergence test)
  uint32_t chol_fail;    // multi-workgroup Cholesky: a pivot broke down
  uint32_t prefer_shift; // the last Cholesky QR of this run needed the shift
  double piv_max, piv_min;  // and the range of its pivots
  double gram_dev;       // max |G - I| of a re-orthogonalization pass's Gram (grid path)
  GridBar bar;           // grid barrier of the multi-workgroup kernels
};

}  // namespace rsvd

#define RSVD_HIP_CHECK(expr)                                   \
  do {                                                         \
    hipError_t _e = (expr);                                    \
    if (_e != hipSuccess) return RSVD_EHIP;                    \
  } while (0)

#define RSVD_LAUNCH_CHECK()                                    \
  do {                                                         \
    hipError_t _e = hipGetLastError();                         \
    if (_e != hipSuccess) return RSVD_EHIP;                    \
  } while (0)
