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

// Arithmetic of a streaming product: FP64 MFMA, FP32 MFMA, or BF16 MFMA (both
// with FP32 accumulation). Operands stay FP64 in memory and are rounded when
// they enter the matrix core.
enum Prec { kPrecF64 = 0, kPrecF32 = 1, kPrecBF16 = 2 };

// ---- wave reductions --------------------------------------------------------
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
// an agent-scope load after a short sleep: about two seconds in all).
constexpr uint32_t kSpinLimit = 1u << 20;

// Barrier over the gridDim.x workgroups of a launch whose whole grid fits on
// the device at once. The last workgroup to arrive resets the counter and
// advances the generation; the others wait for the generation to change.
// Every thread fences at agent scope on both sides, so the data written
// before the barrier by any workgroup (on any XCD) is visible after it.
// A workgroup that has waited kSpinLimit polls raises *abort and leaves;
// waiters see *abort and leave too. Returns false once the barrier has
// been abandoned: the kernel must then return.
__device__ inline bool grid_barrier(uint32_t* count, uint32_t* gen, uint32_t* abort, int* s_ok) {
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    int ok = 1;
    const uint32_t g = __hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t arrived =
        __hip_atomic_fetch_add(count, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) + 1u;
    if (arrived == gridDim.x) {
      __hip_atomic_store(count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      uint32_t spins = 0;
      while (__hip_atomic_load(gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == g) {
        if (__hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) {
          ok = 0;
          break;
        }
        if (++spins > kSpinLimit) {
          __hip_atomic_store(abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          ok = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(8);
      }
    }
    *s_ok = ok;
  }
  __syncthreads();
  __threadfence();
  return *s_ok != 0;
}

// Device-side scalar state of one decomposition, kept in the workspace.
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
  uint32_t bar_count;    // grid barrier of the multi-workgroup kernels
  uint32_t bar_gen;      //   (Jacobi, Cholesky): arrivals, generation
  uint32_t bar_abort;    //   and the abandon word
  uint32_t chol_fail;    // multi-workgroup Cholesky: a pivot broke down
  double piv_max, piv_min;  // and the range of its pivots
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
