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

// Device-side scalar state of one decomposition, kept in the workspace.
struct DevState {
  uint32_t flags;        // RSVD_FLAG_* accumulated by the kernels
  uint32_t qr_shifted;   // the current orthonormalization needs a third pass
  uint32_t qr_householder;  // its Cholesky QR broke down: Householder fallback
  int32_t sweeps;        // Jacobi sweeps used
  int32_t rank;          // chosen rank
  double fro2;           // ||A||_F^2
  double resid2;         // ||A - U S V^T||_F^2
  uint32_t rot_count[64];  // rotations per Jacobi sweep (convergence test)
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
