// Gaussian random projection P (section "Randomized matrix decompositions":
// a random projection matrix P of size N x l applied to V in step 1; one
// draw per decomposition). Entries are i.i.d. N(0, 1) from a counter-based
// generator, so every entry is a pure function of (seed, channel, row, col):
//
//   Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): counter (i, j/4, 0, 0),
//   key (seed, channel) -> four 64-bit words r0..r3; Box-Muller on (r0, r1)
//   and (r2, r3): u1 = ((r >> 11) + 1) 2^-53, u2 = (r' >> 11) 2^-53,
//   z = sqrt(-2 ln u1) cos(2 pi u2), z' = sqrt(-2 ln u1) sin(2 pi u2);
//   P[i][j] = z_{j mod 4}.
//
// One thread produces one 4-column group of one row; consecutive threads
// take consecutive groups of the same row, so stores are contiguous.
#include "common.hpp"
#include "kernels.hpp"
#include "philox.hpp"

namespace rsvd {

namespace {

__global__ void __launch_bounds__(256) omega_kernel(int64_t n, int64_t l, int64_t col0,
                                                    uint64_t seed, uint64_t channel,
                                                    double* __restrict__ out, int64_t ldo) {
  const int64_t g0 = col0 / 4;
  const int64_t g1 = (col0 + l - 1) / 4;
  const int64_t ng = g1 - g0 + 1;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * ng) return;
  const int64_t i = idx / ng;
  const int64_t grp = g0 + idx % ng;
  uint64_t c0 = (uint64_t)i, c1 = (uint64_t)grp, c2 = 0, c3 = 0;
  philox4x64_10(c0, c1, c2, c3, seed, channel);
  double z[4];
  box_muller(c0, c1, z[0], z[1]);
  box_muller(c2, c3, z[2], z[3]);
#pragma unroll
  for (int q = 0; q < 4; q++) {
    const int64_t j = grp * 4 + q;  // global column of the stream
    if (j >= col0 && j < col0 + l) out[i * ldo + (j - col0)] = z[q];
  }
}

}  // namespace

rsvd_status gaussian_omega(int64_t n, int64_t l, int64_t col0, uint64_t seed, uint64_t channel,
                           double* out, int64_t ldo, hipStream_t st) {
  if (n <= 0 || l <= 0) return RSVD_OK;
  const int64_t ng = (col0 + l - 1) / 4 - col0 / 4 + 1;
  const int64_t tot = n * ng;
  hipLaunchKernelGGL(omega_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, n, l,
                     col0, seed, channel, out, ldo);
  RSVD_LAUNCH_CHECK();
  return RSVD_OK;
}

}  // namespace rsvd
