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

namespace rsvd {

namespace {

constexpr uint64_t kPhiloxM0 = 0xD2E7470EE14C6C93ull;
constexpr uint64_t kPhiloxM1 = 0xCA5A826395121157ull;
constexpr uint64_t kPhiloxW0 = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kPhiloxW1 = 0xBB67AE8584CAA73Bull;

__device__ __forceinline__ void philox4x64_10(uint64_t& c0, uint64_t& c1, uint64_t& c2,
                                              uint64_t& c3, uint64_t k0, uint64_t k1) {
#pragma unroll
  for (int r = 0; r < 10; r++) {
    if (r > 0) {
      k0 += kPhiloxW0;
      k1 += kPhiloxW1;
    }
    const uint64_t lo0 = kPhiloxM0 * c0, hi0 = __umul64hi(kPhiloxM0, c0);
    const uint64_t lo1 = kPhiloxM1 * c2, hi1 = __umul64hi(kPhiloxM1, c2);
    const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
}

__device__ __forceinline__ void box_muller(uint64_t ra, uint64_t rb, double& z0, double& z1) {
  const double u1 = ((double)(ra >> 11) + 1.0) * 0x1p-53;
  const double u2 = (double)(rb >> 11) * 0x1p-53;
  const double rad = sqrt(-2.0 * log(u1));
  const double ang = (2.0 * 3.141592653589793) * u2;
  z0 = rad * cos(ang);
  z1 = rad * sin(ang);
}

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
