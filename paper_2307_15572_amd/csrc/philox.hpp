// Counter-based Gaussian draws shared by the projection P and the MLP's
// initial weights: Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11) and the
// Box-Muller transform (see omega.hip for the stream definition).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rsvd {

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

// Entry (i, j) of the standard-normal stream keyed by (k0, k1): counter
// (i, j / 4, 0, 0), value z_{j mod 4}.
__device__ __forceinline__ double philox_normal(uint64_t i, uint64_t j, uint64_t k0, uint64_t k1) {
  uint64_t c0 = i, c1 = j >> 2, c2 = 0, c3 = 0;
  philox4x64_10(c0, c1, c2, c3, k0, k1);
  double z[4];
  box_muller(c0, c1, z[0], z[1]);
  box_muller(c2, c3, z[2], z[3]);
  return z[j & 3];
}

}  // namespace rsvd
