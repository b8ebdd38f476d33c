// The learned (k, p, q) predictor: a 16-64-64-3 MLP (ReLU hidden layers,
// linear head) in FP32, with He-normal initialization, batched inference, and
// a training step that fuses forward, backpropagation of the mean squared
// error and the Adam update (Kingma and Ba 2015) in one launch.
//
// The paper picks R_SVD and the oversampling by hand (section "Randomized
// matrix decompositions"); the predictor maps 16 features of a cheap pilot
// sketch of a channel to (log10 k, p, q) so the main decomposition can be
// sized without adaptive growth.
//
// Parameters: one flat FP32 array, W1 (64 x 16 row-major), b1 (64),
// W2 (64 x 64), b2 (64), W3 (3 x 64), b3 (3): 5443 values.
//
// Training step (B <= 128 samples, one workgroup of 256 threads; the batch's
// activations sit in LDS): Z1 = X W1^T + b1, Z2 = relu(Z1) W2^T + b2,
// Y = relu(Z2) W3^T + b3, loss = mean (Y - T)^2 over B x 3 entries, then the
// gradients layer by layer. Each gradient entry is summed over the batch in
// order by one thread and stays in its registers until the layer's weights
// have been used by the backward pass, then the thread applies Adam to it.
#include <cmath>

#include "common.hpp"
#include "kernels.hpp"
#include "philox.hpp"

namespace rsvd {

namespace {

constexpr int kIn = 16, kHid = 64, kOut = 3;
constexpr int kW1 = 0, kB1 = kW1 + kHid * kIn, kW2 = kB1 + kHid, kB2 = kW2 + kHid * kHid;
constexpr int kW3 = kB2 + kHid, kB3 = kW3 + kOut * kHid, kParams = kB3 + kOut;
static_assert(kParams == 5443, "parameter layout");
constexpr int kMaxBatch = 128;
constexpr int kLd = kHid + 1;  // padded LDS row of the hidden activations

__global__ void __launch_bounds__(256) mlp_init_kernel(float* __restrict__ p, uint64_t seed) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= kParams) return;
  float v = 0.0f;
  if (e < kB1) {  // W1: layer 0
    const int i = (e - kW1) / kIn, j = (e - kW1) % kIn;
    v = (float)(philox_normal(i, j, seed, 0) * sqrt(2.0 / kIn));
  } else if (e >= kW2 && e < kB2) {
    const int i = (e - kW2) / kHid, j = (e - kW2) % kHid;
    v = (float)(philox_normal(i, j, seed, 1) * sqrt(2.0 / kHid));
  } else if (e >= kW3 && e < kB3) {
    const int i = (e - kW3) / kHid, j = (e - kW3) % kHid;
    v = (float)(philox_normal(i, j, seed, 2) * sqrt(2.0 / kHid));
  }
  p[e] = v;
}

// Sizing rules applied to a prediction (documented with rsvd_mlp_predict).
constexpr int kPGrid[14] = {8, 16, 32, 48, 64, 96, 128, 160, 192, 256, 320, 384, 448, 512};
constexpr int kNGrid = 14;
constexpr int kQMax = 4;
constexpr double kRankMargin = 1.05;

// Forward pass of up to 64 samples per workgroup. DECODE: instead of the
// outputs y, write the sizing (k, p, q) decoded from raw = y sd + mean.
template <bool DECODE>
__global__ void __launch_bounds__(256) mlp_forward_kernel(const float* __restrict__ p,
                                                          const float* __restrict__ X, int64_t B,
                                                          float* __restrict__ Y,
                                                          const float* __restrict__ stats,
                                                          const int64_t* __restrict__ n_cap,
                                                          int64_t* __restrict__ kpq) {
  __shared__ float xs[64][kIn];
  __shared__ float h1[64][kLd];
  __shared__ float h2[64][kLd];
  const int64_t s0 = (int64_t)blockIdx.x * 64;
  const int nb = (int)(B - s0 < 64 ? B - s0 : 64);
  for (int e = threadIdx.x; e < nb * kIn; e += blockDim.x) xs[e / kIn][e % kIn] = X[s0 * kIn + e];
  __syncthreads();
  for (int e = threadIdx.x; e < nb * kHid; e += blockDim.x) {
    const int b = e / kHid, j = e % kHid;
    float z = p[kB1 + j];
    for (int i = 0; i < kIn; i++) z += xs[b][i] * p[kW1 + j * kIn + i];
    h1[b][j] = z > 0.0f ? z : 0.0f;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < nb * kHid; e += blockDim.x) {
    const int b = e / kHid, j = e % kHid;
    float z = p[kB2 + j];
    for (int i = 0; i < kHid; i++) z += h1[b][i] * p[kW2 + j * kHid + i];
    h2[b][j] = z > 0.0f ? z : 0.0f;
  }
  __syncthreads();
  if (!DECODE) {
    for (int e = threadIdx.x; e < nb * kOut; e += blockDim.x) {
      const int b = e / kOut, o = e % kOut;
      float y = p[kB3 + o];
      for (int i = 0; i < kHid; i++) y += h2[b][i] * p[kW3 + o * kHid + i];
      Y[(s0 + b) * kOut + o] = y;
    }
    return;
  }
  for (int b = threadIdx.x; b < nb; b += blockDim.x) {
    double raw[kOut];
    for (int o = 0; o < kOut; o++) {
      float y = p[kB3 + o];
      for (int i = 0; i < kHid; i++) y += h2[b][i] * p[kW3 + o * kHid + i];
      raw[o] = (double)y * (double)stats[kOut + o] + (double)stats[o];
    }
    const int64_t cap = n_cap[s0 + b] > 0 ? n_cap[s0 + b] : 1;
    // k: margin, rounded up, within 1 .. cap (NaN or overflow -> cap)
    const double kk = ceil(kRankMargin * exp10(raw[0]));
    const int64_t k = kk < (double)cap ? (kk >= 1.0 ? (int64_t)kk : 1) : cap;
    int pp = kPGrid[kNGrid - 1];
    for (int g = 0; g < kNGrid; g++)
      if ((double)kPGrid[g] >= raw[1]) { pp = kPGrid[g]; break; }
    const double qq = floor(raw[2] + 0.5);  // nearest: the judge catches a q too small
    const int q = qq >= 0.0 ? (qq <= (double)kQMax ? (int)qq : kQMax) : (qq < 0.0 ? 0 : kQMax);
    kpq[(s0 + b) * 3 + 0] = k;
    kpq[(s0 + b) * 3 + 1] = pp;
    kpq[(s0 + b) * 3 + 2] = q;
  }
}

// Raw targets (log10 k, p, q) of B labels, their column means and population
// standard deviations (two passes, each thread summing its samples in order,
// then a fixed-order tree; FP64), and the standardized targets.
__global__ void __launch_bounds__(256) mlp_targets_kernel(const int64_t* __restrict__ labels,
                                                          int64_t B, float* __restrict__ stats,
                                                          float* __restrict__ T) {
  __shared__ double red[kOut][256];
  __shared__ double mean[kOut], sd[kOut];
  const int t = threadIdx.x;
  auto raw = [&](int64_t b, int o) -> double {
    const double v = (double)labels[b * 3 + o];
    return o == 0 ? log10(v > 1.0 ? v : 1.0) : v;
  };
  for (int pass = 0; pass < 2; pass++) {
    double acc[kOut] = {0.0, 0.0, 0.0};
    for (int64_t b = t; b < B; b += blockDim.x)
      for (int o = 0; o < kOut; o++) {
        const double x = raw(b, o);
        acc[o] += pass == 0 ? x : (x - mean[o]) * (x - mean[o]);
      }
    for (int o = 0; o < kOut; o++) red[o][t] = acc[o];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (t < w)
        for (int o = 0; o < kOut; o++) red[o][t] += red[o][t + w];
      __syncthreads();
    }
    if (t < kOut) {
      if (pass == 0) {
        mean[t] = red[t][0] / (double)B;
      } else {
        const double v = sqrt(red[t][0] / (double)B);
        sd[t] = v > 0.0 ? v : 1.0;
      }
    }
    __syncthreads();
  }
  if (t < kOut) {
    stats[t] = (float)mean[t];
    stats[kOut + t] = (float)sd[t];
  }
  for (int64_t e = t; e < B * kOut; e += blockDim.x) {
    const int o = (int)(e % kOut);
    T[e] = (float)((raw(e / kOut, o) - mean[o]) / sd[o]);
  }
}

// Label of one channel from a computed spectrum (rsvd_size_label).
__global__ void size_label_kernel(const double* __restrict__ s, int64_t count, int64_t k,
                                  int64_t n, int64_t l_min, int64_t* __restrict__ kpq) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double best = 0.0;
  int bp = -1, bq = -1;
  const double nn = (double)n;
  for (int q = 0; q <= kQMax; q++) {
    for (int g = 0; g < kNGrid; g++) {
      const int64_t pv = kPGrid[g];
      if (k + pv < n) {
        if (k + pv < l_min) continue;
        // beyond the computed values the ratio only falls: the last one decides
        const int64_t j = k + pv < count ? k + pv : count;
        const double sk = s[k - 1];
        const double r = sk > 0.0 ? s[j - 1] / sk : 0.0;
        if (j <= k || !(pow(r, (double)(4 * q + 2)) <= 1e-8)) continue;
      }
      const double L = (double)(k + pv < n ? k + pv : n);
      const double w = pow(L / 272.0, 1.6);
      const double cost = (2.0 * q + 2.0) * (2.0 * nn * nn * L / 60e12 + 0.44e-3 * w) + 3.2e-3 * w;
      if (bp < 0 || cost < best) {
        best = cost;
        bp = (int)pv;
        bq = q;
      }
    }
  }
  kpq[0] = k;
  kpq[1] = bp;
  kpq[2] = bq;
}

struct AdamArgs {
  float* m;
  float* v;
  float lr, beta1, beta2, eps, bc1, bc2;  // bc = 1 - beta^t
};

// Apply the gradient g of parameter e: Adam update (adam) or store into G.
__device__ __forceinline__ void apply(float* __restrict__ p, int e, float g, bool adam,
                                      const AdamArgs& a, float* __restrict__ G) {
  if (!adam) {
    G[e] = g;
    return;
  }
  const float m = a.beta1 * a.m[e] + (1.0f - a.beta1) * g;
  const float v = a.beta2 * a.v[e] + (1.0f - a.beta2) * g * g;
  a.m[e] = m;
  a.v[e] = v;
  p[e] -= a.lr * (m / a.bc1) / (sqrtf(v / a.bc2) + a.eps);
}

// Loss and gradient of one batch (B <= 128); with adam the gradient is
// applied to p by Adam, else written to G. loss (may be null) gets the loss.
template <bool ADAM>
__global__ void __launch_bounds__(256) mlp_grad_kernel(float* __restrict__ p,
                                                       const float* __restrict__ X,
                                                       const float* __restrict__ T, int B,
                                                       AdamArgs a, float* __restrict__ G,
                                                       float* __restrict__ loss) {
  extern __shared__ float lds[];
  float* xs = lds;                        // B x 16
  float* z1 = xs + kMaxBatch * kIn;       // B x kLd: Z1, later dZ1
  float* z2 = z1 + kMaxBatch * kLd;       // B x kLd: Z2, later dZ2
  float* dy = z2 + kMaxBatch * kLd;       // B x 3
  float* red = dy + kMaxBatch * kOut;     // 256
  const int t = threadIdx.x;
  for (int e = t; e < B * kIn; e += 256) xs[e] = X[e];
  __syncthreads();
  for (int e = t; e < B * kHid; e += 256) {
    const int b = e / kHid, j = e % kHid;
    float z = p[kB1 + j];
    for (int i = 0; i < kIn; i++) z += xs[b * kIn + i] * p[kW1 + j * kIn + i];
    z1[b * kLd + j] = z;
  }
  __syncthreads();
  for (int e = t; e < B * kHid; e += 256) {
    const int b = e / kHid, j = e % kHid;
    float z = p[kB2 + j];
    for (int i = 0; i < kHid; i++) {
      const float h = z1[b * kLd + i];
      z += (h > 0.0f ? h : 0.0f) * p[kW2 + j * kHid + i];
    }
    z2[b * kLd + j] = z;
  }
  __syncthreads();
  // output, residual, loss
  const float scale = 2.0f / (float)(B * kOut);
  float part = 0.0f;
  for (int e = t; e < B * kOut; e += 256) {
    const int b = e / kOut, o = e % kOut;
    float y = p[kB3 + o];
    for (int i = 0; i < kHid; i++) {
      const float h = z2[b * kLd + i];
      y += (h > 0.0f ? h : 0.0f) * p[kW3 + o * kHid + i];
    }
    const float r = y - T[e];
    part += r * r;
    dy[e] = scale * r;
  }
  red[t] = part;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (t < off) red[t] += red[t + off];
    __syncthreads();
  }
  if (t == 0 && loss) *loss = red[0] / (float)(B * kOut);
  // layer 3: gW3[o][j] = sum_b dy[b][o] relu(z2[b][j]); gb3[o] = sum_b dy[b][o]
  float g3 = 0.0f;
  if (t < kOut * kHid) {
    const int o = t / kHid, j = t % kHid;
    for (int b = 0; b < B; b++) {
      const float h = z2[b * kLd + j];
      g3 += dy[b * kOut + o] * (h > 0.0f ? h : 0.0f);
    }
  } else if (t < kOut * kHid + kOut) {
    const int o = t - kOut * kHid;
    for (int b = 0; b < B; b++) g3 += dy[b * kOut + o];
  }
  __syncthreads();
  // dZ2 = (dy W3) * [z2 > 0]   (in place of Z2)
  for (int e = t; e < B * kHid; e += 256) {
    const int b = e / kHid, j = e % kHid;
    float d = 0.0f;
    for (int o = 0; o < kOut; o++) d += dy[b * kOut + o] * p[kW3 + o * kHid + j];
    z2[b * kLd + j] = z2[b * kLd + j] > 0.0f ? d : 0.0f;
  }
  __syncthreads();
  // W3 has been used: apply its gradient
  if (t < kOut * kHid) apply(p, kW3 + t, g3, ADAM, a, G);
  else if (t < kOut * kHid + kOut) apply(p, kB3 + (t - kOut * kHid), g3, ADAM, a, G);
  // layer 2: gW2[j][i] = sum_b dZ2[b][j] relu(z1[b][i]); gb2[j] = sum_b dZ2[b][j]
  float g2[16];
  float gb2 = 0.0f;
#pragma unroll
  for (int r = 0; r < 16; r++) {
    const int e = t + 256 * r, j = e / kHid, i = e % kHid;
    float s = 0.0f;
    for (int b = 0; b < B; b++) {
      const float h = z1[b * kLd + i];
      s += z2[b * kLd + j] * (h > 0.0f ? h : 0.0f);
    }
    g2[r] = s;
  }
  if (t < kHid)
    for (int b = 0; b < B; b++) gb2 += z2[b * kLd + t];
  __syncthreads();
  // dZ1 = (dZ2 W2) * [z1 > 0]   (in place of Z1)
  for (int e = t; e < B * kHid; e += 256) {
    const int b = e / kHid, i = e % kHid;
    float d = 0.0f;
    for (int j = 0; j < kHid; j++) d += z2[b * kLd + j] * p[kW2 + j * kHid + i];
    z1[b * kLd + i] = z1[b * kLd + i] > 0.0f ? d : 0.0f;
  }
  __syncthreads();
  // W2 has been used: apply its gradient
#pragma unroll
  for (int r = 0; r < 16; r++) apply(p, kW2 + t + 256 * r, g2[r], ADAM, a, G);
  if (t < kHid) apply(p, kB2 + t, gb2, ADAM, a, G);
  // layer 1: gW1[i][c] = sum_b dZ1[b][i] x[b][c]; gb1[i] = sum_b dZ1[b][i]
#pragma unroll
  for (int r = 0; r < 4; r++) {
    const int e = t + 256 * r, i = e / kIn, c = e % kIn;
    float s = 0.0f;
    for (int b = 0; b < B; b++) s += z1[b * kLd + i] * xs[b * kIn + c];
    apply(p, kW1 + e, s, ADAM, a, G);
  }
  if (t < kHid) {
    float s = 0.0f;
    for (int b = 0; b < B; b++) s += z1[b * kLd + t];
    apply(p, kB1 + t, s, ADAM, a, G);
  }
}

size_t grad_lds_bytes() {
  return (size_t)(kMaxBatch * kIn + 2 * kMaxBatch * kLd + kMaxBatch * kOut + 256) * sizeof(float);
}

void allow_grad_lds() {
  static bool done = false;
  if (done) return;
  done = true;
  (void)hipFuncSetAttribute((const void*)mlp_grad_kernel<true>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)grad_lds_bytes());
  (void)hipFuncSetAttribute((const void*)mlp_grad_kernel<false>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)grad_lds_bytes());
}

// Features f_i = max(log10(s_i / s_0), -16) of the pilot sketch's singular
// values s (decreasing, l of them); entries beyond l are -16.
__global__ void pilot_feature_kernel(int l, const double* __restrict__ s, float* __restrict__ f) {
  const int i = threadIdx.x;
  if (i >= kIn) return;
  double v = -16.0;
  if (i < l && s[0] > 0.0 && s[i] > 0.0) {
    v = log10(s[i] / s[0]);
    if (!(v >= -16.0)) v = -16.0;
  }
  f[i] = (float)v;
}

}  // namespace

rsvd_status mlp_init(float* p, uint64_t seed, hipStream_t s) {
  hipLaunchKernelGGL(mlp_init_kernel, dim3((kParams + 255) / 256), dim3(256), 0, s, p, seed);
  RSVD_LAUNCH_CHECK();
  return RSVD_OK;
}

rsvd_status mlp_forward(const float* p, const float* X, int64_t B, float* Y, hipStream_t s) {
  if (B <= 0) return RSVD_OK;
  hipLaunchKernelGGL(mlp_forward_kernel<false>, dim3((unsigned)((B + 63) / 64)), dim3(256), 0, s,
                     p, X, B, Y, (const float*)nullptr, (const int64_t*)nullptr, (int64_t*)nullptr);
  RSVD_LAUNCH_CHECK();
  return RSVD_OK;
}

rsvd_status mlp_predict(const float* p, const float* stats, const float* X, int64_t B,
                        const int64_t* n_cap, int64_t* kpq, hipStream_t s) {
  if (B <= 0) return RSVD_OK;
  hipLaunchKernelGGL(mlp_forward_kernel<true>, dim3((unsigned)((B + 63) / 64)), dim3(256), 0, s,
                     p, X, B, (float*)nullptr, stats, n_cap, kpq);
  RSVD_LAUNCH_CHECK();
  return RSVD_OK;
}

rsvd_status mlp_targets(const int64_t* labels, int64_t B, float* stats, float* T, hipStream_t s) {
  hipLaunchKernelGGL(mlp_targets_kernel, dim3(1), dim3(256), 0, s, labels, B, stats, T);
  RSVD_LAUNCH_CHECK();
  return RSVD_OK;
}

rsvd_status size_label(const double* sv, int64_t count, int64_t k, int64_t n, int64_t l_min,
                       int64_t* kpq, hipStream_t s) {
  hipLaunchKernelGGL(size_label_kernel, dim3(1), dim3(64), 0, s, sv, count, k, n, l_min, kpq);
  RSVD_LAUNCH_CHECK();
  return RSVD_OK;
}

rsvd_status mlp_grad(float* p, const float* X, const float* T, int64_t B, bool adam, float* m,
                     float* v, int64_t step, float lr, float* G, float* loss, hipStream_t s) {
  if (B < 1 || B > kMaxBatch) return RSVD_EINVAL;
  allow_grad_lds();
  AdamArgs a{};
  a.m = m;
  a.v = v;
  a.lr = lr;
  a.beta1 = 0.9f;
  a.beta2 = 0.999f;
  a.eps = 1e-8f;
  a.bc1 = (float)(1.0 - std::pow(0.9, (double)step));
  a.bc2 = (float)(1.0 - std::pow(0.999, (double)step));
  if (adam)
    hipLaunchKernelGGL(mlp_grad_kernel<true>, dim3(1), dim3(256), grad_lds_bytes(), s, p, X, T,
                       (int)B, a, G, loss);
  else
    hipLaunchKernelGGL(mlp_grad_kernel<false>, dim3(1), dim3(256), grad_lds_bytes(), s, p, X, T,
                       (int)B, a, G, loss);
  RSVD_LAUNCH_CHECK();
  return RSVD_OK;
}

rsvd_status pilot_features(int l, const double* sig, float* feat, hipStream_t s) {
  hipLaunchKernelGGL(pilot_feature_kernel, dim3(1), dim3(64), 0, s, l, sig, feat);
  RSVD_LAUNCH_CHECK();
  return RSVD_OK;
}

}  // namespace rsvd
