// Prop. 4.1's separable toy on the GPU: the unbiased single-coordinate
// global reset against full random restarts on F(x) = sum_i phi(x_i),
// phi(x) = -x^2/2 - beta x^3/3 on [-1, 1] (basins (0, 1] -> 1 and
// [-1, 0) -> -1 under projected descent, phi(1) < phi(-1)).  One thread per
// independent trial; a trial's point lives in LDS.
#include "common.h"
#include "kernels.h"

namespace mqo {

// uint32 draw -> (2 (w >> 8) + 1 - 2^24) / 2^24: exact, never 0, symmetric.
__device__ __forceinline__ float toy_value(uint32_t w) {
  const int32_t k = (int32_t)(w >> 8);
  return (float)(2 * k + 1 - (1 << 24)) * (1.0f / 16777216.0f);
}

// Projected descent on phi, one rounding per operation in the order written.
__device__ __forceinline__ float toy_descend(float y, float alpha, float beta, int32_t steps) {
  for (int32_t s = 0; s < steps; ++s) {
    float t = y * y;
    t = beta * t;
    t = y + t;
    t = alpha * t;
    y = fminf(fmaxf(y + t, -1.0f), 1.0f);
  }
  return y;
}

__device__ __forceinline__ double toy_phi(float xf, double beta) {
  const double x = xf;
  const double a = x * x;
  const double b = a * x;
  return -0.5 * a - (beta * b) / 3.0;
}

// Start point (restart 0, descended), then `attempts` resets of one
// coordinate, each kept iff phi strictly decreases.  first[t] = the number of
// attempts after which the point is (1, ..., 1) for the first time (0 = at
// the start), else -1.
__global__ __launch_bounds__(256) void k_toy_global_reset(uint64_t seed, int32_t n, float alpha, float beta,
                                                          int32_t steps, int32_t attempts, int32_t trials,
                                                          int32_t *__restrict__ first, float *__restrict__ x_out) {
  extern __shared__ float sx[];  // [n][blockDim.x]
  const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= trials) return;
  float *x = sx + threadIdx.x;
  const int32_t stride = blockDim.x;
  int32_t ones = 0;
  for (int32_t vb = 0; vb * 8 < n; ++vb) {
    uint32_t r[8];
    philox_block8(r, seed, PURPOSE_TOY_START, (uint64_t)t, 0, (uint64_t)vb);
    for (int32_t i = 0; i < 8 && vb * 8 + i < n; ++i) {
      const float y = toy_descend(toy_value(r[i]), alpha, beta, steps);
      x[(vb * 8 + i) * stride] = y;
      ones += y == 1.0f;
    }
  }
  int32_t hit = ones == n ? 0 : -1;
  const double b = beta;
  // The draws and descents of an attempt do not depend on the point, so
  // ILP attempts are drawn and descended together (independent dependency
  // chains); their acceptance tests then run in order.
  constexpr int ILP = 8;
  for (int32_t a0 = 0; a0 < attempts; a0 += ILP) {
    int32_t idx[ILP];
    float y[ILP];
#pragma unroll
    for (int k = 0; k < ILP; ++k) {
      uint32_t r[8];
      philox_block8(r, seed, PURPOSE_TOY_RESET, (uint64_t)t, (uint64_t)(a0 + k), 0);
      idx[k] = (int32_t)(((uint64_t)r[0] * (uint64_t)n) >> 32);
      y[k] = toy_value(r[1]);
    }
    for (int32_t st = 0; st < steps; ++st) {
#pragma unroll
      for (int k = 0; k < ILP; ++k) {
        float u = y[k] * y[k];
        u = beta * u;
        u = y[k] + u;
        u = alpha * u;
        y[k] = fminf(fmaxf(y[k] + u, -1.0f), 1.0f);
      }
    }
#pragma unroll
    for (int k = 0; k < ILP; ++k) {
      if (a0 + k >= attempts) break;
      const float old = x[idx[k] * stride];
      if (toy_phi(y[k], b) < toy_phi(old, b)) {
        x[idx[k] * stride] = y[k];
        ones += (y[k] == 1.0f) - (old == 1.0f);
        if (hit < 0 && ones == n) hit = a0 + k + 1;
      }
    }
  }
  first[t] = hit;
  if (x_out)
    for (int32_t i = 0; i < n; ++i) x_out[(int64_t)t * n + i] = x[i * stride];
}

// Restarts j = 0 .. restarts: the first j whose descended point is
// (1, ..., 1), else -1.
__global__ __launch_bounds__(256) void k_toy_full_restart(uint64_t seed, int32_t n, float alpha, float beta,
                                                          int32_t steps, int32_t restarts, int32_t trials,
                                                          int32_t *__restrict__ first) {
  const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= trials) return;
  int32_t hit = -1;
  for (int32_t j = 0; j <= restarts && hit < 0; ++j) {
    bool all = true;
    for (int32_t vb = 0; vb * 8 < n && all; ++vb) {
      uint32_t r[8];
      philox_block8(r, seed, PURPOSE_TOY_START, (uint64_t)t, (uint64_t)j, (uint64_t)vb);
      for (int32_t i = 0; i < 8 && vb * 8 + i < n && all; ++i)
        all = toy_descend(toy_value(r[i]), alpha, beta, steps) == 1.0f;
    }
    if (all) hit = j;
  }
  first[t] = hit;
}

void launch_toy(int32_t mode, uint64_t seed, int32_t n, float alpha, float beta, int32_t steps, int32_t attempts,
                int32_t trials, int32_t *first, float *x_out, hipStream_t s) {
  const int threads = 256;
  const dim3 grid((unsigned)((trials + threads - 1) / threads));
  if (mode == 0)
    hipLaunchKernelGGL(k_toy_global_reset, grid, dim3(threads), (size_t)n * threads * sizeof(float), s, seed, n,
                       alpha, beta, steps, attempts, trials, first, x_out);
  else
    hipLaunchKernelGGL(k_toy_full_restart, grid, dim3(threads), 0, s, seed, n, alpha, beta, steps, attempts, trials,
                       first);
}

}  // namespace mqo
