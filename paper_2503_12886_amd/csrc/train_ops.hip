// The small dense pieces of the training step around the renderer: the
// weight MLP psi = F(theta) (Eq. 2) forward/backward, and Adam with
// per-attribute learning rates (Sec. A.3).
#include "gbr_internal.h"

namespace gbr {

// ---------------------------------------------------------------- MLP forward
// One block per frame.  Each wave computes whole output units: the 64 lanes
// split the input dimension (coalesced row reads), then a fixed-order DPP
// reduction.  Pre-activations are kept for the backward pass.
constexpr int kMlpThreads = 256;
constexpr int kMlpMaxDim = 1024;

__device__ __forceinline__ float row_dot(const float* __restrict__ wrow, const float* __restrict__ x, int len) {
  const int lane = threadIdx.x & 63;
  float s = 0.0f;
  for (int i = lane; i < len; i += 64) s = __builtin_fmaf(wrow[i], x[i], s);
  s = wave_sum_to63(s);
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, s), 63));
}

__global__ __launch_bounds__(kMlpThreads) void mlp_fwd_kernel(const float* __restrict__ P,
                                                               const float* __restrict__ theta, int d_in,
                                                               int hidden, int K, float* __restrict__ psi,
                                                               float* __restrict__ z1, float* __restrict__ z2) {
  __shared__ float x[kMlpMaxDim], h1[kMlpMaxDim], h2[kMlpMaxDim];
  const int b = blockIdx.x;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  constexpr int NW = kMlpThreads / 64;
  const float* W1 = P;
  const float* b1 = W1 + (int64_t)hidden * d_in;
  const float* W2 = b1 + hidden;
  const float* b2 = W2 + (int64_t)hidden * hidden;
  const float* W3 = b2 + hidden;
  const float* b3 = W3 + (int64_t)K * hidden;
  for (int i = threadIdx.x; i < d_in; i += kMlpThreads) x[i] = theta[(int64_t)b * d_in + i];
  __syncthreads();
  for (int j = w; j < hidden; j += NW) {
    const float z = row_dot(W1 + (int64_t)j * d_in, x, d_in) + b1[j];
    if (lane == 0) { z1[(int64_t)b * hidden + j] = z; h1[j] = fmaxf(z, 0.0f); }
  }
  __syncthreads();
  for (int j = w; j < hidden; j += NW) {
    const float z = row_dot(W2 + (int64_t)j * hidden, h1, hidden) + b2[j];
    if (lane == 0) { z2[(int64_t)b * hidden + j] = z; h2[j] = fmaxf(z, 0.0f); }
  }
  __syncthreads();
  for (int k = w; k < K; k += NW) {
    const float z = row_dot(W3 + (int64_t)k * hidden, h2, hidden) + b3[k];
    if (lane == 0) psi[(int64_t)b * K + k] = z;
  }
}

void launch_mlp_fwd(const float* params, const float* theta, int B, int d_in, int hidden, int K, float* psi,
                    float* z1, float* z2, hipStream_t s) {
  if (B == 0) return;
  hipLaunchKernelGGL(mlp_fwd_kernel, dim3(B), dim3(kMlpThreads), 0, s, params, theta, d_in, hidden, K, psi, z1, z2);
}

// ---------------------------------------------------------------- MLP backward
// Kernel 1 (one block per frame): dz2 = (W3^T dpsi) * [z2 > 0], dz1 = (W2^T dz2) * [z1 > 0].
// Kernel 2 (one thread per parameter): weight/bias gradients summed over the
// frames in frame order.
__global__ __launch_bounds__(kMlpThreads) void mlp_bwd_act_kernel(const float* __restrict__ P,
                                                                   const float* __restrict__ z1,
                                                                   const float* __restrict__ z2,
                                                                   const float* __restrict__ dpsi, int d_in,
                                                                   int hidden, int K, float* __restrict__ dz1,
                                                                   float* __restrict__ dz2) {
  __shared__ float g[64];
  __shared__ float d2[kMlpMaxDim];
  const int b = blockIdx.x;
  const float* W2 = P + (int64_t)hidden * d_in + hidden;
  const float* W3 = W2 + (int64_t)hidden * hidden + hidden;
  for (int k = threadIdx.x; k < K; k += kMlpThreads) g[k] = dpsi[(int64_t)b * K + k];
  __syncthreads();
  for (int i = threadIdx.x; i < hidden; i += kMlpThreads) {
    float s = 0.0f;
    for (int k = 0; k < K; ++k) s = __builtin_fmaf(W3[(int64_t)k * hidden + i], g[k], s);
    const float v = z2[(int64_t)b * hidden + i] > 0.0f ? s : 0.0f;
    d2[i] = v;
    dz2[(int64_t)b * hidden + i] = v;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < hidden; i += kMlpThreads) {
    float s = 0.0f;
    for (int j = 0; j < hidden; ++j) s = __builtin_fmaf(W2[(int64_t)j * hidden + i], d2[j], s);
    dz1[(int64_t)b * hidden + i] = z1[(int64_t)b * hidden + i] > 0.0f ? s : 0.0f;
  }
}

__global__ __launch_bounds__(256) void mlp_bwd_param_kernel(const float* __restrict__ theta,
                                                            const float* __restrict__ z1,
                                                            const float* __restrict__ z2,
                                                            const float* __restrict__ dz1,
                                                            const float* __restrict__ dz2,
                                                            const float* __restrict__ dpsi, int B, int d_in,
                                                            int hidden, int K, float* __restrict__ dP) {
  const int64_t n1 = (int64_t)hidden * d_in, n2 = (int64_t)hidden * hidden, n3 = (int64_t)K * hidden;
  const int64_t total = n1 + hidden + n2 + hidden + n3 + K;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= total) return;
  float s = 0.0f;
  int64_t r = i;
  if (r < n1) {                                    // W1[j][c] = sum_b dz1[b][j] theta[b][c]
    const int j = (int)(r / d_in), c = (int)(r % d_in);
    for (int b = 0; b < B; ++b) s = __builtin_fmaf(dz1[(int64_t)b * hidden + j], theta[(int64_t)b * d_in + c], s);
  } else if ((r -= n1) < hidden) {                 // b1
    for (int b = 0; b < B; ++b) s += dz1[(int64_t)b * hidden + r];
  } else if ((r -= hidden) < n2) {                 // W2[j][c] = sum_b dz2[b][j] relu(z1[b][c])
    const int j = (int)(r / hidden), c = (int)(r % hidden);
    for (int b = 0; b < B; ++b)
      s = __builtin_fmaf(dz2[(int64_t)b * hidden + j], fmaxf(z1[(int64_t)b * hidden + c], 0.0f), s);
  } else if ((r -= n2) < hidden) {                 // b2
    for (int b = 0; b < B; ++b) s += dz2[(int64_t)b * hidden + r];
  } else if ((r -= hidden) < n3) {                 // W3[k][c] = sum_b dpsi[b][k] relu(z2[b][c])
    const int k = (int)(r / hidden), c = (int)(r % hidden);
    for (int b = 0; b < B; ++b)
      s = __builtin_fmaf(dpsi[(int64_t)b * K + k], fmaxf(z2[(int64_t)b * hidden + c], 0.0f), s);
  } else {                                         // b3
    r -= n3;
    for (int b = 0; b < B; ++b) s += dpsi[(int64_t)b * K + r];
  }
  dP[i] = s;
}

void launch_mlp_bwd(const float* params, const float* theta, const float* z1, const float* z2, const float* dpsi,
                    int B, int d_in, int hidden, int K, float* dz1, float* dz2, float* dparams, hipStream_t s) {
  if (B == 0) return;
  hipLaunchKernelGGL(mlp_bwd_act_kernel, dim3(B), dim3(kMlpThreads), 0, s, params, z1, z2, dpsi, d_in, hidden, K,
                     dz1, dz2);
  const int64_t total = (int64_t)hidden * d_in + hidden + (int64_t)hidden * hidden + hidden + (int64_t)K * hidden + K;
  hipLaunchKernelGGL(mlp_bwd_param_kernel, dim3(div_up(total, 256)), dim3(256), 0, s, theta, z1, z2, dz1, dz2, dpsi,
                     B, d_in, hidden, K, dparams);
}

// ---------------------------------------------------------------- Adam
struct LrTable { float v[32]; };

__global__ void adam_tick_kernel(StatusDev* status, int group, float b1, float b2, float* bc) {
  if (status->overflow) return;
  const int t = ++status->adam_step[group];
  bc[0] = (float)(1.0 - pow((double)b1, (double)t));
  bc[1] = (float)(1.0 - pow((double)b2, (double)t));
}

__global__ __launch_bounds__(256) void adam_kernel(const StatusDev* status, const float* __restrict__ bc,
                                                   float* __restrict__ p, const float* __restrict__ g,
                                                   float* __restrict__ m, float* __restrict__ v, int64_t n,
                                                   int64_t split, LrTable lr, float b1, float b2, float eps) {
  if (status->overflow) return;
  const float c1 = bc[0], c2 = bc[1];
  const float rc1 = 1.0f / c1, rsc2 = 1.0f / sqrtf(c2);
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float rate = lr.v[(i >= split ? 16 : 0) + (int)(i & 15)];
    p[i] -= rate * (mi * rc1) / (sqrtf(vi) * rsc2 + eps);
  }
}

void launch_adam(StatusDev* status, int group, float* p, const float* g, float* m, float* v, int64_t n,
                 int64_t split, const float* lr_table_host, float b1, float b2, float eps, hipStream_t s) {
  LrTable lr;
  for (int i = 0; i < 32; ++i) lr.v[i] = lr_table_host[i];
  float* bc = &status->adam_bc[0];
  hipLaunchKernelGGL(adam_tick_kernel, dim3(1), dim3(1), 0, s, status, group, b1, b2, bc);
  if (n == 0) return;
  const unsigned nb = (unsigned)std::min<int64_t>(div_up(n, 256), 8192);
  hipLaunchKernelGGL(adam_kernel, dim3(nb), dim3(256), 0, s, status, bc, p, g, m, v, n, split, lr, b1, b2, eps);
}

}  // namespace gbr
