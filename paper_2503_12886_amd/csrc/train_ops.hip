// The small dense pieces of the training step around the renderer: the
// weight MLP psi = F(theta) (Eq. 2) forward/backward, and Adam with
// per-attribute learning rates (Sec. A.3).
#include "gbr_internal.h"

namespace gbr {

// ---------------------------------------------------------------- MLP forward
// One launch per layer.  A block owns 16 output units for every frame: the 16
// weight rows are staged in LDS once, each thread forms one (frame, unit) dot
// product in input order.  The ReLU of the previous layer is applied when its
// stored pre-activation is read.
constexpr int kRowsPerBlock = 8;
constexpr int kMlpMaxIn = 1024;

__global__ __launch_bounds__(1024) void dense_fwd_kernel(const float* __restrict__ W, const float* __restrict__ bias,
                                                         const float* __restrict__ in, int relu_in, int B, int n_in,
                                                         int n_out, float* __restrict__ out) {
  __shared__ float w[kRowsPerBlock * (kMlpMaxIn + 1)];
  const int ld = n_in | 1;   // odd row stride: the rows a wave reads at once sit in different LDS banks
  const int j0 = blockIdx.x * kRowsPerBlock;
  const int rows = min(kRowsPerBlock, n_out - j0);
  for (int t = threadIdx.x; t < rows * n_in; t += blockDim.x) w[(t / n_in) * ld + t % n_in] = W[(int64_t)j0 * n_in + t];
  __syncthreads();
  for (int q = threadIdx.x; q < B * rows; q += blockDim.x) {
    const int b = q / rows, jj = q % rows;
    const float* x = in + (int64_t)b * n_in;
    const float* wr = w + jj * ld;
    float s = 0.0f;
    if (relu_in) {
#pragma unroll 8
      for (int i = 0; i < n_in; ++i) s = __builtin_fmaf(wr[i], fmaxf(x[i], 0.0f), s);
    } else {
#pragma unroll 8
      for (int i = 0; i < n_in; ++i) s = __builtin_fmaf(wr[i], x[i], s);
    }
    out[(int64_t)b * n_out + j0 + jj] = s + bias[j0 + jj];
  }
}

void launch_mlp_fwd(const float* params, const float* theta, int B, int d_in, int hidden, int K, float* psi,
                    float* z1, float* z2, hipStream_t s) {
  if (B == 0) return;
  const float* W1 = params;
  const float* b1 = W1 + (int64_t)hidden * d_in;
  const float* W2 = b1 + hidden;
  const float* b2 = W2 + (int64_t)hidden * hidden;
  const float* W3 = b2 + hidden;
  const float* b3 = W3 + (int64_t)K * hidden;
  const int thr = std::min(1024, std::max(64, ((B * kRowsPerBlock + 63) / 64) * 64));   // one thread per (frame, row)
  hipLaunchKernelGGL(dense_fwd_kernel, dim3(div_up(hidden, kRowsPerBlock)), dim3(thr), 0, s, W1, b1, theta, 0, B,
                     d_in, hidden, z1);
  hipLaunchKernelGGL(dense_fwd_kernel, dim3(div_up(hidden, kRowsPerBlock)), dim3(thr), 0, s, W2, b2, z1, 1, B,
                     hidden, hidden, z2);
  hipLaunchKernelGGL(dense_fwd_kernel, dim3(div_up(K, kRowsPerBlock)), dim3(thr), 0, s, W3, b3, z2, 1, B, hidden, K,
                     psi);
}

// ---------------------------------------------------------------- MLP backward
// dz2 = (W3^T dpsi) * [z2 > 0], dz1 = (W2^T dz2) * [z1 > 0].  A block owns 64
// units of one frame (a lane per unit, weight rows read coalesced); its 8
// waves each sum an eighth of the contraction, and the eighths are added in
// wave order.  Then one thread per parameter sums over the frames in frame
// order.
constexpr int kActSplit = 8;

__global__ __launch_bounds__(64 * kActSplit) void dense_bwd_act_kernel(const float* __restrict__ W,
                                                                       const float* __restrict__ g,
                                                                       const float* __restrict__ z, int B, int n_g,
                                                                       int n_x, float* __restrict__ dz) {
  __shared__ float part[kActSplit][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i = blockIdx.x * 64 + lane;
  const int b = blockIdx.y;
  const int per = (n_g + kActSplit - 1) / kActSplit;
  const int k0 = w * per, k1 = min(n_g, k0 + per);
  float s = 0.0f;
  if (i < n_x)
    for (int k = k0; k < k1; ++k) s = __builtin_fmaf(W[(int64_t)k * n_x + i], g[(int64_t)b * n_g + k], s);
  part[w][lane] = s;
  __syncthreads();
  if (w == 0 && i < n_x) {
    float t = 0.0f;
#pragma unroll
    for (int q = 0; q < kActSplit; ++q) t += part[q][lane];
    dz[(int64_t)b * n_x + i] = z[(int64_t)b * n_x + i] > 0.0f ? t : 0.0f;
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
  const float* W2 = params + (int64_t)hidden * d_in + hidden;
  const float* W3 = W2 + (int64_t)hidden * hidden + hidden;
  const dim3 ga(div_up(hidden, 64), B);
  hipLaunchKernelGGL(dense_bwd_act_kernel, ga, dim3(64 * kActSplit), 0, s, W3, dpsi, z2, B, K, hidden, dz2);
  hipLaunchKernelGGL(dense_bwd_act_kernel, ga, dim3(64 * kActSplit), 0, s, W2, dz2, z1, B, hidden, hidden, dz1);
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
