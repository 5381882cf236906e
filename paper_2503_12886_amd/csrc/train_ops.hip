// The small dense pieces of the training step around the renderer: the
// weight MLP psi = F(theta) (Eq. 2) forward/backward, and Adam with
// per-attribute learning rates (Sec. A.3).
#include "gbr_internal.h"

namespace gbr {

// ---------------------------------------------------------------- MLP forward
// One workgroup per frame runs the three layers back to back: the layer's
// input vector sits in LDS, each wave forms output units four at a time
// (lanes over the input, weight rows read coalesced, then a fixed-order sum
// across the wave).  Pre-activations are kept (z1, z2 for the backward; the
// ReLU of a layer is applied when the next layer reads them).
constexpr int kMlpThreads = 1024;
constexpr int kMlpWaves = kMlpThreads / 64;
constexpr int kMlpMaxIn = 1024;

__device__ __forceinline__ float wave_sum_f32(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// out[j] = bias[j] + sum_c W[j][c] act(in[c]) for j < n_out; act = ReLU when relu_in.
// A wave forms kRows output units at a time over passes of 256 inputs: lane
// l takes inputs c0 + l + 64 t (t < 4), and every weight load of a pass
// (rows and inputs clamped into range, masked afterwards) is issued before
// the first product, so a layer costs a load latency per pass rather than
// one per input step.
constexpr int kRows = 8;

__device__ __forceinline__ void mlp_layer(const float* __restrict__ W, const float* __restrict__ bias,
                                          const float* in, int n_in, int n_out, bool relu_in,
                                          float* __restrict__ out_g, float* out_l) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int j0 = w * kRows; j0 < n_out; j0 += kMlpWaves * kRows) {
    float s[kRows];
#pragma unroll
    for (int r = 0; r < kRows; ++r) s[r] = 0.0f;
    for (int c0 = 0; c0 < n_in; c0 += 256) {
      float xv[4], wv[kRows][4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int c = c0 + 64 * t + lane;
        const int cc = min(c, n_in - 1);
#pragma unroll
        for (int r = 0; r < kRows; ++r) wv[r][t] = W[(int64_t)min(j0 + r, n_out - 1) * n_in + cc];
        const float v = in[cc];
        xv[t] = c < n_in ? (relu_in ? fmaxf(v, 0.0f) : v) : 0.0f;
      }
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int r = 0; r < kRows; ++r) s[r] = __builtin_fmaf(wv[r][t], xv[t], s[r]);
    }
#pragma unroll
    for (int r = 0; r < kRows; ++r) s[r] = wave_sum_f32(s[r]);
    if (lane < kRows && j0 + lane < n_out) {
      float v = s[0];
#pragma unroll
      for (int r = 1; r < kRows; ++r) v = lane == r ? s[r] : v;
      v += bias[j0 + lane];
      out_g[j0 + lane] = v;
      if (out_l) out_l[j0 + lane] = v;
    }
  }
}

__global__ __launch_bounds__(kMlpThreads) void mlp_fwd_kernel(const float* __restrict__ params,
                                                              const float* __restrict__ theta, int d_in, int hidden,
                                                              int K, float* __restrict__ psi, float* __restrict__ z1,
                                                              float* __restrict__ z2) {
  __shared__ float xa[kMlpMaxIn], xb[kMlpMaxIn];
  const int b = blockIdx.x;
  const float* W1 = params;
  const float* b1 = W1 + (int64_t)hidden * d_in;
  const float* W2 = b1 + hidden;
  const float* b2 = W2 + (int64_t)hidden * hidden;
  const float* W3 = b2 + hidden;
  const float* b3 = W3 + (int64_t)K * hidden;
  for (int t = threadIdx.x; t < d_in; t += kMlpThreads) xa[t] = theta[(int64_t)b * d_in + t];
  __syncthreads();
  mlp_layer(W1, b1, xa, d_in, hidden, false, z1 + (int64_t)b * hidden, xb);
  __syncthreads();
  mlp_layer(W2, b2, xb, hidden, hidden, true, z2 + (int64_t)b * hidden, xa);
  __syncthreads();
  mlp_layer(W3, b3, xa, hidden, K, true, psi + (int64_t)b * K, nullptr);
}

void launch_mlp_fwd(const float* params, const float* theta, int B, int d_in, int hidden, int K, float* psi,
                    float* z1, float* z2, hipStream_t s) {
  if (B == 0) return;
  hipLaunchKernelGGL(mlp_fwd_kernel, dim3(B), dim3(kMlpThreads), 0, s, params, theta, d_in, hidden, K, psi, z1, z2);
}

// ---------------------------------------------------------------- MLP backward
// dz2 = (W3^T dpsi) * [z2 > 0], then dz1 = (W2^T dz2) * [z1 > 0].  Each frame
// takes kActParts workgroups: every one forms the whole of dz2 (K x hidden
// terms; the first one stores it) and its own part of dz1's units.  A unit's
// sum is split over as many threads as the workgroup has for it (weight rows
// read coalesced across units, each thread's loads in flight together), and
// the pieces are added in order.  Then one thread per parameter sums over the
// frames in frame order.
constexpr int kActParts = 4;

// dz[i] = [z[i] > 0] * sum_k W[k][i] g[k] for i in [i0, i1) (g in LDS; dz to
// dz_l (LDS, indexed by i) when non-null and to dz_g (global) when non-null).
__device__ __forceinline__ void mlp_act_back(const float* __restrict__ W, const float* g, int n_g, int n_x, int i0,
                                             int i1, const float* __restrict__ z, float* part, float* dz_l,
                                             float* __restrict__ dz_g) {
  const int nu = i1 - i0;                                          // units, <= kMlpThreads
  const int split = min(16, max(1, kMlpThreads / max(nu, 1)));     // threads per unit
  const int per = (n_g + split - 1) / split;
  const int t = (int)threadIdx.x;
  if (nu > 0 && t < nu * split) {
    const int i = i0 + t % nu, qk = t / nu;
    const int k0 = qk * per, k1 = min(n_g, k0 + per);
    // 16 steps at a time, every weight load issued first (index clamped into
    // range); steps past k1 add 0 * w, which leaves the sum as it is
    float s = 0.0f;
    for (int kb = k0; kb < k1; kb += 16) {
      float wv[16], gv[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int k = min(kb + u, k1 - 1);
        wv[u] = W[(int64_t)k * n_x + i];
        gv[u] = kb + u < k1 ? g[k] : 0.0f;
      }
#pragma unroll
      for (int u = 0; u < 16; ++u) s = __builtin_fmaf(wv[u], gv[u], s);
    }
    part[qk * kMlpMaxIn + (i - i0)] = s;
  }
  __syncthreads();
  for (int u = t; u < nu; u += kMlpThreads) {
    float v = 0.0f;
    for (int qk = 0; qk < split; ++qk) v += part[qk * kMlpMaxIn + u];
    const int i = i0 + u;
    v = z[i] > 0.0f ? v : 0.0f;
    if (dz_l) dz_l[i] = v;
    if (dz_g) dz_g[i] = v;
  }
  __syncthreads();
}

__global__ __launch_bounds__(kMlpThreads) void mlp_bwd_act_kernel(const float* __restrict__ W2,
                                                                  const float* __restrict__ W3,
                                                                  const float* __restrict__ dpsi,
                                                                  const float* __restrict__ z1,
                                                                  const float* __restrict__ z2, int hidden, int K,
                                                                  float* __restrict__ dz1, float* __restrict__ dz2) {
  __shared__ float part[16 * kMlpMaxIn];
  __shared__ float gk[kMlpMaxIn], gh[kMlpMaxIn];
  const int b = blockIdx.x, q = blockIdx.y;
  for (int k = threadIdx.x; k < K; k += kMlpThreads) gk[k] = dpsi[(int64_t)b * K + k];
  __syncthreads();
  mlp_act_back(W3, gk, K, hidden, 0, hidden, z2 + (int64_t)b * hidden, part, gh,
               q == 0 ? dz2 + (int64_t)b * hidden : nullptr);
  const int per = (hidden + kActParts - 1) / kActParts;
  const int i0 = min(hidden, q * per), i1 = min(hidden, i0 + per);
  mlp_act_back(W2, gh, hidden, hidden, i0, i1, z1 + (int64_t)b * hidden, part, nullptr, dz1 + (int64_t)b * hidden);
}

// sum over frames b of x[b xs] * act(y[b ys]) (y absent: of x[b xs]), in frame
// order, one rounding per step; frames are read 16 at a time (index clamped
// into range) so that their loads are in flight together, and the steps past
// the last frame add exact zeros (0 * 0), which leave the sum as it is.
template <bool HAS_Y, bool RELU_Y>
__device__ __forceinline__ float frame_sum(int B, const float* x, int64_t xs, const float* y, int64_t ys) {
  float s = 0.0f;
  for (int b0 = 0; b0 < B; b0 += 16) {
    float xv[16], yv[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int64_t b = min(b0 + u, B - 1);
      const bool in = b0 + u < B;
      const float xl = x[b * xs], yl = HAS_Y ? y[b * ys] : 1.0f;
      xv[u] = in ? xl : 0.0f;
      yv[u] = in ? (RELU_Y ? fmaxf(yl, 0.0f) : yl) : 0.0f;
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) s = HAS_Y ? __builtin_fmaf(xv[u], yv[u], s) : s + xv[u];
  }
  return s;
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
  float s;
  int64_t r = i;
  if (r < n1) {                                    // W1[j][c] = sum_b dz1[b][j] theta[b][c]
    const int j = (int)(r / d_in), c = (int)(r % d_in);
    s = frame_sum<true, false>(B, dz1 + j, hidden, theta + c, d_in);
  } else if ((r -= n1) < hidden) {                 // b1
    s = frame_sum<false, false>(B, dz1 + r, hidden, nullptr, 0);
  } else if ((r -= hidden) < n2) {                 // W2[j][c] = sum_b dz2[b][j] relu(z1[b][c])
    const int j = (int)(r / hidden), c = (int)(r % hidden);
    s = frame_sum<true, true>(B, dz2 + j, hidden, z1 + c, hidden);
  } else if ((r -= n2) < hidden) {                 // b2
    s = frame_sum<false, false>(B, dz2 + r, hidden, nullptr, 0);
  } else if ((r -= hidden) < n3) {                 // W3[k][c] = sum_b dpsi[b][k] relu(z2[b][c])
    const int k = (int)(r / hidden), c = (int)(r % hidden);
    s = frame_sum<true, true>(B, dpsi + k, K, z2 + c, hidden);
  } else {                                         // b3
    r -= n3;
    s = frame_sum<false, false>(B, dpsi + r, K, nullptr, 0);
  }
  dP[i] = s;
}

void launch_mlp_bwd(const float* params, const float* theta, const float* z1, const float* z2, const float* dpsi,
                    int B, int d_in, int hidden, int K, float* dz1, float* dz2, float* dparams, hipStream_t s) {
  if (B == 0) return;
  const float* W2 = params + (int64_t)hidden * d_in + hidden;
  const float* W3 = W2 + (int64_t)hidden * hidden + hidden;
  hipLaunchKernelGGL(mlp_bwd_act_kernel, dim3(B, kActParts), dim3(kMlpThreads), 0, s, W2, W3, dpsi, z1, z2, hidden,
                     K, dz1, dz2);
  const int64_t total = (int64_t)hidden * d_in + hidden + (int64_t)hidden * hidden + hidden + (int64_t)K * hidden + K;
  hipLaunchKernelGGL(mlp_bwd_param_kernel, dim3(div_up(total, 256)), dim3(256), 0, s, theta, z1, z2, dz1, dz2, dpsi,
                     B, d_in, hidden, K, dparams);
}

// ---------------------------------------------------------------- Adam
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
    const float rate = lr.v[(i >= split ? 16 : 0) + (int)(i & 15)];
    adam_update(p[i], m[i], v[i], g[i], rate, b1, b2, rc1, rsc2, eps);
  }
}

void launch_adam_tick(StatusDev* status, int group, float b1, float b2, hipStream_t s) {
  hipLaunchKernelGGL(adam_tick_kernel, dim3(1), dim3(1), 0, s, status, group, b1, b2, &status->adam_bc[group][0]);
}

void launch_adam(StatusDev* status, int group, float* p, const float* g, float* m, float* v, int64_t n,
                 int64_t split, const float* lr_table_host, float b1, float b2, float eps, hipStream_t s) {
  LrTable lr;
  for (int i = 0; i < 32; ++i) lr.v[i] = lr_table_host[i];
  launch_adam_tick(status, group, b1, b2, s);
  if (n == 0) return;
  const unsigned nb = (unsigned)std::min<int64_t>(div_up(n, 256), 8192);
  hipLaunchKernelGGL(adam_kernel, dim3(nb), dim3(256), 0, s, status, &status->adam_bc[group][0], p, g, m, v, n, split, lr,
                     b1, b2, eps);
}

}  // namespace gbr
