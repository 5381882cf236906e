// Linear blending of Gaussian blendshapes (Eq. 1) and its adjoint on the
// gfx950 matrix cores.
//
// Forward:  raw[b][n][f] = sum_{k=0..K} w~[b][k] * bases[k][n][f],  w~[b][0] = 1,
//           w~[b][k] = weights[b][k-1].  A [16 frames x 4 k] times B [4 k x 16
//           features of one Gaussian] per v_mfma_f64_16x16x4f64, accumulated in
//           float64 and rounded to float32 once, so each frame's row is
//           independent of the batch it is blended in.
// Adjoint:  dbases[k][n][f] = sum_b w~[b][k] draw[b][n][f]      (contract over B)
//           dweights[b][k-1] = sum_{n,f} bases[k][n][f] draw[b][n][f]
//                                                              (contract over N*16,
//           one partial per wave, reduced afterwards in wave order)
// both with v_mfma_f32_16x16x4f32.
#include "gbr_internal.h"

namespace gbr {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kBlendMaxSteps = 16;   // K + 1 <= 64

// One wave per (16-frame group, run of Gaussians).  Grid: x over Gaussian runs,
// y over frame groups.  256 threads = 4 waves, each walking kGaussPerWave
// consecutive Gaussians.
constexpr int kGaussPerWave = 4;

__global__ __launch_bounds__(256) void blend_fwd_kernel(const float* __restrict__ bases,
                                                         const float* __restrict__ weights, int B, int K,
                                                         int64_t N, float* __restrict__ raw) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int b0 = blockIdx.y * 16;
  const int steps = (K + 1 + 3) / 4;
  const int row = lane & 15;     // A: frame within group;  B/D: feature
  const int kq = lane >> 4;      // A/B: k within step

  // A fragments (weights), kept for the whole run.
  double afrag[kBlendMaxSteps];
#pragma unroll
  for (int s = 0; s < kBlendMaxSteps; ++s) {
    double a = 0.0;
    const int k = 4 * s + kq;
    const int b = b0 + row;
    if (s < steps && b < B && k <= K) a = (k == 0) ? 1.0 : (double)weights[(int64_t)b * K + (k - 1)];
    afrag[s] = a;
  }

  const int64_t n_begin = ((int64_t)blockIdx.x * 4 + wave) * kGaussPerWave;
  const int64_t slice = N * kNF;
  for (int64_t n = n_begin; n < n_begin + kGaussPerWave && n < N; ++n) {
    d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < kBlendMaxSteps; ++s) {
      if (s < steps) {
        const int k = 4 * s + kq;
        const double bv = (k <= K) ? (double)bases[(int64_t)k * slice + n * kNF + row] : 0.0;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(afrag[s], bv, acc, 0, 0, 0);
      }
    }
    // D layout of the f64 16x16x4 op: lane l, item r holds row 4r + l/16, column l%16.
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int b = b0 + 4 * r + kq;
      if (b < B) raw[((int64_t)b * N + n) * kNF + row] = (row < 14) ? (float)acc[r] : 0.0f;
    }
  }
}

void launch_blend_fwd(const float* bases, const float* weights, int B, int K, int64_t N, float* raw,
                      hipStream_t s) {
  if (N == 0 || B == 0) return;
  dim3 grid(div_up(N, 4 * kGaussPerWave), div_up(B, 16));
  hipLaunchKernelGGL(blend_fwd_kernel, grid, dim3(256), 0, s, bases, weights, B, K, N, raw);
}

// ---------------------------------------------------------------- adjoint
// dbases: one wave per run of Gaussians; M = K+1 slices in row tiles of 16,
// contraction over frames in steps of 4.
template <int MAXT, int MAXS>
__global__ __launch_bounds__(256) void blend_dbases_kernel(const float* __restrict__ draw,
                                                            const float* __restrict__ weights, int B, int K,
                                                            int64_t N, float* __restrict__ dbases,
                                                            int accumulate) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int row = lane & 15, kq = lane >> 4;
  const int ntile = (K + 1 + 15) / 16;
  const int steps = (B + 3) / 4;
  float afrag[MAXT][MAXS];
#pragma unroll
  for (int t = 0; t < MAXT; ++t)
#pragma unroll
    for (int s = 0; s < MAXS; ++s) {
      const int k = 16 * t + row;
      const int b = 4 * s + kq;
      float a = 0.0f;
      if (t < ntile && s < steps && k <= K && b < B) a = (k == 0) ? 1.0f : weights[(int64_t)b * K + (k - 1)];
      afrag[t][s] = a;
    }
  const int64_t n_begin = ((int64_t)blockIdx.x * 4 + wave) * kGaussPerWave;
  const int64_t slice = N * kNF;
  for (int64_t n = n_begin; n < n_begin + kGaussPerWave && n < N; ++n) {
    float bfrag[MAXS];
#pragma unroll
    for (int s = 0; s < MAXS; ++s) {
      const int b = 4 * s + kq;
      bfrag[s] = (s < steps && b < B) ? draw[((int64_t)b * N + n) * kNF + row] : 0.0f;
    }
#pragma unroll
    for (int t = 0; t < MAXT; ++t) {
      if (t < ntile) {
        f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < MAXS; ++s)
          if (s < steps) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(afrag[t][s], bfrag[s], acc, 0, 0, 0);
        // D layout of the f32 16x16x4 op: lane l, item r holds row 4(l/16) + r, column l%16.
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int k = 16 * t + 4 * kq + r;
          if (k <= K) {
            float* dst = &dbases[(int64_t)k * slice + n * kNF + row];
            const float v = (row < 14) ? acc[r] : 0.0f;
            *dst = accumulate ? *dst + v : v;
          }
        }
      }
    }
  }
}

// dweights partials: wave w covers Gaussians [w*G, (w+1)*G) and writes a
// [B][K] partial; frames in row tiles of 16, slices 1..K in column tiles of 16.
constexpr int kDwGaussPerWave = 16;

template <int MAXBT, int MAXKT>
__global__ __launch_bounds__(256) void blend_dweights_kernel(const float* __restrict__ draw,
                                                              const float* __restrict__ bases, int B, int K,
                                                              int64_t N, float* __restrict__ partials) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int row = lane & 15, kq = lane >> 4;
  const int nbt = (B + 15) / 16, nkt = (K + 15) / 16;
  const int64_t gw = (int64_t)blockIdx.x * 4 + wave;
  const int64_t n_begin = gw * kDwGaussPerWave;
  const int64_t slice = N * kNF;
  f4 acc[MAXBT][MAXKT];
#pragma unroll
  for (int i = 0; i < MAXBT; ++i)
#pragma unroll
    for (int j = 0; j < MAXKT; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  for (int64_t n = n_begin; n < n_begin + kDwGaussPerWave && n < N; ++n) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {          // 16 features in 4 steps of 4
      const int f = 4 * s + kq;
      float a[MAXBT], bb[MAXKT];
#pragma unroll
      for (int i = 0; i < MAXBT; ++i) {
        const int b = 16 * i + row;
        a[i] = (i < nbt && b < B && f < 14) ? draw[((int64_t)b * N + n) * kNF + f] : 0.0f;
      }
#pragma unroll
      for (int j = 0; j < MAXKT; ++j) {
        const int k = 16 * j + row + 1;
        bb[j] = (j < nkt && k <= K && f < 14) ? bases[(int64_t)k * slice + n * kNF + f] : 0.0f;
      }
#pragma unroll
      for (int i = 0; i < MAXBT; ++i)
#pragma unroll
        for (int j = 0; j < MAXKT; ++j)
          if (i < nbt && j < nkt) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], bb[j], acc[i][j], 0, 0, 0);
    }
  }
  float* out = partials + gw * (int64_t)B * K;
#pragma unroll
  for (int i = 0; i < MAXBT; ++i)
#pragma unroll
    for (int j = 0; j < MAXKT; ++j)
      if (i < nbt && j < nkt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int b = 16 * i + 4 * kq + r;
          const int k = 16 * j + row;
          if (b < B && k < K) out[(int64_t)b * K + k] = acc[i][j][r];
        }
}

// One block per output: each thread sums a fixed stride of the partials,
// then a fixed-shape tree over the block.
__global__ __launch_bounds__(256) void reduce_partials_kernel(const float* __restrict__ partials, int64_t n_part,
                                                              int BK, float* __restrict__ out, int accumulate) {
  __shared__ float sm[256];
  const int i = blockIdx.x;
  float s = 0.0f;
  for (int64_t p = threadIdx.x; p < n_part; p += 256) s += partials[p * BK + i];
  sm[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sm[threadIdx.x] += sm[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[i] = accumulate ? out[i] + sm[0] : sm[0];
}

int64_t blend_bwd_partials(int B, int K, int64_t N) {
  const int64_t waves = (int64_t)div_up(N, 4 * kDwGaussPerWave) * 4;
  return waves * (int64_t)B * K;
}

void launch_blend_bwd(const float* draw, const float* bases, const float* weights, int B, int K, int64_t N,
                      float* dbases, float* dweights, float* partials, int64_t n_partials, int accumulate,
                      hipStream_t s) {
  if (N == 0 || B == 0) return;
  const dim3 g1(div_up(N, 4 * kGaussPerWave));
  if (B <= 16 && K + 1 <= 32)
    hipLaunchKernelGGL((blend_dbases_kernel<2, 4>), g1, dim3(256), 0, s, draw, weights, B, K, N, dbases, accumulate);
  else
    hipLaunchKernelGGL((blend_dbases_kernel<4, 16>), g1, dim3(256), 0, s, draw, weights, B, K, N, dbases,
                       accumulate);
  if (K == 0) return;
  const dim3 g2(div_up(N, 4 * kDwGaussPerWave));
  if (B <= 16 && K <= 32)
    hipLaunchKernelGGL((blend_dweights_kernel<1, 2>), g2, dim3(256), 0, s, draw, bases, B, K, N, partials);
  else
    hipLaunchKernelGGL((blend_dweights_kernel<4, 4>), g2, dim3(256), 0, s, draw, bases, B, K, N, partials);
  const int64_t n_part = (int64_t)g2.x * 4;
  (void)n_partials;
  hipLaunchKernelGGL(reduce_partials_kernel, dim3(B * K), dim3(256), 0, s, partials, n_part, B * K, dweights,
                     accumulate);
}

}  // namespace gbr
