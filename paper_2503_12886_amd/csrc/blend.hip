// Linear blending of Gaussian blendshapes (Eq. 1) and its adjoint.
//
// Forward:  raw[b][n][f] = sum_{k=0..K} w~[b][k] * bases[k][n][f],  w~[b][0] = 1,
//           w~[b][k] = weights[b][k-1].
// Adjoint:  dbases[k][n][f] = sum_b w~[b][k] draw[b][n][f]       (contract over frames)
//           dweights[b][k-1] = sum_{n,f} bases[k][n][f] draw[b][n][f]
//                                                               (contract over N*16)
//
// The blend and dbases contract over at most K+1 = 64 slices or the batch's
// frames: short contractions whose cost is reading and writing the slices,
// so one thread owns one (Gaussian, feature) element, reads each of its
// inputs once (coalesced across the threads) and writes each output once.
// The blend accumulates in float64 in slice order and rounds once: the
// products of two float32 values are exact in float64, so each frame's
// result is the float64 sum rounded to float32 and does not depend on the
// batch it is blended in.  dweights contracts over N*16 elements into a
// B x K result: a long dense contraction, done on the matrix cores
// (v_mfma_f32_16x16x4f32) with per-wave partials reduced in a fixed order.
#include "gbr_internal.h"

namespace gbr {

typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kBlendThreads = 256;
constexpr int kFrameGroup = 16;        // frames whose weights are staged together

// ---------------------------------------------------------------- forward
// The frames' weights, as float64 with the implicit 1 of slice 0, are laid
// out once in a table that every thread reads at the same address (scalar
// loads: each weight reaches the multiply-adds as a scalar operand).
__global__ void blend_weights_f64_kernel(const float* __restrict__ weights, int K, double* __restrict__ w64) {
  const int b = blockIdx.x, k = threadIdx.x;   // slices past K get weight 0
  w64[(int64_t)b * kBlendW64Stride + k] = (k == 0) ? 1.0 : (k <= K ? (double)weights[(int64_t)b * K + (k - 1)] : 0.0);
}

template <int KM>   // KM >= K + 1: slice values kept in registers
__global__ __launch_bounds__(kBlendThreads) void blend_fwd_kernel(const float* __restrict__ bases,
                                                                   const double* __restrict__ w64, int B, int K,
                                                                   int64_t N, float* __restrict__ raw) {
  const int64_t L = N * kNF;
  const int64_t i = (int64_t)blockIdx.x * kBlendThreads + threadIdx.x;
  if (i >= L) return;
  const bool pad = (i % kNF) >= 14;
  // every load is issued unconditionally (slice index clamped into range) so
  // that they are all in flight together; slices past K are then zeroed
  float x[KM];
#pragma unroll
  for (int k = 0; k < KM; ++k) x[k] = bases[(int64_t)min(k, K) * L + i];
  double v[KM];
#pragma unroll
  for (int k = 0; k < KM; ++k) v[k] = (k <= K) ? (double)x[k] : 0.0;
  for (int b = 0; b < B; ++b) {
    const double* w = w64 + (int64_t)b * kBlendW64Stride;
    double acc = v[0];
#pragma unroll
    for (int k = 1; k < KM; ++k) acc = __builtin_fma(w[k], v[k], acc);   // exact product, one rounding per step
    raw[(int64_t)b * L + i] = pad ? 0.0f : (float)acc;
  }
}

void launch_blend_fwd(const float* bases, const float* weights, int B, int K, int64_t N, float* raw, double* w64,
                      hipStream_t s) {
  if (N == 0 || B == 0) return;
  hipLaunchKernelGGL(blend_weights_f64_kernel, dim3(B), dim3(kBlendW64Stride), 0, s, weights, K, w64);
  const dim3 grid(div_up(N * kNF, kBlendThreads));
  if (K + 1 <= 24)
    hipLaunchKernelGGL(blend_fwd_kernel<24>, grid, dim3(kBlendThreads), 0, s, bases, w64, B, K, N, raw);
  else
    hipLaunchKernelGGL(blend_fwd_kernel<64>, grid, dim3(kBlendThreads), 0, s, bases, w64, B, K, N, raw);
}

// ---------------------------------------------------------------- adjoint: dbases
// One thread per (Gaussian, feature): the frames' draw values are read once
// per group of 16, every slice's sum is kept in a register and added over
// the groups in frame order.  dbases_element forms those sums; the plain
// adjoint writes them, the fused step feeds them to Adam (so both see the
// same gradient).  Every thread of the workgroup must call it (barriers).
template <int KM>
__device__ __forceinline__ void dbases_element(const float* __restrict__ draw, const float* __restrict__ weights,
                                               int B, int K, int64_t L, int64_t i, bool live,
                                               float (&wt)[KM][kFrameGroup], float (&acc)[KM]) {
#pragma unroll
  for (int k = 0; k < KM; ++k) acc[k] = 0.0f;
  for (int b0 = 0; b0 < B; b0 += kFrameGroup) {
    const int nb = min(kFrameGroup, B - b0);
    __syncthreads();
    for (int t = threadIdx.x; t < kFrameGroup * KM; t += kBlendThreads) {
      const int bb = t / KM, k = t % KM;
      float x = 0.0f;
      if (bb < nb && k <= K) x = (k == 0) ? 1.0f : weights[(int64_t)(b0 + bb) * K + (k - 1)];
      wt[k][bb] = x;
    }
    __syncthreads();
    if (!live) continue;
    float d[kFrameGroup];
#pragma unroll
    for (int bb = 0; bb < kFrameGroup; ++bb) d[bb] = draw[(int64_t)(b0 + min(bb, nb - 1)) * L + i];
#pragma unroll
    for (int bb = 0; bb < kFrameGroup; ++bb) d[bb] = (bb < nb) ? d[bb] : 0.0f;   // (weights past nb are 0 too)
#pragma unroll
    for (int k = 0; k < KM; ++k) {
      if (k <= K) {
        float s = 0.0f;
#pragma unroll
        for (int bb = 0; bb < kFrameGroup; ++bb) s = __builtin_fmaf(wt[k][bb], d[bb], s);
        acc[k] += s;
      }
    }
  }
}

template <int KM>
__global__ __launch_bounds__(kBlendThreads) void blend_dbases_kernel(const float* __restrict__ draw,
                                                                      const float* __restrict__ weights, int B,
                                                                      int K, int64_t N, float* __restrict__ dbases,
                                                                      int accumulate) {
  __shared__ float wt[KM][kFrameGroup];   // slice-major: a slice's 16 weights in 4 loads
  const int64_t L = N * kNF;
  const int64_t i = (int64_t)blockIdx.x * kBlendThreads + threadIdx.x;
  const bool live = i < L;
  const bool pad = (i % kNF) >= 14;
  float acc[KM];
  dbases_element<KM>(draw, weights, B, K, L, i, live, wt, acc);
  if (!live) return;
#pragma unroll
  for (int k = 0; k < KM; ++k) {
    if (k <= K) {
      float* dst = &dbases[(int64_t)k * L + i];
      const float v = pad ? 0.0f : acc[k];
      *dst = accumulate ? *dst + v : v;
    }
  }
}

// The Adam step on the bases with the blend adjoint's dbases formed on the
// fly: each thread's K+1 gradients go straight into the update of its
// elements, so dbases is neither written nor read back.  Element k*L + i
// takes the rate lr[(k > 0) * 16 + i % 16].  The whole grid returns on an
// overflowed pass (the flag is uniform), before any barrier.
template <int KM>
__global__ __launch_bounds__(kBlendThreads) void blend_adam_kernel(const float* __restrict__ draw,
                                                                    const float* __restrict__ weights, int B, int K,
                                                                    int64_t N, float* __restrict__ p,
                                                                    float* __restrict__ m, float* __restrict__ v,
                                                                    const StatusDev* status, int group, LrTable lr,
                                                                    float b1, float b2, float eps) {
  __shared__ float wt[KM][kFrameGroup];
  if (status->overflow) return;
  const int64_t L = N * kNF;
  const int64_t i = (int64_t)blockIdx.x * kBlendThreads + threadIdx.x;
  const bool live = i < L;
  const bool pad = (i % kNF) >= 14;
  float acc[KM];
  dbases_element<KM>(draw, weights, B, K, L, i, live, wt, acc);
  if (!live) return;
  const float rc1 = 1.0f / status->adam_bc[group][0], rsc2 = 1.0f / sqrtf(status->adam_bc[group][1]);
#pragma unroll
  for (int k = 0; k < KM; ++k) {
    if (k <= K) {
      const int64_t e = (int64_t)k * L + i;
      const float rate = lr.v[(k > 0 ? 16 : 0) + (int)(i & 15)];
      adam_update(p[e], m[e], v[e], pad ? 0.0f : acc[k], rate, b1, b2, rc1, rsc2, eps);
    }
  }
}

void launch_blend_adam(const float* draw, const float* weights, int B, int K, int64_t N, float* p, float* m, float* v,
                       StatusDev* status, int group, const float* lr_table_host, float b1, float b2, float eps,
                       hipStream_t s) {
  LrTable lr;
  for (int i = 0; i < 32; ++i) lr.v[i] = lr_table_host[i];
  launch_adam_tick(status, group, b1, b2, s);
  if (N == 0 || B == 0) return;
  const dim3 g1(div_up(N * kNF, kBlendThreads));
  if (K + 1 <= 24)
    hipLaunchKernelGGL(blend_adam_kernel<24>, g1, dim3(kBlendThreads), 0, s, draw, weights, B, K, N, p, m, v, status,
                       group, lr, b1, b2, eps);
  else
    hipLaunchKernelGGL(blend_adam_kernel<64>, g1, dim3(kBlendThreads), 0, s, draw, weights, B, K, N, p, m, v, status,
                       group, lr, b1, b2, eps);
}

// ---------------------------------------------------------------- adjoint: dweights
// Wave w covers the flattened elements [w * kDwSpan, (w + 1) * kDwSpan) of
// the N*16 per-slice vectors in blocks of 16: lane (x, q) loads 4 consecutive
// elements (q-th quarter) of frame x's draw and of slice x's (and 16 + x's)
// base; each of the 4 components feeds one 16x16x4 product (frames x slices,
// contracted over the 4 quarters).  The pad features (14, 15) are skipped.
// Writes a [B][K] partial per wave, or per workgroup for small tiles (B <= 16,
// K <= 32: the four waves are added in LDS first, a quarter of the partials).
constexpr int kDwSpan = 256;

template <int MAXBT, int MAXKT>
__global__ __launch_bounds__(256) void blend_dweights_kernel(const float* __restrict__ draw,
                                                              const float* __restrict__ bases, int B, int K,
                                                              int64_t N, float* __restrict__ partials) {
  const int lane = threadIdx.x & 63;
  const int x = lane & 15, q = lane >> 4;
  const int64_t gw = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int64_t L = N * kNF;
  const int64_t e_begin = gw * kDwSpan;
  const int64_t e_end = min(L, e_begin + kDwSpan);
  const int nbt = (B + 15) / 16, nkt = (K + 15) / 16;
  f4 acc[MAXBT][MAXKT];
#pragma unroll
  for (int i = 0; i < MAXBT; ++i)
#pragma unroll
    for (int j = 0; j < MAXKT; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  const f4 zero = {0.f, 0.f, 0.f, 0.f};
  // Blocks of 16 elements, G at a time: every load of a group is issued
  // before its products, and the products of out-of-range tiles are taken on
  // zeros rather than branched around, so that the group's loads are in
  // flight together.  A wave's last group may run past its blocks: those
  // re-read the wave's last block and are zeroed.  The products are summed
  // block by block as without grouping.
  constexpr int G = (MAXBT + MAXKT <= 4) ? 4 : 1;
  const int nit = e_end > e_begin ? (int)((e_end - e_begin) / 16) : 0;   // (uniform; L is a multiple of 16)
  for (int it0 = 0; it0 < nit; it0 += G) {
    f4 a[G][MAXBT], bb[G][MAXKT];
#pragma unroll
    for (int u = 0; u < G; ++u) {
      const bool live = it0 + u < nit;
      const int64_t e = e_begin + (int64_t)min(it0 + u, nit - 1) * 16 + 4 * q;
      // unconditional loads (row and block clamped into range), masked afterwards
#pragma unroll
      for (int i = 0; i < MAXBT; ++i) {
        const int b = 16 * i + x;
        a[u][i] = *reinterpret_cast<const f4*>(draw + (int64_t)min(b, B - 1) * L + e);
        if (!(live && i < nbt && b < B)) a[u][i] = zero;
      }
#pragma unroll
      for (int j = 0; j < MAXKT; ++j) {
        const int k = 16 * j + x + 1;
        bb[u][j] = *reinterpret_cast<const f4*>(bases + (int64_t)min(k, K) * L + e);
        if (!(live && j < nkt && k <= K)) bb[u][j] = zero;
      }
      if (q == 3) {                          // features 14 and 15 are pads
#pragma unroll
        for (int i = 0; i < MAXBT; ++i) { a[u][i][2] = 0.f; a[u][i][3] = 0.f; }
#pragma unroll
        for (int j = 0; j < MAXKT; ++j) { bb[u][j][2] = 0.f; bb[u][j][3] = 0.f; }
      }
    }
    __builtin_amdgcn_sched_barrier(0);      // keep the group's loads ahead of its products
#pragma unroll
    for (int u = 0; u < G; ++u)
#pragma unroll
      for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int i = 0; i < MAXBT; ++i)
#pragma unroll
          for (int j = 0; j < MAXKT; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[u][i][c], bb[u][j][c], acc[i][j], 0, 0, 0);
  }
  // D layout of the f32 16x16x4 op: lane l, item r holds row 4(l/16) + r, column l%16.
  if constexpr (MAXBT * MAXKT <= 2) {
    // small tiles: the block's four waves are added in LDS (wave order) and
    // the block writes one [B][K] partial
    constexpr int TB = 16 * MAXBT, TK = 16 * MAXKT;
    __shared__ float ws[4][TB * TK];
    const int w = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < MAXBT; ++i)
#pragma unroll
      for (int j = 0; j < MAXKT; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) ws[w][(16 * i + 4 * q + r) * TK + 16 * j + x] = acc[i][j][r];
    __syncthreads();
    float* out = partials + (int64_t)blockIdx.x * B * K;
    for (int t = threadIdx.x; t < B * K; t += 256) {
      const int b = t / K, k = t % K;
      const int o = b * TK + k;
      out[t] = ((ws[0][o] + ws[1][o]) + ws[2][o]) + ws[3][o];
    }
  } else {
    float* out = partials + gw * (int64_t)B * K;
#pragma unroll
    for (int i = 0; i < MAXBT; ++i)
#pragma unroll
      for (int j = 0; j < MAXKT; ++j)
        if (i < nbt && j < nkt)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int b = 16 * i + 4 * q + r;
            const int k = 16 * j + x;
            if (b < B && k < K) out[(int64_t)b * K + k] = acc[i][j][r];
          }
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
  const int64_t waves = (int64_t)div_up(N * kNF, 4 * kDwSpan) * 4;
  return waves * (int64_t)B * K;
}

int64_t blend_bwd_partials_used(int B, int K, int64_t N) {
  if (K == 0) return 0;
  const int64_t blocks = (int64_t)div_up(N * kNF, 4 * kDwSpan);
  const bool small = B <= 16 && K <= 32;     // as launch_blend_bwd: a partial per block, else per wave
  return (small ? blocks : 4 * blocks) * (int64_t)B * K;
}

void launch_blend_bwd(const float* draw, const float* bases, const float* weights, int B, int K, int64_t N,
                      float* dbases, float* dweights, float* partials, int64_t n_partials, int accumulate,
                      hipStream_t s) {
  if (N == 0 || B == 0) return;
  const dim3 g1(div_up(N * kNF, kBlendThreads));
  if (dbases && K + 1 <= 24)
    hipLaunchKernelGGL(blend_dbases_kernel<24>, g1, dim3(kBlendThreads), 0, s, draw, weights, B, K, N, dbases,
                       accumulate);
  else if (dbases)
    hipLaunchKernelGGL(blend_dbases_kernel<64>, g1, dim3(kBlendThreads), 0, s, draw, weights, B, K, N, dbases,
                       accumulate);
  if (K == 0) return;
  const dim3 g2(div_up(N * kNF, 4 * kDwSpan));
  const bool small = B <= 16 && K <= 32;
  if (small)
    hipLaunchKernelGGL((blend_dweights_kernel<1, 2>), g2, dim3(256), 0, s, draw, bases, B, K, N, partials);
  else
    hipLaunchKernelGGL((blend_dweights_kernel<4, 4>), g2, dim3(256), 0, s, draw, bases, B, K, N, partials);
  const int64_t n_part = (int64_t)g2.x * (small ? 1 : 4);   // a partial per block (small tiles) or per wave
  (void)n_partials;
  hipLaunchKernelGGL(reduce_partials_kernel, dim3(B * K), dim3(256), 0, s, partials, n_part, B * K, dweights,
                     accumulate);
}

}  // namespace gbr
