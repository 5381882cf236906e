// Per-frame depth order of the visible splats: every valid splat gets its
// frame-local rank in ascending (binary32 depth, splat index) order, the
// order in which the compositing visits Gaussians.  Done once per frame
// instead of once per tile:
//   1. splats are distributed over nbk buckets per frame by their depth bits,
//      scaled between the frame's min and max (monotone in depth);
//   2. a wave ranks each bucket of at most 64 splats by direct comparison;
//      larger buckets go to a block that compares in LDS (<= 2048) or runs
//      the stable radix passes through global memory.
#include "gbr_device.h"

namespace gbr {

constexpr int kMaxBuckets = 8192;   // per frame

__device__ __forceinline__ uint32_t depth_bucket(uint32_t bits, uint32_t mn, uint32_t mx, int nbk) {
  return (uint32_t)(((unsigned long long)(bits - mn) * (unsigned long long)nbk) /
                    ((unsigned long long)(mx - mn) + 1ull));
}

// Bucketing without global atomics.  Workgroup (frame b, block j) takes the
// frame's splats [4096 j, 4096 j + 4096) and histograms their buckets in
// LDS; the histograms of all (frame, block) pairs form a matrix, bucket-major
// with the blocks of a bucket adjacent, whose exclusive scan gives every
// block its own range inside every bucket.  The scatter pass recomputes the
// buckets and places each splat at its block's offset plus its LDS rank.
constexpr int kBucketBlock = 4096;   // splats per workgroup, 16 per thread

__device__ __forceinline__ bool bucket_of(const PassArgs& a, const FrameDev& F, int64_t n, uint32_t mn, uint32_t mx,
                                          uint32_t& bits, uint32_t& bk, int64_t& s) {
  if (n >= F.gauss_count) return false;
  s = F.gauss_base + n;
  if (a.cnt[s] == 0) return false;
  bits = __float_as_uint(a.rec[s * kRecF + 9]);
  bk = depth_bucket(bits, mn, mx, a.nbk);
  return true;
}

__global__ __launch_bounds__(256) void bucket_count_kernel(PassArgs a) {
  __shared__ uint32_t hist[kMaxBuckets];
  const int b = blockIdx.y, blk = blockIdx.x;
  const FrameDev& F = a.frames[b];
  for (int t = threadIdx.x; t < a.nbk; t += 256) hist[t] = 0u;
  __syncthreads();
  const uint32_t mn = a.minmax[2 * b], mx = a.minmax[2 * b + 1];
  for (int i = 0; i < kBucketBlock / 256; ++i) {
    uint32_t bits, bk;
    int64_t s;
    if (bucket_of(a, F, (int64_t)blk * kBucketBlock + i * 256 + threadIdx.x, mn, mx, bits, bk, s))
      atomicAdd(&hist[bk], 1u);
  }
  __syncthreads();
  for (int t = threadIdx.x; t < a.nbk; t += 256)   // every row is written, zeros included
    a.bkt_count[((int64_t)b * a.nbk + t) * a.nblk + blk] = hist[t];
}

__global__ __launch_bounds__(256) void bucket_scatter_kernel(PassArgs a) {
  __shared__ uint32_t hist[kMaxBuckets];
  const int b = blockIdx.y, blk = blockIdx.x;
  const FrameDev& F = a.frames[b];
  if ((int64_t)blk * kBucketBlock >= F.gauss_count) return;
  for (int t = threadIdx.x; t < a.nbk; t += 256) hist[t] = 0u;
  __syncthreads();
  const uint32_t mn = a.minmax[2 * b], mx = a.minmax[2 * b + 1];
  uint32_t rk[kBucketBlock / 256];
#pragma unroll
  for (int i = 0; i < kBucketBlock / 256; ++i) {
    uint32_t bits, bk;
    int64_t s;
    rk[i] = bucket_of(a, F, (int64_t)blk * kBucketBlock + i * 256 + threadIdx.x, mn, mx, bits, bk, s)
                ? atomicAdd(&hist[bk], 1u) : 0u;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < a.nbk; t += 256) hist[t] = a.bkt_moff[((int64_t)b * a.nbk + t) * a.nblk + blk];
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kBucketBlock / 256; ++i) {
    uint32_t bits, bk;
    int64_t s;
    if (bucket_of(a, F, (int64_t)blk * kBucketBlock + i * 256 + threadIdx.x, mn, mx, bits, bk, s))
      a.bkeys[hist[bk] + rk[i]] = ((unsigned long long)bits << 32) | (uint32_t)s;
  }
}

// bkt_start[i] = start of bucket i (frame-major) = the scanned matrix at block 0.
__global__ void bucket_starts_kernel(PassArgs a, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i <= n) a.bkt_start[i] = a.bkt_moff[i * a.nblk];
}

__device__ __forceinline__ void emit_ranked(const PassArgs& a, unsigned long long key, uint32_t pos, uint32_t vbase) {
  const uint32_t s = (uint32_t)key;
  a.depth_sorted[pos] = s;
  a.rank[s] = pos - vbase;
}

// One wave per bucket: keys are unique, so a key's rank is the number of
// smaller keys in the bucket.
__global__ __launch_bounds__(256) void bucket_sort_small_kernel(PassArgs a) {
  const int lane = threadIdx.x & 63;
  const int gb = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (gb >= a.B * a.nbk) return;
  const uint32_t start = a.bkt_start[gb];
  const uint32_t n = a.bkt_start[gb + 1] - start;
  if (n == 0) return;
  if (n > 64) {
    if (lane == 0) a.big_list[atomicAdd(a.big_count, 1u)] = (uint32_t)gb;
    return;
  }
  const int b = gb / a.nbk;
  const uint32_t vbase = a.bkt_start[b * a.nbk];
  const unsigned long long key = (lane < (int)n) ? a.bkeys[start + lane] : ~0ull;
  const uint32_t hi = (uint32_t)(key >> 32), lo = (uint32_t)key;
  uint32_t rank = 0;
  for (uint32_t j = 0; j < n; ++j) {
    const uint32_t khi = (uint32_t)__builtin_amdgcn_readlane((int)hi, (int)j);
    const uint32_t klo = (uint32_t)__builtin_amdgcn_readlane((int)lo, (int)j);
    rank += (khi < hi || (khi == hi && klo < lo)) ? 1u : 0u;
  }
  if (lane < (int)n) emit_ranked(a, key, start + rank, vbase);
}

constexpr int kBigDirect = 2048;

__global__ __launch_bounds__(kSortThreads) void bucket_sort_big_kernel(PassArgs a) {
  __shared__ unsigned long long keys[kBigDirect];
  __shared__ uint32_t hist[kSortWaves * 256];
  __shared__ uint32_t lds_waves[kSortWaves];
  __shared__ uint32_t vary[2];
  const uint32_t count = *a.big_count;
  for (uint32_t item = blockIdx.x; item < count; item += gridDim.x) {
    const int gb = (int)a.big_list[item];
    const uint32_t start = a.bkt_start[gb];
    const int n = (int)(a.bkt_start[gb + 1] - start);
    const int b = gb / a.nbk;
    const uint32_t vbase = a.bkt_start[b * a.nbk];
    __syncthreads();
    if (n <= kBigDirect) {
      for (int i = threadIdx.x; i < n; i += kSortThreads) keys[i] = a.bkeys[start + i];
      __syncthreads();
      for (int i = threadIdx.x; i < n; i += kSortThreads) {
        const unsigned long long k = keys[i];
        uint32_t rank = 0;
        for (int j = 0; j < n; ++j) rank += keys[j] < k ? 1u : 0u;
        emit_ranked(a, k, start + rank, vbase);
      }
    } else {
      unsigned long long* src = a.bkeys + start;
      unsigned long long* alt = a.bkeys_alt + start;
      if (threadIdx.x < 2) vary[threadIdx.x] = 0u;
      __syncthreads();
      const unsigned long long k0 = src[0];
      uint32_t vlo = 0, vhi = 0;
      for (int i = threadIdx.x; i < n; i += kSortThreads) {
        const unsigned long long x = src[i] ^ k0;
        vlo |= (uint32_t)x; vhi |= (uint32_t)(x >> 32);
      }
      if (vlo) atomicOr(&vary[0], vlo);
      if (vhi) atomicOr(&vary[1], vhi);
      __syncthreads();
      const unsigned long long varying = ((unsigned long long)vary[1] << 32) | vary[0];
      int parity = 0;
      for (int shift = 0; shift < 64; shift += 8) {
        if (((varying >> shift) & 255ull) == 0) continue;
        if (parity == 0) radix_pass(src, alt, n, shift, hist, lds_waves);
        else radix_pass(alt, src, n, shift, hist, lds_waves);
        parity ^= 1;
      }
      const unsigned long long* out = parity ? alt : src;
      for (int i = threadIdx.x; i < n; i += kSortThreads) emit_ranked(a, out[i], start + (uint32_t)i, vbase);
    }
  }
}

void launch_depth_order(const PassArgs& a, int64_t max_frame_splats, uint32_t* scan_scratch, hipStream_t s) {
  if (a.B == 0 || max_frame_splats == 0) return;
  const dim3 grid(a.nblk, a.B);
  const int64_t nb = (int64_t)a.B * a.nbk;
  hipLaunchKernelGGL(bucket_count_kernel, grid, dim3(256), 0, s, a);
  launch_scan_u32(a.bkt_count, a.bkt_moff, nb * a.nblk, scan_scratch, a.status, -1, nullptr, s);
  hipLaunchKernelGGL(bucket_starts_kernel, dim3(div_up(nb + 1, 256)), dim3(256), 0, s, a, nb);
  hipLaunchKernelGGL(bucket_scatter_kernel, grid, dim3(256), 0, s, a);
  hipLaunchKernelGGL(bucket_sort_small_kernel, dim3(div_up((int64_t)a.B * a.nbk, 4)), dim3(256), 0, s, a);
  hipLaunchKernelGGL(bucket_sort_big_kernel, dim3(std::min(a.B * a.nbk, 512)), dim3(kSortThreads), 0, s, a);
}

}  // namespace gbr
