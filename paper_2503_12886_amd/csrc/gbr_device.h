// Wave- and block-level building blocks shared by the kernels: prefix scans
// and the stable ballot-ranked LSD radix pass.
#pragma once

#include "gbr_internal.h"

namespace gbr {

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint32_t o = __shfl_up(v, d, 64);
    if (lane >= d) v += o;
  }
  return v;
}

// Exclusive scan of one value per thread across a block of NT threads.
template <int NT>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* lds_waves, uint32_t* total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  constexpr int NW = NT / 64;
  uint32_t inc = wave_incl_scan(v);
  if (lane == 63) lds_waves[w] = inc;
  __syncthreads();
  uint32_t off = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < NW; ++i) {
    uint32_t x = lds_waves[i];
    if (i < w) off += x;
    tot += x;
  }
  __syncthreads();
  if (total) *total = tot;
  return off + inc - v;
}


// Stable LSD radix pass (8-bit digit at `shift`) of n 64-bit keys from src to
// dst by a block of kSortThreads threads.  Wave w owns a contiguous segment of
// the keys, so (wave, step, lane) order is key order and equal digits keep
// their relative order; the rank of a key among equal digits in its step is
// found with ballots over the digit's bits.  src/dst may be LDS or global.
constexpr int kSortThreads = 256;
constexpr int kSortWaves = kSortThreads / 64;
constexpr int kSortCap = 8192;

__device__ __forceinline__ unsigned long long digit_peers(uint32_t d, bool valid) {
  unsigned long long peers = __ballot(valid);
#pragma unroll
  for (int bit = 0; bit < 8; ++bit) {
    const bool on = (d >> bit) & 1u;
    const unsigned long long m = __ballot(on);
    peers &= on ? m : ~m;
  }
  return peers;
}

template <typename SrcT, typename DstT>
__device__ __forceinline__ void radix_pass(SrcT src, DstT dst, int n, int shift, uint32_t* hist,
                                           uint32_t* lds_waves) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int seg = ((n + kSortThreads - 1) / kSortThreads) * 64;
  const int lo = w * seg, hi = min(n, lo + seg);
  for (int i = threadIdx.x; i < kSortWaves * 256; i += kSortThreads) hist[i] = 0u;
  __syncthreads();
  for (int base = lo; base < hi; base += 64) {
    const int k = base + lane;
    const bool valid = k < hi;
    const uint32_t d = valid ? (uint32_t)(src[k] >> shift) & 255u : 0u;
    const unsigned long long peers = digit_peers(d, valid);
    if (valid && lanes_below(peers) == 0) hist[w * 256 + d] += (uint32_t)__popcll(peers);
  }
  __syncthreads();
  // offsets in (digit, wave) order
  uint32_t tot = 0;
  if (threadIdx.x < 256) {
    for (int ww = 0; ww < kSortWaves; ++ww) {
      const uint32_t c = hist[ww * 256 + threadIdx.x];
      hist[ww * 256 + threadIdx.x] = tot;
      tot += c;
    }
  }
  __syncthreads();
  const uint32_t dbase = block_excl_scan<kSortThreads>(threadIdx.x < 256 ? tot : 0u, lds_waves, nullptr);
  if (threadIdx.x < 256)
    for (int ww = 0; ww < kSortWaves; ++ww) hist[ww * 256 + threadIdx.x] += dbase;
  __syncthreads();
  for (int base = lo; base < hi; base += 64) {
    const int k = base + lane;
    const bool valid = k < hi;
    const unsigned long long key = valid ? src[k] : 0ull;
    const uint32_t d = (uint32_t)(key >> shift) & 255u;
    const unsigned long long peers = digit_peers(d, valid);
    const uint32_t below = lanes_below(peers);
    uint32_t at = 0;
    if (valid) at = hist[w * 256 + d];
    if (valid) dst[at + below] = key;
    if (valid && below == 0) hist[w * 256 + d] = at + (uint32_t)__popcll(peers);
  }
  __syncthreads();
}


}  // namespace gbr
