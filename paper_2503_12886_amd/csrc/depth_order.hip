// Per-frame depth order of the visible splats: every valid splat gets its
// frame-local rank in ascending (binary32 depth, splat index) order, the
// order in which the compositing visits Gaussians.  Done once per frame
// instead of once per tile:
//   1. splats are distributed over nbk buckets per frame by their depth bits,
//      scaled between the frame's min and max (monotone in depth);
//   2. buckets are ranked by direct comparison, 32 buckets per workgroup
//      in LDS (or a wave per bucket when they do not fit); large buckets go
//      to workgroups of the same launch that compare in LDS (<= 2048) or
//      run the stable radix passes through global memory.
#include "gbr_device.h"

namespace gbr {

constexpr int kMaxBuckets = 8192;   // per frame

__device__ __forceinline__ uint32_t depth_bucket(uint32_t bits, uint32_t mn, uint32_t mx, int nbk) {
  return (uint32_t)(((unsigned long long)(bits - mn) * (unsigned long long)nbk) /
                    ((unsigned long long)(mx - mn) + 1ull));
}

// Bucketing without global atomics.  Workgroup (frame b, block j) takes the
// frame's splats [8192 j, 8192 j + 8192) and histograms their buckets in
// LDS; the histograms of all (frame, block) pairs form a matrix, bucket-major
// with the blocks of a bucket adjacent, whose exclusive scan gives every
// block its own range inside every bucket.  The scatter pass recomputes the
// buckets and places each splat at its block's offset plus its LDS rank.
// Depth keys come from the compact per-splat key array (invalid splats carry
// 0xffffffff, which no positive depth has); loads are clamped into range and
// issued unconditionally so that a thread's eight loads overlap.
constexpr int kBucketThreads = 1024;
constexpr int kBucketItems = kBucketBlock / kBucketThreads;

// (issued before the frame's depth range is reduced, which they do not need)
__device__ __forceinline__ void load_bucket_keys(const PassArgs& a, const FrameDev& F, int blk, uint32_t* key) {
  const int64_t cnt = F.gauss_count;
#pragma unroll
  for (int i = 0; i < kBucketItems; ++i) {
    const int64_t n = (int64_t)blk * kBucketBlock + i * kBucketThreads + threadIdx.x;
    const int64_t nn = n < cnt ? n : cnt - 1;
    key[i] = cnt > 0 ? a.dkey[F.gauss_base + nn] : 0xffffffffu;
    if (n >= cnt) key[i] = 0xffffffffu;
  }
}

__device__ __forceinline__ void key_buckets(const PassArgs& a, uint32_t mn, uint32_t mx, const uint32_t* key,
                                            uint32_t* bk) {
#pragma unroll
  for (int i = 0; i < kBucketItems; ++i) bk[i] = key[i] != 0xffffffffu ? depth_bucket(key[i], mn, mx, a.nbk) : 0u;
}

// The frame's depth range: the minimum and maximum over the projection's
// per-workgroup slots of frame b (every thread gets it).
__device__ __forceinline__ void frame_depth_range(const PassArgs& a, const FrameDev& F, int b, uint32_t* red,
                                                  uint32_t& mn, uint32_t& mx) {
  const int64_t nbp = (F.gauss_count + 255) / 256;
  const uint32_t* mm = a.blk_mm + 2 * (F.gauss_base / 256 + b);
  uint32_t lo = 0xffffffffu, hi = 0u;
  for (int64_t i = threadIdx.x; i < nbp; i += kBucketThreads) {
    lo = min(lo, mm[2 * i]);
    hi = max(hi, mm[2 * i + 1]);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    lo = min(lo, (uint32_t)__shfl_xor((int)lo, o, 64));
    hi = max(hi, (uint32_t)__shfl_xor((int)hi, o, 64));
  }
  constexpr int NW = kBucketThreads / 64;
  if ((threadIdx.x & 63) == 0) { red[threadIdx.x >> 6] = lo; red[NW + (threadIdx.x >> 6)] = hi; }
  __syncthreads();
  mn = red[0];
  mx = red[NW];
#pragma unroll
  for (int w = 1; w < NW; ++w) { mn = min(mn, red[w]); mx = max(mx, red[NW + w]); }
}

// A block's buckets are split between kBucketParts workgroups (grid x =
// block * kBucketParts + part): each reads the block's keys and handles
// only those in its share of the buckets, so the pass fills twice as many
// CUs as there are (frame, block) pairs.  nbk is a power of two >= 64.
constexpr int kBucketParts = 2;

__global__ __launch_bounds__(kBucketThreads) void bucket_count_kernel(PassArgs a) {
  __shared__ uint32_t hist[kMaxBuckets / kBucketParts];
  __shared__ uint32_t red[2 * (kBucketThreads / 64)];
  const int b = blockIdx.y, blk = blockIdx.x / kBucketParts;
  const int per = a.nbk / kBucketParts;
  const uint32_t lo = (uint32_t)((blockIdx.x % kBucketParts) * per);
  const FrameDev& F = a.frames[b];
  uint32_t key[kBucketItems], bk[kBucketItems];
  load_bucket_keys(a, F, blk, key);
  for (int t = threadIdx.x; t < per; t += kBucketThreads) hist[t] = 0u;
  uint32_t mn, mx;
  frame_depth_range(a, F, b, red, mn, mx);
  key_buckets(a, mn, mx, key, bk);
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kBucketItems; ++i)
    if (key[i] != 0xffffffffu && bk[i] - lo < (uint32_t)per) atomicAdd(&hist[bk[i] - lo], 1u);
  __syncthreads();
  for (int t = threadIdx.x; t < per; t += kBucketThreads)   // every row is written, zeros included
    a.bkt_count[((int64_t)b * a.nbk + lo + t) * a.nblk + blk] = hist[t];
}

__global__ __launch_bounds__(kBucketThreads) void bucket_scatter_kernel(PassArgs a) {
  __shared__ uint32_t hist[kMaxBuckets / kBucketParts];
  __shared__ uint32_t red[2 * (kBucketThreads / 64)];
  const int b = blockIdx.y, blk = blockIdx.x / kBucketParts;
  const int per = a.nbk / kBucketParts;
  const uint32_t lo = (uint32_t)((blockIdx.x % kBucketParts) * per);
  const FrameDev& F = a.frames[b];
  if ((int64_t)blk * kBucketBlock >= F.gauss_count) return;
  // the keys and this block's offsets in its buckets are read first: neither
  // depends on the depth range or the LDS ranks
  uint32_t key[kBucketItems], bk[kBucketItems], rk[kBucketItems];
  load_bucket_keys(a, F, blk, key);
  constexpr int kOffPer = kMaxBuckets / kBucketParts / kBucketThreads;
  uint32_t moff[kOffPer];
#pragma unroll
  for (int j = 0; j < kOffPer; ++j) {
    const int t = (int)threadIdx.x + j * kBucketThreads;
    moff[j] = t < per ? a.bkt_moff[((int64_t)b * a.nbk + lo + t) * a.nblk + blk] : 0u;
  }
  for (int t = threadIdx.x; t < per; t += kBucketThreads) hist[t] = 0u;
  uint32_t mn, mx;
  frame_depth_range(a, F, b, red, mn, mx);
  key_buckets(a, mn, mx, key, bk);
  __syncthreads();
  bool mine[kBucketItems];
#pragma unroll
  for (int i = 0; i < kBucketItems; ++i) {
    mine[i] = key[i] != 0xffffffffu && bk[i] - lo < (uint32_t)per;
    rk[i] = mine[i] ? atomicAdd(&hist[bk[i] - lo], 1u) : 0u;
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kOffPer; ++j) {
    const int t = (int)threadIdx.x + j * kBucketThreads;
    if (t < per) hist[t] = moff[j];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kBucketItems; ++i) {
    if (!mine[i]) continue;
    const int64_t s = F.gauss_base + (int64_t)blk * kBucketBlock + i * kBucketThreads + threadIdx.x;
    a.bkeys[hist[bk[i] - lo] + rk[i]] = ((unsigned long long)key[i] << 32) | (uint32_t)s;
  }
}


__device__ __forceinline__ void emit_ranked(const PassArgs& a, unsigned long long key, uint32_t pos, uint32_t vbase) {
  const uint32_t s = (uint32_t)key;
  a.depth_sorted[pos] = s;
  a.rank[s] = pos - vbase;
}

// Ranks within buckets.  Keys are unique, so a key's rank is the number of
// smaller keys in its bucket.  One launch does both parts:
//  * the ranking workgroups take 32 consecutive buckets each: when their
//    keys fit in LDS, every thread ranks keys against the keys of their
//    bucket there; otherwise a wave per bucket compares through lane reads.
//    Buckets of more than kRankMax keys (kWaveMax on the wave path: the cap
//    follows from the 32 buckets' total alone) are left to
//  * the large-bucket workgroups, which come first in the grid (so that
//    their longer work starts early): workgroup s of ns checks the buckets
//    s, s + ns, ..., recomputing each one's cap from the bucket starts, and
//    sorts those above it one at a time (comparison in LDS up to kBigDirect
//    keys, else stable radix passes over the varying key bytes).
// The bucket count per frame is a power of two of at least 64, so a ranking
// workgroup's buckets belong to one frame.
constexpr int kRankBuckets = 32;
constexpr int kRankKeys = 2048;
constexpr uint32_t kRankMax = 128;
constexpr uint32_t kWaveMax = 64;
constexpr int kBigDirect = 2048;
constexpr int kOrderThreads = 256;
static_assert(kSortThreads == kOrderThreads, "the radix passes run on the workgroup");
static_assert(kBigDirect <= kRankKeys, "both parts share the key array");

// the cap of bucket gb (the size above which it is a large bucket)
__device__ __forceinline__ uint32_t bucket_cap(const PassArgs& a, int gb, int nb) {
  const int g0 = gb - gb % kRankBuckets, g1 = min(nb, g0 + kRankBuckets);
  return a.bkt_start[g1] - a.bkt_start[g0] <= (uint32_t)kRankKeys ? kRankMax : kWaveMax;
}

__device__ void sort_large_buckets(const PassArgs& a, int s, int ns, unsigned long long* keys, uint32_t* hist,
                                   uint32_t* lds_waves, uint32_t* vary, uint32_t* list, uint32_t* nlist) {
  const int nb = a.B * a.nbk;
  for (int round = s; round < nb; round += ns * kOrderThreads) {
    if (threadIdx.x == 0) *nlist = 0u;
    __syncthreads();
    const int gb = round + ns * (int)threadIdx.x;
    if (gb < nb) {
      const uint32_t n = a.bkt_start[gb + 1] - a.bkt_start[gb];
      if (n > kWaveMax && n > bucket_cap(a, gb, nb)) list[atomicAdd(nlist, 1u)] = (uint32_t)gb;
    }
    __syncthreads();
    const uint32_t count = *nlist;
    for (uint32_t item = 0; item < count; ++item) {
      const int g = (int)list[item];
      const uint32_t start = a.bkt_start[g];
      const int n = (int)(a.bkt_start[g + 1] - start);
      const uint32_t vbase = a.bkt_start[(g / a.nbk) * a.nbk];
      __syncthreads();
      if (n <= kBigDirect) {
        for (int i = threadIdx.x; i < n; i += kOrderThreads) keys[i] = a.bkeys[start + i];
        __syncthreads();
        for (int i = threadIdx.x; i < n; i += kOrderThreads) {
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
        for (int i = threadIdx.x; i < n; i += kOrderThreads) {
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
        for (int i = threadIdx.x; i < n; i += kOrderThreads) emit_ranked(a, out[i], start + (uint32_t)i, vbase);
      }
    }
    __syncthreads();   // the list is rewritten by the next round
  }
}

__device__ void rank_buckets(const PassArgs& a, int blk, unsigned long long* keys, uint32_t* bs, uint32_t* vb) {
  const int nb = a.B * a.nbk;
  const int gb0 = blk * kRankBuckets;
  const int nbl = min(nb - gb0, kRankBuckets);
  if (threadIdx.x <= nbl) bs[threadIdx.x] = a.bkt_start[gb0 + threadIdx.x];
  if (threadIdx.x == 0) *vb = a.bkt_start[(gb0 / a.nbk) * a.nbk];
  __syncthreads();
  const uint32_t k0 = bs[0], nk = bs[nbl] - k0;
  const uint32_t cap = nk <= (uint32_t)kRankKeys ? kRankMax : kWaveMax;
  const uint32_t vbase = *vb;
  if (nk <= (uint32_t)kRankKeys) {
    for (uint32_t i = threadIdx.x; i < nk; i += kOrderThreads) keys[i] = a.bkeys[k0 + i];
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < nk; i += kOrderThreads) {
      // bucket of key i: the last j with bs[j] <= k0 + i
      int lo = 0, hi = nbl - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (bs[mid] <= k0 + i) lo = mid; else hi = mid - 1;
      }
      const uint32_t j0 = bs[lo] - k0, j1 = bs[lo + 1] - k0;
      if (j1 - j0 > cap) continue;
      const unsigned long long k = keys[i];
      uint32_t rank = 0;
      for (uint32_t j = j0; j < j1; ++j) rank += keys[j] < k ? 1u : 0u;
      emit_ranked(a, k, k0 + j0 + rank, vbase);
    }
    return;
  }
  const int lane = threadIdx.x & 63;
  for (int j = threadIdx.x >> 6; j < nbl; j += kOrderThreads / 64) {
    const uint32_t start = bs[j], n = bs[j + 1] - start;
    if (n == 0 || n > cap) continue;
    const unsigned long long key = (lane < (int)n) ? a.bkeys[start + lane] : ~0ull;
    const uint32_t hi = (uint32_t)(key >> 32), lo = (uint32_t)key;
    uint32_t rank = 0;
    for (uint32_t q = 0; q < n; ++q) {
      const uint32_t khi = (uint32_t)__builtin_amdgcn_readlane((int)hi, (int)q);
      const uint32_t klo = (uint32_t)__builtin_amdgcn_readlane((int)lo, (int)q);
      rank += (khi < hi || (khi == hi && klo < lo)) ? 1u : 0u;
    }
    if (lane < (int)n) emit_ranked(a, key, start + rank, vbase);
  }
}

// Workgroups [0, ns) sort the large buckets, the rest rank 32 buckets each.
__global__ __launch_bounds__(kOrderThreads) void bucket_order_kernel(PassArgs a, int ns) {
  __shared__ unsigned long long keys[kRankKeys];
  __shared__ uint32_t hist[kSortWaves * 256];
  __shared__ uint32_t lds_waves[kSortWaves];
  __shared__ uint32_t vary[2];
  __shared__ uint32_t list[kOrderThreads];
  __shared__ uint32_t nlist;
  __shared__ uint32_t bs[kRankBuckets + 1];
  __shared__ uint32_t vb;
  if ((int)blockIdx.x < ns) sort_large_buckets(a, (int)blockIdx.x, ns, keys, hist, lds_waves, vary, list, &nlist);
  else rank_buckets(a, (int)blockIdx.x - ns, keys, bs, &vb);
}

void launch_depth_order(const PassArgs& a, int64_t max_frame_splats, uint32_t* scan_scratch, const ScanJob& side,
                        hipStream_t s) {
  if (a.B == 0 || max_frame_splats == 0) {
    launch_scan_u32(side.in, side.out, side.n, side.block_sums, a.status, side.cap_check, side.total_out, s,
                    side.strided, side.stride);
    return;
  }
  const dim3 grid(a.nblk * kBucketParts, a.B);
  const int64_t nb = (int64_t)a.B * a.nbk;
  hipLaunchKernelGGL(bucket_count_kernel, grid, dim3(kBucketThreads), 0, s, a);
  // the scan also writes each bucket's start (its first workgroup's offset) to bkt_start
  const ScanJob buckets{a.bkt_count, a.bkt_moff, nb * a.nblk, scan_scratch, -1, nullptr, a.bkt_start, a.nblk};
  launch_scan_u32_pair(buckets, side, a.status, s);
  hipLaunchKernelGGL(bucket_scatter_kernel, grid, dim3(kBucketThreads), 0, s, a);
  const int ns = std::min(div_up(nb, kOrderThreads), 512);   // large-bucket workgroups: 256 buckets each at most
  hipLaunchKernelGGL(bucket_order_kernel, dim3(ns + div_up(nb, kRankBuckets)), dim3(kOrderThreads), 0, s, a, ns);
}

}  // namespace gbr
