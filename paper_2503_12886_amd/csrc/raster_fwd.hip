// Forward half of the batch-parallel rasterizer (Sec. 3.2): preprocess of
// every (frame, Gaussian), tile binning, per-tile depth order and front-to-back
// compositing, for all frames of a batch with no host synchronisation.
#include "gbr_internal.h"

namespace gbr {

// ---------------------------------------------------------------- fills
__global__ void fill_u32_kernel(uint32_t* p, uint32_t v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
__global__ void fill_f32_kernel(float* p, float v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
void launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)std::min<int64_t>(div_up(n, 256), 4096)), dim3(256), 0, s, p, v, n);
}
void launch_fill_f32(float* p, float v, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(fill_f32_kernel, dim3((unsigned)std::min<int64_t>(div_up(n, 256), 4096)), dim3(256), 0, s, p, v, n);
}

// ---------------------------------------------------------------- exclusive scan (u32)
// Three phases: per-block totals, a one-block scan of the totals (which also
// publishes the grand total and checks it against a capacity), per-block
// rescan with the block offset.  Integer sums, so the order does not matter
// for the result.
constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanBlock = kScanThreads * kScanItems;

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

__global__ __launch_bounds__(kScanThreads) void scan_totals_kernel(const uint32_t* __restrict__ in, int64_t n,
                                                                    uint32_t* __restrict__ block_sums) {
  __shared__ uint32_t lw[kScanThreads / 64];
  const int64_t base = (int64_t)blockIdx.x * kScanBlock;
  uint32_t s = 0;
  for (int i = 0; i < kScanItems; ++i) {
    const int64_t k = base + (int64_t)i * kScanThreads + threadIdx.x;
    if (k < n) s += in[k];
  }
  uint32_t tot;
  block_excl_scan<kScanThreads>(s, lw, &tot);
  if (threadIdx.x == 0) block_sums[blockIdx.x] = tot;
}

__global__ __launch_bounds__(1024) void scan_blocksums_kernel(uint32_t* __restrict__ block_sums, int nb,
                                                              StatusDev* status, int64_t cap_check,
                                                              unsigned long long* total_out) {
  __shared__ uint32_t lw[16];
  __shared__ unsigned long long carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int base = 0; base < nb; base += 1024) {
    const int k = base + threadIdx.x;
    const uint32_t v = (k < nb) ? block_sums[k] : 0u;
    uint32_t tot;
    const uint32_t ex = block_excl_scan<1024>(v, lw, &tot);
    const unsigned long long c = carry;
    if (k < nb) block_sums[k] = (uint32_t)(c + ex);
    __syncthreads();
    if (threadIdx.x == 0) carry = c + tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (total_out) *total_out = carry;
    if (cap_check >= 0 && carry > (unsigned long long)cap_check) status->overflow |= 1u;
  }
}

__global__ __launch_bounds__(kScanThreads) void scan_apply_kernel(const uint32_t* __restrict__ in, int64_t n,
                                                                   const uint32_t* __restrict__ block_sums,
                                                                   uint32_t* __restrict__ out) {
  __shared__ uint32_t tile[kScanBlock];
  __shared__ uint32_t lw[kScanThreads / 64];
  const int64_t base = (int64_t)blockIdx.x * kScanBlock;
  for (int i = 0; i < kScanItems; ++i) {
    const int idx = i * kScanThreads + threadIdx.x;
    const int64_t k = base + idx;
    tile[idx] = (k < n) ? in[k] : 0u;
  }
  __syncthreads();
  uint32_t local[kScanItems];
  uint32_t s = 0;
  for (int i = 0; i < kScanItems; ++i) {
    local[i] = tile[threadIdx.x * kScanItems + i];
    s += local[i];
  }
  uint32_t ex = block_excl_scan<kScanThreads>(s, lw, nullptr) + block_sums[blockIdx.x];
  for (int i = 0; i < kScanItems; ++i) {
    tile[threadIdx.x * kScanItems + i] = ex;
    ex += local[i];
  }
  __syncthreads();
  for (int i = 0; i < kScanItems; ++i) {
    const int idx = i * kScanThreads + threadIdx.x;
    const int64_t k = base + idx;
    if (k < n) out[k] = tile[idx];
  }
  // out[n] = grand total, written by the block that holds the last element
  if (threadIdx.x == kScanThreads - 1 && base <= n && n < base + kScanBlock) {
    out[n] = ex;  // ex of the last thread is the running total after its items
  }
}

int64_t scan_scratch_words(int64_t n) { return div_up(n + 1, kScanBlock) + 1; }

void launch_scan_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* block_sums, StatusDev* status,
                     int64_t cap_check, unsigned long long* total_out, hipStream_t s) {
  const int nb = div_up(n + 1, kScanBlock);
  hipLaunchKernelGGL(scan_totals_kernel, dim3(nb), dim3(kScanThreads), 0, s, in, n, block_sums);
  hipLaunchKernelGGL(scan_blocksums_kernel, dim3(1), dim3(1024), 0, s, block_sums, nb, status, cap_check, total_out);
  hipLaunchKernelGGL(scan_apply_kernel, dim3(nb), dim3(kScanThreads), 0, s, in, n, block_sums, out);
}

// ---------------------------------------------------------------- preprocess
// One thread per (frame, Gaussian).  Activations and EWA projection in
// float64 (so that the integer decisions -- which pixels and tiles a Gaussian
// may reach, and its binary32 depth key -- are exactly reproducible), the
// per-pixel record rounded to float32.  Each block also counts, in LDS, how
// many entries its Gaussians add to every tile of the frame, and flushes the
// non-zero counts with one global atomic each.
struct Projected {
  bool valid;
  double mx, my, A, Bq, C, o, tz;
  int x0, x1, y0, y1;
};

__device__ __forceinline__ void project_gaussian(const float* __restrict__ g, const FrameDev& F, Projected& p) {
  p.valid = false;
  const float4 v0 = reinterpret_cast<const float4*>(g)[0];
  const float4 v1 = reinterpret_cast<const float4*>(g)[1];
  const float4 v2 = reinterpret_cast<const float4*>(g)[2];
  const double mu0 = v0.x, mu1 = v0.y, mu2 = v0.z;
  const double tx = (double)F.R[0] * mu0 + (double)F.R[1] * mu1 + (double)F.R[2] * mu2 + (double)F.t[0];
  const double ty = (double)F.R[3] * mu0 + (double)F.R[4] * mu1 + (double)F.R[5] * mu2 + (double)F.t[1];
  const double tz = (double)F.R[6] * mu0 + (double)F.R[7] * mu1 + (double)F.R[8] * mu2 + (double)F.t[2];
  p.tz = tz;
  if (!(tz > (double)F.near_z)) return;
  double qw = v0.w, qx = v1.x, qy = v1.y, qz = v1.z;
  const double qinv = 1.0 / sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
  qw *= qinv; qx *= qinv; qy *= qinv; qz *= qinv;
  const double s0 = exp((double)v1.w), s1 = exp((double)v2.x), s2 = exp((double)v2.y);
  p.o = 1.0 / (1.0 + exp(-(double)v2.z));
  // rotation of the unit quaternion, columns scaled: M = R(q) diag(s)
  const double M00 = (1.0 - 2.0 * (qy * qy + qz * qz)) * s0, M01 = 2.0 * (qx * qy - qw * qz) * s1,
               M02 = 2.0 * (qx * qz + qw * qy) * s2;
  const double M10 = 2.0 * (qx * qy + qw * qz) * s0, M11 = (1.0 - 2.0 * (qx * qx + qz * qz)) * s1,
               M12 = 2.0 * (qy * qz - qw * qx) * s2;
  const double M20 = 2.0 * (qx * qz - qw * qy) * s0, M21 = 2.0 * (qy * qz + qw * qx) * s1,
               M22 = (1.0 - 2.0 * (qx * qx + qy * qy)) * s2;
  // W = J Rcam, the 2x3 local affine map of the perspective projection
  const double iz = 1.0 / tz;
  const double jx = (double)F.fx * iz, jy = (double)F.fy * iz;
  const double ux = -jx * tx * iz, uy = -jy * ty * iz;
  double W0[3], W1[3];
  for (int j = 0; j < 3; ++j) {
    W0[j] = jx * (double)F.R[j] + ux * (double)F.R[6 + j];
    W1[j] = jy * (double)F.R[3 + j] + uy * (double)F.R[6 + j];
  }
  // V = W M;  Sigma2 = V V^T + lowpass I
  const double V00 = W0[0] * M00 + W0[1] * M10 + W0[2] * M20;
  const double V01 = W0[0] * M01 + W0[1] * M11 + W0[2] * M21;
  const double V02 = W0[0] * M02 + W0[1] * M12 + W0[2] * M22;
  const double V10 = W1[0] * M00 + W1[1] * M10 + W1[2] * M20;
  const double V11 = W1[0] * M01 + W1[1] * M11 + W1[2] * M21;
  const double V12 = W1[0] * M02 + W1[1] * M12 + W1[2] * M22;
  const double sa = V00 * V00 + V01 * V01 + V02 * V02 + kLowPass;
  const double sb = V00 * V10 + V01 * V11 + V02 * V12;
  const double sc = V10 * V10 + V11 * V11 + V12 * V12 + kLowPass;
  p.mx = (double)F.fx * tx * iz + (double)F.cx;
  p.my = (double)F.fy * ty * iz + (double)F.cy;
  const double det = sa * sc - sb * sb;
  if (!(det > 0.0)) return;
  p.A = sc / det; p.Bq = -sb / det; p.C = sa / det;
  // alpha >= 1/255 needs q <= 2 ln(255 o); axis-aligned half extents of that ellipse
  const double thr = 2.0 * log(255.0 * p.o);
  if (!(thr >= 0.0)) return;
  const double ex = sqrt(thr * sa) + kBoxPad, ey = sqrt(thr * sc) + kBoxPad;
  double fx0 = ceil(p.mx - ex - 0.5), fx1 = floor(p.mx + ex - 0.5);
  double fy0 = ceil(p.my - ey - 0.5), fy1 = floor(p.my + ey - 0.5);
  fx0 = fmax(fx0, 0.0); fy0 = fmax(fy0, 0.0);
  fx1 = fmin(fx1, (double)(F.W - 1)); fy1 = fmin(fy1, (double)(F.H - 1));
  if (fx0 > fx1 || fy0 > fy1) return;
  p.x0 = (int)fx0; p.x1 = (int)fx1; p.y0 = (int)fy0; p.y1 = (int)fy1;
  p.valid = true;
}

__global__ __launch_bounds__(256) void preprocess_kernel(PassArgs a, const float* __restrict__ raw) {
  __shared__ uint32_t hist[kMaxFrameTilesLds];
  const int b = blockIdx.y;
  const FrameDev& F = a.frames[b];
  const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if ((int64_t)blockIdx.x * 256 >= F.gauss_count) return;   // uniform per block
  const bool lds = F.n_tiles <= kMaxFrameTilesLds;
  if (lds)
    for (int t = threadIdx.x; t < F.n_tiles; t += 256) hist[t] = 0u;
  __syncthreads();
  int4 r = make_int4(0, 0, -1, -1);
  if (n < F.gauss_count) {
    const int64_t s = F.gauss_base + n;
    Projected p;
    project_gaussian(raw + s * kNF, F, p);
    float* rec = a.rec + s * kRecF;
    uint32_t count = 0;
    if (p.valid) {
      const int T = a.tile;
      r = make_int4(p.x0 / T, p.y0 / T, p.x1 / T, p.y1 / T);
      count = (uint32_t)((r.z - r.x + 1) * (r.w - r.y + 1));
      const float4 r0 = make_float4((float)p.mx, (float)p.my, (float)(-0.5 * kLog2e * p.A), (float)(-kLog2e * p.Bq));
      const float4 r1 = make_float4((float)(-0.5 * kLog2e * p.C), (float)p.o, raw[s * kNF + 11], raw[s * kNF + 12]);
      const float4 r2 = make_float4(raw[s * kNF + 13], (float)p.tz, 0.0f, 0.0f);
      reinterpret_cast<float4*>(rec)[0] = r0;
      reinterpret_cast<float4*>(rec)[1] = r1;
      reinterpret_cast<float4*>(rec)[2] = r2;
    } else {
      reinterpret_cast<float4*>(rec)[2] = make_float4(0.0f, (float)p.tz, 0.0f, 0.0f);
    }
    a.rect[s] = r;
    a.cnt[s] = count;
  }
  for (int ty = r.y; ty <= r.w; ++ty)
    for (int tx = r.x; tx <= r.z; ++tx) {
      const int t = ty * F.ntx + tx;
      if (lds) atomicAdd(&hist[t], 1u);
      else atomicAdd(&a.tile_count[F.tile_base + t], 1u);
    }
  __syncthreads();
  if (lds)
    for (int t = threadIdx.x; t < F.n_tiles; t += 256) {
      const uint32_t c = hist[t];
      if (c) atomicAdd(&a.tile_count[F.tile_base + t], c);
    }
}

void launch_preprocess(const PassArgs& a, const float* raw, int64_t max_frame_splats, hipStream_t s) {
  if (a.B == 0 || max_frame_splats == 0) return;
  hipLaunchKernelGGL(preprocess_kernel, dim3(div_up(max_frame_splats, 256), a.B), dim3(256), 0, s, a, raw);
}

// ---------------------------------------------------------------- scatter
// Each block reserves, per tile, one contiguous range of slots for all its
// Gaussians' entries (one global atomic per tile and block), then hands out
// slots inside the range with LDS atomics.  The order inside a tile is
// arbitrary here; the per-tile sort that follows makes it unique.
__global__ __launch_bounds__(256) void scatter_kernel(PassArgs a) {
  __shared__ uint32_t hist[kMaxFrameTilesLds];
  if (a.status->overflow) return;
  const int b = blockIdx.y;
  const FrameDev& F = a.frames[b];
  const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if ((int64_t)blockIdx.x * 256 >= F.gauss_count) return;
  const bool lds = F.n_tiles <= kMaxFrameTilesLds;
  if (lds)
    for (int t = threadIdx.x; t < F.n_tiles; t += 256) hist[t] = 0u;
  __syncthreads();
  int4 r = make_int4(0, 0, -1, -1);
  int64_t s = F.gauss_base + n;
  unsigned long long key_hi = 0;
  if (n < F.gauss_count && a.cnt[s] > 0) {
    r = a.rect[s];
    key_hi = (unsigned long long)__float_as_uint(a.rec[s * kRecF + 9]) << 32;
  }
  if (lds) {
    for (int ty = r.y; ty <= r.w; ++ty)
      for (int tx = r.x; tx <= r.z; ++tx) atomicAdd(&hist[ty * F.ntx + tx], 1u);
    __syncthreads();
    for (int t = threadIdx.x; t < F.n_tiles; t += 256) {
      const uint32_t c = hist[t];
      if (c) hist[t] = atomicAdd(&a.tile_cursor[F.tile_base + t], c);
    }
    __syncthreads();
  }
  const unsigned long long key = key_hi | (unsigned long long)(uint32_t)s;
  for (int ty = r.y; ty <= r.w; ++ty)
    for (int tx = r.x; tx <= r.z; ++tx) {
      const int t = ty * F.ntx + tx;
      const uint32_t slot = lds ? atomicAdd(&hist[t], 1u) : atomicAdd(&a.tile_cursor[F.tile_base + t], 1u);
      a.keys[(uint64_t)a.tile_start[F.tile_base + t] + slot] = key;
    }
}

void launch_scatter(const PassArgs& a, int64_t max_frame_splats, hipStream_t s) {
  if (a.B == 0 || max_frame_splats == 0) return;
  hipLaunchKernelGGL(scatter_kernel, dim3(div_up(max_frame_splats, 256), a.B), dim3(256), 0, s, a);
}

// ---------------------------------------------------------------- per-tile sort
// Stable LSD radix sort of a tile's 64-bit keys (binary32 depth bits << 32 |
// splat index) with 8-bit digits, skipping digits on which all keys agree.
// 8 waves; wave w owns a contiguous segment of the keys, so (wave, step,
// lane) order is key order and the ranking below is stable.  Lists of up to
// kSortCap keys live in LDS; longer ones ping-pong through global memory.
constexpr int kSortThreads = 512;
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

__global__ __launch_bounds__(kSortThreads) void tile_sort_kernel(PassArgs a) {
  extern __shared__ unsigned long long smem_keys[];
  unsigned long long* bufA = smem_keys;
  unsigned long long* bufB = smem_keys + kSortCap;
  uint32_t* hist = reinterpret_cast<uint32_t*>(smem_keys + 2 * kSortCap);
  uint32_t* lds_waves = hist + kSortWaves * 256;
  uint32_t* vary = lds_waves + kSortWaves;
  if (a.status->overflow) return;
  const int g = blockIdx.x;
  const uint32_t start = a.tile_start[g];
  const int n = (int)(a.tile_start[g + 1] - start);
  if (n == 0) return;
  unsigned long long* gkeys = a.keys + start;
  unsigned long long* galt = a.keys_alt + start;
  const bool in_lds = n <= kSortCap;
  if (threadIdx.x < 2) vary[threadIdx.x] = 0u;
  __syncthreads();
  const unsigned long long k0 = gkeys[0];
  uint32_t vlo = 0, vhi = 0;
  for (int i = threadIdx.x; i < n; i += kSortThreads) {
    const unsigned long long k = gkeys[i];
    if (in_lds) bufA[i] = k;
    const unsigned long long x = k ^ k0;
    vlo |= (uint32_t)x; vhi |= (uint32_t)(x >> 32);
  }
  if (vlo) atomicOr(&vary[0], vlo);
  if (vhi) atomicOr(&vary[1], vhi);
  __syncthreads();
  const unsigned long long varying = ((unsigned long long)vary[1] << 32) | vary[0];
  int parity = 0;   // 0: data in A (or gkeys), 1: in B (or galt)
  for (int shift = 0; shift < 64; shift += 8) {
    if (((varying >> shift) & 255ull) == 0) continue;
    if (in_lds) {
      if (parity == 0) radix_pass(bufA, bufB, n, shift, hist, lds_waves);
      else radix_pass(bufB, bufA, n, shift, hist, lds_waves);
    } else {
      if (parity == 0) radix_pass(gkeys, galt, n, shift, hist, lds_waves);
      else radix_pass(galt, gkeys, n, shift, hist, lds_waves);
    }
    parity ^= 1;
  }
  const unsigned long long* out = in_lds ? (parity ? bufB : bufA) : (parity ? galt : gkeys);
  // sorted splat indices, and the map from each entry's emission slot
  // (splat's emission offset + row-major index of the tile in its rect) to
  // its sorted position
  const int b = frame_of_tile(a.frames, a.B, g);
  const FrameDev& F = a.frames[b];
  const int lt = g - F.tile_base;
  const int tx = lt % F.ntx, ty = lt / F.ntx;
  for (int i = threadIdx.x; i < n; i += kSortThreads) {
    const uint32_t s = (uint32_t)out[i];
    a.sorted[start + i] = s;
    const int4 r = a.rect[s];
    const uint32_t j = (uint32_t)((ty - r.y) * (r.z - r.x + 1) + (tx - r.x));
    a.pos[a.soff[s] + j] = start + i;
  }
}

void launch_tile_sort(const PassArgs& a, hipStream_t s) {
  if (a.n_tiles == 0) return;
  const size_t lds = 2 * kSortCap * sizeof(unsigned long long) + (kSortWaves * 256 + kSortWaves + 2) * sizeof(uint32_t);
  static bool attr_set = false;   // more than 64 KB of dynamic LDS must be requested explicitly
  if (!attr_set) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(tile_sort_kernel),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    attr_set = true;
  }
  hipLaunchKernelGGL(tile_sort_kernel, dim3(a.n_tiles), dim3(kSortThreads), lds, s, a);
}

// ---------------------------------------------------------------- compositing
// One workgroup per tile.  T = 8: 64 threads, one pixel each; T = 16: 256
// threads, one pixel each; T = 32: 256 threads, a 2x2 pixel block each.
// CHUNK sorted entries at a time are staged in LDS and read by every thread
// (broadcast); the tile stops when all its pixels have stopped.
template <int T> struct TileShape {
  static constexpr int NT = (T == 8) ? 64 : 256;
  static constexpr int PXW = (T == 32) ? 2 : 1;     // pixels per thread along x and y
  static constexpr int PX = PXW * PXW;
  static constexpr int TPR = T / PXW;               // threads per pixel row
  static constexpr int NW = NT / 64;
};

// alpha of a splat at a pixel, bit-identical wherever it is evaluated:
// power = ca dx^2 + cb dx dy + cc dy^2 (= -q/2 in log2 units), alpha = o 2^power.
__device__ __forceinline__ float splat_alpha(float4 r0, float4 r1, float px, float py, float& dx, float& dy,
                                             float& pw_raw, float& g2) {
#pragma clang fp contract(off)
  dx = px - r0.x;
  dy = py - r0.y;
  float pw = (r0.z * dx) * dx;
  pw = __builtin_fmaf(r0.w * dx, dy, pw);
  pw = __builtin_fmaf(r1.x * dy, dy, pw);
  pw_raw = pw;
  pw = fminf(pw, 0.0f);
  g2 = __builtin_amdgcn_exp2f(pw);
  return r1.y * g2;
}

template <int T, int CHUNK>
__global__ __launch_bounds__(TileShape<T>::NT) void composite_fwd_kernel(PassArgs a, float* __restrict__ images) {
  using S = TileShape<T>;
  __shared__ float4 s0[CHUNK];
  __shared__ float4 s1[CHUNK];
  __shared__ float s2[CHUNK];
  __shared__ uint32_t s_last;
  if (a.status->overflow) return;
  const int g = blockIdx.x;
  const int b = frame_of_tile(a.frames, a.B, g);
  const FrameDev& F = a.frames[b];
  const int lt = g - F.tile_base;
  const int tx = lt % F.ntx, ty = lt / F.ntx;
  const uint32_t start = a.tile_start[g], end = a.tile_start[g + 1];
  const int lx0 = (threadIdx.x % S::TPR) * S::PXW, ly0 = (threadIdx.x / S::TPR) * S::PXW;
  float T_[S::PX], C0[S::PX], C1[S::PX], C2[S::PX];
  uint32_t last[S::PX];
  bool done[S::PX];
  int pxi[S::PX], pyi[S::PX];
#pragma unroll
  for (int p = 0; p < S::PX; ++p) {
    pxi[p] = tx * T + lx0 + (p % S::PXW);
    pyi[p] = ty * T + ly0 + (p / S::PXW);
    T_[p] = 1.0f; C0[p] = C1[p] = C2[p] = 0.0f; last[p] = 0;
    done[p] = !(pxi[p] < F.W && pyi[p] < F.H);
  }
  if (threadIdx.x == 0) s_last = 0;
  for (uint32_t cb = start; cb < end; cb += CHUNK) {
    const int n = (int)min((uint32_t)CHUNK, end - cb);
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += S::NT) {
      const float4* rec = reinterpret_cast<const float4*>(a.rec + (int64_t)a.sorted[cb + i] * kRecF);
      s0[i] = rec[0]; s1[i] = rec[1]; s2[i] = rec[2].x;
    }
    __syncthreads();
    bool all_done = true;
#pragma unroll
    for (int p = 0; p < S::PX; ++p) all_done &= done[p];
    if (!all_done) {
      for (int i = 0; i < n; ++i) {
        const float4 r0 = s0[i], r1 = s1[i];
#pragma unroll
        for (int p = 0; p < S::PX; ++p) {
          if (done[p]) continue;
          float dx, dy, pwr, g2;
          const float al0 = splat_alpha(r0, r1, (float)pxi[p] + 0.5f, (float)pyi[p] + 0.5f, dx, dy, pwr, g2);
          if (al0 < kAlphaMin) continue;
          const float al = fminf(al0, kAlphaMax);
          const float tn = T_[p] * (1.0f - al);
          if (tn < kTMin) { done[p] = true; continue; }
          const float w = al * T_[p];
          C0[p] = __builtin_fmaf(w, r1.z, C0[p]);
          C1[p] = __builtin_fmaf(w, r1.w, C1[p]);
          C2[p] = __builtin_fmaf(w, s2[i], C2[p]);
          T_[p] = tn;
          last[p] = cb - start + i + 1;
        }
      }
    }
    bool mine = false;
#pragma unroll
    for (int p = 0; p < S::PX; ++p) mine |= !done[p];
    if (__syncthreads_count(mine) == 0) break;
  }
  uint32_t my_last = 0;
#pragma unroll
  for (int p = 0; p < S::PX; ++p) {
    if (pxi[p] < F.W && pyi[p] < F.H) {
      const int64_t pix = (int64_t)pyi[p] * F.W + pxi[p];
      const int64_t hw = (int64_t)F.W * F.H;
      float* img = images + F.pix_base * 3;
      img[pix] = C0[p] + T_[p] * F.bg[0];
      img[hw + pix] = C1[p] + T_[p] * F.bg[1];
      img[2 * hw + pix] = C2[p] + T_[p] * F.bg[2];
      a.n_iter[F.pix_base + pix] = last[p];
      a.t_final[F.pix_base + pix] = T_[p];
      my_last = max(my_last, last[p]);
    }
  }
  __syncthreads();
  if (my_last) atomicMax(&s_last, my_last);
  __syncthreads();
  if (threadIdx.x == 0) a.tile_last[g] = s_last;
}

void launch_composite_fwd(const PassArgs& a, float* images, int chunk, hipStream_t s) {
  if (a.n_tiles == 0) return;
  const dim3 grid(a.n_tiles);
#define GBR_FWD(TT, CC) \
  hipLaunchKernelGGL((composite_fwd_kernel<TT, CC>), grid, dim3(TileShape<TT>::NT), 0, s, a, images)
#define GBR_FWD_T(TT)                      \
  if (chunk == 64) GBR_FWD(TT, 64);        \
  else if (chunk == 128) GBR_FWD(TT, 128); \
  else GBR_FWD(TT, 256);
  if (a.tile == 8) { GBR_FWD_T(8) }
  else if (a.tile == 16) { GBR_FWD_T(16) }
  else { GBR_FWD_T(32) }
#undef GBR_FWD_T
#undef GBR_FWD
}

}  // namespace gbr
