// Forward half of the batch-parallel rasterizer (Sec. 3.2): preprocess of
// every (frame, Gaussian), tile binning, per-tile depth order and front-to-back
// compositing, for all frames of a batch with no host synchronisation.
#include "gbr_device.h"
#include "tangent_ops.h"

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
// out[k] = sum of in[0..k), out[n] = the grand total.  Two passes:
// per-block totals, then every block adds the totals of the blocks before it
// (read directly, summed in 64 bits) to its own rescan.  The grand total is
// published (and checked against a capacity) by the workgroup that writes
// out[n].  Integer sums, so the order does not matter for the result.  One
// launch pair can carry two independent scans: the first job's blocks come
// first in the grid, then the second's.
constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanBlock = kScanThreads * kScanItems;

struct ScanJobs {
  ScanJob j0, j1;
  int nb0;   // blocks of the first job
};

// The job of this workgroup (chosen field by field, uniformly) and its block index within it.
__device__ __forceinline__ ScanJob scan_job(const ScanJobs& J, int* blk) {
  const bool second = (int)blockIdx.x >= J.nb0;
  *blk = (int)blockIdx.x - (second ? J.nb0 : 0);
  ScanJob j;
  j.in = second ? J.j1.in : J.j0.in;
  j.out = second ? J.j1.out : J.j0.out;
  j.n = second ? J.j1.n : J.j0.n;
  j.block_sums = second ? J.j1.block_sums : J.j0.block_sums;
  j.cap_check = second ? J.j1.cap_check : J.j0.cap_check;
  j.total_out = second ? J.j1.total_out : J.j0.total_out;
  j.strided = second ? J.j1.strided : J.j0.strided;
  j.stride = second ? J.j1.stride : J.j0.stride;
  return j;
}

__device__ __forceinline__ void publish_total(unsigned long long total, StatusDev* status, int64_t cap_check,
                                              unsigned long long* total_out) {
  if (total_out) *total_out = total;
  if (cap_check >= 0 && total > (unsigned long long)cap_check) status->overflow |= 1u;
}

__device__ __forceinline__ void scan_totals_block(const ScanJob& J, int blk, uint32_t* lw) {
  const uint32_t* __restrict__ in = J.in;
  const int64_t n = J.n;
  const int64_t base = (int64_t)blk * kScanBlock;
  // loads issued unconditionally (index clamped into range), then masked
  uint32_t v[kScanItems];
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    const int64_t k = base + (int64_t)i * kScanThreads + threadIdx.x;
    v[i] = (n > 0) ? in[min(k, n - 1)] : 0u;
  }
  uint32_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) s += (base + (int64_t)i * kScanThreads + threadIdx.x < n) ? v[i] : 0u;
  uint32_t tot;
  block_excl_scan<kScanThreads>(s, lw, &tot);
  if (threadIdx.x == 0) J.block_sums[blk] = tot;
}

__global__ __launch_bounds__(kScanThreads) void scan_totals_kernel(ScanJobs jobs) {
  __shared__ uint32_t lw[kScanThreads / 64];
  int blk;
  const ScanJob J = scan_job(jobs, &blk);
  scan_totals_block(J, blk, lw);
}

__global__ __launch_bounds__(kScanThreads) void scan_apply_kernel(ScanJobs jobs, StatusDev* status) {
  __shared__ uint32_t tile[kScanBlock];
  __shared__ uint32_t lw[kScanThreads / 64];
  __shared__ unsigned long long wsum[kScanThreads / 64];
  int blk;
  const ScanJob J = scan_job(jobs, &blk);
  const uint32_t* __restrict__ in = J.in;
  const uint32_t* __restrict__ block_sums = J.block_sums;
  uint32_t* __restrict__ out = J.out;
  uint32_t* __restrict__ strided = J.strided;
  const int64_t n = J.n;
  const int stride = J.stride;
  const int64_t base = (int64_t)blk * kScanBlock;
  uint32_t v[kScanItems];
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) v[i] = (n > 0) ? in[min(base + i * kScanThreads + threadIdx.x, n - 1)] : 0u;
  // this block's offset: the totals of the blocks before it
  unsigned long long part = 0;
  for (int k = threadIdx.x; k < blk; k += kScanThreads) part += block_sums[k];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o, 64);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = part;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    const int idx = i * kScanThreads + threadIdx.x;
    tile[idx] = (base + idx < n) ? v[i] : 0u;
  }
  __syncthreads();
  unsigned long long off = 0;
#pragma unroll
  for (int w = 0; w < kScanThreads / 64; ++w) off += wsum[w];
  uint32_t local[kScanItems];
  uint32_t s = 0;
  for (int i = 0; i < kScanItems; ++i) {
    local[i] = tile[threadIdx.x * kScanItems + i];
    s += local[i];
  }
  uint32_t ex = block_excl_scan<kScanThreads>(s, lw, nullptr);
  for (int i = 0; i < kScanItems; ++i) {
    tile[threadIdx.x * kScanItems + i] = ex;
    ex += local[i];
  }
  __syncthreads();
  for (int i = 0; i < kScanItems; ++i) {
    const int idx = i * kScanThreads + threadIdx.x;
    const int64_t k = base + idx;
    if (k < n) {
      const uint32_t val = (uint32_t)(off + tile[idx]);
      out[k] = val;
      if (strided && (uint32_t)k % (uint32_t)stride == 0u) strided[(uint32_t)k / (uint32_t)stride] = val;
    }
  }
  // out[n] = grand total, written by the block that holds position n
  if (threadIdx.x == kScanThreads - 1 && base <= n && n < base + kScanBlock) {
    const unsigned long long total = off + ex;   // ex of the last thread: the block's running total
    out[n] = (uint32_t)total;
    if (strided && (uint32_t)n % (uint32_t)stride == 0u) strided[(uint32_t)n / (uint32_t)stride] = (uint32_t)total;
    publish_total(total, status, J.cap_check, J.total_out);
  }
}

int64_t scan_scratch_words(int64_t n) { return div_up(n + 1, kScanBlock) + 1; }

void launch_scan_u32_pair(const ScanJob& j0, const ScanJob& j1, StatusDev* status, hipStream_t s) {
  ScanJobs J;
  J.j0 = j0;
  J.j1 = j1;
  J.j0.stride = j0.stride < 1 ? 1 : j0.stride;
  J.j1.stride = j1.stride < 1 ? 1 : j1.stride;
  J.nb0 = (int)div_up(j0.n + 1, kScanBlock);
  const int nb = J.nb0 + (j1.in ? (int)div_up(j1.n + 1, kScanBlock) : 0);
  hipLaunchKernelGGL(scan_totals_kernel, dim3(nb), dim3(kScanThreads), 0, s, J);
  hipLaunchKernelGGL(scan_apply_kernel, dim3(nb), dim3(kScanThreads), 0, s, J, status);
}

void launch_scan_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* block_sums, StatusDev* status,
                     int64_t cap_check, unsigned long long* total_out, hipStream_t s, uint32_t* strided,
                     int stride) {
  const ScanJob j0{in, out, n, block_sums, cap_check, total_out, strided, stride};
  const ScanJob none{nullptr, nullptr, 0, nullptr, -1, nullptr, nullptr, 1};
  launch_scan_u32_pair(j0, none, status, s);
}

// ---------------------------------------------------------------- preprocess
// One thread per (frame, Gaussian).  Activations and EWA projection in
// float64 (so that the integer decisions -- which pixels and tiles a Gaussian
// may reach, and its binary32 depth key -- are exactly reproducible), the
// per-pixel record rounded to float32.  Each block also reduces its splats'
// depth keys to a minimum and maximum, stored in the block's own slot (the
// depth passes take the frame's range, which scales the depth buckets, from
// those slots).  The pass's first kernel, it also clears the pass's counters
// (tile-class counts, overflow flag) in block (0, 0).
struct Projected {
  bool valid;
  double mx, my, A, Bq, C, o, tz;
  int x0, x1, y0, y1;
};

// v0, v1, v2: the first three float4 of a blended record (position,
// quaternion, log-scales, opacity logit, red).
__device__ __forceinline__ void project_gaussian(const float4 v0, const float4 v1, const float4 v2, const FrameDev& F,
                                                 Projected& p) {
  p.valid = false;
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

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = min(v, (uint32_t)__shfl_xor((int)v, o, 64));
  return v;
}
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, o, 64));
  return v;
}

__global__ __launch_bounds__(256) void preprocess_kernel(PassArgs a, const float* __restrict__ raw) {
  __shared__ uint32_t wmin[4], wmax[4];
  const int b = blockIdx.y;
  const FrameDev& F = a.frames[b];
  const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (blockIdx.x == 0 && b == 0) {   // the pass's counters: this is its first kernel
    if (threadIdx.x < 66) a.cls_cnt[threadIdx.x] = 0u;
    if (threadIdx.x == 0) { a.status->overflow = 0u; a.status->entries = 0ull; }
  }
  if ((int64_t)blockIdx.x * 256 >= F.gauss_count) return;   // uniform per block
  const int tsh = __ffs(a.tile) - 1;                         // tile is a power of two
  uint32_t dmin = 0xffffffffu, dmax = 0u;
  if (n < F.gauss_count) {
    const int64_t s = F.gauss_base + n;
    const float4* src = reinterpret_cast<const float4*>(raw + s * kNF);
    float4 v0 = src[0], v1 = src[1];
    const float4 col = src[2];              // log-scales 1-2, opacity logit, red
    const float4 col2 = src[3];             // green, blue
    if (a.tg.on) tangent_deform(a.tg, b, n, v0, v1, v0, v1);   // tangent space -> frame b's mesh
    Projected p;
    project_gaussian(v0, v1, col, F, p);
    float* rec = a.rec + s * kRecF;
    int4 r = make_int4(0, 0, -1, -1);
    uint32_t count = 0, key = 0xffffffffu;
    if (p.valid) {
      r = make_int4(p.x0 >> tsh, p.y0 >> tsh, p.x1 >> tsh, p.y1 >> tsh);
      count = (uint32_t)((r.z - r.x + 1) * (r.w - r.y + 1));
      const float4 r0 = make_float4((float)p.mx, (float)p.my, (float)(-0.5 * kLog2e * p.A), (float)(-kLog2e * p.Bq));
      const float4 r1 = make_float4((float)(-0.5 * kLog2e * p.C), (float)log2(p.o), col.w, col2.x);
      const float4 r2 = make_float4(col2.y, (float)p.tz,
                                    __uint_as_float((uint32_t)p.x0 | ((uint32_t)p.x1 << 16)),
                                    __uint_as_float((uint32_t)p.y0 | ((uint32_t)p.y1 << 16)));
      reinterpret_cast<float4*>(rec)[0] = r0;
      reinterpret_cast<float4*>(rec)[1] = r1;
      reinterpret_cast<float4*>(rec)[2] = r2;
      key = __float_as_uint(r2.y);
      dmin = key; dmax = key;
    } else {
      reinterpret_cast<float4*>(rec)[2] = make_float4(0.0f, (float)p.tz, 0.0f, 0.0f);
    }
    a.rect[s] = r;
    a.cnt[s] = count;
    a.dkey[s] = key;
  }
  // the block's depth range (wave reductions), stored in its own slot: the
  // depth passes reduce the frame's slots, so nothing is cleared or merged
  dmin = wave_min_u32(dmin);
  dmax = wave_max_u32(dmax);
  if ((threadIdx.x & 63) == 0) { wmin[threadIdx.x >> 6] = dmin; wmax[threadIdx.x >> 6] = dmax; }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t* mm = a.blk_mm + 2 * (F.gauss_base / 256 + b + blockIdx.x);
    mm[0] = min(min(wmin[0], wmin[1]), min(wmin[2], wmin[3]));
    mm[1] = max(max(wmax[0], wmax[1]), max(wmax[2], wmax[3]));
  }
}

bool launch_preprocess(const PassArgs& a, const float* raw, int64_t max_frame_splats, hipStream_t s) {
  if (a.B == 0 || max_frame_splats == 0) return false;
  hipLaunchKernelGGL(preprocess_kernel, dim3(div_up(max_frame_splats, 256), a.B), dim3(256), 0, s, a, raw);
  return true;
}

// ---------------------------------------------------------------- binning
// A tile's list is the set of frame-local depth ranks of the splats that
// overlap it.  Each tile owns a row of bitmap_words words (bit r = rank r);
// reading a row's set bits in ascending order gives the tile's list in depth
// order, so no entry array is scattered or sorted.  Rows are cut into
// segments of seg_words words, and the set bits of every segment are counted
// once (seg_cnt): the tile's entry count is their sum, and the compositing
// places each segment in the tile's order from those counts alone, reading
// only the segments it consumes.
//
// Rows are built by rank: workgroup j of a frame takes the splats of ranks
// [32 SW j, 32 SW (j + 1)), which own segment j (words [SW j, SW (j + 1)))
// of every row.  Each splat ORs its bit into an LDS copy of those SW words
// for every tile of its rect; the workgroup then stores the bit count of
// every tile's segment and the segments that have set bits.  Every count is
// written by exactly one workgroup, and a segment whose count is zero is
// never read (its words keep whatever an earlier pass left there), so
// nothing needs clearing and rows of empty tiles cost no stores.
// In LDS a tile's segment takes SW + 1 words: the lanes of a half-wave OR
// into the same word offset of their (scattered) tiles, and with a stride of
// SW words those tiles would share a couple of banks; an odd stride spreads
// them over all of them.  Frames with more tiles than the LDS copy holds set
// the bits in memory with atomics after clearing the rows, and count the
// segments in a second pass.
constexpr int kRowBuildWords = 2048 * 9;     // LDS words (72 KB): 2048 tiles at SW = 8, 1084 at SW = 16

int bitmap_seg_words(int max_frame_tiles, int64_t row_words) {
  int sw = (int64_t)max_frame_tiles * 17 <= kRowBuildWords ? 16 : 8;
  while (row_words / sw > kMaxRowSegs) sw *= 2;
  return sw;
}

template <int SW>
__global__ __launch_bounds__(32 * SW) void bitmap_rows_kernel(PassArgs a) {
  constexpr int NT = 32 * SW;                 // one thread per rank of the segment
  constexpr int ST = SW + 1;                  // LDS words per tile
  __shared__ __align__(16) uint32_t words[kRowBuildWords];
  const int b = blockIdx.y;
  const FrameDev& F = a.frames[b];
  const uint32_t vbase = a.bkt_start[b * a.nbk];
  const uint32_t nv = a.bkt_start[(b + 1) * a.nbk] - vbase;
  const uint32_t r0 = blockIdx.x * (uint32_t)NT;
  if (r0 >= nv || a.status->overflow) return;
  const int nw4 = F.n_tiles * (SW / 4);
  const int nz4 = (F.n_tiles * ST + 3) / 4;   // <= kRowBuildWords / 4 (a multiple of 4 words)
  uint4* w4 = reinterpret_cast<uint4*>(words);
  for (int q = threadIdx.x; q < nz4; q += NT) w4[q] = make_uint4(0u, 0u, 0u, 0u);
  __syncthreads();
  const uint32_t r = r0 + threadIdx.x;
  if (r < nv) {
    const uint32_t s = a.depth_sorted[vbase + r];
    const int4 rc = a.rect[s];
    const uint32_t bit = 1u << (r & 31u);
    const int wl = (int)((r >> 5) & (SW - 1));
    for (int ty = rc.y; ty <= rc.w; ++ty)
      for (int tx = rc.x; tx <= rc.z; ++tx) atomicOr(&words[(ty * F.ntx + tx) * ST + wl], bit);
  }
  __syncthreads();
  // every tile's bit count, also kept in its segment's pad word
  const int seg = (int)blockIdx.x;
  uint16_t* cnt = a.seg_cnt + (int64_t)F.tile_base * a.seg_stride + seg;
  for (int t = threadIdx.x; t < F.n_tiles; t += NT) {
    uint32_t c = 0;
#pragma unroll
    for (int k = 0; k < SW; ++k) c += __popc(words[t * ST + k]);
    cnt[(int64_t)t * a.seg_stride] = (uint16_t)c;
    words[t * ST + SW] = c;
  }
  __syncthreads();
  // the segments with set bits (16-byte stores; rows and segments are 64-byte aligned)
  uint32_t* rows = a.tbits + (int64_t)F.tile_base * a.bitmap_words + (int64_t)seg * SW;
  for (int q = threadIdx.x; q < nw4; q += NT) {
    const int t = q / (SW / 4), k = q % (SW / 4);
    const uint32_t* src = words + t * ST + 4 * k;
    if (words[t * ST + SW] == 0u) continue;
    reinterpret_cast<uint4*>(rows + (int64_t)t * a.bitmap_words)[k] = make_uint4(src[0], src[1], src[2], src[3]);
  }
}

__global__ __launch_bounds__(256) void bitmap_rows_atomic_kernel(PassArgs a) {
  const int b = blockIdx.y;
  const FrameDev& F = a.frames[b];
  const uint32_t vbase = a.bkt_start[b * a.nbk];
  const uint32_t nv = a.bkt_start[(b + 1) * a.nbk] - vbase;
  const uint32_t r = blockIdx.x * 256u + threadIdx.x;
  if (r >= nv || a.status->overflow) return;
  const uint32_t s = a.depth_sorted[vbase + r];
  const int4 rc = a.rect[s];
  const uint32_t bit = 1u << (r & 31u);
  uint32_t* base = a.tbits + (int64_t)F.tile_base * a.bitmap_words + (r >> 5);
  for (int ty = rc.y; ty <= rc.w; ++ty)
    for (int tx = rc.x; tx <= rc.z; ++tx) atomicOr(base + (int64_t)(ty * F.ntx + tx) * a.bitmap_words, bit);
}

// Bit counts of the segments of rows set in memory: a thread per (tile, segment).
__global__ __launch_bounds__(256) void seg_count_kernel(PassArgs a) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= (int64_t)a.n_tiles * a.seg_stride || a.status->overflow) return;
  const int64_t g = i / a.seg_stride;
  const int sg = (int)(i % a.seg_stride);
  const uint4* src = reinterpret_cast<const uint4*>(a.tbits + g * a.bitmap_words + (int64_t)sg * a.seg_words);
  uint32_t c = 0;
  for (int k = 0; k < a.seg_words / 4; ++k) {
    const uint4 v = src[k];
    c += __popc(v.x) + __popc(v.y) + __popc(v.z) + __popc(v.w);
  }
  a.seg_cnt[i] = (uint16_t)c;
}

void launch_bitmap_rows(const PassArgs& a, int64_t max_frame_splats, int max_frame_tiles, hipStream_t s) {
  if (a.B == 0 || max_frame_splats == 0) return;
  const bool in_lds = (int64_t)max_frame_tiles * (a.seg_words + 1) <= kRowBuildWords;
  if (in_lds && a.seg_words == 32) {
    hipLaunchKernelGGL(bitmap_rows_kernel<32>, dim3(div_up(max_frame_splats, 1024), a.B), dim3(1024), 0, s, a);
  } else if (in_lds && a.seg_words == 16) {
    hipLaunchKernelGGL(bitmap_rows_kernel<16>, dim3(div_up(max_frame_splats, 512), a.B), dim3(512), 0, s, a);
  } else if (in_lds && a.seg_words == 8) {
    hipLaunchKernelGGL(bitmap_rows_kernel<8>, dim3(div_up(max_frame_splats, 256), a.B), dim3(256), 0, s, a);
  } else {
    launch_fill_u32(a.tbits, 0u, (int64_t)a.n_tiles * a.bitmap_words, s);
    hipLaunchKernelGGL(bitmap_rows_atomic_kernel, dim3(div_up(max_frame_splats, 256), a.B), dim3(256), 0, s, a);
    hipLaunchKernelGGL(seg_count_kernel, dim3(div_up((int64_t)a.n_tiles * a.seg_stride, 256)), dim3(256), 0, s, a);
  }
}

// A tile's entry count is the sum of its row's segment counts: one wave per
// tile, lanes over the segments.  The first 128 counts are read (clamped to
// the row) before the frame's segment count is known, which only masks
// them, so that their loads overlap the frame lookup.
__global__ __launch_bounds__(256) void tile_count_kernel(PassArgs a) {
  // (the wave's tile, declared uniform so that the frame lookup runs on scalar loads)
  const int g = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
  if (g >= a.n_tiles) return;
  const int lane = threadIdx.x & 63;
  const uint16_t* sc = a.seg_cnt + (int64_t)g * a.seg_stride;
  const uint32_t last = (uint32_t)a.seg_stride - 1u;
  const uint32_t v0 = sc[min((uint32_t)lane, last)], v1 = sc[min((uint32_t)lane + 64u, last)];
  const int b = frame_of_tile(a.frames, a.B, g);
  const uint32_t nv = a.bkt_start[(b + 1) * a.nbk] - a.bkt_start[b * a.nbk];
  const uint32_t nseg = ((nv + 31) / 32 + a.seg_words - 1) / a.seg_words;
  uint32_t c = ((uint32_t)lane < nseg ? v0 : 0u) + ((uint32_t)lane + 64u < nseg ? v1 : 0u);
  for (uint32_t q = lane + 128; q < nseg; q += 64) c += sc[q];
  for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
  if (lane == 0) a.tile_count[g] = c;
}

void launch_tile_count(const PassArgs& a, hipStream_t s) {
  if (a.n_tiles == 0) return;
  hipLaunchKernelGGL(tile_count_kernel, dim3(div_up(a.n_tiles, 4)), dim3(256), 0, s, a);
}

// ---------------------------------------------------------------- tile classes
// Forward: work = list length; backward: entries the forward pass used (also
// written out as the tile's last used position).  A workgroup of 1024 tiles
// counts its tiles per class in LDS, reserves one range per class in the
// class lists (33 global atomics), and writes its tiles there.  The forward
// classification needs only the tile counts, so it runs in the tile scan's
// first launch (workgroups after the scan's, 4 tiles per thread).
template <int NTH>
__device__ __forceinline__ void classify_block(const PassArgs& a, int blk, bool backward, uint32_t* cnt,
                                               uint32_t* base) {
  constexpr int PER = 1024 / NTH;   // tiles per thread
  if (threadIdx.x < 33) cnt[threadIdx.x] = 0u;
  __syncthreads();
  int c[PER];
  uint32_t slot[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int g = blk * 1024 + k * NTH + (int)threadIdx.x;
    c[k] = -1;
    slot[k] = 0;
    if (g < a.n_tiles) {
      uint32_t work;
      if (backward) {                     // the tile's last used position: the largest of its quadrants'
        const uint4 ql = reinterpret_cast<const uint4*>(a.qlast)[g];
        work = max(max(ql.x, ql.y), max(ql.z, ql.w));
        a.tile_last[g] = work;
      } else {
        work = a.tile_count[g];
      }
      c[k] = work_class(work);
      slot[k] = atomicAdd(&cnt[c[k]], 1u);
    }
  }
  __syncthreads();
  uint32_t* gcnt = a.cls_cnt + (backward ? 33 : 0);
  if (threadIdx.x < 33) base[threadIdx.x] = cnt[threadIdx.x] ? atomicAdd(&gcnt[threadIdx.x], cnt[threadIdx.x]) : 0u;
  __syncthreads();
  uint32_t* lists = backward ? a.order_bwd : a.order_fwd;
#pragma unroll
  for (int k = 0; k < PER; ++k)
    if (c[k] >= 0) lists[(int64_t)c[k] * a.n_tiles + base[c[k]] + slot[k]] = (uint32_t)(blk * 1024 + k * NTH + threadIdx.x);
}

__global__ __launch_bounds__(1024) void classify_tiles_kernel(PassArgs a, int backward) {
  __shared__ uint32_t cnt[33], base[33];
  classify_block<1024>(a, (int)blockIdx.x, backward != 0, cnt, base);
}

void launch_classify_tiles(const PassArgs& a, bool backward, hipStream_t s) {
  if (a.n_tiles == 0) return;
  hipLaunchKernelGGL(classify_tiles_kernel, dim3(div_up(a.n_tiles, 1024)), dim3(1024), 0, s, a, backward ? 1 : 0);
}

// The tile scan's totals pass (workgroups [0, nb)) and the forward
// classification (the rest, 1024 tiles each) in one launch.
__global__ __launch_bounds__(kScanThreads) void tile_totals_classify_kernel(ScanJobs jobs, PassArgs a) {
  __shared__ uint32_t lw[kScanThreads / 64];
  __shared__ uint32_t cnt[33], base[33];
  if ((int)blockIdx.x < jobs.nb0) scan_totals_block(jobs.j0, (int)blockIdx.x, lw);
  else classify_block<kScanThreads>(a, (int)blockIdx.x - jobs.nb0, false, cnt, base);
}

void launch_tile_scan_classify(const PassArgs& a, uint32_t* block_sums, int64_t cap_check,
                               unsigned long long* total_out, hipStream_t s) {
  ScanJobs J;
  J.j0 = ScanJob{a.tile_count, a.tile_start, a.n_tiles, block_sums, cap_check, total_out, nullptr, 1};
  J.j1 = ScanJob{nullptr, nullptr, 0, nullptr, -1, nullptr, nullptr, 1};
  J.nb0 = (int)div_up((int64_t)a.n_tiles + 1, kScanBlock);
  const int ncls = a.n_tiles > 0 ? div_up(a.n_tiles, 1024) : 0;
  hipLaunchKernelGGL(tile_totals_classify_kernel, dim3(J.nb0 + ncls), dim3(kScanThreads), 0, s, J, a);
  hipLaunchKernelGGL(scan_apply_kernel, dim3(J.nb0), dim3(kScanThreads), 0, s, J, a.status);
}

// ---------------------------------------------------------------- complete lists
// The whole sorted list of every tile, from its bitmap row: each thread owns
// a run of words, a block prefix count places its set bits, which it writes
// as splat indices (rank -> splat through the frame's depth order).  The
// forward pass orders each tile only as far as it composites; this pass
// completes the lists on request.
__global__ __launch_bounds__(256) void tile_lists_kernel(PassArgs a) {
  __shared__ uint32_t lw[4];
  if (a.status->overflow) return;
  const int g = blockIdx.x;
  const uint32_t start = a.tile_start[g];
  if (a.tile_start[g + 1] == start) return;
  const int b = frame_of_tile(a.frames, a.B, g);
  const uint32_t vbase = a.bkt_start[b * a.nbk];
  const uint32_t nv = a.bkt_start[(b + 1) * a.nbk] - vbase;
  const uint32_t W = (nv + 31) / 32;
  const uint32_t* row = a.tbits + (int64_t)g * a.bitmap_words;
  const uint16_t* segc = a.seg_cnt + (int64_t)g * a.seg_stride;
  const uint32_t sh = (uint32_t)__ffs(a.seg_words) - 1u;
  // the words of a segment with no set bits are not stored: read as zero
  auto word = [&](uint32_t w) { return segc[w >> sh] ? row[w] : 0u; };
  const uint32_t wpt = (W + 255) / 256;
  const uint32_t w0 = min(W, threadIdx.x * wpt), w1 = min(W, w0 + wpt);
  uint32_t c = 0;
  for (uint32_t w = w0; w < w1; ++w) c += __popc(word(w));
  uint32_t out = start + block_excl_scan<256>(c, lw, nullptr);
  for (uint32_t w = w0; w < w1; ++w) {
    uint32_t bits = word(w);
    while (bits) {
      const uint32_t bit = __ffs(bits) - 1u;
      bits &= bits - 1u;
      a.sorted[out++] = a.depth_sorted[vbase + w * 32u + bit];
    }
  }
}

void launch_tile_lists(const PassArgs& a, hipStream_t s) {
  if (a.n_tiles == 0) return;
  hipLaunchKernelGGL(tile_lists_kernel, dim3(a.n_tiles), dim3(256), 0, s, a);
}

// ---------------------------------------------------------------- compositing
// One workgroup per tile (pixels to threads: TileMap).
// CHUNK sorted entries at a time are staged in LDS and read by every thread
// (broadcast); the tile stops when all its pixels have stopped.
template <int T> using TileShape = TileMap<T>;

// Whether a splat's alpha >= 1/255 region may reach the rectangle
// [x0, x1] x [y0, y1] of pixel centres: the maximum of the concave power
// ca dx^2 + cb dx dy + cc dy^2 over the rectangle (the mean inside: 0; else
// the best point of the four edges) against -log2(255) - log2(o), less a margin
// of 0.01 that keeps the test conservative under float32 rounding (at that
// margin alpha is 0.7 % below the threshold).  A splat that cannot reach a
// pixel is never taken there, so skipping it changes nothing.
__device__ __forceinline__ bool strip_reach(float4 r0, float4 r1, float x0, float x1, float y0, float y1) {
  const float ca = r0.z, cb = r0.w, cc = r1.x;
  x0 -= r0.x; x1 -= r0.x; y0 -= r0.y; y1 -= r0.y;
  if (x0 <= 0.0f && x1 >= 0.0f && y0 <= 0.0f && y1 >= 0.0f) return true;
  const float kx = -cb / (2.0f * cc), ky = -cb / (2.0f * ca);
  float best = -INFINITY;
  {
    const float ya = fminf(fmaxf(kx * x0, y0), y1), yb = fminf(fmaxf(kx * x1, y0), y1);
    best = fmaxf(best, ca * x0 * x0 + cb * x0 * ya + cc * ya * ya);
    best = fmaxf(best, ca * x1 * x1 + cb * x1 * yb + cc * yb * yb);
    const float xa = fminf(fmaxf(ky * y0, x0), x1), xb = fminf(fmaxf(ky * y1, x0), x1);
    best = fmaxf(best, ca * xa * xa + cb * xa * y0 + cc * y0 * y0);
    best = fmaxf(best, ca * xb * xb + cb * xb * y1 + cc * y1 * y1);
  }
  return best >= -kLog2_255 - r1.y - 0.01f;
}

// alpha of a splat at a pixel, bit-identical wherever it is evaluated:
// power = ca dx^2 + cb dx dy + cc dy^2 (= -q/2 in log2 units) plus lo =
// log2(opacity), clamped at lo (q >= 0), and alpha = 2^power = o 2^(-q/2 log2 e).
// The clamp is one v_min_f32 (min(power, lo) for every non-NaN power);
// written as such because fminf would first canonicalise lo, one more
// instruction per (entry, pixel).
__device__ __forceinline__ float splat_alpha(float4 r0, float4 r1, float px, float py, float& dx, float& dy,
                                             float& pw_raw) {
#pragma clang fp contract(off)
  dx = px - r0.x;
  dy = py - r0.y;
  float pw = __builtin_fmaf(r0.z * dx, dx, r1.y);
  pw = __builtin_fmaf(r0.w * dx, dy, pw);
  pw = __builtin_fmaf(r1.x * dy, dy, pw);
  pw_raw = pw;
  float pc;
  asm("v_min_f32 %0, %1, %2" : "=v"(pc) : "v"(pw), "v"(r1.y));
  return __builtin_amdgcn_exp2f(pc);
}

// A staged candidate: mean, log2-scaled conic, log2 opacity, colour, and the
// position after it in the tile's list.
struct __align__(16) StagedRec {
  float4 r0;    // mx my ca cb
  float4 r1;    // cc lo r g (lo = log2 opacity)
  float cb;     // b
  uint32_t next;  // list position after this entry
  float pad[2];
};

// One wave per (tile, quadrant): each wave composites its quadrant's pixels
// on its own, with no barrier shared with the other quadrants of the tile,
// and stops as soon as its own pixels have stopped.  While a chunk's records
// are staged, the entries whose alpha >= 1/255 region may reach the wave's
// pixels are compacted into LDS in list order (a lane tests an entry); the
// compositing then walks that dense array 4 at a time with a uniform counter.
// Per (entry, pixel) the front-to-back step is written on the pixel's signed
// transmittance Te (its transmittance while it runs; once it has stopped,
// minus the transmittance at the stop), so every decision is a vector
// compare and select: no per-entry mask logic on the scalar unit.  The tile's list is read
// in depth order from its bitmap row, a chunk at a time, as the compositing
// consumes it: a cursor walks the row's segments 64 at a time (their bit
// counts, prefix-summed across the wave, place each segment in the tile's
// order), and the words of the segments that overlap the chunk are read a
// word per lane.  Entries behind the wave's stop are never ordered, mapped
// to splats or read.  The consumed part of the sorted list is written out
// for the backward pass (the quadrant waves of a tile write identical
// values), with a per-quadrant contribution byte per entry and the
// quadrant's last used position.  The quadrant waves of a tile get block
// indices of the same residue mod 8, so that they run on one XCD and share
// its L2.
template <int T, int CHUNK>
__global__ __launch_bounds__(64, T == 32 ? 1 : 7) void composite_fwd_kernel(PassArgs a, float* __restrict__ images) {
  using S = TileShape<T>;
  constexpr int NQ = S::NW;             // quadrants per tile
  constexpr int U = 4;                  // entries evaluated together (independent alphas)
  __shared__ StagedRec sr[CHUNK + U];   // the chunk's splat records (one LDS address per entry)
  __shared__ uint32_t list[CHUNK];      // ranks of the chunk being staged
  __shared__ uint32_t ovs[64], ovp[64]; // segments of a window that overlap the chunk: id, first position
  if (a.status->overflow) return;
  const int lane = threadIdx.x;
  int r = blockIdx.x, q = 0;
  if (NQ > 1) {
    const int grp = blockIdx.x / (8 * NQ), within = blockIdx.x % (8 * NQ);
    q = within / 8;
    r = grp * 8 + within % 8;
  }
  const int g = tile_of_rank(a.cls_cnt, a.order_fwd, a.n_tiles, r);
  if (g < 0) return;
  const int b = frame_of_tile(a.frames, a.B, g);
  const FrameDev& F = a.frames[b];
  const int lt = g - F.tile_base;
  const int tx = lt % F.ntx, ty = lt / F.ntx;
  const uint32_t start = a.tile_start[g], end = a.tile_start[g + 1];
  const int vt = q * 64 + lane;         // this lane's thread index in the tile's pixel map
  const int lx0 = S::lx0(vt), ly0 = S::ly0(vt);
  // Te: transmittance while the pixel runs; once it has stopped, minus the
  // transmittance at the stop (-0 outside the frame).  last: list position
  // after the last entry taken; lastk: candidate slot + 1 of the last entry
  // taken in the current chunk (0: none)
  float Te[S::PX], C0[S::PX], C1[S::PX], C2[S::PX], pxf[S::PX], pyf[S::PX];
  uint32_t last[S::PX], lastk[S::PX];
  bool inside[S::PX];
  bool mine = false;
#pragma unroll
  for (int p = 0; p < S::PX; ++p) {
    const int px = tx * T + lx0 + (p % S::PXW), py = ty * T + ly0 + (p / S::PXW);
    pxf[p] = (float)px + 0.5f;
    pyf[p] = (float)py + 0.5f;
    inside[p] = px < F.W && py < F.H;
    Te[p] = inside[p] ? 1.0f : 0.0f;
    C0[p] = C1[p] = C2[p] = 0.0f; last[p] = 0; lastk[p] = 0;
    mine |= inside[p];
  }
  const uint32_t* row = a.tbits + (int64_t)g * a.bitmap_words;
  const uint16_t* segc = a.seg_cnt + (int64_t)g * a.seg_stride;
  const int SW = a.seg_words;
  const uint32_t sh = (uint32_t)__ffs(SW) - 1u;
  uint32_t vbase = 0, nseg = 0, nv = 0;
  if (end > start) {
    vbase = a.bkt_start[b * a.nbk];
    nv = a.bkt_start[(b + 1) * a.nbk] - vbase;
    nseg = ((nv + 31) / 32 + SW - 1) / SW;
  }
  // the wave's quadrant origin (pixel centre of its first lane's first pixel);
  // entries are culled against the rectangle of its pixels still running
  static_assert(S::LPR == 8, "the live-rectangle fold assumes 8 lanes per quadrant row");
  const float qx0 = (float)(tx * T + S::qx(vt) * S::QW) + 0.5f;
  const float qy0 = (float)(ty * T + S::qy(vt) * S::QW) + 0.5f;
  uint32_t wseg = 0, wpos = 0;          // cursor: a segment starting at or before the chunk, its first position
  bool live = __ballot(mine) != 0ull;
  for (uint32_t cb = start; live && cb < end; cb += CHUNK) {
    const int n = (int)min((uint32_t)CHUNK, end - cb);
    const uint32_t c0 = cb - start, c1 = c0 + (uint32_t)n;
    // ---- ranks of positions [c0, c1) into list[] ----
    while (true) {
      const uint32_t sg = wseg + (uint32_t)lane;
      const uint32_t cnt = segc[min(sg, nseg - 1u)] * (sg < nseg ? 1u : 0u);
      const uint32_t inc = wave_incl_scan(cnt);
      const uint32_t p0 = wpos + inc - cnt;          // first position of segment sg
      const uint32_t wtot = __shfl(inc, 63);
      const bool ov = cnt != 0u && p0 < c1 && p0 + cnt > c0;
      const unsigned long long om = __ballot(ov);
      const int nov = __popcll(om);
      if (ov) {
        const uint32_t k = lanes_below(om);
        ovs[k] = sg;
        ovp[k] = p0;
      }
      __syncthreads();
      for (int k0 = 0; k0 < nov; k0 += 64 >> sh) {
        const int k = k0 + (lane >> sh);
        const int kc = min(k, nov - 1);
        const uint32_t wi = (uint32_t)lane & (uint32_t)(SW - 1);
        const uint32_t wq = ovs[kc] * (uint32_t)SW + wi;
        uint32_t bits = row[wq];
        if (k >= nov) bits = 0u;
        const uint32_t c = __popc(bits);
        uint32_t incw = c;
        for (int d = 1; d < SW; d <<= 1) {
          const uint32_t o = __shfl_up(incw, d, SW);
          if ((int)wi >= d) incw += o;
        }
        uint32_t pos = ovp[kc] + incw - c;
        while (bits) {
          const uint32_t bit = __ffs(bits) - 1u;
          bits &= bits - 1u;
          if (pos >= c0 && pos < c1) list[pos - c0] = wq * 32u + bit;
          ++pos;
        }
      }
      __syncthreads();
      const bool more = wpos + wtot < c1 && wseg + 64u < nseg;   // the chunk goes on past this window
      if (!more) {
        // next chunk: from the segment holding position c1 (or the next window)
        const unsigned long long past = __ballot(sg < nseg && p0 + cnt > c1);
        if (past) {
          const int j = __ffsll((long long)past) - 1;
          wpos = __shfl(p0, j);
          wseg += (uint32_t)j;
        } else {
          wseg += 64u;
          wpos += wtot;
        }
        break;
      }
      wseg += 64u;
      wpos += wtot;
    }
    // ---- the rectangle of the pixel centres still running: lanes are 8 per
    // row, so a column runs if any of its 8 lanes does, a row if its byte of
    // the wave mask is nonzero ----
    float sx0, sx1, sy0, sy1;
    {
      bool run = false;
#pragma unroll
      for (int p = 0; p < S::PX; ++p) run |= Te[p] > 0.0f;
      const unsigned long long M = __ballot(run);
      unsigned long long cm8 = M | (M >> 32);
      cm8 |= cm8 >> 16;
      cm8 |= cm8 >> 8;
      cm8 &= 0xffull;
      unsigned long long rm = M | (M >> 4);
      rm |= rm >> 2;
      rm |= rm >> 1;
      rm &= 0x0101010101010101ull;
      const int c0l = __ffsll((long long)cm8) - 1, c1l = 63 - __clzll((long long)cm8);
      const int r0l = (__ffsll((long long)rm) - 1) >> 3, r1l = (63 - __clzll((long long)rm)) >> 3;
      sx0 = qx0 + (float)(c0l * S::PXW);
      sx1 = qx0 + (float)(c1l * S::PXW + S::PXW - 1);
      sy0 = qy0 + (float)(r0l * S::PXW);
      sy1 = qy0 + (float)(r1l * S::PXW + S::PXW - 1);
    }
    // ---- the chunk's records; the candidates compacted in list order ----
    constexpr int NB = (CHUNK + 63) / 64;
    int kslot[NB];                        // this lane's entry of block j: its candidate slot, or -1
    int ncand = 0;                        // (uniform)
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int i = j * 64 + lane;
      kslot[j] = -1;
      if (j * 64 >= n) continue;
      float4 q0 = make_float4(0.f, 0.f, 0.f, 0.f), q1 = q0;
      float qb = 0.f;
      bool c = false;
      if (i < n) {
        const uint32_t sp = a.depth_sorted[vbase + min(list[i], nv - 1u)];   // (every rank is written)
        a.sorted[cb + i] = sp;
        const float4* rec = reinterpret_cast<const float4*>(a.rec + (int64_t)sp * kRecF);
        q0 = rec[0]; q1 = rec[1]; qb = rec[2].x;
        c = live && strip_reach(q0, q1, sx0, sx1, sy0, sy1);
      }
      const unsigned long long m = __ballot(c);
      if (c) {
        const int k = ncand + (int)lanes_below(m);
        kslot[j] = k;
        sr[k].r0 = q0; sr[k].r1 = q1; sr[k].cb = qb; sr[k].next = c0 + (uint32_t)i + 1u;
      }
      ncand += __popcll(m);
    }
    if (lane < U) {                       // padding entries: opacity 0 (log2 -1e30), never taken; their
      sr[ncand + lane].r1 = make_float4(0.f, -1e30f, 0.f, 0.f);   // colour 0 (its mean and conic may be
      sr[ncand + lane].cb = 0.f;                                   // anything: min(power, -1e30) = -1e30)
    }
    __syncthreads();
    // ---- compositing: the candidates in list order, U at a time ----
    uint32_t took4 = 0u;                  // lane g: bit u = some pixel took candidate 4 g + u
    for (int k = 0; live && k < ncand; k += U) {
      float4 r0[U], r1[U];
      float cb2[U];
#pragma unroll
      for (int u = 0; u < U; ++u) { r0[u] = sr[k + u].r0; r1[u] = sr[k + u].r1; cb2[u] = sr[k + u].cb; }
      unsigned long long tm[U];
#pragma unroll
      for (int u = 0; u < U; ++u) tm[u] = 0ull;
#pragma unroll
      for (int p = 0; p < S::PX; ++p) {
        float al[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          float dx, dy, pwr;
          al[u] = splat_alpha(r0[u], r1[u], pxf[p], pyf[p], dx, dy, pwr);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          // the front-to-back step: alpha below 1/255 is skipped (w = 0, Te
          // passes unchanged), T (1 - alpha) < 1e-4 stops the pixel before
          // this entry (Te -> -T); a stopped pixel has Te <= 0, so its tn <= 0
          // stops it again (Te kept: -|Te|) and it takes nothing
          const float w = (al[u] >= kAlphaMin) ? fminf(al[u], kAlphaMax) : 0.0f;
          const float tn = __builtin_fmaf(-w, Te[p], Te[p]);   // T (1 - alpha), rounded once
          const bool stop = tn < kTMin;
          const float wgt = stop ? 0.0f : w * Te[p];
          C0[p] = __builtin_fmaf(wgt, r1[u].z, C0[p]);
          C1[p] = __builtin_fmaf(wgt, r1[u].w, C1[p]);
          C2[p] = __builtin_fmaf(wgt, cb2[u], C2[p]);
          Te[p] = stop ? -fabsf(Te[p]) : tn;   // one select with source modifiers
          const bool take = wgt > 0.0f;   // w >= 1/255 and Te >= 1e-4: never 0 when taken
          lastk[p] = take ? (uint32_t)(k + u + 1) : lastk[p];
          tm[u] |= __builtin_amdgcn_ballot_w64(take);
        }
      }
      // bit u: some pixel took candidate k + u; formed on the scalar unit
      // (the masks are uniform; the compiler builds it with vector ORs)
      uint32_t m4 = 0u;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        uint32_t bit;
        asm("s_cmp_lg_u64 %1, 0\n\ts_cselect_b32 %0, %2, 0" : "=s"(bit) : "s"(tm[u]), "i"(1 << u) : "scc");
        m4 |= bit;
      }
      took4 = (lane == k / U) ? m4 : took4;
      bool mine_now = false;
#pragma unroll
      for (int p = 0; p < S::PX; ++p) mine_now |= Te[p] > 0.0f;
      if (__ballot(mine_now) == 0ull) live = false;
    }
    // the list position after each pixel's last entry taken in this chunk
#pragma unroll
    for (int p = 0; p < S::PX; ++p) {
      if (lastk[p]) last[p] = sr[lastk[p] - 1].next;
      lastk[p] = 0;
    }
    // the quadrant's contribution byte of every entry of the chunk
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int i = j * 64 + lane;
      const int ks = kslot[j];
      const uint32_t t4 = (uint32_t)__shfl((int)took4, ks < 0 ? 0 : ks / U);
      if (i < n) a.cmask[((int64_t)(cb + i) << 2) + q] = (ks >= 0) ? (uint8_t)((t4 >> (ks % U)) & 1u) : (uint8_t)0;
    }
    __syncthreads();
  }
  uint32_t my_last = 0;
#pragma unroll
  for (int p = 0; p < S::PX; ++p) {
    if (inside[p]) {
      const int px = (int)pxf[p], py = (int)pyf[p];
      const int64_t pix = (int64_t)py * F.W + px;
      const int64_t hw = (int64_t)F.W * F.H;
      float* img = images + F.pix_base * 3;
      const float Tfin = fabsf(Te[p]);
      img[pix] = C0[p] + Tfin * F.bg[0];
      img[hw + pix] = C1[p] + Tfin * F.bg[1];
      img[2 * hw + pix] = C2[p] + Tfin * F.bg[2];
      a.n_iter[F.pix_base + pix] = last[p];
      a.t_final[F.pix_base + pix] = Tfin;
      my_last = max(my_last, last[p]);
    }
  }
  my_last = wave_max_u32(my_last);
  if (lane < 4 && (lane == q || NQ == 1)) a.qlast[g * 4 + lane] = lane == q ? my_last : 0u;
}

void launch_composite_fwd(const PassArgs& a, float* images, int chunk, hipStream_t s) {
  if (a.n_tiles == 0) return;
  const int nq = a.tile == 8 ? 1 : 4;
  const dim3 grid(nq == 1 ? a.n_tiles : div_up(a.n_tiles, 8) * 8 * nq);
#define GBR_FWD(TT, CC) hipLaunchKernelGGL((composite_fwd_kernel<TT, CC>), grid, dim3(64), 0, s, a, images)
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

// Contributors per pixel, on request: the entries before the pixel's stop
// position whose alpha reaches 1/255 (every such entry was taken, nothing
// after the stop was).  Reads the complete per-tile lists; a workgroup per
// tile, a thread per pixel.  Diagnostic only, not part of a pass.
__global__ __launch_bounds__(256) void count_contrib_kernel(PassArgs a) {
  const int g = blockIdx.x;
  if (a.status->overflow || g >= a.n_tiles) return;
  const int b = frame_of_tile(a.frames, a.B, g);
  const FrameDev& F = a.frames[b];
  const int T = a.tile;
  const int lt = g - F.tile_base;
  const int tx = lt % F.ntx, ty = lt / F.ntx;
  const uint32_t start = a.tile_start[g];
  for (int q = threadIdx.x; q < T * T; q += 256) {
    const int px = tx * T + q % T, py = ty * T + q / T;
    if (px >= F.W || py >= F.H) continue;
    const int64_t pix = F.pix_base + (int64_t)py * F.W + px;
    const uint32_t nit = a.n_iter[pix];
    uint32_t c = 0;
    for (uint32_t i = 0; i < nit; ++i) {
      const float4* rec = reinterpret_cast<const float4*>(a.rec + (int64_t)a.sorted[start + i] * kRecF);
      float dx, dy, pwr;
      const float al = splat_alpha(rec[0], rec[1], (float)px + 0.5f, (float)py + 0.5f, dx, dy, pwr);
      c += al >= kAlphaMin ? 1u : 0u;
    }
    a.n_contrib[pix] = c;
  }
}

void launch_count_contrib(const PassArgs& a, hipStream_t s) {
  if (a.n_tiles == 0) return;
  hipLaunchKernelGGL(count_contrib_kernel, dim3(a.n_tiles), dim3(256), 0, s, a);
}

}  // namespace gbr
