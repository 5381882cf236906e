// Internal definitions shared by the libgbr kernels and the host side of the
// library (device structs, launch helpers, wave-level primitives).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gbr {

constexpr int kNF = 16;                    // stored floats per blended Gaussian
constexpr float kAlphaMin = 1.0f / 255.0f; // contribution threshold
constexpr float kAlphaMax = 0.99f;         // opacity clamp
constexpr float kTMin = 1e-4f;             // transmittance stop
constexpr double kLowPass = 0.3;           // px^2 added to the 2D covariance
constexpr double kBoxPad = 0.01;           // px added to the alpha-support box
constexpr double kLog2e = 1.4426950408889634;
constexpr float kLog2_255 = 7.99435343685886f;   // log2(255): alpha >= 1/255 <=> log2(alpha) >= -kLog2_255
constexpr double kLn2 = 0.6931471805599453;
constexpr int kRecF = 12;
constexpr int kPartF = 12;          // floats per partial record: 9 values, padded to 48 B (3 x 16-B loads)                  // floats per splat record
constexpr int kMaxFrameTilesLds = 4096;    // per-frame tile histogram kept in LDS

// Per-frame table entry, built on the host for every render and uploaded
// with the pass.
struct FrameDev {
  float fx, fy, cx, cy;
  float R[9];
  float t[3];
  float near_z;
  float bg[3];
  int32_t W, H, ntx, nty;
  int32_t tile_base;   // first global tile id of the frame
  int32_t n_tiles;
  int64_t pix_base;    // first pixel of the frame in the packed pixel space
  int64_t gauss_base;  // first splat of the frame
  int64_t gauss_count;
};

// Device-side status of a pass; read once per step by gbr_query_status.
struct StatusDev {
  unsigned long long entries;
  unsigned int overflow;
  unsigned int pad0;
  int32_t adam_step[4];
  float loss;
  float adam_bc[4][2];     // per group: bias corrections 1 - beta^t of its last Adam step
  float pad1;
};

// Tangent-space binding of a pass (Sec. 3.1, Eq. 4): when `on`, the pass
// reads tangent-space Gaussians (every frame holds the same N, bound to
// triangle tri[n] at barycentric coordinates bary[n]), carries each to its
// frame's deformed mesh inside the projection, and the adjoint returns the
// gradient in tangent space.  frames: [B][F][16] per-(frame, triangle) TBN
// matrix and frame quaternion (gbr_tangent_frames).
struct TangentArgs {
  const int32_t* tri;
  const float* bary;
  const float* verts;       // [B][V][3]
  const int32_t* faces;     // [F][3]
  const float* frames;      // [B][F][16]
  int64_t N;
  int32_t V, F;
  int32_t on;
  int32_t pad;
};

// Everything the pass kernels need, passed by value.

struct PassArgs {
  const FrameDev* frames;
  int32_t B;
  int32_t tile;
  int32_t n_tiles;          // total tiles of the pass
  int32_t pad;
  int64_t n_splats;
  int64_t n_pixels;
  int64_t cap_entries;
  StatusDev* status;
  // splat stage
  float* rec;               // [S][12]: mx my ca cb | cc lo r g | b depth box_x box_y (lo = log2 opacity)
                            //   box_x = x0 | x1 << 16, box_y = y0 | y1 << 16 (pixel box, as bits)
  int4* rect;               // [S] inclusive tile rect (tx0, ty0, tx1, ty1)
  uint32_t* cnt;            // [S] tiles touched
  uint32_t* soff;           // [S] exclusive scan of cnt (emission offsets)
  uint32_t* dkey;           // [S] binary32 depth bits of a valid splat, 0xffffffff otherwise
  // tile stage
  uint32_t* tile_count;     // [tiles]
  uint32_t* tile_start;     // [tiles + 1]
  uint32_t* tile_last;      // [tiles] entries used by the tile's last pixel (the largest of qlast)
  uint32_t* qlast;          // [tiles][4] entries used by the last pixel of each quadrant (wave) of the tile
  uint32_t* tbits;          // [tiles][bitmap_words] per-tile bitmaps of frame-local depth ranks
  uint16_t* seg_cnt;        // [tiles][seg_stride] set bits of each row segment
  uint32_t* sorted;         // [E] splat index in tile order
  uint32_t* order_fwd;      // [33][tiles] tiles by class of list length (scheduling only)
  uint32_t* order_bwd;      // [33][tiles] tiles by class of entries used by the forward pass
  uint32_t* cls_cnt;        // [2][33] tiles per class (forward, backward)
  // per-frame depth order
  int32_t nbk;              // depth buckets per frame
  int32_t nblk;             // workgroups of kBucketBlock splats per frame in the bucket passes
  int32_t bitmap_words;     // words per tile bitmap row (largest frame's splats / 32, rounded up to 16)
  int32_t seg_words;        // words per row segment (8 or 16); a segment's set bits are counted once
  int32_t seg_stride;       // segments per row = bitmap_words / seg_words
  uint32_t* blk_mm;         // [2 per projection workgroup] min, max binary32 depth bits of its valid splats;
                            // frame b's workgroup j at gauss_base / 256 + b + j (frames never share one)
                            //   (a 128-byte line per frame, so frames' atomics do not share a line)
  uint32_t* bkt_count;      // [B * nbk][nblk] per-block bucket counts
  uint32_t* bkt_moff;       // [B * nbk * nblk + 1] their exclusive scan
  uint32_t* bkt_start;      // [B * nbk + 1] exclusive scan; frame b's valid splats start at bkt_start[b * nbk]
  unsigned long long* bkeys;      // [S] (depth bits << 32) | splat, grouped by bucket
  unsigned long long* bkeys_alt;  // [S] ping-pong for large buckets
  uint32_t* depth_sorted;   // [S] valid splats of each frame in (depth, index) order
  uint32_t* rank;           // [S] frame-local position of a valid splat in that order
  // pixel stage
  uint32_t* n_iter;         // [pixels] list position after the last contributor
  uint32_t* n_contrib;      // [pixels] number of contributors (computed on request)
  float* t_final;           // [pixels]
  float* part;              // [E][kPartF] per-entry gradient partials (9 used), by emission slot
  uint8_t* part_flag;       // [E] 1 where the entry's partial is written; zeroed at allocation, set by the
                            // backward compositing, and reset to 0 by the gather that reads it
  uint8_t* cmask;           // [E][4] byte w = 1: some pixel of quadrant w of the tile took this entry (forward)
  TangentArgs tg;           // tangent-space binding (tg.on = 0: the pass reads deformed-space Gaussians)
};

__device__ __forceinline__ int frame_of_tile(const FrameDev* frames, int B, int g) {
  int lo = 0, hi = B - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (frames[mid].tile_base <= g) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ int frame_of_splat(const FrameDev* frames, int B, int64_t s) {
  int lo = 0, hi = B - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (frames[mid].gauss_base <= s) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// popcount(mask & lanes below this one)
__device__ __forceinline__ uint32_t lanes_below(unsigned long long mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

template <int CTRL, int ROW_MASK, int BANK_MASK, bool BOUND_CTRL>
__device__ __forceinline__ float dpp_mov(float x) {
  return __builtin_bit_cast(float,
      __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), CTRL, ROW_MASK, BANK_MASK, BOUND_CTRL));
}

// Pixels of a tile and the threads that composite them.  T = 8: 64 threads,
// one pixel each; T = 16: 256 threads, one pixel each; T = 32: 256 threads,
// a 2x2 pixel block each.  Each wave covers a square quadrant of the tile
// (the whole tile when T = 8), its lanes row-major inside it: compact wave
// footprints let whole waves skip a splat or stop early.  The forward and
// backward passes share this map (the forward's per-wave contribution bits
// are read by the backward's waves).
template <int T> struct TileMap {
  static constexpr int NT = (T == 8) ? 64 : 256;
  static constexpr int PXW = (T == 32) ? 2 : 1;     // pixels per thread along x and y
  static constexpr int PX = PXW * PXW;
  static constexpr int NW = NT / 64;
  static constexpr int QW = (NW == 1) ? T : T / 2;  // side of a wave's quadrant, pixels
  static constexpr int LPR = QW / PXW;              // lanes per quadrant row
  __device__ static int qx(int tid) { return (tid >> 6) & 1; }
  __device__ static int qy(int tid) { return (tid >> 6) >> 1; }
  __device__ static int lx0(int tid) { return qx(tid) * QW + ((tid & 63) % LPR) * PXW; }
  __device__ static int ly0(int tid) { return qy(tid) * QW + ((tid & 63) / LPR) * PXW; }
};

// Longest-first tile scheduling.  Workgroups start in blockIdx order, so the
// compositing passes visit tiles by descending work: a tile goes to the list
// of its work class (floor(log2(work)); class 32 = no work, last), and a
// workgroup finds its tile by walking the 33 class counts.  Scheduling only:
// a tile's result does not depend on when it runs.
__device__ __forceinline__ int work_class(uint32_t work) { return work ? 31 - __clz(work) : 32; }

__device__ __forceinline__ int tile_of_rank(const uint32_t* cnt, const uint32_t* lists, int n_tiles, int r) {
  uint32_t acc = 0;
  for (int i = 0; i < 33; ++i) {
    const int c = (i < 32) ? 31 - i : 32;
    const uint32_t k = cnt[c];
    if ((uint32_t)r < acc + k) return (int)lists[(int64_t)c * n_tiles + (r - acc)];
    acc += k;
  }
  return -1;
}

// Lane swaps of gfx950: after swap32(x, y), x holds (x lanes 0-31, y lanes
// 0-31) and y holds (x lanes 32-63, y lanes 32-63); after swap16(x, y), by
// rows of 16 lanes, x holds (x0, y0, x2, y2) and y holds (x1, y1, x3, y3).
// Adding the two results folds two values into one register at half the
// lane count each.  Written as inline assembly (both operands are read and
// written in place), several swaps per statement, with two wait states
// before the first (after the VALU writes of the operands) and after the
// last.
#define GBR_SWAP_PAIR(op, i, j) op " %" #i ", %" #j "\n\t"
__device__ __forceinline__ void fold32x9(float* x, float* y) {   // x[c] <- x[c] + y[c] folded, c < 9
  asm volatile("s_nop 1\n\t"
               GBR_SWAP_PAIR("v_permlane32_swap_b32", 0, 9) GBR_SWAP_PAIR("v_permlane32_swap_b32", 1, 10)
               GBR_SWAP_PAIR("v_permlane32_swap_b32", 2, 11) GBR_SWAP_PAIR("v_permlane32_swap_b32", 3, 12)
               GBR_SWAP_PAIR("v_permlane32_swap_b32", 4, 13) GBR_SWAP_PAIR("v_permlane32_swap_b32", 5, 14)
               GBR_SWAP_PAIR("v_permlane32_swap_b32", 6, 15) GBR_SWAP_PAIR("v_permlane32_swap_b32", 7, 16)
               GBR_SWAP_PAIR("v_permlane32_swap_b32", 8, 17) "s_nop 1"
               : "+v"(x[0]), "+v"(x[1]), "+v"(x[2]), "+v"(x[3]), "+v"(x[4]), "+v"(x[5]), "+v"(x[6]), "+v"(x[7]),
                 "+v"(x[8]), "+v"(y[0]), "+v"(y[1]), "+v"(y[2]), "+v"(y[3]), "+v"(y[4]), "+v"(y[5]), "+v"(y[6]),
                 "+v"(y[7]), "+v"(y[8]));
#pragma unroll
  for (int c = 0; c < 9; ++c) x[c] += y[c];
}
__device__ __forceinline__ void fold16x9(float* x, float* y) {   // x[c] <- x[c] + y[c] folded, c < 9
  asm volatile("s_nop 1\n\t"
               GBR_SWAP_PAIR("v_permlane16_swap_b32", 0, 9) GBR_SWAP_PAIR("v_permlane16_swap_b32", 1, 10)
               GBR_SWAP_PAIR("v_permlane16_swap_b32", 2, 11) GBR_SWAP_PAIR("v_permlane16_swap_b32", 3, 12)
               GBR_SWAP_PAIR("v_permlane16_swap_b32", 4, 13) GBR_SWAP_PAIR("v_permlane16_swap_b32", 5, 14)
               GBR_SWAP_PAIR("v_permlane16_swap_b32", 6, 15) GBR_SWAP_PAIR("v_permlane16_swap_b32", 7, 16)
               GBR_SWAP_PAIR("v_permlane16_swap_b32", 8, 17) "s_nop 1"
               : "+v"(x[0]), "+v"(x[1]), "+v"(x[2]), "+v"(x[3]), "+v"(x[4]), "+v"(x[5]), "+v"(x[6]), "+v"(x[7]),
                 "+v"(x[8]), "+v"(y[0]), "+v"(y[1]), "+v"(y[2]), "+v"(y[3]), "+v"(y[4]), "+v"(y[5]), "+v"(y[6]),
                 "+v"(y[7]), "+v"(y[8]));
#pragma unroll
  for (int c = 0; c < 9; ++c) x[c] += y[c];
}
#undef GBR_SWAP_PAIR

inline int div_up(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

}  // namespace gbr

// Kernel launchers (defined in the .hip files).
namespace gbr {
void launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s);
void launch_fill_f32(float* p, float v, int64_t n, hipStream_t s);
constexpr int kBucketBlock = 8192;      // splats per workgroup in the depth-bucket passes
constexpr int kBlendMaxFrames = 4096;   // frames per gbr_blend call (rows of the float64 weight table)
constexpr int kBlendW64Stride = 64;     // K + 1 <= 64
void launch_blend_fwd(const float* bases, const float* weights, int B, int K, int64_t N, float* raw, double* w64,
                      hipStream_t s);
void launch_blend_bwd(const float* draw, const float* bases, const float* weights, int B, int K, int64_t N,
                      float* dbases, float* dweights, float* partials, int64_t n_partials, int accumulate,
                      hipStream_t s);
int64_t blend_bwd_partials(int B, int K, int64_t N);
// floats of partials launch_blend_bwd actually writes and reads for this shape
int64_t blend_bwd_partials_used(int B, int K, int64_t N);
// Exclusive scan of in[0, n) into out[0, n] (out[n] = total).  With strided
// non-null, also strided[j] = out[j * stride] for every j * stride <= n.
// The grand total is stored to total_out when non-null, and sets the
// overflow flag when it exceeds cap_check (>= 0).  block_sums holds
// scan_scratch_words(n) words.
struct ScanJob {
  const uint32_t* in;
  uint32_t* out;
  int64_t n;
  uint32_t* block_sums;
  int64_t cap_check;
  unsigned long long* total_out;
  uint32_t* strided;
  int stride;
};
void launch_scan_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* block_sums, StatusDev* status,
                     int64_t cap_check, unsigned long long* total_out, hipStream_t s, uint32_t* strided = nullptr,
                     int stride = 1);
// Two independent scans in the same two launches (distinct block_sums).
void launch_scan_u32_pair(const ScanJob& j0, const ScanJob& j1, StatusDev* status, hipStream_t s);
int64_t scan_scratch_words(int64_t n);
// Returns whether it launched (no frame has Gaussians otherwise): the
// launch also clears the pass's counters.
bool launch_preprocess(const PassArgs& a, const float* raw, int64_t max_frame_splats, hipStream_t s);
// Words per bitmap row segment for frames of up to max_frame_tiles tiles
// (the workgroup that builds a segment of every row of a frame holds them in LDS).
constexpr int kMaxRowSegs = 1024;   // segments per bitmap row at most (the compositing lists them in LDS)
int bitmap_seg_words(int max_frame_tiles, int64_t row_words);
void launch_bitmap_rows(const PassArgs& a, int64_t max_frame_splats, int max_frame_tiles, hipStream_t s);
void launch_tile_lists(const PassArgs& a, hipStream_t s);
void launch_tile_count(const PassArgs& a, hipStream_t s);
void launch_count_contrib(const PassArgs& a, hipStream_t s);
void launch_classify_tiles(const PassArgs& a, bool backward, hipStream_t s);
// The tile scan (tile_count -> tile_start, total to total_out, checked against
// cap_check) with the forward classification of the tiles in its first launch.
void launch_tile_scan_classify(const PassArgs& a, uint32_t* block_sums, int64_t cap_check,
                               unsigned long long* total_out, hipStream_t s);

// The depth order of every frame's splats.  side is an independent scan whose
// input is ready when the pass starts, run in the bucket scan's launches.
void launch_depth_order(const PassArgs& a, int64_t max_frame_splats, uint32_t* scan_scratch, const ScanJob& side,
                        hipStream_t s);
void launch_composite_fwd(const PassArgs& a, float* images, int chunk, hipStream_t s);
void launch_composite_bwd(const PassArgs& a, const float* dimages, const float* images, int chunk, hipStream_t s);
void launch_gather_bwd(const PassArgs& a, const float* raw, float* draw, int64_t max_frame_splats, hipStream_t s);
void launch_tangent_frames(const float* verts, const int32_t* faces, const float* face_uv, int B, int V, int F,
                           float* frames, hipStream_t s);
void launch_tangent_fwd(const float* raw_t, const int32_t* tri, const float* bary, const float* verts,
                        const int32_t* faces, const float* frames, int B, int64_t N, int V, int F, float* raw_d,
                        hipStream_t s);
void launch_tangent_bwd(const float* draw_d, const int32_t* tri, const float* frames, int B, int64_t N, int F,
                        float* draw_t, hipStream_t s);
void launch_color_init_apply(const float* draw_i, const float* draw_1, int B, int64_t N, float delta, float* bases,
                             uint8_t* done, hipStream_t s);
void launch_loss(const PassArgs& a, const float* images, const float* targets, int kind, float* dimages,
                 float* partials, int64_t n_partials, hipStream_t s);
int64_t loss_partials(int64_t n_floats);
void launch_mlp_fwd(const float* params, const float* theta, int B, int d_in, int hidden, int K, float* psi,
                    float* z1, float* z2, hipStream_t s);
void launch_mlp_bwd(const float* params, const float* theta, const float* z1, const float* z2, const float* dpsi,
                    int B, int d_in, int hidden, int K, float* dz1, float* dz2, float* dparams, hipStream_t s);
// Adam's update of one element (Sec. A.3), shared by the plain step and the
// step fused with the blend adjoint so that both form the same values.
// rc1 = 1 / (1 - b1^t), rsc2 = 1 / sqrt(1 - b2^t).
struct LrTable { float v[32]; };
__device__ __forceinline__ void adam_update(float& p, float& m, float& v, float g, float rate, float b1, float b2,
                                            float rc1, float rsc2, float eps) {
  const float mi = b1 * m + (1.0f - b1) * g;
  const float vi = b2 * v + (1.0f - b2) * g * g;
  m = mi;
  v = vi;
  p -= rate * (mi * rc1) / (sqrtf(vi) * rsc2 + eps);
}
void launch_adam_tick(StatusDev* status, int group, float b1, float b2, hipStream_t s);
void launch_blend_adam(const float* draw, const float* weights, int B, int K, int64_t N, float* p, float* m, float* v,
                       StatusDev* status, int group, const float* lr_table_host, float b1, float b2, float eps,
                       hipStream_t s);
void launch_adam(StatusDev* status, int group, float* p, const float* g, float* m, float* v, int64_t n,
                 int64_t split, const float* lr_table_host, float b1, float b2, float eps, hipStream_t s);
}  // namespace gbr
