// C ABI of libgbr: context and workspace management, host-side validation,
// and the enqueue order of the batch-parallel pass (preprocess and rasterize
// of a whole batch of frames with no host synchronisation in between; the
// only synchronisation of a training step is gbr_query_status).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <vector>

#include "gbr.h"
#include "gbr_internal.h"

using namespace gbr;

namespace {

constexpr int kSlots = 5;          // pinned frame-table slots; the last one is used under graph capture
constexpr int kCaptureSlot = kSlots - 1;
constexpr int kMaxK = 63;
constexpr int kMaxFramesHard = 4096;
constexpr int64_t kMaxBitmapWords = 32768;   // 128 KB bitmap row per tile: frames of up to 1,048,576 Gaussians

// A failed HIP call is reported once: its error is also taken out of HIP's
// last-error state, which the launch checks read, so that it does not
// surface again at an unrelated later call.
#define GBR_HIP(x)                 \
  do {                             \
    hipError_t e_ = (x);           \
    if (e_ != hipSuccess) {        \
      (void)hipGetLastError();     \
      return GBR_ERR_HIP;          \
    }                              \
  } while (0)

template <typename T>
int dalloc(T** p, int64_t count) {
  *p = nullptr;
  if (count <= 0) count = 1;
  if (hipMalloc(reinterpret_cast<void**>(p), sizeof(T) * (size_t)count) != hipSuccess) return GBR_ERR_OOM;
  return GBR_OK;
}

template <typename T>
void dfree(T*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

// Clears the per-pass counters (the status and the tile-class counts of both
// schedules, 66 words) for a pass whose projection, which clears them
// otherwise, does not run: no frame has Gaussians.  One block of 256.
__global__ void begin_pass_kernel(PassArgs a) {
  if (threadIdx.x < 66) a.cls_cnt[threadIdx.x] = 0u;
  if (threadIdx.x == 0) { a.status->overflow = 0u; a.status->entries = 0ull; }
}

__global__ void clear_overflow_kernel(StatusDev* status) { status->overflow = 0u; }

// A status record of the host ring: the device status and the number of the
// post that wrote it.
struct StatusRec {
  StatusDev st;
  unsigned long long seq;
};
constexpr int kStatusSlots = 4;   // records of the ring (gbr_status_post / gbr_status_wait)

// Post n (the device counts its posts in the order it runs them) copies the
// status into record n mod kStatusSlots of the host ring, then stores n with
// a system-scope release, so that the host sees the record whole once it
// sees n.
__global__ void status_post_kernel(const StatusDev* __restrict__ d, StatusRec* ring, unsigned long long* count) {
  const unsigned long long n = *count + 1ull;
  *count = n;
  StatusRec* r = ring + n % kStatusSlots;
  r->st = *d;
  __hip_atomic_store(&r->seq, n, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

}  // namespace

// ---- scratch of the allocation-free entry point (gbr_blend_backward_noalloc)
// The dweights partials live in this fixed device array instead of a
// context's workspace.  In host code `scratch` only names the symbol: its
// device address is taken once per device with hipGetSymbolAddress (that
// device current) and only that address is passed to kernels.
constexpr int64_t kNoAllocScratchFloats = int64_t(1) << 20;   // 4 MiB per device
static __device__ __align__(256) float scratch[kNoAllocScratchFloats];
constexpr int kNoAllocMaxDevices = 64;
static std::mutex g_scratch_mu;
static float* g_scratch_addr[kNoAllocMaxDevices] = {};

static int scratch_of_current_device(float** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kNoAllocMaxDevices) return GBR_ERR_HIP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return GBR_ERR_HIP;
    g_scratch_addr[dev] = static_cast<float*>(p);
  }
  *out = g_scratch_addr[dev];
  return GBR_OK;
}

struct gbr_ctx {
  gbr_config cfg;
  int tile = 16, chunk = 64;
  int64_t cap_entries = 0, cap_splats = 0, cap_pixels = 0, cap_tiles = 0;
  int cap_frames = 0;
  // device workspace
  FrameDev* d_frames = nullptr;
  StatusDev* d_status = nullptr;
  float* rec = nullptr;
  int4* rect = nullptr;
  uint32_t *cnt = nullptr, *soff = nullptr, *dkey = nullptr;
  uint32_t *tile_count = nullptr, *tile_start = nullptr, *tile_last = nullptr, *qlast = nullptr;
  uint32_t* tbits = nullptr;        // [cap_tbits] per-tile rank bitmap rows
  int64_t cap_tbits = 0;
  uint16_t* seg_cnt = nullptr;      // [cap_seg] set bits per row segment
  int64_t cap_seg = 0;
  int seg_words = 16, max_frame_tiles = 0;
  uint32_t* sorted = nullptr;
  uint32_t *order_fwd = nullptr, *order_bwd = nullptr, *cls_cnt = nullptr;
  uint8_t* part_flag = nullptr;
  uint8_t* cmask = nullptr;
  // per-frame depth order
  uint32_t *blk_mm = nullptr, *bkt_count = nullptr, *bkt_moff = nullptr, *bkt_start = nullptr;
  unsigned long long *bkeys = nullptr, *bkeys_alt = nullptr;
  uint32_t *depth_sorted = nullptr, *rank = nullptr;
  int64_t cap_bkt = 0, cap_bkt_cells = 0;
  int nbk = 64, nblk = 1;
  float* part = nullptr;
  uint32_t* n_iter = nullptr;
  uint32_t* n_contrib = nullptr;
  float* t_final = nullptr;
  uint32_t* scan_scratch = nullptr;
  uint32_t* scan_scratch_splat = nullptr;   // block sums of the per-splat count scan
  int64_t cap_scan_words = 0;
  float* draw_scratch = nullptr;
  float *ci_ones = nullptr, *ci_draw = nullptr;   // colour initialisation: all-ones images, second adjoint
  float* loss_part = nullptr;
  float* blend_part = nullptr;
  double* blend_w64 = nullptr;     // [kBlendMaxFrames][kBlendW64Stride]
  int64_t blend_part_n = 0;
  float *mlp_z1 = nullptr, *mlp_z2 = nullptr, *mlp_dz1 = nullptr, *mlp_dz2 = nullptr;
  // host staging
  FrameDev* h_frames = nullptr;    // [kSlots][cap_frames] pinned
  hipEvent_t slot_ev[kSlots] = {};
  bool slot_used[kSlots] = {};
  int next_slot = 0;
  // bumped whenever a buffer that captured work may reference is freed and
  // allocated again; a graph records it and refuses to launch once it moved
  uint64_t alloc_gen = 0;
  StatusDev* h_status = nullptr;   // pinned: gbr_query_status's record
  StatusRec* h_ring = nullptr;     // pinned, coherent, [kStatusSlots]: the posted records
  StatusRec* d_ring = nullptr;     // the device's address of h_ring
  unsigned long long* d_posts = nullptr;   // posts the device has run
  int64_t posts = 0;               // posts enqueued (eagerly, or by launches of graphs holding them)
  int64_t capture_posts = 0;       // posts in the graph being captured
  // frame table of captured passes (host capture slot): whether the device
  // table holds it, and whether the graph being captured uses it
  bool frames_replay_ready = false;
  bool capture_uses_frames = false;
  int capture_frames_B = 0;
  hipStream_t post_stream = nullptr;   // the stream of the latest post
  // pass state
  bool capturing = false;
  bool have_pre = false, have_raster = false;
  bool cls_clean = false;          // tile-class counts cleared by the last enqueued pass start, not yet used
  int B = 0;
  int64_t n_splats = 0, n_pixels = 0, max_frame_splats = 0;
  int n_tiles = 0;
  const float* last_raw = nullptr;
  std::vector<FrameDev> frames_host;
  // kernel timing
  bool timing_on[GBR_K_COUNT] = {};
  hipEvent_t t_ev[GBR_K_COUNT][2] = {};
  bool t_recorded[GBR_K_COUNT] = {};       // an eager launch was bracketed since timing was enabled
  unsigned long long* t_stamp = nullptr;   // [GBR_K_COUNT][4]: start, sum of ticks, launches, unused
  int wall_khz = 0;                        // wall-clock rate of the device
  // tangent-space binding of the last pass (gbr_render_tangent); off for gbr_render
  TangentArgs tg{};
  // MLP state
  const float* mlp_theta = nullptr;
  int mlp_B = 0, mlp_din = 0, mlp_hidden = 0, mlp_K = 0;
  bool have_mlp = false;
};

struct gbr_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  gbr_ctx* ctx = nullptr;         // the context whose buffers the captured work uses
  uint64_t alloc_gen = 0;         // its allocation generation at capture
  int64_t posts = 0;              // status posts the graph holds
  bool uses_frames = false;       // a captured pass reads the capture slot's frame table
};

namespace {

PassArgs make_args(gbr_ctx* c) {
  PassArgs a;
  std::memset(&a, 0, sizeof(a));
  a.frames = c->d_frames;
  a.B = c->B;
  a.tile = c->tile;
  a.n_tiles = c->n_tiles;
  a.n_splats = c->n_splats;
  a.n_pixels = c->n_pixels;
  a.cap_entries = c->cap_entries;
  a.status = c->d_status;
  a.rec = c->rec; a.rect = c->rect; a.cnt = c->cnt; a.soff = c->soff; a.dkey = c->dkey;
  a.tile_count = c->tile_count; a.tile_start = c->tile_start;
  a.tile_last = c->tile_last; a.qlast = c->qlast;
  a.order_fwd = c->order_fwd; a.order_bwd = c->order_bwd; a.cls_cnt = c->cls_cnt;
  a.tbits = c->tbits; a.sorted = c->sorted; a.part_flag = c->part_flag; a.cmask = c->cmask;
  a.nbk = c->nbk;
  a.nblk = c->nblk;
  a.bitmap_words = (int32_t)(((c->max_frame_splats + 31) / 32 + 31) / 32 * 32);
  a.seg_words = c->seg_words;
  a.seg_stride = a.bitmap_words / a.seg_words;
  a.seg_cnt = c->seg_cnt;
  a.blk_mm = c->blk_mm; a.bkt_count = c->bkt_count; a.bkt_moff = c->bkt_moff; a.bkt_start = c->bkt_start;
  a.bkeys = c->bkeys; a.bkeys_alt = c->bkeys_alt; a.depth_sorted = c->depth_sorted; a.rank = c->rank;
  a.n_iter = c->n_iter; a.n_contrib = c->n_contrib; a.t_final = c->t_final; a.part = c->part;
  a.tg = c->tg;
  return a;
}

// Launch brackets of one kernel while its timing is enabled.
//  * Eagerly: a pair of HIP events on the launch stream, read by
//    gbr_timing_read (duration of the most recent launch).
//  * Always: two one-lane stamp kernels on the same stream that read the
//    GPU's constant-rate wall clock before and after the launch and add the
//    difference to a device accumulator (gbr_timing_accum). Stamp kernels are
//    ordinary launches, so a captured graph repeats them on every replay;
//    an event recorded during capture is only a dependency inside the graph
//    and keeps the timestamp of its last eager record.
__global__ void timer_stamp_kernel(unsigned long long* slot, int phase) {
  if (threadIdx.x != 0) return;
  const unsigned long long now = wall_clock64();
  if (phase == 0) {
    slot[0] = now;
  } else {
    slot[1] += now - slot[0];
    slot[2] += 1ULL;
  }
}

struct KTimer {
  gbr_ctx* c; int k; hipStream_t s; bool on;
  KTimer(gbr_ctx* c_, int k_, hipStream_t s_)
      : c(c_), k(k_), s(s_), on(k_ >= 0 && k_ < GBR_K_COUNT && c_->timing_on[k_]) {
    if (!on) return;
    timer_stamp_kernel<<<1, 64, 0, s>>>(c->t_stamp + 4 * k, 0);
    if (!c->capturing) (void)hipEventRecord(c->t_ev[k][0], s);   // events bracket the kernel alone
  }
  ~KTimer() {
    if (!on) return;
    if (!c->capturing) {
      (void)hipEventRecord(c->t_ev[k][1], s);
      c->t_recorded[k] = true;
    }
    timer_stamp_kernel<<<1, 64, 0, s>>>(c->t_stamp + 4 * k, 1);
  }
};

bool finite(float x) { return std::isfinite(x); }

int check_tiling(int tile, int chunk) {
  if (tile != 8 && tile != 16 && tile != 32) return GBR_ERR_INVALID_ARG;
  if (chunk != 64 && chunk != 128 && chunk != 256) return GBR_ERR_INVALID_ARG;
  return GBR_OK;
}

int alloc_entries(gbr_ctx* c, int64_t cap) {
  ++c->alloc_gen;
  dfree(c->sorted); dfree(c->part); dfree(c->part_flag); dfree(c->cmask);
  int rc = GBR_OK;
  if ((rc = dalloc(&c->sorted, cap))) return rc;
  if ((rc = dalloc(&c->part_flag, cap + 64))) return rc;   // gather reads 64-entry flag windows
  // every pass leaves the flags zero (the gather resets what it reads), so
  // they are cleared once here
  if (hipMemset(c->part_flag, 0, (size_t)cap + 64) != hipSuccess) return GBR_ERR_HIP;
  if ((rc = dalloc(&c->cmask, 4 * cap))) return rc;   // a byte per quadrant
  if ((rc = dalloc(&c->part, cap * kPartF))) return rc;
  c->cap_entries = cap;
  return GBR_OK;
}

int alloc_buckets(gbr_ctx* c, int64_t n, int64_t cells) {
  ++c->alloc_gen;
  dfree(c->bkt_count); dfree(c->bkt_moff); dfree(c->bkt_start);
  c->cap_bkt = 0; c->cap_bkt_cells = 0;
  int rc = GBR_OK;
  if ((rc = dalloc(&c->bkt_count, cells))) return rc;
  if ((rc = dalloc(&c->bkt_moff, cells + 1))) return rc;
  if ((rc = dalloc(&c->bkt_start, n + 1))) return rc;
  c->cap_bkt = n; c->cap_bkt_cells = cells;
  return GBR_OK;
}

void free_all(gbr_ctx* c) {
  dfree(c->d_frames); dfree(c->d_status); dfree(c->rec); dfree(c->rect); dfree(c->cnt); dfree(c->soff); dfree(c->dkey);
  dfree(c->tile_count); dfree(c->tile_start); dfree(c->tile_last); dfree(c->qlast); dfree(c->tbits); dfree(c->seg_cnt);
  dfree(c->order_fwd); dfree(c->order_bwd); dfree(c->cls_cnt);
  dfree(c->sorted); dfree(c->part); dfree(c->part_flag); dfree(c->cmask);
  dfree(c->blk_mm); dfree(c->bkt_count); dfree(c->bkt_moff); dfree(c->bkt_start);
  dfree(c->bkeys); dfree(c->bkeys_alt); dfree(c->depth_sorted); dfree(c->rank);
  dfree(c->n_iter); dfree(c->n_contrib); dfree(c->t_final); dfree(c->scan_scratch); dfree(c->scan_scratch_splat);
  dfree(c->draw_scratch);
  dfree(c->ci_ones); dfree(c->ci_draw);
  dfree(c->loss_part); dfree(c->blend_part); dfree(c->blend_w64);
  dfree(c->mlp_z1); dfree(c->mlp_z2); dfree(c->mlp_dz1); dfree(c->mlp_dz2);
  dfree(c->t_stamp);
  if (c->h_frames) (void)hipHostFree(c->h_frames);
  if (c->h_status) (void)hipHostFree(c->h_status);
  if (c->h_ring) (void)hipHostFree(c->h_ring);
  dfree(c->d_posts);
  c->h_frames = nullptr; c->h_status = nullptr; c->h_ring = nullptr; c->d_ring = nullptr;
  for (int i = 0; i < kSlots; ++i)
    if (c->slot_ev[i]) (void)hipEventDestroy(c->slot_ev[i]);
  for (int k = 0; k < GBR_K_COUNT; ++k)
    for (int j = 0; j < 2; ++j)
      if (c->t_ev[k][j]) (void)hipEventDestroy(c->t_ev[k][j]);
}

// Validates the frame list and fills the device frame table (host copy).
int build_frames(gbr_ctx* c, const int64_t* goff, const gbr_camera* cams, int B, std::vector<FrameDev>& out,
                 int* n_tiles, int64_t* n_pix, int64_t* n_spl, int64_t* max_fs) {
  if (B < 1 || !goff || !cams) return GBR_ERR_INVALID_ARG;
  if (B > c->cap_frames) return GBR_ERR_CAPACITY;
  if (goff[0] != 0) return GBR_ERR_INVALID_ARG;
  out.resize(B);
  int64_t tiles = 0, pix = 0, mfs = 0;
  for (int b = 0; b < B; ++b) {
    const gbr_camera& k = cams[b];
    if (goff[b + 1] < goff[b]) return GBR_ERR_INVALID_ARG;
    if (k.width < 1 || k.height < 1 || k.width > 16384 || k.height > 16384) return GBR_ERR_INVALID_ARG;
    if (!finite(k.fx) || !finite(k.fy) || !finite(k.cx) || !finite(k.cy) || k.fx == 0.f || k.fy == 0.f)
      return GBR_ERR_INVALID_ARG;
    for (int i = 0; i < 9; ++i) if (!finite(k.R[i])) return GBR_ERR_INVALID_ARG;
    for (int i = 0; i < 3; ++i) if (!finite(k.t[i]) || !finite(k.bg[i])) return GBR_ERR_INVALID_ARG;
    if (!finite(k.near_z) || k.near_z < 0.f) return GBR_ERR_INVALID_ARG;
    FrameDev& F = out[b];
    F.fx = k.fx; F.fy = k.fy; F.cx = k.cx; F.cy = k.cy;
    std::memcpy(F.R, k.R, sizeof(F.R));
    std::memcpy(F.t, k.t, sizeof(F.t));
    F.near_z = k.near_z;
    std::memcpy(F.bg, k.bg, sizeof(F.bg));
    F.W = k.width; F.H = k.height;
    F.ntx = (k.width + c->tile - 1) / c->tile;
    F.nty = (k.height + c->tile - 1) / c->tile;
    F.n_tiles = F.ntx * F.nty;
    F.tile_base = (int32_t)tiles;
    F.pix_base = pix;
    F.gauss_base = goff[b];
    F.gauss_count = goff[b + 1] - goff[b];
    tiles += F.n_tiles;
    pix += (int64_t)k.width * k.height;
    mfs = std::max(mfs, F.gauss_count);
  }
  if (goff[B] > c->cap_splats || pix > c->cap_pixels || tiles > c->cap_tiles) return GBR_ERR_CAPACITY;
  *n_tiles = (int)tiles; *n_pix = pix; *n_spl = goff[B]; *max_fs = mfs;
  return GBR_OK;
}

// The frame table of a pass.  Eagerly it goes up through one of the
// rotating host slots.  A captured pass leaves it in the capture slot and
// records no copy: gbr_graph_launch uploads that slot before a replay when
// the device table is not already it (after the capture, a restaging, or an
// eager pass), so an unchanged batch costs no copy per replay.
int stage_and_upload(gbr_ctx* c, hipStream_t s) {
  if (c->capturing) {
    std::memcpy(c->h_frames + (int64_t)kCaptureSlot * c->cap_frames, c->frames_host.data(), sizeof(FrameDev) * c->B);
    c->capture_frames_B = c->B;
    c->capture_uses_frames = true;
    c->frames_replay_ready = false;
    return GBR_OK;
  }
  const int slot = c->next_slot;
  c->next_slot = (c->next_slot + 1) % (kSlots - 1);
  if (c->slot_used[slot]) GBR_HIP(hipEventSynchronize(c->slot_ev[slot]));
  FrameDev* h = c->h_frames + (int64_t)slot * c->cap_frames;
  std::memcpy(h, c->frames_host.data(), sizeof(FrameDev) * c->B);
  GBR_HIP(hipMemcpyAsync(c->d_frames, h, sizeof(FrameDev) * c->B, hipMemcpyHostToDevice, s));
  GBR_HIP(hipEventRecord(c->slot_ev[slot], s));
  c->slot_used[slot] = true;
  c->frames_replay_ready = false;   // the device table is this pass's now
  return GBR_OK;
}

int enqueue_preprocess(gbr_ctx* c, const float* raw, hipStream_t s) {
  int rc = stage_and_upload(c, s);
  if (rc) return rc;
  PassArgs a = make_args(c);
  bool projected;
  {
    KTimer t(c, GBR_K_PREPROCESS, s);
    projected = launch_preprocess(a, raw, c->max_frame_splats, s);   // also clears the pass's counters
  }
  if (!projected) hipLaunchKernelGGL(begin_pass_kernel, dim3(1), dim3(256), 0, s, a);
  c->cls_clean = true;
  {
    KTimer t(c, GBR_K_DEPTH_ORDER, s);
    // the scan of the splats' tile counts (preprocess output) shares the bucket scan's launches
    const ScanJob splat_scan{c->cnt, c->soff, c->n_splats, c->scan_scratch_splat, -1, nullptr, nullptr, 1};
    launch_depth_order(a, c->max_frame_splats, c->scan_scratch, splat_scan, s);
  }
  {
    KTimer t(c, GBR_K_BINNING, s);
    launch_bitmap_rows(a, c->max_frame_splats, c->max_frame_tiles, s);
    launch_tile_count(a, s);
  }
  {
    KTimer t(c, GBR_K_TILE_SCAN, s);
    // the forward classification (by list length) runs in the scan's first launch
    launch_tile_scan_classify(a, c->scan_scratch, c->cap_entries, &c->d_status->entries, s);
  }
  GBR_HIP(hipGetLastError());
  c->last_raw = raw;
  c->have_pre = true;
  c->have_raster = false;
  return GBR_OK;
}

int enqueue_rasterize(gbr_ctx* c, float* images, hipStream_t s) {
  PassArgs a = make_args(c);
  {
    KTimer t(c, GBR_K_TILE_SORT, s);
    // the forward schedule was built with the tile scan; the backward one
    // starts empty: cleared at the pass start, or here when the pass is
    // rasterised again
    if (!c->cls_clean) launch_fill_u32(c->cls_cnt + 33, 0u, 33, s);
    c->cls_clean = false;
  }
  {
    KTimer t(c, GBR_K_COMPOSITE_FWD, s);
    launch_composite_fwd(a, images, c->chunk, s);
  }
  launch_classify_tiles(a, true, s);
  GBR_HIP(hipGetLastError());
  c->have_raster = true;
  return GBR_OK;
}

int set_pass(gbr_ctx* c, const float* raw, const int64_t* goff, const gbr_camera* cams, int B) {
  if (!raw) return GBR_ERR_INVALID_ARG;
  std::vector<FrameDev> fr;
  int nt; int64_t np, ns, mfs;
  int rc = build_frames(c, goff, cams, B, fr, &nt, &np, &ns, &mfs);
  if (rc) return rc;
  if ((mfs + 31) / 32 > kMaxBitmapWords) return GBR_ERR_CAPACITY;
  int nbk = 64;
  while (nbk < 8192 && (int64_t)nbk * 8 < mfs) nbk *= 2;
  const int nblk = (int)std::max<int64_t>(1, (mfs + kBucketBlock - 1) / kBucketBlock);
  if ((int64_t)B * nbk > c->cap_bkt || (int64_t)B * nbk * nblk > c->cap_bkt_cells) {
    if (c->capturing) return GBR_ERR_STATE;
    GBR_HIP(hipDeviceSynchronize());
    rc = alloc_buckets(c, (int64_t)B * nbk, (int64_t)B * nbk * nblk);
    if (rc) return rc;
  }
  const int64_t scan_words = scan_scratch_words((int64_t)B * nbk * nblk);
  if (scan_words > c->cap_scan_words) {   // the bucket-count matrix is the longest scan of a pass
    if (c->capturing) return GBR_ERR_STATE;
    GBR_HIP(hipDeviceSynchronize());
    ++c->alloc_gen;
    dfree(c->scan_scratch);
    c->cap_scan_words = 0;
    rc = dalloc(&c->scan_scratch, scan_words);
    if (rc) return rc;
    c->cap_scan_words = scan_words;
  }
  int mft = 0;
  for (const FrameDev& f : fr) mft = std::max(mft, f.n_tiles);
  const int64_t row_words = ((mfs + 31) / 32 + 31) / 32 * 32;
  const int seg_words = bitmap_seg_words(mft, row_words);
  const int64_t need_bits = std::max<int64_t>(1, (int64_t)nt * row_words);
  if (need_bits > c->cap_tbits) {
    if (c->capturing) return GBR_ERR_STATE;
    GBR_HIP(hipDeviceSynchronize());
    ++c->alloc_gen;
    dfree(c->tbits);
    c->cap_tbits = 0;
    rc = dalloc(&c->tbits, need_bits);
    if (rc) return rc;
    c->cap_tbits = need_bits;
  }
  const int64_t need_seg = std::max<int64_t>(1, (int64_t)nt * (row_words / seg_words));
  if (need_seg > c->cap_seg) {
    if (c->capturing) return GBR_ERR_STATE;
    GBR_HIP(hipDeviceSynchronize());
    ++c->alloc_gen;
    dfree(c->seg_cnt);
    c->cap_seg = 0;
    rc = dalloc(&c->seg_cnt, need_seg);
    if (rc) return rc;
    c->cap_seg = need_seg;
  }
  c->frames_host.swap(fr);
  c->B = B; c->n_tiles = nt; c->n_pixels = np; c->n_splats = ns; c->max_frame_splats = mfs;
  c->nbk = nbk;
  c->nblk = nblk;
  c->seg_words = seg_words;
  c->max_frame_tiles = mft;
  return GBR_OK;
}

// Device bytes of a context's workspace from its capacities: the sizes
// gbr_create allocates, grown by a pass (depth buckets, scan scratch, tile
// bitmap rows and their segment counts) and by gbr_reserve (entries).  One
// formula serves gbr_memory (a context's current bytes) and gbr_plan_bytes
// (what a context sized for a batch would hold).
struct WorkspaceCaps {
  int64_t frames, splats, pixels, tiles, entries, bkt, bkt_cells, scan_words, tbits, seg, ci_pixels, ci_splats;
  bool timing;
};

int64_t workspace_bytes(const WorkspaceCaps& k) {
  auto n = [](int64_t c) { return c < 1 ? (int64_t)1 : c; };   // dalloc allocates at least one element
  int64_t b = 0;
  b += n(k.frames) * (int64_t)sizeof(FrameDev) + (int64_t)sizeof(StatusDev) + 8;   // + the post counter
  b += n(k.splats * kRecF) * 4 + n(k.splats) * 16 + n(k.splats) * 4 + n(k.splats + 1) * 4 + n(k.splats) * 4;
  b += (n(k.tiles) + n(k.tiles + 1) + n(k.tiles) + n(4 * k.tiles) + 2 * n(33 * k.tiles)) * 4 + 66 * 4;
  b += n(2 * ((int64_t)div_up(k.splats, 256) + k.frames + 1)) * 4;   // projection workgroups' depth ranges
  b += (n(k.splats) * 2) * 8 + n(k.splats) * 4 * 2;                       // bucket keys, order, rank
  b += (n(k.bkt_cells) + n(k.bkt_cells + 1) + n(k.bkt + 1)) * 4;  // depth buckets
  b += 3 * n(k.pixels) * 4;                                                  // n_iter, n_contrib, t_final
  b += n(k.scan_words) * 4 + n(scan_scratch_words(k.splats)) * 4 + n(k.splats * kNF) * 4;
  b += n(2 * loss_partials(3 * k.pixels) + 2) * 4;
  b += n(4 * k.splats + 4096LL * k.frames + 64LL * 64 * 8) * 4;
  b += (int64_t)kBlendMaxFrames * kBlendW64Stride * 8 + 4 * n(k.frames * 1024) * 4;
  b += n(k.entries) * 4 + n(k.entries + 64) + n(4 * k.entries) + n(k.entries * kPartF) * 4;   // sorted, flags, cmask, part
  b += n(k.tbits) * 4 + n(k.seg) * 2;
  if (k.ci_pixels) b += n(3 * k.ci_pixels) * 4 + n(k.ci_splats * kNF) * 4;
  if (k.timing) b += 4 * GBR_K_COUNT * 8;
  return b;
}

// The pass-dependent capacities for frames of up to mfs splats (bucket
// count and blocks as set_pass chooses them) over n_tiles tiles, the largest
// frame having max_frame_tiles.
void pass_caps(int B, int64_t mfs, int64_t n_tiles, int max_frame_tiles, int64_t* bkt, int64_t* cells,
               int64_t* scan_words, int64_t* tbits, int64_t* seg) {
  int nbk = 64;
  while (nbk < 8192 && (int64_t)nbk * 8 < mfs) nbk *= 2;
  const int64_t nblk = std::max<int64_t>(1, (mfs + kBucketBlock - 1) / kBucketBlock);
  *bkt = (int64_t)B * nbk;
  *cells = (int64_t)B * nbk * nblk;
  *scan_words = scan_scratch_words(*cells);
  const int64_t row_words = ((mfs + 31) / 32 + 31) / 32 * 32;
  const int sw = bitmap_seg_words(max_frame_tiles, row_words);
  *tbits = std::max<int64_t>(1, n_tiles * row_words);
  *seg = std::max<int64_t>(1, n_tiles * (row_words / sw));
}

WorkspaceCaps caps_at_create(const gbr_config* cfg) {
  WorkspaceCaps k{};
  k.frames = cfg->max_frames;
  k.splats = cfg->max_splats;
  k.pixels = cfg->max_pixels;
  const int64_t edge = 2 * (int64_t)std::ceil(std::sqrt((double)cfg->max_pixels)) / 8 + 1;
  k.tiles = cfg->max_pixels / 64 + (int64_t)cfg->max_frames * (2 * edge + 1);
  k.entries = cfg->max_entries;
  k.bkt = 64LL * cfg->max_frames;
  k.bkt_cells = 64LL * cfg->max_frames;
  k.scan_words = scan_scratch_words(std::max<int64_t>(std::max<int64_t>(k.splats, k.tiles), 8192LL * k.frames));
  k.tbits = 0;
  k.seg = 0;
  return k;
}

}  // namespace

extern "C" {

const char* gbr_strerror(int code) {
  switch (code) {
    case GBR_OK: return "ok";
    case GBR_ERR_INVALID_ARG: return "invalid argument";
    case GBR_ERR_CAPACITY: return "capacity exceeded (frames, splats, pixels or tiles)";
    case GBR_ERR_OOM: return "device out of memory";
    case GBR_ERR_HIP: return "HIP runtime error";
    case GBR_ERR_STATE: return "call out of order (no preceding render/forward)";
    case GBR_ERR_OVERFLOW: return "tile-entry capacity overflowed in the last pass";
    default: return "unknown error";
  }
}

int gbr_create(const gbr_config* cfg, gbr_ctx** out) {
  if (!cfg || !out) return GBR_ERR_INVALID_ARG;
  *out = nullptr;
  if (check_tiling(cfg->tile, cfg->chunk)) return GBR_ERR_INVALID_ARG;
  if (cfg->max_frames < 1 || cfg->max_frames > kMaxFramesHard || cfg->max_splats < 1 || cfg->max_pixels < 1 ||
      cfg->max_entries < 1 || cfg->max_splats >= (int64_t)UINT32_MAX || cfg->max_entries >= (int64_t)UINT32_MAX)
    return GBR_ERR_INVALID_ARG;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || cfg->device < 0 || cfg->device >= ndev) return GBR_ERR_HIP;
  if (hipSetDevice(cfg->device) != hipSuccess) return GBR_ERR_HIP;
  gbr_ctx* c = new gbr_ctx();
  c->cfg = *cfg;
  c->tile = cfg->tile; c->chunk = cfg->chunk;
  c->cap_frames = cfg->max_frames;
  c->cap_splats = cfg->max_splats;
  c->cap_pixels = cfg->max_pixels;
  // tiles at the smallest tile size, plus partial edge tiles of every frame
  c->cap_tiles = caps_at_create(cfg).tiles;
  int rc = GBR_OK;
#define TRY(x) do { if ((rc = (x))) { free_all(c); delete c; return rc; } } while (0)
  TRY(dalloc(&c->d_frames, c->cap_frames));
  TRY(dalloc(&c->d_status, 1));
  TRY(dalloc(&c->rec, c->cap_splats * kRecF));
  TRY(dalloc(&c->rect, c->cap_splats));
  TRY(dalloc(&c->cnt, c->cap_splats));
  TRY(dalloc(&c->soff, c->cap_splats + 1));
  TRY(dalloc(&c->dkey, c->cap_splats));
  TRY(dalloc(&c->tile_count, c->cap_tiles));
  TRY(dalloc(&c->tile_start, c->cap_tiles + 1));
  TRY(dalloc(&c->tile_last, c->cap_tiles));
  TRY(dalloc(&c->qlast, 4 * c->cap_tiles));
  TRY(dalloc(&c->order_fwd, 33 * c->cap_tiles));
  TRY(dalloc(&c->order_bwd, 33 * c->cap_tiles));
  TRY(dalloc(&c->cls_cnt, 66));
  TRY(dalloc(&c->blk_mm, 2 * ((int64_t)div_up(c->cap_splats, 256) + c->cap_frames + 1)));
  TRY(dalloc(&c->bkeys, c->cap_splats));
  TRY(dalloc(&c->bkeys_alt, c->cap_splats));
  TRY(dalloc(&c->depth_sorted, c->cap_splats));
  TRY(dalloc(&c->rank, c->cap_splats));
  TRY(alloc_buckets(c, 64LL * c->cap_frames, 64LL * c->cap_frames));
  TRY(dalloc(&c->n_iter, c->cap_pixels));
  TRY(dalloc(&c->n_contrib, c->cap_pixels));
  TRY(dalloc(&c->t_final, c->cap_pixels));
  c->cap_scan_words = scan_scratch_words(std::max<int64_t>(std::max<int64_t>(c->cap_splats, c->cap_tiles),
                                                            (int64_t)8192 * c->cap_frames));
  TRY(dalloc(&c->scan_scratch, c->cap_scan_words));
  TRY(dalloc(&c->scan_scratch_splat, scan_scratch_words(c->cap_splats)));
  TRY(dalloc(&c->draw_scratch, c->cap_splats * kNF));
  TRY(dalloc(&c->loss_part, 2 * loss_partials(3 * c->cap_pixels) + 2));
  c->blend_part_n = 4 * c->cap_splats + 4096LL * c->cap_frames + 64LL * 64 * 8;
  TRY(dalloc(&c->blend_part, c->blend_part_n));
  TRY(dalloc(&c->blend_w64, (int64_t)kBlendMaxFrames * kBlendW64Stride));
  TRY(dalloc(&c->mlp_z1, (int64_t)c->cap_frames * 1024));
  TRY(dalloc(&c->mlp_z2, (int64_t)c->cap_frames * 1024));
  TRY(dalloc(&c->mlp_dz1, (int64_t)c->cap_frames * 1024));
  TRY(dalloc(&c->mlp_dz2, (int64_t)c->cap_frames * 1024));
  TRY(alloc_entries(c, cfg->max_entries));
  if (hipHostMalloc(reinterpret_cast<void**>(&c->h_frames), sizeof(FrameDev) * kSlots * c->cap_frames,
                    hipHostMallocDefault) != hipSuccess) TRY(GBR_ERR_OOM);
  if (hipHostMalloc(reinterpret_cast<void**>(&c->h_status), sizeof(StatusDev), hipHostMallocDefault) != hipSuccess)
    TRY(GBR_ERR_OOM);
  if (hipHostMalloc(reinterpret_cast<void**>(&c->h_ring), sizeof(StatusRec) * kStatusSlots,
                    hipHostMallocCoherent) != hipSuccess)
    TRY(GBR_ERR_OOM);
  std::memset(c->h_ring, 0, sizeof(StatusRec) * kStatusSlots);
  if (hipHostGetDevicePointer(reinterpret_cast<void**>(&c->d_ring), c->h_ring, 0) != hipSuccess) TRY(GBR_ERR_HIP);
  TRY(dalloc(&c->d_posts, 1));
  if (hipMemset(c->d_posts, 0, sizeof(unsigned long long)) != hipSuccess) TRY(GBR_ERR_HIP);
  for (int i = 0; i < kSlots; ++i)
    if (hipEventCreateWithFlags(&c->slot_ev[i], hipEventDisableTiming) != hipSuccess) TRY(GBR_ERR_HIP);
  StatusDev zero;
  std::memset(&zero, 0, sizeof(zero));
  if (hipMemcpy(c->d_status, &zero, sizeof(zero), hipMemcpyHostToDevice) != hipSuccess) TRY(GBR_ERR_HIP);
#undef TRY
  *out = c;
  return GBR_OK;
}

int gbr_destroy(gbr_ctx* c) {
  if (!c) return GBR_ERR_INVALID_ARG;
  (void)hipSetDevice(c->cfg.device);
  (void)hipDeviceSynchronize();
  free_all(c);
  delete c;
  return GBR_OK;
}

int gbr_memory(gbr_ctx* c, int64_t* device_bytes) {
  if (!c || !device_bytes) return GBR_ERR_INVALID_ARG;
  WorkspaceCaps k{};
  k.frames = c->cap_frames; k.splats = c->cap_splats; k.pixels = c->cap_pixels; k.tiles = c->cap_tiles;
  k.entries = c->cap_entries; k.bkt = c->cap_bkt; k.bkt_cells = c->cap_bkt_cells; k.scan_words = c->cap_scan_words;
  k.tbits = c->cap_tbits; k.seg = c->cap_seg;
  k.ci_pixels = c->ci_ones ? c->cap_pixels : 0;
  k.ci_splats = c->ci_ones ? c->cap_splats : 0;
  k.timing = c->t_stamp != nullptr;
  *device_bytes = workspace_bytes(k);
  return GBR_OK;
}

int gbr_plan_bytes(const gbr_config* cfg, int32_t B, const int64_t* gauss_offsets, const int32_t* widths,
                   const int32_t* heights, int64_t entries, int64_t* device_bytes) {
  if (!cfg || !gauss_offsets || !widths || !heights || !device_bytes || B < 1 || B > cfg->max_frames ||
      entries < 0 || check_tiling(cfg->tile, cfg->chunk))
    return GBR_ERR_INVALID_ARG;
  WorkspaceCaps k = caps_at_create(cfg);
  int64_t mfs = 0, n_tiles = 0, pix = 0;
  int mft = 0;
  for (int b = 0; b < B; ++b) {
    const int64_t nb = gauss_offsets[b + 1] - gauss_offsets[b];
    if (nb < 0 || widths[b] < 1 || heights[b] < 1) return GBR_ERR_INVALID_ARG;
    mfs = std::max(mfs, nb);
    const int t = ((widths[b] + cfg->tile - 1) / cfg->tile) * ((heights[b] + cfg->tile - 1) / cfg->tile);
    n_tiles += t;
    mft = std::max(mft, t);
    pix += (int64_t)widths[b] * heights[b];
  }
  if (gauss_offsets[B] > cfg->max_splats || pix > cfg->max_pixels || n_tiles > k.tiles) return GBR_ERR_CAPACITY;
  int64_t bkt, cells, scan_words, tbits, seg;
  pass_caps(B, mfs, n_tiles, mft, &bkt, &cells, &scan_words, &tbits, &seg);
  // a pass grows a buffer only beyond its current capacity
  if (bkt > k.bkt || cells > k.bkt_cells) { k.bkt = bkt; k.bkt_cells = cells; }
  k.scan_words = std::max(k.scan_words, scan_words);
  k.tbits = tbits;
  k.seg = seg;
  k.entries = std::max(k.entries, entries);
  *device_bytes = workspace_bytes(k);
  return GBR_OK;
}

int gbr_reserve(gbr_ctx* c, int64_t max_entries) {
  if (!c || max_entries < 1 || max_entries >= (int64_t)UINT32_MAX) return GBR_ERR_INVALID_ARG;
  if (c->capturing) return GBR_ERR_STATE;
  if (max_entries <= c->cap_entries) return GBR_OK;
  GBR_HIP(hipDeviceSynchronize());
  int rc = alloc_entries(c, max_entries);
  c->have_raster = false;
  return rc;
}

int gbr_set_tiling(gbr_ctx* c, int32_t tile, int32_t chunk) {
  if (!c || check_tiling(tile, chunk)) return GBR_ERR_INVALID_ARG;
  if (c->capturing) return GBR_ERR_STATE;
  c->tile = tile; c->chunk = chunk;
  c->have_pre = c->have_raster = false;
  return GBR_OK;
}

int gbr_blend(gbr_ctx* c, const float* bases, const float* weights, int32_t B, int32_t K, int64_t N, float* raw,
              void* stream) {
  if (!c || !bases || !raw || B < 1 || B > kBlendMaxFrames || K < 0 || K > kMaxK || N < 1 || (K > 0 && !weights))
    return GBR_ERR_INVALID_ARG;
  {
    KTimer t(c, GBR_K_BLEND, (hipStream_t)stream);
    launch_blend_fwd(bases, weights, B, K, N, raw, c->blend_w64, (hipStream_t)stream);
  }
  GBR_HIP(hipGetLastError());
  return GBR_OK;
}

static int preprocess_impl(gbr_ctx* c, const float* raw, const int64_t* goff, const gbr_camera* cams, int32_t B,
                           void* stream) {
  int rc = set_pass(c, raw, goff, cams, B);
  if (rc) return rc;
  return enqueue_preprocess(c, raw, (hipStream_t)stream);
}

int gbr_preprocess(gbr_ctx* c, const float* raw, const int64_t* goff, const gbr_camera* cams, int32_t B,
                   void* stream) {
  if (!c) return GBR_ERR_INVALID_ARG;
  c->tg.on = 0;
  return preprocess_impl(c, raw, goff, cams, B, stream);
}

int gbr_entry_count(gbr_ctx* c, void* stream, int64_t* entries) {
  if (!c || !entries) return GBR_ERR_INVALID_ARG;
  if (!c->have_pre) return GBR_ERR_STATE;
  if (c->capturing) return GBR_ERR_STATE;
  hipStream_t s = (hipStream_t)stream;
  GBR_HIP(hipMemcpyAsync(c->h_status, c->d_status, sizeof(StatusDev), hipMemcpyDeviceToHost, s));
  GBR_HIP(hipStreamSynchronize(s));
  *entries = (int64_t)c->h_status->entries;
  if (*entries > c->cap_entries) {
    int rc = gbr_reserve(c, *entries + *entries / 4 + 1024);
    if (rc) return rc;
    hipLaunchKernelGGL(clear_overflow_kernel, dim3(1), dim3(1), 0, s, c->d_status);
    GBR_HIP(hipGetLastError());
  }
  return GBR_OK;
}

int gbr_rasterize(gbr_ctx* c, float* images, void* stream) {
  if (!c || !images) return GBR_ERR_INVALID_ARG;
  if (!c->have_pre) return GBR_ERR_STATE;
  return enqueue_rasterize(c, images, (hipStream_t)stream);
}

int gbr_render(gbr_ctx* c, const float* raw, const int64_t* goff, const gbr_camera* cams, int32_t B, float* images,
               void* stream) {
  if (!c || !images) return GBR_ERR_INVALID_ARG;
  c->tg.on = 0;
  int rc = preprocess_impl(c, raw, goff, cams, B, stream);
  if (rc) return rc;
  return enqueue_rasterize(c, images, (hipStream_t)stream);
}

int gbr_render_tangent(gbr_ctx* c, const float* raw_t, const int32_t* tri, const float* bary, const float* verts,
                       const int32_t* faces, const float* frames, int64_t N, int32_t V, int32_t F,
                       const gbr_camera* cams, int32_t B, float* images, void* stream) {
  if (!c || !raw_t || !tri || !bary || !verts || !faces || !frames || !images || N < 1 || V < 1 || F < 1 || B < 1)
    return GBR_ERR_INVALID_ARG;
  if ((int64_t)B * N > c->cap_splats) return GBR_ERR_CAPACITY;
  std::vector<int64_t> goff(B + 1);
  for (int b = 0; b <= B; ++b) goff[b] = (int64_t)b * N;
  c->tg = TangentArgs{tri, bary, verts, faces, frames, N, V, F, 1, 0};
  int rc = preprocess_impl(c, raw_t, goff.data(), cams, B, stream);
  if (rc) {
    c->tg.on = 0;
    return rc;
  }
  return enqueue_rasterize(c, images, (hipStream_t)stream);
}

int gbr_render_backward(gbr_ctx* c, const float* dimages, float* draw, void* stream) {
  if (!c || !dimages || !draw) return GBR_ERR_INVALID_ARG;
  if (!c->have_raster) return GBR_ERR_STATE;
  hipStream_t s = (hipStream_t)stream;
  PassArgs a = make_args(c);
  {
    KTimer t(c, GBR_K_COMPOSITE_BWD, s);
    launch_composite_bwd(a, dimages, nullptr, c->chunk, s);
  }
  {
    KTimer t(c, GBR_K_GATHER_BWD, s);
    launch_gather_bwd(a, c->last_raw, draw, c->max_frame_splats, s);
  }
  GBR_HIP(hipGetLastError());
  return GBR_OK;
}

int gbr_blend_backward(gbr_ctx* c, const float* draw, const float* bases, const float* weights, int32_t B,
                       int32_t K, int64_t N, float* dbases, float* dweights, int32_t accumulate, void* stream) {
  if (!c || !draw || !bases || B < 1 || B > 64 || K < 0 || K > kMaxK || N < 1) return GBR_ERR_INVALID_ARG;
  if (K > 0 && (!weights || !dweights)) return GBR_ERR_INVALID_ARG;
  if ((int64_t)B * N > c->cap_splats) return GBR_ERR_CAPACITY;
  if (blend_bwd_partials(B, K, N) > c->blend_part_n) return GBR_ERR_CAPACITY;
  {
    KTimer t(c, GBR_K_BLEND_BWD, (hipStream_t)stream);
    launch_blend_bwd(draw, bases, weights, B, K, N, dbases, dweights, c->blend_part, c->blend_part_n, accumulate,
                     (hipStream_t)stream);
  }
  GBR_HIP(hipGetLastError());
  return GBR_OK;
}

int gbr_blend_backward_noalloc(const float* draw, const float* bases, const float* weights, int32_t B, int32_t K,
                               int64_t N, float* dbases, float* dweights, int32_t accumulate, void* stream) {
  if (!draw || !bases || B < 1 || B > 64 || K < 0 || K > kMaxK || N < 1) return GBR_ERR_INVALID_ARG;
  if (K > 0 && (!weights || !dweights)) return GBR_ERR_INVALID_ARG;
  if (N > (int64_t)INT32_MAX / kNF) return GBR_ERR_INVALID_ARG;
  if (blend_bwd_partials_used(B, K, N) > kNoAllocScratchFloats) return GBR_ERR_CAPACITY;
  float* part = nullptr;
  const int rc = scratch_of_current_device(&part);
  if (rc) return rc;
  launch_blend_bwd(draw, bases, weights, B, K, N, dbases, dweights, part, kNoAllocScratchFloats, accumulate,
                   (hipStream_t)stream);
  GBR_HIP(hipGetLastError());
  return GBR_OK;
}

int gbr_backward(gbr_ctx* c, const float* dimages, const float* bases, const float* weights, int32_t K,
                 float* dbases, float* dweights, void* stream) {
  if (!c) return GBR_ERR_INVALID_ARG;
  if (!c->have_raster) return GBR_ERR_STATE;
  const int64_t N = c->frames_host.empty() ? 0 : c->frames_host[0].gauss_count;
  for (int b = 0; b < c->B; ++b)
    if (c->frames_host[b].gauss_count != N || c->frames_host[b].gauss_base != (int64_t)b * N)
      return GBR_ERR_INVALID_ARG;
  int rc = gbr_render_backward(c, dimages, c->draw_scratch, stream);
  if (rc) return rc;
  return gbr_blend_backward(c, c->draw_scratch, bases, weights, c->B, K, N, dbases, dweights, 0, stream);
}

int gbr_blend_adam_step(gbr_ctx* c, int32_t group, const float* draw, const float* weights, int32_t B, int32_t K,
                        int64_t N, float* bases, float* m, float* v, const float* lr_table, float beta1, float beta2,
                        float eps, void* stream) {
  if (!c || group < 0 || group > 3 || !draw || !bases || !m || !v || !lr_table || B < 1 || B > 64 || K < 0 ||
      K > kMaxK || N < 1 || (K > 0 && !weights))
    return GBR_ERR_INVALID_ARG;
  if ((int64_t)B * N > c->cap_splats) return GBR_ERR_CAPACITY;
  if (!(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f && eps >= 0.f)) return GBR_ERR_INVALID_ARG;
  for (int i = 0; i < 32; ++i)
    if (!finite(lr_table[i])) return GBR_ERR_INVALID_ARG;
  {
    KTimer t(c, GBR_K_ADAM, (hipStream_t)stream);
    launch_blend_adam(draw, weights, B, K, N, bases, m, v, c->d_status, group, lr_table, beta1, beta2, eps,
                      (hipStream_t)stream);
  }
  GBR_HIP(hipGetLastError());
  return GBR_OK;
}

int gbr_tangent_frames(gbr_ctx* c, const float* verts, const int32_t* faces, const float* face_uv, int32_t B,
                       int32_t V, int32_t F, float* frames, void* stream) {
  if (!c || !verts || !faces || !face_uv || !frames || B < 1 || V < 3 || F < 1) return GBR_ERR_INVALID_ARG;
  launch_tangent_frames(verts, faces, face_uv, B, V, F, frames, (hipStream_t)stream);
  GBR_HIP(hipGetLastError());
  return GBR_OK;
}

int gbr_tangent_transform(gbr_ctx* c, const float* raw_t, const int32_t* tri, const float* bary, const float* verts,
                          const int32_t* faces, const float* frames, int32_t B, int64_t N, int32_t V, int32_t F,
                          float* raw_d, void* stream) {
  if (!c || !raw_t || !tri || !bary || !verts || !faces || !frames || !raw_d || B < 1 || N < 1 || V < 3 || F < 1)
    return GBR_ERR_INVALID_ARG;
  launch_tangent_fwd(raw_t, tri, bary, verts, faces, frames, B, N, V, F, raw_d, (hipStream_t)stream);
  GBR_HIP(hipGetLastError());
  return GBR_OK;
}

int gbr_tangent_backward(gbr_ctx* c, const float* draw_d, const int32_t* tri, const float* frames, int32_t B,
                         int64_t N, int32_t F, float* draw_t, void* stream) {
  if (!c || !draw_d || !tri || !frames || !draw_t || B < 1 || N < 1 || F < 1) return GBR_ERR_INVALID_ARG;
  launch_tangent_bwd(draw_d, tri, frames, B, N, F, draw_t, (hipStream_t)stream);
  GBR_HIP(hipGetLastError());
  return GBR_OK;
}

int gbr_color_init(gbr_ctx* c, const float* targets, float* bases, float delta, uint8_t* done, void* stream) {
  if (!c || !targets || !bases || !done || !(delta >= 0.0f)) return GBR_ERR_INVALID_ARG;
  if (!c->have_raster) return GBR_ERR_STATE;
  const int64_t N = c->frames_host.empty() ? 0 : c->frames_host[0].gauss_count;
  for (int b = 0; b < c->B; ++b)
    if (c->frames_host[b].gauss_count != N || c->frames_host[b].gauss_base != (int64_t)b * N)
      return GBR_ERR_INVALID_ARG;
  if (c->capturing) return GBR_ERR_STATE;
  if (!c->ci_ones) {
    GBR_HIP(hipDeviceSynchronize());
    int rc = dalloc(&c->ci_ones, 3 * c->cap_pixels);
    if (!rc) rc = dalloc(&c->ci_draw, c->cap_splats * kNF);
    if (rc) { dfree(c->ci_ones); dfree(c->ci_draw); return rc; }
  }
  hipStream_t s = (hipStream_t)stream;
  launch_fill_f32(c->ci_ones, 1.0f, 3 * c->n_pixels, s);
  int rc = gbr_render_backward(c, targets, c->draw_scratch, stream);
  if (rc) return rc;
  rc = gbr_render_backward(c, c->ci_ones, c->ci_draw, stream);
  if (rc) return rc;
  launch_color_init_apply(c->draw_scratch, c->ci_draw, c->B, N, delta, bases, done, s);
  GBR_HIP(hipGetLastError());
  return GBR_OK;
}

int gbr_loss(gbr_ctx* c, const float* images, const float* targets, int32_t kind, float* dimages, void* stream) {
  if (!c || !images || !targets || !dimages || (kind != 1 && kind != 2)) return GBR_ERR_INVALID_ARG;
  if (!c->have_pre) return GBR_ERR_STATE;
  PassArgs a = make_args(c);
  {
    KTimer t(c, GBR_K_LOSS, (hipStream_t)stream);
    launch_loss(a, images, targets, kind, dimages, c->loss_part, 0, (hipStream_t)stream);
  }
  GBR_HIP(hipGetLastError());
  return GBR_OK;
}

int gbr_mlp_forward(gbr_ctx* c, const float* params, const float* theta, int32_t B, int32_t d_in, int32_t hidden,
                    int32_t K, float* psi, void* stream) {
  if (!c || !params || !theta || !psi || B < 1 || d_in < 1 || d_in > 1024 || hidden < 1 || hidden > 1024 || K < 1 ||
      K > 64)
    return GBR_ERR_INVALID_ARG;
  if (B > c->cap_frames) return GBR_ERR_CAPACITY;
  {
    KTimer t(c, GBR_K_MLP, (hipStream_t)stream);
    launch_mlp_fwd(params, theta, B, d_in, hidden, K, psi, c->mlp_z1, c->mlp_z2, (hipStream_t)stream);
  }
  GBR_HIP(hipGetLastError());
  c->mlp_theta = theta; c->mlp_B = B; c->mlp_din = d_in; c->mlp_hidden = hidden; c->mlp_K = K;
  c->have_mlp = true;
  return GBR_OK;
}

int gbr_mlp_backward(gbr_ctx* c, const float* params, const float* dpsi, float* dparams, void* stream) {
  if (!c || !params || !dpsi || !dparams) return GBR_ERR_INVALID_ARG;
  if (!c->have_mlp) return GBR_ERR_STATE;
  {
    KTimer t(c, GBR_K_MLP, (hipStream_t)stream);
    launch_mlp_bwd(params, c->mlp_theta, c->mlp_z1, c->mlp_z2, dpsi, c->mlp_B, c->mlp_din, c->mlp_hidden,
                   c->mlp_K, c->mlp_dz1, c->mlp_dz2, dparams, (hipStream_t)stream);
  }
  GBR_HIP(hipGetLastError());
  return GBR_OK;
}

int gbr_adam_step(gbr_ctx* c, int32_t group, float* params, const float* grads, float* m, float* v, int64_t n,
                  int64_t split, const float* lr_table, float beta1, float beta2, float eps, void* stream) {
  if (!c || group < 0 || group > 3 || n < 0 || !lr_table || (n > 0 && (!params || !grads || !m || !v)))
    return GBR_ERR_INVALID_ARG;
  if (!(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f && eps >= 0.f)) return GBR_ERR_INVALID_ARG;
  for (int i = 0; i < 32; ++i)
    if (!finite(lr_table[i])) return GBR_ERR_INVALID_ARG;
  {
    KTimer t(c, group == 0 ? GBR_K_ADAM : GBR_K_COUNT, (hipStream_t)stream);
    launch_adam(c->d_status, group, params, grads, m, v, n, split, lr_table, beta1, beta2, eps,
                (hipStream_t)stream);
  }
  GBR_HIP(hipGetLastError());
  return GBR_OK;
}

static void fill_status(const gbr_ctx* c, const StatusDev& h, gbr_status* out) {
  out->entries = (int64_t)h.entries;
  out->entries_capacity = c->cap_entries;
  out->overflow = (int32_t)h.overflow;
  for (int i = 0; i < 4; ++i) out->adam_steps[i] = h.adam_step[i];
  out->loss = h.loss;
}

int gbr_query_status(gbr_ctx* c, void* stream, gbr_status* out) {
  if (!c || !out) return GBR_ERR_INVALID_ARG;
  if (c->capturing) return GBR_ERR_STATE;
  hipStream_t s = (hipStream_t)stream;
  GBR_HIP(hipMemcpyAsync(c->h_status, c->d_status, sizeof(StatusDev), hipMemcpyDeviceToHost, s));
  GBR_HIP(hipStreamSynchronize(s));
  fill_status(c, *c->h_status, out);
  return GBR_OK;
}

int gbr_status_post(gbr_ctx* c, void* stream) {
  if (!c) return GBR_ERR_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(status_post_kernel, dim3(1), dim3(1), 0, s, c->d_status, c->d_ring, c->d_posts);
  GBR_HIP(hipGetLastError());
  if (c->capturing) {
    ++c->capture_posts;
  } else {
    ++c->posts;
    c->post_stream = s;
  }
  return GBR_OK;
}

int gbr_status_posts(gbr_ctx* c, int64_t* n) {
  if (!c || !n) return GBR_ERR_INVALID_ARG;
  *n = c->posts;
  return GBR_OK;
}

int gbr_status_wait(gbr_ctx* c, int64_t n, gbr_status* out) {
  if (!c || !out || n < 1) return GBR_ERR_INVALID_ARG;
  if (n > c->posts) return GBR_ERR_STATE;   // never enqueued: it would not arrive
  StatusRec* r = c->h_ring + n % kStatusSlots;
  const unsigned long long want = (unsigned long long)n;
  for (uint64_t spin = 1;; ++spin) {
    unsigned long long seq = __atomic_load_n(&r->seq, __ATOMIC_ACQUIRE);
    if (seq == want) {
      StatusDev st;
      std::memcpy(&st, (const void*)&r->st, sizeof(st));
      __atomic_thread_fence(__ATOMIC_ACQUIRE);
      if (__atomic_load_n(&r->seq, __ATOMIC_ACQUIRE) != want) return GBR_ERR_STATE;   // overwritten meanwhile
      fill_status(c, st, out);
      return GBR_OK;
    }
    if (seq > want) return GBR_ERR_STATE;   // overwritten: more than kStatusSlots posts ahead of the waits
    if (spin % 4096 == 0) {                  // the stream's state: an error, or done without this post
      const hipError_t q = hipStreamQuery(c->post_stream);
      if (q == hipSuccess) {
        if (__atomic_load_n(&r->seq, __ATOMIC_ACQUIRE) == want) continue;
        return GBR_ERR_STATE;
      }
      if (q != hipErrorNotReady) {
        (void)hipGetLastError();
        return GBR_ERR_HIP;
      }
    }
    __builtin_ia32_pause();
  }
}

int gbr_stage_frames(gbr_ctx* c, const int64_t* goff, const gbr_camera* cams, int32_t B) {
  if (!c) return GBR_ERR_INVALID_ARG;
  if (!c->have_pre || B != c->B) return GBR_ERR_STATE;
  std::vector<FrameDev> fr;
  int nt; int64_t np, ns, mfs;
  int rc = build_frames(c, goff, cams, B, fr, &nt, &np, &ns, &mfs);
  if (rc) return rc;
  for (int b = 0; b < B; ++b) {
    const FrameDev &x = fr[b], &y = c->frames_host[b];
    if (x.W != y.W || x.H != y.H || x.gauss_base != y.gauss_base || x.gauss_count != y.gauss_count)
      return GBR_ERR_INVALID_ARG;
  }
  c->frames_host.swap(fr);
  std::memcpy(c->h_frames + (int64_t)kCaptureSlot * c->cap_frames, c->frames_host.data(), sizeof(FrameDev) * B);
  c->frames_replay_ready = false;   // the next replay uploads it
  return GBR_OK;
}

int gbr_graph_begin(gbr_ctx* c, void* stream) {
  if (!c || c->capturing) return GBR_ERR_STATE;
  GBR_HIP(hipStreamBeginCapture((hipStream_t)stream, hipStreamCaptureModeRelaxed));
  c->capturing = true;
  c->capture_posts = 0;
  c->capture_uses_frames = false;
  return GBR_OK;
}

int gbr_graph_end(gbr_ctx* c, void* stream, gbr_graph** out) {
  if (!c || !out || !c->capturing) return GBR_ERR_STATE;
  c->capturing = false;
  gbr_graph* g = new gbr_graph();
  if (hipStreamEndCapture((hipStream_t)stream, &g->graph) != hipSuccess) { delete g; return GBR_ERR_HIP; }
  if (hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGraphDestroy(g->graph);
    delete g;
    return GBR_ERR_HIP;
  }
  g->ctx = c;
  g->alloc_gen = c->alloc_gen;
  g->posts = c->capture_posts;
  g->uses_frames = c->capture_uses_frames;
  *out = g;
  return GBR_OK;
}

int gbr_graph_launch(gbr_graph* g, void* stream) {
  if (!g) return GBR_ERR_INVALID_ARG;
  if (g->ctx->alloc_gen != g->alloc_gen) return GBR_ERR_STATE;   // a buffer it uses was reallocated
  gbr_ctx* c = g->ctx;
  if (g->uses_frames && !c->frames_replay_ready) {
    GBR_HIP(hipMemcpyAsync(c->d_frames, c->h_frames + (int64_t)kCaptureSlot * c->cap_frames,
                           sizeof(FrameDev) * c->capture_frames_B, hipMemcpyHostToDevice, (hipStream_t)stream));
    c->frames_replay_ready = true;
  }
  GBR_HIP(hipGraphLaunch(g->exec, (hipStream_t)stream));
  if (g->posts) {
    g->ctx->posts += g->posts;
    g->ctx->post_stream = (hipStream_t)stream;
  }
  return GBR_OK;
}

int gbr_graph_destroy(gbr_graph* g) {
  if (!g) return GBR_ERR_INVALID_ARG;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
  return GBR_OK;
}

int gbr_autotune(gbr_ctx* c, const float* raw, const int64_t* goff, const gbr_camera* cams, int32_t B,
                 float* images, float* dimages, float* draw, void* stream, int32_t* best_tile, int32_t* best_chunk,
                 float* times_ms) {
  if (!c || !raw || !images || !dimages || !draw) return GBR_ERR_INVALID_ARG;
  if (c->capturing) return GBR_ERR_STATE;
  hipStream_t s = (hipStream_t)stream;
  const int tiles[3] = {8, 16, 32}, chunks[3] = {64, 128, 256};
  hipEvent_t e0, e1;
  GBR_HIP(hipEventCreate(&e0));
  GBR_HIP(hipEventCreate(&e1));
  float best = 1e30f;
  int bt = c->tile, bc = c->chunk;
  int rc = GBR_OK;
  for (int ti = 0; ti < 3 && !rc; ++ti)
    for (int ci = 0; ci < 3 && !rc; ++ci) {
      rc = gbr_set_tiling(c, tiles[ti], chunks[ci]);
      if (rc) break;
      // make sure the entry buffers fit this tile size
      rc = gbr_preprocess(c, raw, goff, cams, B, stream);
      if (rc) break;
      int64_t e = 0;
      rc = gbr_entry_count(c, stream, &e);
      if (rc) break;
      float ms = 0.f;
      for (int rep = 0; rep < 3 && !rc; ++rep) {
        (void)hipEventRecord(e0, s);
        rc = gbr_render(c, raw, goff, cams, B, images, stream);
        if (!rc) rc = gbr_render_backward(c, dimages, draw, stream);
        (void)hipEventRecord(e1, s);
        (void)hipEventSynchronize(e1);
        float t = 0.f;
        (void)hipEventElapsedTime(&t, e0, e1);
        if (rep == 0 || t < ms) ms = t;
      }
      if (times_ms) times_ms[ti * 3 + ci] = ms;
      if (!rc && ms < best) { best = ms; bt = tiles[ti]; bc = chunks[ci]; }
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  rc = gbr_set_tiling(c, bt, bc);
  if (best_tile) *best_tile = bt;
  if (best_chunk) *best_chunk = bc;
  return rc;
}

int gbr_inspect(gbr_ctx* c, int32_t what, void* dst, int64_t* bytes) {
  if (!c || !dst || !bytes) return GBR_ERR_INVALID_ARG;
  if (!c->have_pre) return GBR_ERR_STATE;
  GBR_HIP(hipDeviceSynchronize());
  const void* src = nullptr;
  int64_t n = 0;
  StatusDev st;
  GBR_HIP(hipMemcpy(&st, c->d_status, sizeof(st), hipMemcpyDeviceToHost));
  const int64_t entries = std::min<int64_t>((int64_t)st.entries, c->cap_entries);
  if (what >= 4 && !c->have_raster) return GBR_ERR_STATE;
  switch (what) {
    case 1: src = c->rec; n = c->n_splats * kRecF * 4; break;
    case 2: src = c->rect; n = c->n_splats * 16; break;
    case 3: src = c->tile_start; n = ((int64_t)c->n_tiles + 1) * 4; break;
    case 4:   // the complete per-tile lists (the forward may have ordered only what it consumed)
      launch_tile_lists(make_args(c), nullptr);
      GBR_HIP(hipDeviceSynchronize());
      src = c->sorted; n = entries * 4; break;
    case 10: src = c->sorted; n = entries * 4; break;   // as the pass left it
    case 5: src = c->n_iter; n = c->n_pixels * 4; break;
    case 6: src = c->t_final; n = c->n_pixels * 4; break;
    case 7: src = c->tile_last; n = (int64_t)c->n_tiles * 4; break;
    case 8:   // contributors per pixel, counted on request from the complete lists
      launch_tile_lists(make_args(c), nullptr);
      launch_count_contrib(make_args(c), nullptr);
      GBR_HIP(hipDeviceSynchronize());
      src = c->n_contrib; n = c->n_pixels * 4; break;
    case 9: {   // one byte per entry, bit w = quadrant w's byte, valid below the quadrant's last position
      if (*bytes < entries) return GBR_ERR_CAPACITY;
      std::vector<uint32_t> q4((size_t)entries), ts((size_t)c->n_tiles + 1), ql((size_t)c->n_tiles * 4);
      if (entries > 0) GBR_HIP(hipMemcpy(q4.data(), c->cmask, (size_t)entries * 4, hipMemcpyDeviceToHost));
      GBR_HIP(hipMemcpy(ts.data(), c->tile_start, ts.size() * 4, hipMemcpyDeviceToHost));
      GBR_HIP(hipMemcpy(ql.data(), c->qlast, ql.size() * 4, hipMemcpyDeviceToHost));
      uint8_t* d8 = static_cast<uint8_t*>(dst);
      std::memset(d8, 0, (size_t)entries);
      for (int g = 0; g < c->n_tiles; ++g) {
        for (int64_t i = ts[g]; i < (int64_t)ts[g + 1] && i < entries; ++i) {
          const uint32_t v = q4[(size_t)i];
          uint8_t m = 0;
          for (int w = 0; w < 4; ++w)
            if ((uint32_t)(i - ts[g]) < ql[(size_t)g * 4 + w] && ((v >> (8 * w)) & 1u)) m |= (uint8_t)(1u << w);
          d8[i] = m;
        }
      }
      *bytes = entries;
      return GBR_OK;
    }
    case 11: src = c->qlast; n = (int64_t)c->n_tiles * 16; break;
    default: return GBR_ERR_INVALID_ARG;
  }
  if (*bytes < n) return GBR_ERR_CAPACITY;
  if (n > 0) GBR_HIP(hipMemcpy(dst, src, (size_t)n, hipMemcpyDeviceToHost));
  *bytes = n;
  return GBR_OK;
}

int gbr_timing(gbr_ctx* c, int32_t which, int32_t enable) {
  if (!c || which < 0 || which >= GBR_K_COUNT) return GBR_ERR_INVALID_ARG;
  if (c->capturing) return GBR_ERR_STATE;
  if (enable && !c->t_ev[which][0]) {
    GBR_HIP(hipEventCreate(&c->t_ev[which][0]));
    GBR_HIP(hipEventCreate(&c->t_ev[which][1]));
  }
  if (enable && !c->t_stamp) {
    int rc = dalloc(&c->t_stamp, 4 * GBR_K_COUNT);
    if (rc) return rc;
    GBR_HIP(hipDeviceGetAttribute(&c->wall_khz, hipDeviceAttributeWallClockRate, c->cfg.device));
    if (c->wall_khz <= 0) return GBR_ERR_HIP;
    GBR_HIP(hipMemset(c->t_stamp, 0, sizeof(unsigned long long) * 4 * GBR_K_COUNT));
  }
  if (enable) {
    // restart the accumulator after everything queued so far
    GBR_HIP(hipDeviceSynchronize());
    GBR_HIP(hipMemset(c->t_stamp + 4 * which, 0, sizeof(unsigned long long) * 4));
  }
  c->timing_on[which] = enable != 0;
  if (enable) c->t_recorded[which] = false;
  return GBR_OK;
}

int gbr_timing_accum(gbr_ctx* c, int32_t which, int32_t reset, double* total_ms, int64_t* launches) {
  if (!c || !total_ms || !launches || which < 0 || which >= GBR_K_COUNT) return GBR_ERR_INVALID_ARG;
  if (c->capturing) return GBR_ERR_STATE;
  if (!c->t_stamp) return GBR_ERR_STATE;
  unsigned long long h[4];
  GBR_HIP(hipDeviceSynchronize());
  GBR_HIP(hipMemcpy(h, c->t_stamp + 4 * which, sizeof(h), hipMemcpyDeviceToHost));
  *total_ms = (double)h[1] / (double)c->wall_khz;
  *launches = (int64_t)h[2];
  if (reset) GBR_HIP(hipMemset(c->t_stamp + 4 * which, 0, sizeof(h)));
  return GBR_OK;
}

int gbr_timing_read(gbr_ctx* c, int32_t which, float* ms) {
  if (!c || !ms || which < 0 || which >= GBR_K_COUNT) return GBR_ERR_INVALID_ARG;
  // no eager launch of the kernel since its timing was enabled: nothing to
  // read (asking HIP would leave its error state set for the next call)
  if (!c->t_ev[which][0] || !c->t_recorded[which]) return GBR_ERR_STATE;
  GBR_HIP(hipEventSynchronize(c->t_ev[which][1]));
  GBR_HIP(hipEventElapsedTime(ms, c->t_ev[which][0], c->t_ev[which][1]));
  return GBR_OK;
}

}  // extern "C"
