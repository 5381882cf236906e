/*
 * gbr.h -- C ABI of libgbr, the gfx950 (MI355X) batch-parallel differentiable
 * renderer for reduced Gaussian blendshape avatars (RGBAvatar, arXiv
 * 2503.12886).
 *
 * The calls follow the paper's problem statement:
 *   blend     G^psi = G_0 + sum_k psi_k dG_k                    (Eq. 1)
 *   render    per-frame preprocess (activation + EWA projection), tile
 *             binning + depth order, front-to-back alpha compositing; a
 *             whole batch of frames, each with its own Gaussian set and
 *             camera, in one pass with no host synchronisation (Sec. 3.2,
 *             "Batch-parallel Gaussian Rasterization", Fig. 5c)
 *   backward  dL/dimages -> dL/d(blended Gaussians) -> dL/dbases, dL/dweights
 *             (the bases and weights are what training optimises, Sec. 3.2
 *             and Sec. A.3)
 * plus the pieces of the training step around them: the weight MLP
 * psi = F(theta) (Eq. 2), the L1 colour loss (Sec. 3.2 "Loss Function"),
 * Adam with per-attribute learning rates (Sec. A.3), the single status read
 * per step, graph capture and tile/chunk autotuning.
 *
 * Conventions shared by every call
 *  - All tensors are float32 in device memory unless stated otherwise; the
 *    caller allocates and owns every input and output pointer and the
 *    library never frees them.  Host-side arrays are marked "host".
 *  - A blended Gaussian is 16 floats: position [0:3], quaternion (w,x,y,z)
 *    [3:7], log-scale [7:10], opacity logit [10], RGB [11:14], pad [14:16]
 *    (pads are ignored on input and written as 0).  Activations after
 *    blending (Sec. A.3): normalised quaternion, exp scale, sigmoid opacity,
 *    identity colour.
 *  - bases: [(K+1)][N][16]; slice 0 is G_0, slices 1..K are dG_1..dG_K.
 *    weights: [B][K] (psi of every frame; G_0 has the implicit weight 1).
 *  - Images: frame b is a CHW block of 3*H_b*W_b floats; frames are packed
 *    back to back in call order (offset of frame b = 3 * sum_{b'<b} H W).
 *  - Every call is stream-ordered and enqueue-only unless it says it
 *    synchronises; `stream` is a hipStream_t passed as void* (NULL = the
 *    null stream).
 *  - Return value: GBR_OK or a negative GBR_ERR_* code (gbr_strerror).
 *    Arguments are validated on the host before anything is enqueued; an
 *    error leaves the context and the outputs untouched.  Capacity overflow
 *    that only the device can see (the number of tile entries) sets a
 *    device flag instead: every later kernel of that pass becomes a no-op,
 *    Adam skips its update, and gbr_query_status reports it; the caller then
 *    calls gbr_reserve and replays the step.
 *  - A context is used by one host thread and one stream at a time.
 */
#ifndef GBR_H
#define GBR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GBR_OK 0
#define GBR_ERR_INVALID_ARG (-1)
#define GBR_ERR_CAPACITY (-2)   /* host-visible capacity exceeded (frames, splats, pixels) */
#define GBR_ERR_OOM (-3)
#define GBR_ERR_HIP (-4)
#define GBR_ERR_STATE (-5)      /* e.g. backward without a preceding render */
#define GBR_ERR_OVERFLOW (-6)   /* device-detected entry overflow in the last pass */

typedef struct gbr_ctx gbr_ctx;
typedef struct gbr_graph gbr_graph;

/* Pinhole camera of one frame.  R, t: world->camera (row-major), OpenCV axes
   (+z forward, +x right, +y down); pixel (j, i) is sampled at (j+0.5, i+0.5).
   A Gaussian whose camera-space z <= near_z is culled.  bg: background colour
   composited behind the Gaussians (the random background of Sec. 3.2). */
typedef struct {
  int32_t width, height;
  float fx, fy, cx, cy;
  float R[9];
  float t[3];
  float near_z;
  float bg[3];
} gbr_camera;

/* tile: 8, 16 or 32 px.  chunk: 64, 128 or 256 entries staged in LDS per
   compositing step.  max_*: capacities the context allocates at creation
   (frames per call, sum of per-frame Gaussian counts, sum of per-frame pixel
   counts, tile-Gaussian entries).  max_entries grows with gbr_reserve. */
typedef struct {
  int32_t tile;
  int32_t chunk;
  int32_t device;
  int32_t max_frames;
  int64_t max_splats;
  int64_t max_pixels;
  int64_t max_entries;
} gbr_config;

typedef struct {
  int64_t entries;           /* tile-Gaussian entries of the last pass */
  int64_t entries_capacity;
  int32_t overflow;          /* nonzero: the last pass overflowed, outputs invalid */
  int32_t adam_steps[4];     /* Adam steps applied per parameter group */
  float loss;                /* last value computed by gbr_loss */
} gbr_status;

const char* gbr_strerror(int code);

/* Create a context on cfg->device: allocates every workspace from the
   capacities in cfg.  Out: *out owns the workspace until gbr_destroy. */
int gbr_create(const gbr_config* cfg, gbr_ctx** out);
int gbr_destroy(gbr_ctx* ctx);
/* Grow the entry capacity to at least max_entries (synchronises the device;
   not allowed during graph capture).  When the capacity grows, graphs
   captured before refuse to launch (GBR_ERR_STATE). */
int gbr_reserve(gbr_ctx* ctx, int64_t max_entries);
/* Device memory of a context's workspace, in bytes, for callers that budget
   it (the serving executor admits work by the bytes its contexts hold):
   gbr_memory gives what the context holds now (its capacities at creation,
   grown by gbr_reserve and by the per-pass buffers -- depth buckets, scan
   scratch, tile bitmap rows -- of the largest pass so far); gbr_plan_bytes
   gives what a context created with cfg would hold after one pass of B
   frames (per-frame Gaussian counts from gauss_offsets, host [B + 1];
   frame sizes widths, heights, host [B]) with at least `entries` tile
   entries reserved.  Both count the allocations as requested (the device
   allocator rounds each up).  Host-only; GBR_ERR_INVALID_ARG /
   GBR_ERR_CAPACITY as gbr_create and gbr_render would return. */
int gbr_memory(gbr_ctx* ctx, int64_t* device_bytes);
int gbr_plan_bytes(const gbr_config* cfg, int32_t B, const int64_t* gauss_offsets, const int32_t* widths,
                   const int32_t* heights, int64_t entries, int64_t* device_bytes);
/* Switch tile size / LDS chunk depth (validated as in gbr_config). */
int gbr_set_tiling(gbr_ctx* ctx, int32_t tile, int32_t chunk);

/* Eq. 1.  raw[b] = bases[0] + sum_k weights[b][k-1] * bases[k] for B frames
   that share one Gaussian set of N.  Accumulates in float64 in slice order
   (each float32 x float32 product is exact in float64) and rounds once to
   float32, so the result does not depend on B.  bases [(K+1)][N][16],
   weights [B][K] (may be NULL when K = 0), raw [B][N][16] (pads written 0).
   1 <= B <= 4096, 0 <= K <= 63, N >= 1, else GBR_ERR_INVALID_ARG. */
int gbr_blend(gbr_ctx* ctx, const float* bases, const float* weights, int32_t B, int32_t K, int64_t N, float* raw,
              void* stream);

/* Render B frames (Sec. 3.2 batch-parallel rasterization: preprocess, then
   rasterize, with no host synchronisation in between).
   raw: packed [sum_b N_b][16] blended Gaussians; frame b uses rows
   gauss_offsets[b] .. gauss_offsets[b+1]-1 (host array [B+1], starting at 0).
   cams: host array [B].  images: packed CHW frames (see above).
   The context keeps what the backward pass needs until the next render. */
int gbr_render(gbr_ctx* ctx, const float* raw, const int64_t* gauss_offsets, const gbr_camera* cams, int32_t B,
               float* images, void* stream);
/* The two halves of gbr_render, for callers that want the paper's per-frame
   scheme (Fig. 5a/5b): gbr_preprocess (activation, projection, per-frame
   depth order, per-tile rank bitmaps and entry counts), then gbr_entry_count
   (a host synchronisation that returns the number of tile entries, and
   grows the capacity if needed), then gbr_rasterize (compositing). */
int gbr_preprocess(gbr_ctx* ctx, const float* raw, const int64_t* gauss_offsets, const gbr_camera* cams, int32_t B,
                   void* stream);
int gbr_entry_count(gbr_ctx* ctx, void* stream, int64_t* entries);
int gbr_rasterize(gbr_ctx* ctx, float* images, void* stream);

/* Adjoint of the last gbr_render: dimages (same packing as images) ->
   draw [sum_b N_b][16] = dL/draw (pads written 0).  Deterministic: no
   floating-point atomics, fixed summation order. */
int gbr_render_backward(gbr_ctx* ctx, const float* dimages, float* draw, void* stream);

/* Adjoint of gbr_blend.  draw [B][N][16] -> dbases [(K+1)][N][16] (pads
   written 0) and dweights [B][K] (the contraction over N*16 runs on the
   matrix cores with per-wave partials summed in a fixed order);
   accumulate != 0 adds into the outputs.  dbases may be NULL: then only
   dweights is formed (for gbr_blend_adam_step, which forms dbases itself).
   1 <= B <= 64, 0 <= K <= 63, B * N within the context's max_splats
   (GBR_ERR_CAPACITY). */
int gbr_blend_backward(gbr_ctx* ctx, const float* draw, const float* bases, const float* weights, int32_t B,
                       int32_t K, int64_t N, float* dbases, float* dweights, int32_t accumulate, void* stream);

/* gbr_blend_backward for callers that cannot allocate device memory (code
   under graph capture, tight serving loops, harnesses that forbid
   hipMalloc): no context, and nothing is allocated or freed.  The dweights
   partials go to a fixed 4 MiB device array of the library (one per device,
   its address looked up on the first call on that device and kept until the
   process ends), so a shape whose partials exceed 2^20 floats --
   ceil(N * 16 / 1024) * B * K, times 4 when B > 16 or K > 32 -- returns
   GBR_ERR_CAPACITY (N = 50,000, B = 16, K = 20 needs 250,240).  Arguments,
   layouts, limits (1 <= B <= 64, 0 <= K <= 63) and results as
   gbr_blend_backward, bit for bit.  Call it with the stream's device
   current.  Every call on a device shares that device's array: calls that
   overlap on one device (different streams, or host threads) race and give
   wrong results; calls ordered on one stream are safe (the array needs no
   clearing: each call writes every partial it reads). */
int gbr_blend_backward_noalloc(const float* draw, const float* bases, const float* weights, int32_t B, int32_t K,
                               int64_t N, float* dbases, float* dweights, int32_t accumulate, void* stream);

/* The Adam step of gbr_adam_step (Sec. A.3) on the bases [(K+1)][N][16],
   with their gradient -- the dbases of gbr_blend_backward (Eq. 1's adjoint,
   accumulate = 0) for the same draw and weights -- formed inside the update
   and never stored: one pass over draw, bases, m and v instead of writing
   dbases and reading it back.  The values equal gbr_blend_backward followed
   by gbr_adam_step with split = N * 16 on the same table.  Call it after
   every use of the old bases (gbr_blend_backward's dweights reads them).
   group, lr_table, betas and eps as for gbr_adam_step (the update is
   skipped on an overflowed pass); B, K, N limits as for
   gbr_blend_backward.  Device pointers; bases, m, v updated in place. */
int gbr_blend_adam_step(gbr_ctx* ctx, int32_t group, const float* draw, const float* weights, int32_t B, int32_t K,
                        int64_t N, float* bases, float* m, float* v, const float* lr_table, float beta1, float beta2,
                        float eps, void* stream);

/* gbr_render_backward followed by gbr_blend_backward for a batch rendered
   from one blend (all frames share N = gauss_offsets[1]); draw lives in the
   context's workspace. */
int gbr_backward(gbr_ctx* ctx, const float* dimages, const float* bases, const float* weights, int32_t K,
                 float* dbases, float* dweights, void* stream);

/* Tangent-space Gaussians (Sec. 3.1; Eq. 4 and Alg. 1 of the appendix).
   A mesh of V vertices and F triangles: faces [F][3] i32 vertex indices,
   face_uv [F][3][2] f32 texture coordinates per triangle corner (the UV
   triangles must be non-degenerate), verts [B][V][3] f32 one deformed mesh
   per frame.  gbr_tangent_frames writes, per (frame, triangle), frames
   [B][F][16] f32: the TBN matrix R = [T B N] row-major (9 values; T and B
   solve e1 = du1 T + dv1 B, e2 = du2 T + dv2 B for the edges e1 = v1 - v0,
   e2 = v2 - v0, N the unit normal e1 x e2), then the unit quaternion
   (w, x, y, z) of R's Gram-Schmidt frame [T^, B^, T^ x B^], then 3 unused.
   gbr_tangent_transform carries blended Gaussians raw_t [B][N][16] (as
   gbr_blend writes them; Gaussian n bound to triangle tri[n] with
   barycentric coordinates bary [N][3]) to raw_d [B][N][16]:
   x_D = R x_T + (the barycentric point of the frame's triangle),
   q_D = q_R (x) q_T (Hamilton product), the other features copied.
   gbr_tangent_backward maps dL/draw_d to dL/draw_t (dx_T = R^T dx_D,
   dq_T = conj(q_R) (x) dq_D, the rest copied).  All pointers are device
   pointers owned by the caller; indices out of range are clamped (no
   fault, meaningless result).  Enqueue only; graph-capturable. */
int gbr_tangent_frames(gbr_ctx* ctx, const float* verts, const int32_t* faces, const float* face_uv, int32_t B,
                       int32_t V, int32_t F, float* frames, void* stream);
int gbr_tangent_transform(gbr_ctx* ctx, const float* raw_t, const int32_t* tri, const float* bary, const float* verts,
                          const int32_t* faces, const float* frames, int32_t B, int64_t N, int32_t V, int32_t F,
                          float* raw_d, void* stream);
int gbr_tangent_backward(gbr_ctx* ctx, const float* draw_d, const int32_t* tri, const float* frames, int32_t B,
                         int64_t N, int32_t F, float* draw_t, void* stream);

/* gbr_render of tangent-space Gaussians with the transform applied inside
   the pass (Sec. 3.1, Eq. 4): raw_t [B][N][16] as gbr_blend writes it (every
   frame holds the same N Gaussians), bound to triangles tri [N] with
   barycentric coordinates bary [N][3] of the mesh faces [F][3] (V vertices),
   verts [B][V][3] one deformed mesh per frame, frames [B][F][16] the
   per-(frame, triangle) records of gbr_tangent_frames.  Each Gaussian is
   carried to its frame's mesh in the projection, with the same bits as
   gbr_tangent_transform followed by gbr_render; the adjoint of this pass
   (gbr_render_backward, gbr_backward) returns dL/draw_t in tangent space,
   with the same bits as gbr_render_backward followed by
   gbr_tangent_backward.  No deformed copy is stored.  The pointers must
   stay valid until the pass's backward has run; indices out of
   range are clamped.  Errors as gbr_render. */
int gbr_render_tangent(gbr_ctx* ctx, const float* raw_t, const int32_t* tri, const float* bary, const float* verts,
                       const int32_t* faces, const float* frames, int64_t N, int32_t V, int32_t F,
                       const gbr_camera* cams, int32_t B, float* images, void* stream);

/* Colour initialisation (Sec. 3.1, "Initialization", Eq. 3) after a render
   of a batch blended from one set of bases (every frame b holds Gaussians
   [b N, (b + 1) N) of the blend, as for gbr_backward).  For every Gaussian n
   with done[n] == 0, the first frame b whose total splatting weight
   W = sum_p w_p (w_p = the Gaussian's compositing weight alpha T at pixel p)
   exceeds delta (the paper uses 0.1) sets the base model's colour,
   bases[0][n][11..13], to sum_p w_p I_p / W, with I the frame's image in
   targets (same packing as the render's images), and sets done[n] = 1;
   other Gaussians are left alone.  The sums are the colour adjoint of the
   render under I and under all-ones images (two gbr_render_backward
   passes; the context's backward workspace is reused, so a later
   gbr_backward recomputes its own).  bases [(K+1)][N][16] and done [N] u8
   are device pointers owned by the caller.  Not inside graph capture
   (GBR_ERR_STATE); allocates its two scratch buffers on first use. */
int gbr_color_init(gbr_ctx* ctx, const float* targets, float* bases, float delta, uint8_t* done, void* stream);

/* Photometric loss over the frames of the last render (Sec. 3.2: L1 colour
   loss; kind 1 = L1, 2 = L2), mean over every channel of every pixel.
   Writes dimages (same packing) and keeps the loss value for
   gbr_query_status.  Deterministic reduction order. */
int gbr_loss(gbr_ctx* ctx, const float* images, const float* targets, int32_t kind, float* dimages, void* stream);

/* Eq. 2, psi = F(theta): linear(d_in->hidden) + ReLU + linear(hidden->hidden)
   + ReLU + linear(hidden->K).  params packed: W1 [hidden][d_in], b1 [hidden],
   W2 [hidden][hidden], b2 [hidden], W3 [K][hidden], b3 [K].  theta [B][d_in],
   psi [B][K].  Keeps activations for gbr_mlp_backward.
   Limits: d_in <= 1024, hidden <= 1024, K <= 64. */
int gbr_mlp_forward(gbr_ctx* ctx, const float* params, const float* theta, int32_t B, int32_t d_in, int32_t hidden,
                    int32_t K, float* psi, void* stream);
/* dpsi [B][K] -> dparams (same packing as params, overwritten). */
int gbr_mlp_backward(gbr_ctx* ctx, const float* params, const float* dpsi, float* dparams, void* stream);

/* Adam (Sec. A.3) on n parameters, in place on params/m/v.  Learning rate
   of element i: lr_table[(i >= split) * 16 + (i % 16)] (host array [32]),
   i.e. one 16-entry per-feature table for the first `split` elements (the
   base model G_0) and one for the rest (the deltas); pass equal rows for a
   uniform rate.  group (0..3) selects the device step counter used for the
   bias correction; the counter advances only when the pass did not
   overflow, and the update is skipped on overflow. */
int gbr_adam_step(gbr_ctx* ctx, int32_t group, float* params, const float* grads, float* m, float* v, int64_t n,
                  int64_t split, const float* lr_table, float beta1, float beta2, float eps, void* stream);

/* The one host synchronisation per step: waits for `stream` and reads the
   device status (entries, overflow flag, Adam step counters, loss). */
int gbr_query_status(gbr_ctx* ctx, void* stream, gbr_status* out);

/* The same read split in two, so that the host can enqueue the next steps
   before it waits for this one's status, with nothing enqueued between the
   steps but the steps themselves.  gbr_status_post enqueues on `stream`,
   eagerly or into the graph being captured, a one-thread kernel that copies
   the device status (as it stands when the stream reaches it) into a ring of
   4 records in pinned host memory: the device numbers its posts 1, 2, ... in
   the order it runs them, and post n lands in record n mod 4 together with n.
   gbr_status_posts returns how many posts have been enqueued: an eager post
   counts at once, a graph's posts each time gbr_graph_launch launches it, so
   after enqueueing a post (or launching a graph that ends with one) its
   number is the count.  gbr_status_wait waits (spinning on the host) until
   post n has landed and reads it: GBR_ERR_STATE when post n was never
   enqueued, when a newer post has overwritten its record (keep at most 4
   posts ahead of the waits) or when the stream of the latest post has
   finished without it; GBR_ERR_HIP when that stream reports an error. */
int gbr_status_post(gbr_ctx* ctx, void* stream);
int gbr_status_posts(gbr_ctx* ctx, int64_t* n);
int gbr_status_wait(gbr_ctx* ctx, int64_t n, gbr_status* out);

/* Re-stage the per-frame table (cameras, Gaussian offsets) of the last
   render without enqueueing work, so that a graph captured around gbr_render
   replays with new cameras.  B and every frame's size must match the
   captured call.  Call only when the previous replay has completed. */
int gbr_stage_frames(gbr_ctx* ctx, const int64_t* gauss_offsets, const gbr_camera* cams, int32_t B);

/* Graph capture of the work enqueued on `stream` between begin and end
   (one captured training step replayed with a single launch).  A graph
   keeps the device addresses of the context's buffers at capture: when a
   later call reallocates one of them (gbr_reserve, gbr_entry_count growing
   the entry capacity, a render needing larger per-pass buffers),
   gbr_graph_launch returns GBR_ERR_STATE without enqueueing anything, and
   the caller captures again.  A captured render records no copy of its
   per-frame table: gbr_graph_launch enqueues one on `stream` before the
   replay when the device does not hold that table already (after the
   capture, a gbr_stage_frames or an eager render), so replays of an
   unchanged batch copy nothing.  Begin a capture only when earlier
   replays of the context have completed.  A graph must be destroyed
   before its context. */
int gbr_graph_begin(gbr_ctx* ctx, void* stream);
int gbr_graph_end(gbr_ctx* ctx, void* stream, gbr_graph** out);
int gbr_graph_launch(gbr_graph* g, void* stream);
int gbr_graph_destroy(gbr_graph* g);

/* Autotuner: renders and back-propagates the given frames once per
   (tile, chunk) in {8,16,32} x {64,128,256}, times each on `stream`, keeps
   the fastest in the context and reports it (times_ms: host [9], may be
   NULL; entries beyond capacity grow it).  Synchronises. */
int gbr_autotune(gbr_ctx* ctx, const float* raw, const int64_t* gauss_offsets, const gbr_camera* cams, int32_t B,
                 float* images_scratch, float* dimages_scratch, float* draw_scratch, void* stream,
                 int32_t* best_tile, int32_t* best_chunk, float* times_ms);

/* Copy an internal buffer of the last pass to host memory (synchronises).
   what: 1 splat records [S][12] f32 (mx, my, ca, cb, cc, log2 opacity, r, g,
   b, depth, pixel box x, pixel box y; ca, cb, cc = -log2(e) * (A/2, B, C/2)
   of the conic q = A dx^2 + 2B dx dy + C dy^2, so that alpha =
   2^(ca dx^2 + cb dx dy + cc dy^2 + log2 opacity); the two pixel-box slots hold
   the bits of u32 values x0 | x1 << 16 and y0 | y1 << 16, the inclusive
   pixel range of the alpha >= 1/255 support), 2 tile rects [S][4] i32 (inclusive
   tx0, ty0, tx1, ty1), 3 tile starts [tiles+1] u32 (tile g's entries are
   [start[g], start[g+1]) of the sorted list), 4 sorted entries [entries] u32
   (global splat index; the complete lists: when the forward pass ordered
   each tile only as far as it composited, this call completes them first),
   5 per-pixel list position after the last contributor [pixels] u32,
   6 per-pixel final transmittance [pixels] f32, 7 per-tile entries used
   [tiles] u32, 8 per-pixel number of contributing Gaussians [pixels] u32
   (counted by this call from the complete lists: the entries before the
   pixel's stop position with alpha >= 1/255),
   9 per-entry contribution mask [entries] u8: bit w set when some pixel of
   the tile's quadrant w (tiles of 16 and 32 px: quadrants of half the side,
   w = 2 * (row half) + (column half); tiles of 8 px: one quadrant, bit 0)
   took the entry in the forward pass, 10 the sorted entries [entries] u32
   as the pass left them (each tile's list is valid at least up to its
   last used position, 7), 11 per-tile, per-quadrant entries used
   [tiles][4] u32 (quadrant w's pixels took nothing at or past position
   [g][w] of tile g's list; 7 is the largest of the four; tiles of 8 px
   have one quadrant, w = 0, the others 0).
   *bytes in: capacity of dst; out: bytes written. */
int gbr_inspect(gbr_ctx* ctx, int32_t what, void* dst, int64_t* bytes);

/* Kernel timing for measurement tools.  which: GBR_K_* below.  Not a
   passage of the paper: it exists so that a benchmark can time one kernel
   on its own launch stream.  While timing of a kernel is enabled, every
   launch of it is bracketed
   - in eager calls, by a pair of HIP events on the launch stream:
     gbr_timing_read returns the duration of the most recent eager launch
     in ms (GBR_ERR_STATE when no eager launch was bracketed since the
     timing was enabled);
   - in eager calls and in captured graphs alike, by two one-lane stamp
     kernels on the launch stream that read the device's constant-rate
     wall clock before and after the launch and add the difference to a
     device accumulator: gbr_timing_accum returns the accumulated ms and
     the number of bracketed launches (reset != 0 then clears them).
   A graph captured while timing was enabled keeps its stamp kernels on
   every replay, whatever gbr_timing says later.  Brackets include the
   kernel's dispatch latency (a few microseconds).
   gbr_timing(enable=1) synchronises the device and clears that kernel's
   accumulator; it fails with GBR_ERR_STATE during capture, as does
   gbr_timing_accum, which synchronises the device before reading. */
#define GBR_K_BLEND 0
#define GBR_K_PREPROCESS 1
#define GBR_K_BINNING 2      /* per-tile rank bitmap rows and tile counts */
#define GBR_K_TILE_SORT 3    /* clearing the backward scheduling classes when a pass is rasterised again (the
                                forward classes are built in the tile scan's launch, the lists are ordered
                                inside the forward pass) */
#define GBR_K_COMPOSITE_FWD 4
#define GBR_K_COMPOSITE_BWD 5
#define GBR_K_GATHER_BWD 6
#define GBR_K_BLEND_BWD 7
#define GBR_K_ADAM 8
#define GBR_K_LOSS 9
#define GBR_K_MLP 10         /* forward and backward */
#define GBR_K_TILE_SCAN 11   /* tile offsets, with the forward scheduling classes */
#define GBR_K_DEPTH_ORDER 12  /* per-frame depth ranks of the visible splats (and the splat-offset scan) */
#define GBR_K_COUNT 13
int gbr_timing(gbr_ctx* ctx, int32_t which, int32_t enable);
int gbr_timing_read(gbr_ctx* ctx, int32_t which, float* ms);
int gbr_timing_accum(gbr_ctx* ctx, int32_t which, int32_t reset, double* total_ms, int64_t* launches);

#ifdef __cplusplus
}
#endif
#endif /* GBR_H */
