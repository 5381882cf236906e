// Backward half of the batch-parallel rasterizer: per-tile reverse traversal
// of the compositing recurrence, per-entry partial gradients reduced across
// the tile's pixels without atomics, a fixed-order gather per splat, and the
// adjoint of activation + EWA projection.  Also the photometric loss.
#include "gbr_internal.h"
#include "tangent_ops.h"

namespace gbr {

template <int T> using TileShapeB = TileMap<T>;

// Must stay bit-identical to the forward kernel's alpha: power = ca dx^2 +
// cb dx dy + cc dy^2 + lo (lo = log2 opacity), alpha = 2^min(power, lo).
// The clamp is one v_min_f32 (min(power, lo) for every non-NaN power);
// written as such because fminf would first canonicalise lo, one more
// instruction per (entry, pixel).
__device__ __forceinline__ float splat_alpha_b(float4 r0, float4 r1, float px, float py, float& dx, float& dy,
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

// Per-entry partial, summed over the tile's pixels, in units of t = alpha *
// dL/dalpha (the gradient with respect to the power is t ln 2):
//   (sum t dx, sum t dy, sum t dx^2, sum t dx dy, sum t dy^2, sum t,
//    d r, d g, d b)
// with (dx, dy) the pixel's offset from the mean.  The splat's gradients
// follow once per splat, after the sums: the power's coefficients ca, cb, cc
// get ln 2 times the three second moments, the mean -ln 2 (2 ca, cb; cb,
// 2 cc) times the first moments, the opacity logit (1 - o) sum t.  Along the
// traversal each lane keeps only the transmittance and <colour behind,
// dL/dout>.
// A wave's sum over its lanes is taken in a fixed order (lane folds, then
// in-row shifts); the block then adds its waves in order and writes the
// entry's partial, by emission slot, only if some pixel contributed; a byte
// flag marks it.

// Folds one entry into a lane's back-to-front state (transmittance in front
// of the entry, colour behind it) and returns its partial in acc.  Lanes
// whose pixel did not take the entry add exact zeros and keep their state.
template <int PX>
__device__ __forceinline__ void entry_grad(const float4 r0, const float4 r1, const float cbl, const uint32_t li,
                                           const float* pxf, const float* pyf, const uint32_t* nit, float* T_,
                                           float* SG, const float* G0, const float* G1, const float* G2,
                                           float* acc) {
#pragma unroll
  for (int p = 0; p < PX; ++p) {
    float dx, dy, pwr;
    const float a0 = splat_alpha_b(r0, r1, pxf[p], pyf[p], dx, dy, pwr);
    const bool take = li < nit[p] && a0 >= kAlphaMin;
    // an untaken entry folds with alpha 0: 1/(1 - 0) = 1 exactly, so the
    // transmittance passes through unchanged and the weight is 0
    const float al = take ? fminf(a0, kAlphaMax) : 0.0f;
    const float inv = __builtin_amdgcn_rcpf(1.0f - al);
    const float Ti = T_[p] * inv;                     // transmittance in front of this entry
    const float wgt = al * Ti;
    const float cg = r1.z * G0[p] + r1.w * G1[p] + cbl * G2[p];   // <colour, dL/dout>
    const float dal = Ti * cg - SG[p] * inv;          // d out / d alpha
    SG[p] += wgt * cg;                                // <colour behind, dL/dout>
    T_[p] = Ti;
    // min(0.99, .) passes the gradient only below the clamp
    const float t = (take && a0 < kAlphaMax) ? a0 * dal : 0.0f;
    // power clamped at log2 o (q < 0 by rounding): no gradient to the conic or mean
    const float tq = (pwr > r1.y) ? 0.0f : t;
    const float p1 = tq * dx, p2 = tq * dy;
    const float v[9] = {p1, p2, p1 * dx, p1 * dy, p2 * dy, t, wgt * G0[p], wgt * G1[p], wgt * G2[p]};
    // the first pixel assigns (adding it to 0 would cost an instruction per value)
#pragma unroll
    for (int c = 0; c < 9; ++c) acc[c] = (p == 0) ? v[c] : acc[c] + v[c];
  }
}

// The sums over the 16 lanes of each row of 9 values, transposed into one
// register: at each halving step two registers are paired, each lane keeping
// one of the two values and adding its partner's copy of it (partners by
// row_ror:8, row_half_mirror, quad_perm xor 2, then xor 1), so 21 VALU
// operations replace 36 in-row shifts.  Lane i of a row ends with the row's
// total of value 8 when i is odd, else of value 4 i1 + 2 i2 + i3 (i1, i2, i3
// the bits 1 to 3 of i); every lane's total covers each of the 16 lanes once.
// In the first two steps the two halves of a pair are whole DPP banks (4
// lanes), so each half is one DPP add that writes only its banks, in place
// (inline assembly: two wait states before DPP reads of VALU results);
// the last two steps select between the registers.
template <int CTRL>
__device__ __forceinline__ float pair_fold(float x, float y, bool hi) {
  const float z = hi ? y : x, w = hi ? x : y;
  return z + dpp_mov<CTRL, 0xf, 0xf, false>(w);
}
#define GBR_BANK_PAIR(ctrl, x, y, mx, my)                                                    \
  "v_add_f32_dpp %" #x ", %" #x ", %" #x " " ctrl " row_mask:0xf bank_mask:" mx "\n\t"     \
  "v_add_f32_dpp %" #x ", %" #y ", %" #y " " ctrl " row_mask:0xf bank_mask:" my "\n\t"
__device__ __forceinline__ float rows_transposed9(const float (&v)[9], int lane) {
  constexpr int kQuadXor2 = 0x4e, kQuadXor1 = 0xb1;
  float a0 = v[0], a1 = v[2], a2 = v[4], a3 = v[6], a4 = v[8];
  // partners 8 apart: the first value in lanes 0-7 (banks 0, 1), the second in 8-15
  asm volatile("s_nop 1\n\t"
               GBR_BANK_PAIR("row_ror:8", 0, 5, "0x3", "0xc") GBR_BANK_PAIR("row_ror:8", 1, 6, "0x3", "0xc")
               GBR_BANK_PAIR("row_ror:8", 2, 7, "0x3", "0xc") GBR_BANK_PAIR("row_ror:8", 3, 8, "0x3", "0xc")
               "v_add_f32_dpp %4, %4, %4 row_ror:8 row_mask:0xf bank_mask:0xf"
               : "+v"(a0), "+v"(a1), "+v"(a2), "+v"(a3), "+v"(a4)
               : "v"(v[1]), "v"(v[3]), "v"(v[5]), "v"(v[7]));
  // partners mirrored inside 8 lanes: the first value in banks 0 and 2, the second in 1 and 3
  asm volatile("s_nop 1\n\t"
               GBR_BANK_PAIR("row_half_mirror", 0, 3, "0x5", "0xa") GBR_BANK_PAIR("row_half_mirror", 1, 4, "0x5", "0xa")
               "v_add_f32_dpp %2, %2, %2 row_half_mirror row_mask:0xf bank_mask:0xf"
               : "+v"(a0), "+v"(a2), "+v"(a4)
               : "v"(a1), "v"(a3));
  const bool b1 = lane & 2, b0 = lane & 1;
  const float d0 = pair_fold<kQuadXor2>(a0, a2, b1);
  const float d1 = a4 + dpp_mov<kQuadXor2, 0xf, 0xf, false>(a4);
  return pair_fold<kQuadXor1>(d0, d1, b0);
}
#undef GBR_BANK_PAIR

// Adds rows 0 and 1, and rows 2 and 3, lane by lane (each half-wave's two
// rows end with the same sums): a lane swap of the register with its copy.
__device__ __forceinline__ float row_pair_sum(float x) {
  float y = x;
  asm volatile("s_nop 1\n\tv_permlane16_swap_b32 %0, %1\n\ts_nop 1" : "+v"(x), "+v"(y));
  return x + y;
}

template <int T, int CHUNK>
__global__ __launch_bounds__(TileShapeB<T>::NT, T == 16 ? 8 : 1) void composite_bwd_kernel(PassArgs a,
                                                                         const float* __restrict__ dimages) {
  static_assert(CHUNK <= 256, "a group's chunk positions are packed one byte each");
  using S = TileShapeB<T>;
  constexpr int U = 4;                      // entries folded per step (independent alphas)
  __shared__ float4 s0[CHUNK];
  __shared__ float4 s1[CHUNK];
  __shared__ float4 s2[CHUNK];             // .x only: 16-byte slots share the LDS address of s0 and s1
  __shared__ float red[CHUNK][S::NW][9];
  __shared__ uint32_t wany[CHUNK];         // byte w: wave w wrote red[i][w]
  __shared__ uint32_t cm[CHUNK];          // byte w: quadrant w took the entry
  __shared__ uint32_t sid[CHUNK];
  if (a.status->overflow) return;
  const int g = tile_of_rank(a.cls_cnt + 33, a.order_bwd, a.n_tiles, blockIdx.x);
  if (g < 0) return;
  const uint32_t L = a.tile_last[g];
  if (L == 0) return;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint32_t Lw = a.qlast[g * 4 + w];    // this wave's quadrant took nothing at or past Lw
  const int b = frame_of_tile(a.frames, a.B, g);
  const FrameDev& F = a.frames[b];
  const int lt = g - F.tile_base;
  const int tx = lt % F.ntx, ty = lt / F.ntx;
  const uint32_t start = a.tile_start[g];
  const int lx0 = S::lx0(threadIdx.x), ly0 = S::ly0(threadIdx.x);
  float T_[S::PX], SG[S::PX], G0[S::PX], G1[S::PX], G2[S::PX];
  uint32_t nit[S::PX];
  float pxf[S::PX], pyf[S::PX];
  const float* img_g = dimages + F.pix_base * 3;
  const int64_t hw = (int64_t)F.W * F.H;
#pragma unroll
  for (int p = 0; p < S::PX; ++p) {
    const int px = tx * T + lx0 + (p % S::PXW), py = ty * T + ly0 + (p / S::PXW);
    pxf[p] = (float)px + 0.5f;
    pyf[p] = (float)py + 0.5f;
    nit[p] = 0; T_[p] = 1.0f; SG[p] = 0.0f; G0[p] = G1[p] = G2[p] = 0.0f;
    if (px < F.W && py < F.H) {
      const int64_t pix = (int64_t)py * F.W + px;
      nit[p] = a.n_iter[F.pix_base + pix];
      T_[p] = a.t_final[F.pix_base + pix];
      G0[p] = img_g[pix]; G1[p] = img_g[hw + pix]; G2[p] = img_g[2 * hw + pix];
      // <colour behind the current entry, dL/dout>, starts at <T_end * background, dL/dout>
      SG[p] = T_[p] * (F.bg[0] * G0[p] + F.bg[1] * G1[p] + F.bg[2] * G2[p]);
    }
  }
  uint8_t* wany8 = reinterpret_cast<uint8_t*>(wany);
  for (int ce = (int)L; ce > 0; ce -= CHUNK) {
    const int cbeg = max(0, ce - CHUNK);
    const int n = ce - cbeg;
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += S::NT) {
      const uint32_t sp = a.sorted[start + cbeg + i];
      const float4* rec = reinterpret_cast<const float4*>(a.rec + (int64_t)sp * kRecF);
      s0[i] = rec[0]; s1[i] = rec[1]; s2[i] = make_float4(rec[2].x, 0.0f, 0.0f, 0.0f);
      cm[i] = reinterpret_cast<const uint32_t*>(a.cmask)[start + cbeg + i];
      sid[i] = sp;
      wany[i] = 0u;
    }
    __syncthreads();
    // Entries this wave's pixels took in the forward pass (its contribution
    // mask bit), visited back to front in groups of 4.  A pixel takes an
    // entry here exactly when it took it in the forward pass (the same alpha
    // bits, the same stop position), so every visited entry has a
    // contributing pixel in the wave and its partial is written unchecked.
    for (int gb = (n - 1) & ~63; gb >= 0; gb -= 64) {
      const int idx = gb + lane;
      unsigned long long m = __ballot(idx < n && (uint32_t)(cbeg + idx) < Lw && ((cm[idx] >> (8 * w)) & 1u));
      while (m) {
        int e[U];
        int cnt = 0;
#pragma unroll
        for (int u = 0; u < U; ++u) {
          e[u] = -1;
          if (m) {
            const int hb = 63 - __clzll((long long)m);
            m &= ~(1ull << hb);
            e[u] = gb + hb;
            ++cnt;
          }
        }
        if (cnt <= 2) {
          // a short group (the tail of a chunk): two entries, one lane-swap
          // fold (entry 0 in lanes 0-31, entry 1 in 32-63), the transposed
          // row sums, then each half-wave's two rows added
          float acc2[2][9];
#pragma unroll
          for (int u = 0; u < 2; ++u) {
            const int i = e[u] < 0 ? e[0] : e[u];
            const uint32_t li = e[u] < 0 ? 0xffffffffu : (uint32_t)(cbeg + i);
            entry_grad<S::PX>(s0[i], s1[i], s2[i].x, li, pxf, pyf, nit, T_, SG, G0, G1, G2, acc2[u]);
          }
          fold32x9(acc2[0], acc2[1]);
          const float tot = row_pair_sum(rows_transposed9(acc2[0], lane));
          const int li = lane & 15;
          if ((lane & 16) == 0 && ((li & 1) == 0 || li == 1)) {   // rows 0 and 2, one lane per value
            const int u = lane >> 5;
            const int eu = u == 0 ? e[0] : e[1];
            const int c = (li & 1) ? 8 : (((li >> 1) & 1) << 2) | (((li >> 2) & 1) << 1) | ((li >> 3) & 1);
            if (u < cnt) {
              red[eu][w][c] = tot;
              if (li == 1) wany8[eu * 4 + w] = 1;
            }
          }
          continue;
        }
        float acc[U][9];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          // an absent entry is folded as an untaken one (zeros, state kept)
          const int i = e[u] < 0 ? e[0] : e[u];
          const uint32_t li = e[u] < 0 ? 0xffffffffu : (uint32_t)(cbeg + i);
          entry_grad<S::PX>(s0[i], s1[i], s2[i].x, li, pxf, pyf, nit, T_, SG, G0, G1, G2, acc[u]);
        }
        // Sums of the 4 x 9 partials over the wave's 64 lanes, in a fixed
        // order: fold lanes 32 apart (entries 0|1 and 2|3 into one register
        // per value), then 16 apart (all four entries of a value in one
        // register, a row each: row r holds entry (r >> 1) | ((r & 1) << 1)),
        // then the transposed in-row sums, which leave each of the entry's 9
        // totals in its own lane of the row.
        fold32x9(acc[0], acc[1]);
        fold32x9(acc[2], acc[3]);
        fold16x9(acc[0], acc[2]);
        const float tot = rows_transposed9(acc[0], lane);
        // the group's chunk positions (< CHUNK <= 256), one byte each, so that
        // a lane picks its row's entry with one shift
        const uint32_t epack = (uint32_t)(e[0] & 0xff) | ((uint32_t)(e[1] & 0xff) << 8) |
                               ((uint32_t)(e[2] & 0xff) << 16) | ((uint32_t)(e[3] & 0xff) << 24);
        const int li = lane & 15;
        if ((li & 1) == 0 || li == 1) {   // one lane per value of the row
          const int r = lane >> 4, u = (r >> 1) | ((r & 1) << 1);
          const int eu = (int)((epack >> (8 * u)) & 0xffu);
          const int c = (li & 1) ? 8 : (((li >> 1) & 1) << 2) | (((li >> 2) & 1) << 1) | ((li >> 3) & 1);
          if (u < cnt) {
            red[eu][w][c] = tot;
            if (li == 1) wany8[eu * 4 + w] = 1;
          }
        }
      }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += S::NT) {
      const uint32_t wa = wany[i];
      if (wa == 0u) continue;
      float v[9];   // -0 + x is x for every x, so the first wave's add folds away
#pragma unroll
      for (int c = 0; c < 9; ++c) v[c] = -0.0f;
#pragma unroll
      for (int ww = 0; ww < S::NW; ++ww) {
        if (!((wa >> (8 * ww)) & 0xffu)) continue;
#pragma unroll
        for (int c = 0; c < 9; ++c) v[c] += red[i][ww][c];
      }
      // emission slot: the splat's offset + row-major index of this tile in its rect
      const uint32_t sp = sid[i];
      const int4 r = a.rect[sp];
      const uint32_t e = a.soff[sp] + (uint32_t)((ty - r.y) * (r.z - r.x + 1) + (tx - r.x));
      float4* dst = reinterpret_cast<float4*>(a.part + (int64_t)e * kPartF);
      dst[0] = make_float4(v[0], v[1], v[2], v[3]);
      dst[1] = make_float4(v[4], v[5], v[6], v[7]);
      dst[2] = make_float4(v[8], 0.0f, 0.0f, 0.0f);
      a.part_flag[e] = 1;
    }
  }
}

void launch_composite_bwd(const PassArgs& a, const float* dimages, const float* images, int chunk, hipStream_t s) {
  (void)images;
  if (a.n_tiles == 0) return;
  const dim3 grid(a.n_tiles);
#define GBR_BWD(TT, CC) \
  hipLaunchKernelGGL((composite_bwd_kernel<TT, CC>), grid, dim3(TileShapeB<TT>::NT), 0, s, a, dimages)
#define GBR_BWD_T(TT)                      \
  if (chunk == 64) GBR_BWD(TT, 64);        \
  else if (chunk == 128) GBR_BWD(TT, 128); \
  else GBR_BWD(TT, 256);
  if (a.tile == 8) { GBR_BWD_T(8) }
  else if (a.tile == 16) { GBR_BWD_T(16) }
  else { GBR_BWD_T(32) }
#undef GBR_BWD_T
#undef GBR_BWD
}

// ---------------------------------------------------------------- gather + projection adjoint
// One thread per splat.  It sums its entries' partials in row-major tile
// order (unflagged entries -- no contributing pixel, or past the tile's last
// used position -- are zero): the flags of a 64-entry window are read as four
// 16-byte loads, then the flagged partials 4 at a time, all loads in flight
// before any is used, and each consumed flag is reset to 0 for the next
// pass.  It then chains the 9 sums back through the conic, the EWA
// projection and the activations in float64 and writes the splat's draw
// row.  (As two passes, the sums written to the row and read back, it took
// 12 us more: the adjoint's lower occupancy hides the gather's loads well
// enough.)
// Flag bytes (0 or 1) of 4 entries -> 4 bits.
__device__ __forceinline__ uint32_t flag_nibble(uint32_t w) {
  return (w & 1u) | ((w >> 7) & 2u) | ((w >> 14) & 4u) | ((w >> 21) & 8u);
}

// The 9 sums of a splat over its c entries from off on (acc zeroed by the caller).
__device__ __forceinline__ void gather_splat_sums(const PassArgs& a, uint32_t off, uint32_t c, float (&acc)[9]) {
  const uint32_t end = off + c;
  const uint32_t* fw = reinterpret_cast<const uint32_t*>(a.part_flag);   // padded by 64 bytes past the capacity
  // windows of 64 entries starting at a multiple of 16: the 16 flag words
  // are read as four aligned 16-byte loads and turned into a bit mask of
  // the flagged entries, whose partials are then read 4 at a time (all 4
  // in flight together)
  for (uint32_t e0 = off & ~15u; e0 < end; e0 += 64) {
    uint32_t w[16];
    const uint4* fq = reinterpret_cast<const uint4*>(fw + (e0 >> 2));
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const uint4 x = fq[k];
      w[4 * k] = x.x; w[4 * k + 1] = x.y; w[4 * k + 2] = x.z; w[4 * k + 3] = x.w;
    }
    unsigned long long m = 0ull;
#pragma unroll
    for (int k = 0; k < 16; ++k) m |= (unsigned long long)flag_nibble(w[k]) << (4 * k);
    // keep [off, end) only
    const uint32_t lo = off > e0 ? off - e0 : 0u;
    const uint32_t hi = end - e0 < 64u ? end - e0 : 64u;
    m &= (hi >= 64u ? ~0ull : ((1ull << hi) - 1ull)) & ~((1ull << lo) - 1ull);
    while (m) {
      uint32_t e[4];
      bool v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        v[u] = m != 0ull;
        e[u] = v[u] ? e0 + (uint32_t)(__ffsll((long long)m) - 1) : off;   // off: in range, unused
        m &= m - 1ull;
      }
      float4 q[4][3];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const float4* src = reinterpret_cast<const float4*>(a.part + (int64_t)e[u] * kPartF);
        q[u][0] = src[0]; q[u][1] = src[1]; q[u][2] = src[2];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (!v[u]) continue;
        // the flag goes back to 0 for the next pass (only this splat's
        // flags are written; neighbours mask this entry out of their windows)
        a.part_flag[e[u]] = 0;
        acc[0] += q[u][0].x; acc[1] += q[u][0].y; acc[2] += q[u][0].z; acc[3] += q[u][0].w;
        acc[4] += q[u][1].x; acc[5] += q[u][1].y; acc[6] += q[u][1].z; acc[7] += q[u][1].w;
        acc[8] += q[u][2].x;
      }
    }
  }
}

// A workgroup per (frame, 64 of its splats): the frame is the grid's y
// index, so its camera is read at uniform addresses.  One-wave workgroups
// let the chip's last round of waves be filled finely (the splats' gathers
// differ in length).
constexpr int kAdjThreads = 64;
__global__ __launch_bounds__(kAdjThreads) void proj_adjoint_kernel(PassArgs a, const float* __restrict__ raw,
                                                                   float* __restrict__ draw) {
  const int b = blockIdx.y;
  const FrameDev& F = a.frames[b];
  const int64_t n = (int64_t)blockIdx.x * kAdjThreads + threadIdx.x;
  if (n >= F.gauss_count) return;
  const int64_t s = F.gauss_base + n;
  float4* out = reinterpret_cast<float4*>(draw + s * kNF);
  // the overflow flag, the count, the entry offset and the splat's blended
  // Gaussian are read together, so that one load latency precedes the
  // gather instead of three
  const uint32_t ovf = a.status->overflow, c = a.cnt[s], off = a.soff[s];
  const float4* src = reinterpret_cast<const float4*>(raw + s * kNF);
  float4 v0 = src[0], v1 = src[1];
  const float4 v2 = src[2];
  // (an empty use before the branch, or the compiler sinks the last two
  // loads past it and waits for the count first)
  asm volatile("" ::"v"(ovf), "v"(off), "v"(v0.x), "v"(v0.y), "v"(v0.z), "v"(v0.w), "v"(v1.x), "v"(v1.y), "v"(v1.z),
               "v"(v1.w), "v"(v2.x), "v"(v2.y), "v"(v2.z));
  if (ovf || c == 0) {
    const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
    out[0] = z; out[1] = z; out[2] = z; out[3] = z;
    return;
  }
  float acc[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) acc[k] = 0.0f;
  gather_splat_sums(a, off, c, acc);

  // ---- recompute the forward quantities (float64) ----
  if (a.tg.on) tangent_deform(a.tg, b, n, v0, v1, v0, v1);   // as the forward pass did
  const float gp[11] = {v0.x, v0.y, v0.z, v0.w, v1.x, v1.y, v1.z, v1.w, v2.x, v2.y, v2.z};
  const double mu0 = gp[0], mu1 = gp[1], mu2 = gp[2];
  double R[9], tcam[3];
  for (int i = 0; i < 9; ++i) R[i] = F.R[i];
  for (int i = 0; i < 3; ++i) tcam[i] = R[3 * i] * mu0 + R[3 * i + 1] * mu1 + R[3 * i + 2] * mu2 + (double)F.t[i];
  const double tx = tcam[0], ty = tcam[1], tz = tcam[2];
  const double qraw[4] = {gp[3], gp[4], gp[5], gp[6]};
  const double qn2 = qraw[0] * qraw[0] + qraw[1] * qraw[1] + qraw[2] * qraw[2] + qraw[3] * qraw[3];
  const double qlen = sqrt(qn2);
  const double qw = qraw[0] / qlen, qx = qraw[1] / qlen, qy = qraw[2] / qlen, qz = qraw[3] / qlen;
  const double sc[3] = {exp((double)gp[7]), exp((double)gp[8]), exp((double)gp[9])};
  const double o = 1.0 / (1.0 + exp(-(double)gp[10]));
  double Rq[9];
  Rq[0] = 1.0 - 2.0 * (qy * qy + qz * qz); Rq[1] = 2.0 * (qx * qy - qw * qz); Rq[2] = 2.0 * (qx * qz + qw * qy);
  Rq[3] = 2.0 * (qx * qy + qw * qz); Rq[4] = 1.0 - 2.0 * (qx * qx + qz * qz); Rq[5] = 2.0 * (qy * qz - qw * qx);
  Rq[6] = 2.0 * (qx * qz - qw * qy); Rq[7] = 2.0 * (qy * qz + qw * qx); Rq[8] = 1.0 - 2.0 * (qx * qx + qy * qy);
  double M[9];
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 3; ++k) M[3 * i + k] = Rq[3 * i + k] * sc[k];
  const double iz = 1.0 / tz;
  const double fx = F.fx, fy = F.fy;
  const double jx = fx * iz, jy = fy * iz, ux = -fx * tx * iz * iz, uy = -fy * ty * iz * iz;
  double Wm[6];
  for (int k = 0; k < 3; ++k) {
    Wm[k] = jx * R[k] + ux * R[6 + k];
    Wm[3 + k] = jy * R[3 + k] + uy * R[6 + k];
  }
  double V[6];
  for (int i = 0; i < 2; ++i)
    for (int k = 0; k < 3; ++k) V[3 * i + k] = Wm[3 * i] * M[k] + Wm[3 * i + 1] * M[3 + k] + Wm[3 * i + 2] * M[6 + k];
  const double sa = V[0] * V[0] + V[1] * V[1] + V[2] * V[2] + kLowPass;
  const double sb = V[0] * V[3] + V[1] * V[4] + V[2] * V[5];
  const double scc = V[3] * V[3] + V[4] * V[4] + V[5] * V[5] + kLowPass;
  const double det = sa * scc - sb * sb;
  const double QA = scc / det, QB = -sb / det, QC = sa / det;

  // ---- record-space gradient -> conic coefficients of q = A dx^2 + 2B dx dy + C dy^2 ----
  // dL/dpower = ln 2 * alpha * dL/dalpha, so the moments of t carry a factor ln 2
  double am[5];
  for (int k = 0; k < 5; ++k) am[k] = (double)acc[k] * kLn2;
  const double dA = am[2] * (-0.5 * kLog2e);
  const double dB = am[3] * (-kLog2e);      // cb = -log2e * B  (coefficient of dx dy is 2B)
  const double dC = am[4] * (-0.5 * kLog2e);
  // conic -> Sigma2 (symmetric):  dS = -Q dQ Q with dQ = [[dA, dB/2], [dB/2, dC]]
  const double h = 0.5 * dB;
  const double t00 = QA * dA + QB * h, t01 = QA * h + QB * dC;
  const double t10 = QB * dA + QC * h, t11 = QB * h + QC * dC;
  const double g00 = -(t00 * QA + t01 * QB);
  const double g01 = -(t00 * QB + t01 * QC);
  const double g11 = -(t10 * QB + t11 * QC);
  // Sigma2 = V V^T + c I:  dV = 2 G V
  double dV[6];
  for (int k = 0; k < 3; ++k) {
    dV[k] = 2.0 * (g00 * V[k] + g01 * V[3 + k]);
    dV[3 + k] = 2.0 * (g01 * V[k] + g11 * V[3 + k]);
  }
  // V = W M:  dW = dV M^T,  dM = W^T dV
  double dW[6], dM[9];
  for (int i = 0; i < 2; ++i)
    for (int k = 0; k < 3; ++k)
      dW[3 * i + k] = dV[3 * i] * M[3 * k] + dV[3 * i + 1] * M[3 * k + 1] + dV[3 * i + 2] * M[3 * k + 2];
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 3; ++k) dM[3 * i + k] = Wm[i] * dV[k] + Wm[3 + i] * dV[3 + k];
  // W rows: jx R0 + ux R2, jy R1 + uy R2  ->  d(jx), d(ux), d(jy), d(uy)
  double djx = 0, dux = 0, djy = 0, duy = 0;
  for (int k = 0; k < 3; ++k) {
    djx += dW[k] * R[k]; dux += dW[k] * R[6 + k];
    djy += dW[3 + k] * R[3 + k]; duy += dW[3 + k] * R[6 + k];
  }
  // jx = fx/tz, ux = -fx tx/tz^2, jy = fy/tz, uy = -fy ty/tz^2; mean = (fx tx/tz + cx, fy ty/tz + cy)
  // mean: d power / d mean = -(2 ca dx + cb dy, cb dx + 2 cc dy), summed as (sum dpw dx, sum dpw dy)
  const double ca = -0.5 * kLog2e * QA, cbq = -kLog2e * QB, cc = -0.5 * kLog2e * QC;
  const double dmx = -(2.0 * ca * am[0] + cbq * am[1]);
  const double dmy = -(cbq * am[0] + 2.0 * cc * am[1]);
  double dtx = dux * (-fx * iz * iz) + dmx * fx * iz;
  double dty = duy * (-fy * iz * iz) + dmy * fy * iz;
  double dtz = djx * (-fx * iz * iz) + dux * (2.0 * fx * tx * iz * iz * iz) + djy * (-fy * iz * iz) +
               duy * (2.0 * fy * ty * iz * iz * iz) - dmx * fx * tx * iz * iz - dmy * fy * ty * iz * iz;
  float res[16];
  for (int k = 0; k < 3; ++k) res[k] = (float)(R[k] * dtx + R[3 + k] * dty + R[6 + k] * dtz);
  // M = Rq diag(s):  dRq = dM diag(s),  ds_k = sum_i dM_ik Rq_ik
  double dRq[9], ds[3];
  for (int k = 0; k < 3; ++k) {
    ds[k] = dM[k] * Rq[k] + dM[3 + k] * Rq[3 + k] + dM[6 + k] * Rq[6 + k];
    for (int i = 0; i < 3; ++i) dRq[3 * i + k] = dM[3 * i + k] * sc[k];
  }
  // d Rq / d (w, x, y, z) of the unit quaternion
  double dq[4];
  dq[0] = 2.0 * (qz * (dRq[3] - dRq[1]) + qy * (dRq[2] - dRq[6]) + qx * (dRq[7] - dRq[5]));
  dq[1] = 2.0 * (qy * (dRq[1] + dRq[3]) + qz * (dRq[2] + dRq[6]) + qw * (dRq[7] - dRq[5]) - 2.0 * qx * (dRq[4] + dRq[8]));
  dq[2] = 2.0 * (qx * (dRq[1] + dRq[3]) + qw * (dRq[2] - dRq[6]) + qz * (dRq[5] + dRq[7]) - 2.0 * qy * (dRq[0] + dRq[8]));
  dq[3] = 2.0 * (qw * (dRq[3] - dRq[1]) + qx * (dRq[2] + dRq[6]) + qy * (dRq[5] + dRq[7]) - 2.0 * qz * (dRq[0] + dRq[4]));
  const double dotq = qw * dq[0] + qx * dq[1] + qy * dq[2] + qz * dq[3];
  const double qh[4] = {qw, qx, qy, qz};
  for (int k = 0; k < 4; ++k) res[3 + k] = (float)((dq[k] - qh[k] * dotq) / qlen);
  for (int k = 0; k < 3; ++k) res[7 + k] = (float)(ds[k] * sc[k]);
  // alpha = 2^(... + log2 o), o = sigmoid(logit):  dL/dlogit = (1 - o) * sum alpha dL/dalpha
  res[10] = (float)((double)acc[5] * (1.0 - o));
  res[11] = acc[6]; res[12] = acc[7]; res[13] = acc[8];
  res[14] = 0.0f; res[15] = 0.0f;
  float4 o0 = make_float4(res[0], res[1], res[2], res[3]);
  float4 o1 = make_float4(res[4], res[5], res[6], res[7]);
  if (a.tg.on) tangent_adjoint(tangent_frame(a.tg, b, n), o0, o1, o0, o1);   // back to tangent space
  out[0] = o0;
  out[1] = o1;
  out[2] = make_float4(res[8], res[9], res[10], res[11]);
  out[3] = make_float4(res[12], res[13], res[14], res[15]);
}

// ---------------------------------------------------------------- colour initialisation (Eq. 3)
// draw_i / draw_1: the colour adjoint of the last render under the target
// images and under all-ones images, i.e. per (frame, Gaussian) the sums of
// w_p I_p and of w_p over the pixels (w_p the Gaussian's compositing weight).
// A thread per Gaussian: if not yet initialised, the first frame whose
// weight exceeds delta sets the base colour to their ratio.
__global__ __launch_bounds__(256) void color_init_apply_kernel(const float* __restrict__ draw_i,
                                                               const float* __restrict__ draw_1, int B, int64_t N,
                                                               float delta, float* __restrict__ bases,
                                                               uint8_t* __restrict__ done) {
  const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (n >= N || done[n]) return;
  for (int b = 0; b < B; ++b) {
    const int64_t r = ((int64_t)b * N + n) * kNF;
    const float w = draw_1[r + 11];
    if (w > delta) {
      bases[n * kNF + 11] = draw_i[r + 11] / w;
      bases[n * kNF + 12] = draw_i[r + 12] / w;
      bases[n * kNF + 13] = draw_i[r + 13] / w;
      done[n] = 1;
      return;
    }
  }
}

void launch_color_init_apply(const float* draw_i, const float* draw_1, int B, int64_t N, float delta, float* bases,
                             uint8_t* done, hipStream_t s) {
  if (N == 0) return;
  hipLaunchKernelGGL(color_init_apply_kernel, dim3(div_up(N, 256)), dim3(256), 0, s, draw_i, draw_1, B, N, delta,
                     bases, done);
}

void launch_gather_bwd(const PassArgs& a, const float* raw, float* draw, int64_t max_frame_splats, hipStream_t s) {
  if (a.n_splats == 0 || max_frame_splats == 0) return;
  hipLaunchKernelGGL(proj_adjoint_kernel, dim3(div_up(max_frame_splats, kAdjThreads), a.B), dim3(kAdjThreads), 0, s, a,
                     raw, draw);
}

// ---------------------------------------------------------------- loss
// kind 1: mean |x - y| (Sec. 3.2 L1 colour loss), kind 2: mean (x - y)^2.
// Per-block float64 partial sums, then one block sums them in order.
constexpr int kLossThreads = 256;
constexpr int kLossPerBlock = kLossThreads * 16;

__global__ __launch_bounds__(kLossThreads) void loss_kernel(const float* __restrict__ x, const float* __restrict__ y,
                                                             int64_t n, int kind, float* __restrict__ dx,
                                                             double* __restrict__ partials,
                                                             const StatusDev* status) {
  __shared__ double sm[kLossThreads];
  const int64_t base = (int64_t)blockIdx.x * kLossPerBlock;
  const float inv = 1.0f / (float)n;
  // loads issued unconditionally (index clamped into range, n >= 1), then masked
  float xv[16], yv[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int64_t k = min(base + (int64_t)i * kLossThreads + threadIdx.x, n - 1);
    xv[i] = x[k];
    yv[i] = y[k];
  }
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int64_t k = base + (int64_t)i * kLossThreads + threadIdx.x;
    if (k < n) {
      const float d = xv[i] - yv[i];
      if (kind == 1) {
        s += fabs((double)d);
        dx[k] = (d > 0.0f ? inv : (d < 0.0f ? -inv : 0.0f));
      } else {
        s += (double)d * (double)d;
        dx[k] = 2.0f * d * inv;
      }
    }
  }
  sm[threadIdx.x] = s;
  __syncthreads();
  for (int w = kLossThreads / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) sm[threadIdx.x] += sm[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = sm[0];
  (void)status;
}

// Thread t adds partials t, t + 256, ... in order (16 loads in flight at a
// time; a missing one adds 0), then a fixed tree over the threads.
__global__ void loss_final_kernel(const double* __restrict__ partials, int nb, int64_t n, StatusDev* status) {
  __shared__ double sm[256];
  double s = 0.0;
  for (int i0 = threadIdx.x; i0 < nb; i0 += 16 * 256) {
    double v[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int i = i0 + j * 256;
      v[j] = i < nb ? partials[i] : 0.0;
    }
#pragma unroll
    for (int j = 0; j < 16; ++j) s += v[j];
  }
  sm[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sm[threadIdx.x] += sm[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) status->loss = (float)(sm[0] / (double)n);
}

int64_t loss_partials(int64_t n_floats) { return div_up(n_floats, kLossPerBlock); }

void launch_loss(const PassArgs& a, const float* images, const float* targets, int kind, float* dimages,
                 float* partials, int64_t n_partials, hipStream_t s) {
  const int64_t n = a.n_pixels * 3;
  if (n == 0) return;
  const int nb = div_up(n, kLossPerBlock);
  (void)n_partials;
  double* part = reinterpret_cast<double*>(partials);
  hipLaunchKernelGGL(loss_kernel, dim3(nb), dim3(kLossThreads), 0, s, images, targets, n, kind, dimages, part,
                     a.status);
  hipLaunchKernelGGL(loss_final_kernel, dim3(1), dim3(256), 0, s, part, nb, n, a.status);
}

}  // namespace gbr
