/*
 * FP64 reference for the Gaussian splatting renderer that the reduced
 * Gaussian blendshape avatar is rendered with (Sec. 3.2 "Batch-parallel
 * Gaussian Rasterization" and Sec. A.3 "Implementation Details": the
 * rasterizer builds on the original 3D Gaussian Splatting renderer).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU path is
 * checked against.  It is plain, slow, single-threaded double-precision C,
 * written from the mathematics, and shares no code, header or constant table
 * with the GPU library.  Only tests, the smoke check and the CPU-baseline leg
 * of the benchmark may load it.
 *
 * Conventions (the paper leaves them open; each is a stated reading):
 *  - a blended Gaussian is 16 floats: position x[0:3], quaternion q[3:7]
 *    stored (w,x,y,z), log-scale s[7:10], opacity logit [10], RGB [11:14],
 *    two unused pad slots [14:16];
 *  - activations after blending (Sec. A.3 says activations follow the
 *    blending): q normalised, s = exp, opacity = sigmoid, colour identity;
 *  - camera: world->camera rotation R (row-major) and translation t, OpenCV
 *    axes (+z forward), pinhole fx, fy, cx, cy, pixel (j, i) sampled at
 *    (j + 0.5, i + 0.5);
 *  - EWA projection with the local affine Jacobian of the perspective map
 *    and a 0.3 px^2 low-pass added to the 2D covariance;
 *  - a Gaussian contributes to a pixel iff alpha >= 1/255, alpha =
 *    min(0.99, o * exp(-q/2)); front-to-back compositing in ascending
 *    (depth, index) order, depth = camera-space z rounded to binary32, and a
 *    pixel stops *before* the Gaussian that would take its transmittance
 *    below 1e-4; output = colour + T_end * background.
 *
 * Compile with -ffp-contract=off so that the arithmetic is what is written.
 */
#define _GNU_SOURCE   /* qsort_r */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NF 16                 /* floats per blended Gaussian */
#define NCAM 20               /* doubles per camera record */
#define NPROJ 24              /* doubles per projected Gaussian */
#define ALPHA_MIN (1.0 / 255.0)
#define ALPHA_MAX 0.99
#define T_MIN 1e-4
#define LOWPASS 0.3
#define BOX_PAD 0.01          /* px added to the exact alpha-support box */

/* camera record: fx fy cx cy R[9] t[3] near bg[3] */
typedef struct {
  double fx, fy, cx, cy, R[9], t[3], near_z, bg[3];
} cam_t;

static void cam_load(const double* c, cam_t* k) {
  k->fx = c[0]; k->fy = c[1]; k->cx = c[2]; k->cy = c[3];
  for (int i = 0; i < 9; ++i) k->R[i] = c[4 + i];
  for (int i = 0; i < 3; ++i) k->t[i] = c[13 + i];
  k->near_z = c[16];
  for (int i = 0; i < 3; ++i) k->bg[i] = c[17 + i];
}

/* Rotation matrix of a unit quaternion (w, x, y, z), row-major. */
static void quat_to_rot(const double q[4], double R[9]) {
  double w = q[0], x = q[1], y = q[2], z = q[3];
  R[0] = 1.0 - 2.0 * (y * y + z * z); R[1] = 2.0 * (x * y - w * z);       R[2] = 2.0 * (x * z + w * y);
  R[3] = 2.0 * (x * y + w * z);       R[4] = 1.0 - 2.0 * (x * x + z * z); R[5] = 2.0 * (y * z - w * x);
  R[6] = 2.0 * (x * z - w * y);       R[7] = 2.0 * (y * z + w * x);       R[8] = 1.0 - 2.0 * (x * x + y * y);
}

/* Everything the forward pass derives for one Gaussian, kept for the adjoint. */
typedef struct {
  int valid;
  double mu[3], qn[4], qnorm, s[3], o, col[3];
  double Rq[9], M[9], S3[9];     /* rotation, M = R diag(s), Sigma3 = M M^T */
  double tc[3];                  /* camera-space position */
  double J[6], Tm[6];            /* 2x3 Jacobian and Tm = J Rcam */
  double S2[4];                  /* 2x2 covariance incl. low-pass */
  double det, Q[4];              /* conic Q = S2^-1 (symmetric) */
  double mx, my, depth;
  float key;                     /* binary32 depth used for ordering */
  double ex, ey;                 /* half extents of the alpha-support box */
  int px0, px1, py0, py1;        /* inclusive pixel box, clipped */
} proj_t;

static void project_one(const double* raw, const cam_t* cam, int W, int H, proj_t* p) {
  memset(p, 0, sizeof(*p));
  for (int i = 0; i < 3; ++i) p->mu[i] = raw[i];
  double qq = 0.0;
  for (int i = 0; i < 4; ++i) qq += raw[3 + i] * raw[3 + i];
  p->qnorm = sqrt(qq);
  for (int i = 0; i < 4; ++i) p->qn[i] = raw[3 + i] / p->qnorm;
  for (int i = 0; i < 3; ++i) p->s[i] = exp(raw[7 + i]);
  p->o = 1.0 / (1.0 + exp(-raw[10]));
  for (int i = 0; i < 3; ++i) p->col[i] = raw[11 + i];

  quat_to_rot(p->qn, p->Rq);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) p->M[3 * i + j] = p->Rq[3 * i + j] * p->s[j];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double a = 0.0;
      for (int k = 0; k < 3; ++k) a += p->M[3 * i + k] * p->M[3 * j + k];
      p->S3[3 * i + j] = a;
    }

  for (int i = 0; i < 3; ++i) {
    double a = cam->t[i];
    for (int k = 0; k < 3; ++k) a += cam->R[3 * i + k] * p->mu[k];
    p->tc[i] = a;
  }
  double tx = p->tc[0], ty = p->tc[1], tz = p->tc[2];
  p->depth = tz;
  p->key = (float)tz;
  if (!(tz > cam->near_z)) return;

  p->J[0] = cam->fx / tz; p->J[1] = 0.0;            p->J[2] = -cam->fx * tx / (tz * tz);
  p->J[3] = 0.0;          p->J[4] = cam->fy / tz;   p->J[5] = -cam->fy * ty / (tz * tz);
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 3; ++j) {
      double a = 0.0;
      for (int k = 0; k < 3; ++k) a += p->J[3 * i + k] * cam->R[3 * k + j];
      p->Tm[3 * i + j] = a;
    }
  /* S2 = Tm S3 Tm^T + lowpass I */
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      double a = 0.0;
      for (int k = 0; k < 3; ++k)
        for (int l = 0; l < 3; ++l) a += p->Tm[3 * i + k] * p->S3[3 * k + l] * p->Tm[3 * j + l];
      p->S2[2 * i + j] = a + (i == j ? LOWPASS : 0.0);
    }
  p->mx = cam->fx * tx / tz + cam->cx;
  p->my = cam->fy * ty / tz + cam->cy;
  p->det = p->S2[0] * p->S2[3] - p->S2[1] * p->S2[2];
  if (!(p->det > 0.0)) return;
  p->Q[0] = p->S2[3] / p->det;
  p->Q[1] = -p->S2[1] / p->det;
  p->Q[2] = -p->S2[2] / p->det;
  p->Q[3] = p->S2[0] / p->det;

  /* alpha >= 1/255  <=>  q <= 2 ln(255 o); the ellipse {d : d^T Q d <= c}
     has axis-aligned half extents sqrt(c S2_00), sqrt(c S2_11). */
  double c = 2.0 * log(255.0 * p->o);
  if (!(c >= 0.0)) return;
  p->ex = sqrt(c * p->S2[0]) + BOX_PAD;
  p->ey = sqrt(c * p->S2[3]) + BOX_PAD;
  /* pixels whose centre j + 0.5 lies in [mx - ex, mx + ex] */
  double fx0 = ceil(p->mx - p->ex - 0.5), fx1 = floor(p->mx + p->ex - 0.5);
  double fy0 = ceil(p->my - p->ey - 0.5), fy1 = floor(p->my + p->ey - 0.5);
  if (fx0 < 0.0) fx0 = 0.0;
  if (fy0 < 0.0) fy0 = 0.0;
  if (fx1 > W - 1.0) fx1 = W - 1.0;
  if (fy1 > H - 1.0) fy1 = H - 1.0;
  if (fx0 > fx1 || fy0 > fy1) return;
  p->px0 = (int)fx0; p->px1 = (int)fx1; p->py0 = (int)fy0; p->py1 = (int)fy1;
  p->valid = 1;
}

/* ---- projection, exported for stage checks ---------------------------------- */
/* out per Gaussian (NPROJ doubles):
   valid mx my S00 S01 S11 A B C depth key o r g b px0 px1 py0 py1 ex ey tx ty tz */
int oracle_project(int64_t N, const double* raw, const double* camd, int W, int H, double* out) {
  cam_t cam; cam_load(camd, &cam);
  for (int64_t n = 0; n < N; ++n) {
    proj_t p; project_one(raw + NF * n, &cam, W, H, &p);
    double* o = out + NPROJ * n;
    o[0] = p.valid; o[1] = p.mx; o[2] = p.my;
    o[3] = p.S2[0]; o[4] = p.S2[1]; o[5] = p.S2[3];
    o[6] = p.Q[0]; o[7] = p.Q[1]; o[8] = p.Q[3];
    o[9] = p.depth; o[10] = (double)p.key; o[11] = p.o;
    o[12] = p.col[0]; o[13] = p.col[1]; o[14] = p.col[2];
    o[15] = p.valid ? p.px0 : -1; o[16] = p.valid ? p.px1 : -1;
    o[17] = p.valid ? p.py0 : -1; o[18] = p.valid ? p.py1 : -1;
    o[19] = p.ex; o[20] = p.ey;
    o[21] = p.tc[0]; o[22] = p.tc[1]; o[23] = p.tc[2];
  }
  return 0;
}

/* ---- depth order ------------------------------------------------------------- */
/* The projections are passed to the comparator as qsort_r's context, so
   concurrent calls (one frame per thread) do not share any state. */
static int cmp_depth(const void* a, const void* b, void* ctx) {
  const proj_t* P = (const proj_t*)ctx;
  int64_t i = *(const int64_t*)a, j = *(const int64_t*)b;
  float ki = P[i].key, kj = P[j].key;
  if (ki < kj) return -1;
  if (ki > kj) return 1;
  return (i < j) ? -1 : (i > j);
}

/* Per-pixel contributor record kept by the forward walk for the adjoint. */
typedef struct { int64_t g; double a, G, alpha, T, dx, dy; } contrib_t;

/* ---- ambiguity margins ---------------------------------------------------------
   A binary32 implementation of the compositing can take a different discrete
   decision from this double-precision walk only where a decision's value is
   within that implementation's error of its threshold.  The margins below are
   first-order bounds on those errors, for an implementation whose inputs are
   the projected quantities (mean, conic, opacity) each rounded to binary32 and
   whose arithmetic is binary32 throughout (u = 2^-24 per operation):

   alpha = o exp(-q/2) with q = A dx^2 + 2 B dx dy + C dy^2, dx = px - mx,
   dy = py - my.  With S = (|A| dx^2 + 2 |B dx dy| + |C| dy^2) / 2 (the
   exponent's terms) and ln o:
     - the rounded mean moves dx by u |mx| and the subtraction rounds by
       u |dx|: d(q/2)/dmx = -(A dx + B dy), so the exponent moves by at most
       u (|mx| + |dx|) |A dx + B dy| (likewise in y);
     - the rounded conic coefficients: u S; two products per term: 2 u S; the
       three additions (partial sums bounded by S + |ln o|): 3 u (S + |ln o|);
       a change of base to exp2: u (S + |ln o|); the rounded opacity: u |ln o|;
     - the exponential itself: 2 ulp, 4 u relative.
   The relative error of alpha is at most the exponent's absolute error plus
   4 u.  A product (1 - alpha_i) over the taken entries then carries, per
   factor, alpha/(1 - alpha) times alpha's relative error (u for the clamped
   0.99, whose binary32 value is within u of it), one rounding for 1 - alpha
   and one for the product: the transmittance's relative error is at most the
   sum over the factors so far.  The thresholds 1/255, 0.99 and 1e-4 are
   themselves within u of their binary32 values. */
#define U32 (1.0 / 16777216.0)

static double alpha_rel_bound(const proj_t* p, double dx, double dy) {
  double gx = fabs(p->Q[0] * dx + p->Q[1] * dy), gy = fabs(p->Q[1] * dx + p->Q[3] * dy);
  double S = 0.5 * (fabs(p->Q[0]) * dx * dx + 2.0 * fabs(p->Q[1] * dx * dy) + fabs(p->Q[3]) * dy * dy);
  double lo = fabs(log(p->o));
  double e = (fabs(p->mx) + fabs(dx)) * gx + (fabs(p->my) + fabs(dy)) * gy + 7.0 * S + 5.0 * lo;
  return U32 * (e + 4.0);
}

/* Walk one pixel's candidates (already in depth order), compositing front to
   back.  Writes the pixel colour, the final transmittance, and the
   contributor list; returns the number of contributors.  `flags` collects the
   decisions that sit within a margin of their threshold: 1 = alpha vs 1/255,
   2 = transmittance stop, 4 = alpha vs the 0.99 clamp.  With eps_a < 0 the
   margins are the binary32 error bounds above (per entry and per pixel);
   otherwise eps_a and eps_t are fixed relative margins for alpha and for the
   transmittance. */
static int64_t composite_pixel(const proj_t* P, const int64_t* cand, int64_t ncand, double px, double py,
                               const double bg[3], double eps_a, double eps_t, double out[3], double* Tend,
                               contrib_t* rec, unsigned* flags) {
  const int derived = eps_a < 0.0;
  double T = 1.0, C[3] = {0.0, 0.0, 0.0};
  double rho = 0.0;                  /* bound on T's relative error so far (derived margins) */
  int64_t n = 0;
  for (int64_t k = 0; k < ncand; ++k) {
    const proj_t* p = &P[cand[k]];
    double dx = px - p->mx, dy = py - p->my;
    double q = p->Q[0] * dx * dx + 2.0 * p->Q[1] * dx * dy + p->Q[3] * dy * dy;
    if (q < 0.0) q = 0.0;
    double G = exp(-0.5 * q);
    double a = p->o * G;
    double ea = derived ? alpha_rel_bound(p, dx, dy) + U32 : eps_a;
    if (fabs(a - ALPHA_MIN) <= ea * a) *flags |= 1u;
    if (a < ALPHA_MIN) continue;
    if (fabs(a - ALPHA_MAX) <= ea * a) *flags |= 4u;
    double alpha = a < ALPHA_MAX ? a : ALPHA_MAX;
    double Tn = T * (1.0 - alpha);
    double ef = (alpha / (1.0 - alpha)) * (a < ALPHA_MAX ? ea : U32) + 2.0 * U32;
    double et = derived ? rho + ef + U32 : eps_t;
    if (fabs(Tn - T_MIN) <= et * Tn) *flags |= 2u;
    if (Tn < T_MIN) break;
    for (int c = 0; c < 3; ++c) C[c] += alpha * T * p->col[c];
    if (rec) {
      rec[n].g = cand[k]; rec[n].a = a; rec[n].G = G; rec[n].alpha = alpha;
      rec[n].T = T; rec[n].dx = dx; rec[n].dy = dy;
    }
    ++n;
    T = Tn;
    rho += ef;
  }
  for (int c = 0; c < 3; ++c) out[c] = C[c] + T * bg[c];
  *Tend = T;
  return n;
}

/* For checks of the margins: the unclamped alpha of Gaussian gidx[m] at the
   point (px[m], py[m]) and the bound on its relative error used above. */
int oracle_alpha_bounds(int64_t N, const double* raw, const double* camd, int W, int H, int64_t M,
                        const int64_t* gidx, const double* px, const double* py, double* alpha, double* bound) {
  cam_t cam; cam_load(camd, &cam);
  for (int64_t m = 0; m < M; ++m) {
    if (gidx[m] < 0 || gidx[m] >= N) return -1;
    proj_t p; project_one(raw + NF * gidx[m], &cam, W, H, &p);
    double dx = px[m] - p.mx, dy = py[m] - p.my;
    double q = p.Q[0] * dx * dx + 2.0 * p.Q[1] * dx * dy + p.Q[3] * dy * dy;
    if (q < 0.0) q = 0.0;
    alpha[m] = p.o * exp(-0.5 * q);
    bound[m] = alpha_rel_bound(&p, dx, dy);
  }
  return 0;
}

/* Candidate lists per 16x16 block of pixels: every valid Gaussian whose pixel
   box meets the block, in depth order.  This only narrows the per-pixel loop;
   the alpha test above decides what contributes. */
#define OB 16
typedef struct { int64_t* idx; int64_t n, cap; } list_t;

static void push(list_t* l, int64_t g) {
  if (l->n == l->cap) {
    l->cap = l->cap ? 2 * l->cap : 64;
    l->idx = (int64_t*)realloc(l->idx, sizeof(int64_t) * l->cap);
  }
  l->idx[l->n++] = g;
}

typedef struct {
  proj_t* P;
  int64_t* order; int64_t nvalid;
  list_t* blocks; int nbx, nby;
} scene_t;

static int scene_build(int64_t N, const double* raw, const cam_t* cam, int W, int H, scene_t* s) {
  s->P = (proj_t*)malloc(sizeof(proj_t) * (N > 0 ? N : 1));
  s->order = (int64_t*)malloc(sizeof(int64_t) * (N > 0 ? N : 1));
  if (!s->P || !s->order) return -1;
  s->nvalid = 0;
  for (int64_t n = 0; n < N; ++n) {
    project_one(raw + NF * n, cam, W, H, &s->P[n]);
    if (s->P[n].valid) s->order[s->nvalid++] = n;
  }
  qsort_r(s->order, (size_t)s->nvalid, sizeof(int64_t), cmp_depth, s->P);
  s->nbx = (W + OB - 1) / OB; s->nby = (H + OB - 1) / OB;
  s->blocks = (list_t*)calloc((size_t)s->nbx * s->nby, sizeof(list_t));
  if (!s->blocks) return -1;
  for (int64_t k = 0; k < s->nvalid; ++k) {
    const proj_t* p = &s->P[s->order[k]];
    for (int by = p->py0 / OB; by <= p->py1 / OB; ++by)
      for (int bx = p->px0 / OB; bx <= p->px1 / OB; ++bx) push(&s->blocks[by * s->nbx + bx], s->order[k]);
  }
  return 0;
}

static void scene_free(scene_t* s) {
  if (s->blocks)
    for (int b = 0; b < s->nbx * s->nby; ++b) free(s->blocks[b].idx);
  free(s->blocks); free(s->order); free(s->P);
}

/* ---- forward render ---------------------------------------------------------- */
/* image: [3][H][W]; T_end, n_contrib, flags: [H][W] (any may be NULL). */
int oracle_render(int64_t N, const double* raw, const double* camd, int W, int H, double* image, double* T_end,
                  int32_t* n_contrib, uint8_t* flags, double eps_a, double eps_t) {
  cam_t cam; cam_load(camd, &cam);
  scene_t s; memset(&s, 0, sizeof(s));
  if (scene_build(N, raw, &cam, W, H, &s)) { scene_free(&s); return -1; }
  for (int i = 0; i < H; ++i)
    for (int j = 0; j < W; ++j) {
      const list_t* l = &s.blocks[(i / OB) * s.nbx + (j / OB)];
      double out[3], Te; unsigned f = 0;
      int64_t n = composite_pixel(s.P, l->idx, l->n, j + 0.5, i + 0.5, cam.bg, eps_a, eps_t, out, &Te, NULL, &f);
      for (int c = 0; c < 3; ++c) image[((int64_t)c * H + i) * W + j] = out[c];
      if (T_end) T_end[(int64_t)i * W + j] = Te;
      if (n_contrib) n_contrib[(int64_t)i * W + j] = (int32_t)n;
      if (flags) flags[(int64_t)i * W + j] = (uint8_t)f;
    }
  scene_free(&s);
  return 0;
}

/* ---- adjoint ----------------------------------------------------------------- */
/* Gradients of the loss with respect to the projected quantities of one
   Gaussian: mean (mx, my), conic entries Q00, Q01 (= Q10, counted once as in
   q = Q00 dx^2 + 2 Q01 dx dy + Q11 dy^2), Q11, opacity, colour. */
typedef struct { double dmx, dmy, dQ00, dQ01, dQ11, dop, dcol[3]; } dproj_t;

/* Chain one Gaussian's projected-quantity gradient back to its 16 raw floats. */
static void project_adjoint(const proj_t* p, const cam_t* cam, const dproj_t* d, double* draw) {
  /* conic -> S2:  Q = S2^-1,  dS2 = -Q dQ Q  with dQ the full symmetric matrix */
  double dQ[4] = {d->dQ00, 0.5 * d->dQ01, 0.5 * d->dQ01, d->dQ11};
  double tmp[4], dS2[4];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) tmp[2 * i + j] = p->Q[2 * i] * dQ[j] + p->Q[2 * i + 1] * dQ[2 + j];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) dS2[2 * i + j] = -(tmp[2 * i] * p->Q[j] + tmp[2 * i + 1] * p->Q[2 + j]);

  /* S2 = Tm S3 Tm^T + c I:  dS3 = Tm^T dS2 Tm,  dTm = 2 dS2 Tm S3 (all symmetric) */
  double dS3[9], dTm[6], TS[6];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double a = 0.0;
      for (int k = 0; k < 2; ++k)
        for (int l = 0; l < 2; ++l) a += p->Tm[3 * k + i] * dS2[2 * k + l] * p->Tm[3 * l + j];
      dS3[3 * i + j] = a;
    }
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 3; ++j) {
      double a = 0.0;
      for (int k = 0; k < 3; ++k) a += p->Tm[3 * i + k] * p->S3[3 * k + j];
      TS[3 * i + j] = a;
    }
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 3; ++j) {
      double a = 0.0;
      for (int k = 0; k < 2; ++k) a += dS2[2 * i + k] * TS[3 * k + j];
      dTm[3 * i + j] = 2.0 * a;
    }

  /* Tm = J Rcam:  dJ = dTm Rcam^T */
  double dJ[6];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 3; ++j) {
      double a = 0.0;
      for (int k = 0; k < 3; ++k) a += dTm[3 * i + k] * cam->R[3 * j + k];
      dJ[3 * i + j] = a;
    }

  double tx = p->tc[0], ty = p->tc[1], tz = p->tc[2];
  double fx = cam->fx, fy = cam->fy;
  double dt[3] = {0.0, 0.0, 0.0};
  /* J entries as functions of t */
  dt[2] += dJ[0] * (-fx / (tz * tz));
  dt[0] += dJ[2] * (-fx / (tz * tz));
  dt[2] += dJ[2] * (2.0 * fx * tx / (tz * tz * tz));
  dt[2] += dJ[4] * (-fy / (tz * tz));
  dt[1] += dJ[5] * (-fy / (tz * tz));
  dt[2] += dJ[5] * (2.0 * fy * ty / (tz * tz * tz));
  /* projected mean */
  dt[0] += d->dmx * fx / tz;
  dt[1] += d->dmy * fy / tz;
  dt[2] += -d->dmx * fx * tx / (tz * tz) - d->dmy * fy * ty / (tz * tz);
  /* t = Rcam mu + tcam */
  for (int k = 0; k < 3; ++k) {
    double a = 0.0;
    for (int i = 0; i < 3; ++i) a += cam->R[3 * i + k] * dt[i];
    draw[k] = a;
  }

  /* S3 = M M^T:  dM = (dS3 + dS3^T) M;  M = Rq diag(s) */
  double dM[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double a = 0.0;
      for (int k = 0; k < 3; ++k) a += (dS3[3 * i + k] + dS3[3 * k + i]) * p->M[3 * k + j];
      dM[3 * i + j] = a;
    }
  double ds[3], dR[9];
  for (int j = 0; j < 3; ++j) {
    double a = 0.0;
    for (int i = 0; i < 3; ++i) a += p->Rq[3 * i + j] * dM[3 * i + j];
    ds[j] = a;
  }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) dR[3 * i + j] = dM[3 * i + j] * p->s[j];

  /* rotation matrix entries as functions of the unit quaternion */
  double w = p->qn[0], x = p->qn[1], y = p->qn[2], z = p->qn[3];
  double dqn[4];
  dqn[0] = 2.0 * (-z * dR[1] + y * dR[2] + z * dR[3] - x * dR[5] - y * dR[6] + x * dR[7]);
  dqn[1] = 2.0 * (y * dR[1] + z * dR[2] + y * dR[3] - 2.0 * x * dR[4] - w * dR[5] + z * dR[6] + w * dR[7] -
                  2.0 * x * dR[8]);
  dqn[2] = 2.0 * (-2.0 * y * dR[0] + x * dR[1] + w * dR[2] + x * dR[3] + z * dR[5] - w * dR[6] + z * dR[7] -
                  2.0 * y * dR[8]);
  dqn[3] = 2.0 * (-2.0 * z * dR[0] - w * dR[1] + x * dR[2] + w * dR[3] - 2.0 * z * dR[4] + y * dR[5] +
                  x * dR[6] + y * dR[7]);
  /* normalisation */
  double dot = 0.0;
  for (int i = 0; i < 4; ++i) dot += p->qn[i] * dqn[i];
  for (int i = 0; i < 4; ++i) draw[3 + i] = (dqn[i] - p->qn[i] * dot) / p->qnorm;
  /* exp, sigmoid, identity */
  for (int j = 0; j < 3; ++j) draw[7 + j] = ds[j] * p->s[j];
  draw[10] = d->dop * p->o * (1.0 - p->o);
  for (int c = 0; c < 3; ++c) draw[11 + c] = d->dcol[c];
  draw[14] = 0.0; draw[15] = 0.0;
}

/* dimage: [3][H][W] = dL/d(output image).  draw: [N][16] = dL/d(blended raw),
   overwritten.  Optional dproj_out: [N][9] gradients w.r.t. (mx, my, Q00, Q01,
   Q11, o, r, g, b) for stage checks. */
/* The adjoint of the rendering: dimage -> draw [N][16] (and the projected-
   quantity gradients dproj_out [N][9] if not NULL: d mean x, y, d conic
   A, 2B, C, d opacity, d colour).  If dproj_mag is not NULL it receives, per
   Gaussian and projected quantity, the sum over pixels of the magnitudes of
   the per-pixel terms that the gradient is the sum of, each term's magnitude
   formed from the magnitudes of its factors (the alpha gradient's colour
   and background-behind parts taken separately), for error bounds of an
   implementation that forms and sums them in binary32. */
int oracle_render_grad(int64_t N, const double* raw, const double* camd, int W, int H, const double* dimage,
                       double* draw, double* dproj_out, double* dproj_mag) {
  cam_t cam; cam_load(camd, &cam);
  scene_t s; memset(&s, 0, sizeof(s));
  if (scene_build(N, raw, &cam, W, H, &s)) { scene_free(&s); return -1; }
  dproj_t* dp = (dproj_t*)calloc((size_t)(N > 0 ? N : 1), sizeof(dproj_t));
  dproj_t* dm = (dproj_t*)calloc((size_t)(N > 0 ? N : 1), sizeof(dproj_t));   /* magnitudes */
  int64_t maxc = 1;
  for (int b = 0; b < s.nbx * s.nby; ++b) if (s.blocks[b].n > maxc) maxc = s.blocks[b].n;
  contrib_t* rec = (contrib_t*)malloc(sizeof(contrib_t) * maxc);
  double* suffix = (double*)malloc(sizeof(double) * 3 * (maxc + 1));
  if (!dp || !dm || !rec || !suffix) { free(dp); free(dm); free(rec); free(suffix); scene_free(&s); return -1; }

  for (int i = 0; i < H; ++i)
    for (int j = 0; j < W; ++j) {
      const list_t* l = &s.blocks[(i / OB) * s.nbx + (j / OB)];
      double out[3], Te; unsigned f = 0;
      int64_t n = composite_pixel(s.P, l->idx, l->n, j + 0.5, i + 0.5, cam.bg, 0.0, 0.0, out, &Te, rec, &f);
      double g[3];
      for (int c = 0; c < 3; ++c) g[c] = dimage[((int64_t)c * H + i) * W + j];
      /* suffix[k] = sum_{m >= k} alpha_m T_m col_m + T_end bg */
      for (int c = 0; c < 3; ++c) suffix[3 * n + c] = Te * cam.bg[c];
      for (int64_t k = n - 1; k >= 0; --k) {
        const proj_t* p = &s.P[rec[k].g];
        for (int c = 0; c < 3; ++c) suffix[3 * k + c] = suffix[3 * (k + 1) + c] + rec[k].alpha * rec[k].T * p->col[c];
      }
      for (int64_t k = 0; k < n; ++k) {
        const contrib_t* r = &rec[k];
        const proj_t* p = &s.P[r->g];
        dproj_t* d = &dp[r->g];
        dproj_t* m = &dm[r->g];
        /* out = sum_m alpha_m T_m col_m + T_end bg, T_{m} = prod_{l<m} (1 - alpha_l) */
        double dalpha = 0.0, dalpha_mag = 0.0;
        for (int c = 0; c < 3; ++c) {
          d->dcol[c] += r->alpha * r->T * g[c];
          m->dcol[c] += fabs(r->alpha * r->T * g[c]);
          dalpha += g[c] * (r->T * p->col[c] - suffix[3 * (k + 1) + c] / (1.0 - r->alpha));
          dalpha_mag += fabs(g[c]) * (r->T * fabs(p->col[c]) + fabs(suffix[3 * (k + 1) + c]) / (1.0 - r->alpha));
        }
        double da = (r->a < ALPHA_MAX) ? dalpha : 0.0;       /* min(0.99, a) */
        d->dop += r->G * da;
        double dG = p->o * da;
        double dq = -0.5 * r->G * dG;                         /* G = exp(-q/2) */
        d->dQ00 += dq * r->dx * r->dx;
        d->dQ01 += dq * 2.0 * r->dx * r->dy;
        d->dQ11 += dq * r->dy * r->dy;
        double ddx = dq * (2.0 * p->Q[0] * r->dx + 2.0 * p->Q[1] * r->dy);
        double ddy = dq * (2.0 * p->Q[1] * r->dx + 2.0 * p->Q[3] * r->dy);
        d->dmx -= ddx;                                        /* dx = px - mx */
        d->dmy -= ddy;
        /* magnitudes: each factor by the magnitudes it is formed from (the
           alpha gradient's two colour terms taken apart) */
        if (r->a < ALPHA_MAX) {
          double dq_mag = 0.5 * r->G * p->o * dalpha_mag;
          m->dop += r->G * dalpha_mag;
          m->dQ00 += dq_mag * r->dx * r->dx;
          m->dQ01 += dq_mag * 2.0 * fabs(r->dx * r->dy);
          m->dQ11 += dq_mag * r->dy * r->dy;
          m->dmx += dq_mag * (2.0 * fabs(p->Q[0] * r->dx) + 2.0 * fabs(p->Q[1] * r->dy));
          m->dmy += dq_mag * (2.0 * fabs(p->Q[1] * r->dx) + 2.0 * fabs(p->Q[3] * r->dy));
        }
      }
    }

  for (int64_t n = 0; n < N; ++n) {
    double* dr = draw + NF * n;
    for (int k = 0; k < NF; ++k) dr[k] = 0.0;
    if (s.P[n].valid) project_adjoint(&s.P[n], &cam, &dp[n], dr);
    if (dproj_out) {
      double* o = dproj_out + 9 * n;
      o[0] = dp[n].dmx; o[1] = dp[n].dmy; o[2] = dp[n].dQ00; o[3] = dp[n].dQ01; o[4] = dp[n].dQ11;
      o[5] = dp[n].dop; o[6] = dp[n].dcol[0]; o[7] = dp[n].dcol[1]; o[8] = dp[n].dcol[2];
    }
    if (dproj_mag) {
      double* o = dproj_mag + 9 * n;
      o[0] = dm[n].dmx; o[1] = dm[n].dmy; o[2] = dm[n].dQ00; o[3] = dm[n].dQ01; o[4] = dm[n].dQ11;
      o[5] = dm[n].dop; o[6] = dm[n].dcol[0]; o[7] = dm[n].dcol[1]; o[8] = dm[n].dcol[2];
    }
  }
  free(dp); free(dm); free(rec); free(suffix);
  scene_free(&s);
  return 0;
}

/* Per-pixel contributor lists as Gaussian indices (for structure checks):
   writes up to `cap` indices per pixel into lists[(i*W+j)*cap ...], counts
   into n_contrib.  Returns 0, or 1 if any pixel had more than `cap`. */
/* The projection's adjoint alone: projected-quantity gradients dproj [N][9]
   (as oracle_render_grad writes them) -> draw [N][16]. */
int oracle_project_adjoint(int64_t N, const double* raw, const double* camd, int W, int H, const double* dproj,
                           double* draw) {
  cam_t cam; cam_load(camd, &cam);
  for (int64_t n = 0; n < N; ++n) {
    proj_t p; project_one(raw + NF * n, &cam, W, H, &p);
    double* dr = draw + NF * n;
    for (int k = 0; k < NF; ++k) dr[k] = 0.0;
    if (!p.valid) continue;
    const double* i = dproj + 9 * n;
    dproj_t d;
    memset(&d, 0, sizeof(d));
    d.dmx = i[0]; d.dmy = i[1]; d.dQ00 = i[2]; d.dQ01 = i[3]; d.dQ11 = i[4];
    d.dop = i[5]; d.dcol[0] = i[6]; d.dcol[1] = i[7]; d.dcol[2] = i[8];
    project_adjoint(&p, &cam, &d, dr);
  }
  return 0;
}

int oracle_contributors(int64_t N, const double* raw, const double* camd, int W, int H, int32_t cap,
                        int64_t* lists, int32_t* n_contrib) {
  cam_t cam; cam_load(camd, &cam);
  scene_t s; memset(&s, 0, sizeof(s));
  if (scene_build(N, raw, &cam, W, H, &s)) { scene_free(&s); return -1; }
  int64_t maxc = 1;
  for (int b = 0; b < s.nbx * s.nby; ++b) if (s.blocks[b].n > maxc) maxc = s.blocks[b].n;
  contrib_t* rec = (contrib_t*)malloc(sizeof(contrib_t) * maxc);
  int over = 0;
  for (int i = 0; i < H; ++i)
    for (int j = 0; j < W; ++j) {
      const list_t* l = &s.blocks[(i / OB) * s.nbx + (j / OB)];
      double out[3], Te; unsigned f = 0;
      int64_t n = composite_pixel(s.P, l->idx, l->n, j + 0.5, i + 0.5, cam.bg, 0.0, 0.0, out, &Te, rec, &f);
      int64_t base = ((int64_t)i * W + j) * cap;
      for (int64_t k = 0; k < n && k < cap; ++k) lists[base + k] = rec[k].g;
      if (n > cap) over = 1;
      n_contrib[(int64_t)i * W + j] = (int32_t)n;
    }
  free(rec);
  scene_free(&s);
  return over;
}
