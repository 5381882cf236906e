// The tangent-space transform of one Gaussian and its adjoint (Sec. 3.1,
// Eq. 4; Alg. 1 of the appendix), shared by the stand-alone transform
// kernels and the pass kernels that apply it on the fly, so that both form
// the same bits: x_D = R x_T + t (t the barycentric point of the Gaussian's
// triangle on the frame's deformed mesh, R = [T B N]), q_D = q_R (x) q_T;
// dx_T = R^T dx_D, dq_T = conj(q_R) (x) dq_D.  Formed in float64 from the
// float32 inputs and rounded once.
#pragma once

#include "gbr_internal.h"

namespace gbr {

constexpr int kFrameF = 16;   // floats per (frame, triangle) record: R row-major, q_R (w, x, y, z), 3 unused

__device__ __forceinline__ void qmul(const double p[4], const double q[4], double o[4]) {
  o[0] = p[0] * q[0] - p[1] * q[1] - p[2] * q[2] - p[3] * q[3];
  o[1] = p[0] * q[1] + p[1] * q[0] + p[2] * q[3] - p[3] * q[2];
  o[2] = p[0] * q[2] - p[1] * q[3] + p[2] * q[0] + p[3] * q[1];
  o[3] = p[0] * q[3] + p[1] * q[2] - p[2] * q[1] + p[3] * q[0];
}

// The (frame, triangle) record of Gaussian n in frame b (triangle index clamped).
__device__ __forceinline__ const float* tangent_frame(const TangentArgs& tg, int b, int64_t n) {
  const int f = min(max(tg.tri[n], 0), tg.F - 1);
  return tg.frames + ((int64_t)b * tg.F + f) * kFrameF;
}

// The first two float4 of a tangent-space record (position, quaternion,
// first log-scale) carried to frame b's deformed mesh; the rest passes.
__device__ __forceinline__ void tangent_deform(const TangentArgs& tg, int b, int64_t n, float4 a0, float4 a1,
                                               float4& d0, float4& d1) {
  const int f = min(max(tg.tri[n], 0), tg.F - 1);
  const float* fr = tg.frames + ((int64_t)b * tg.F + f) * kFrameF;
  const float* vb = tg.verts + (int64_t)b * tg.V * 3;
  double t[3] = {0.0, 0.0, 0.0};
  for (int k = 0; k < 3; ++k) {
    const int v = min(max(tg.faces[3 * f + k], 0), tg.V - 1);
    const double w = tg.bary[n * 3 + k];
    for (int c = 0; c < 3; ++c) t[c] += w * (double)vb[(int64_t)v * 3 + c];
  }
  const double x[3] = {a0.x, a0.y, a0.z};
  double xd[3];
  for (int r = 0; r < 3; ++r)
    xd[r] = (double)fr[3 * r] * x[0] + (double)fr[3 * r + 1] * x[1] + (double)fr[3 * r + 2] * x[2] + t[r];
  const double qr[4] = {fr[9], fr[10], fr[11], fr[12]};
  const double qt[4] = {a0.w, a1.x, a1.y, a1.z};
  double qd[4];
  qmul(qr, qt, qd);
  d0 = make_float4((float)xd[0], (float)xd[1], (float)xd[2], (float)qd[0]);
  d1 = make_float4((float)qd[1], (float)qd[2], (float)qd[3], a1.w);
}

// The adjoint of tangent_deform on the first two float4 of a gradient record.
__device__ __forceinline__ void tangent_adjoint(const float* fr, float4 g0, float4 g1, float4& o0, float4& o1) {
  const double gx[3] = {g0.x, g0.y, g0.z};
  double dx[3];
  for (int c = 0; c < 3; ++c)
    dx[c] = (double)fr[c] * gx[0] + (double)fr[3 + c] * gx[1] + (double)fr[6 + c] * gx[2];   // R^T gx
  const double qc[4] = {fr[9], -(double)fr[10], -(double)fr[11], -(double)fr[12]};
  const double gq[4] = {g0.w, g1.x, g1.y, g1.z};
  double dq[4];
  qmul(qc, gq, dq);
  o0 = make_float4((float)dx[0], (float)dx[1], (float)dx[2], (float)dq[0]);
  o1 = make_float4((float)dq[1], (float)dq[2], (float)dq[3], g1.w);
}

}  // namespace gbr
