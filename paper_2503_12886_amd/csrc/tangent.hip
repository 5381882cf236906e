// Tangent-space Gaussians (Sec. 3.1; Eq. 4 and Alg. 1 of the appendix):
// every Gaussian is bound to a mesh triangle with fixed barycentric
// coordinates, and its position and rotation live in that triangle's
// tangent frame.  Per frame, the deformed mesh gives each triangle a TBN
// matrix R = [T B N] (T, B solving e1 = du1 T + dv1 B, e2 = du2 T + dv2 B;
// N the unit normal) and the Gaussians are carried to the deformed space:
// x_D = R x_T + t (t the barycentric point), q_D = q_R (x) q_T with q_R the
// unit quaternion of R's Gram-Schmidt frame [T^, B^, T^ x B^]; the other
// attributes pass through.  The adjoint is dx_T = R^T dx_D,
// dq_T = conj(q_R) (x) dq_D.  Frame quantities are formed in float64 from
// the float32 inputs and rounded once.
#include "tangent_ops.h"

namespace gbr {

// frames: [B][F][kFrameF]: R row-major (R[i][j] = component i of column j), q_R (w, x, y, z)

__device__ __forceinline__ void quat_of_frame(const double G[9], double q[4]) {
  const double tr = G[0] + G[4] + G[8];
  if (tr > 0.0) {
    const double s = 2.0 * sqrt(1.0 + tr);
    q[0] = 0.25 * s; q[1] = (G[7] - G[5]) / s; q[2] = (G[2] - G[6]) / s; q[3] = (G[3] - G[1]) / s;
  } else if (G[0] > G[4] && G[0] > G[8]) {
    const double s = 2.0 * sqrt(1.0 + G[0] - G[4] - G[8]);
    q[0] = (G[7] - G[5]) / s; q[1] = 0.25 * s; q[2] = (G[1] + G[3]) / s; q[3] = (G[2] + G[6]) / s;
  } else if (G[4] > G[8]) {
    const double s = 2.0 * sqrt(1.0 + G[4] - G[0] - G[8]);
    q[0] = (G[2] - G[6]) / s; q[1] = (G[1] + G[3]) / s; q[2] = 0.25 * s; q[3] = (G[5] + G[7]) / s;
  } else {
    const double s = 2.0 * sqrt(1.0 + G[8] - G[0] - G[4]);
    q[0] = (G[3] - G[1]) / s; q[1] = (G[2] + G[6]) / s; q[2] = (G[5] + G[7]) / s; q[3] = 0.25 * s;
  }
  const double inv = 1.0 / sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  const double sg = q[0] >= 0.0 ? inv : -inv;
  for (int k = 0; k < 4; ++k) q[k] *= sg;
}

__global__ __launch_bounds__(256) void tbn_kernel(const float* __restrict__ verts, const int32_t* __restrict__ faces,
                                                  const float* __restrict__ face_uv, int B, int V, int F,
                                                  float* __restrict__ frames) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= (int64_t)B * F) return;
  const int b = (int)(i / F), f = (int)(i % F);
  int vi[3];
  for (int k = 0; k < 3; ++k) vi[k] = min(max(faces[3 * f + k], 0), V - 1);   // out-of-range indices clamped
  const float* vb = verts + (int64_t)b * V * 3;
  double p[3][3];
  for (int k = 0; k < 3; ++k)
    for (int c = 0; c < 3; ++c) p[k][c] = vb[(int64_t)vi[k] * 3 + c];
  const float* uv = face_uv + (int64_t)f * 6;
  const double du1 = (double)uv[2] - uv[0], dv1 = (double)uv[3] - uv[1];
  const double du2 = (double)uv[4] - uv[0], dv2 = (double)uv[5] - uv[1];
  double e1[3], e2[3], T[3], Bt[3], N[3];
  for (int c = 0; c < 3; ++c) { e1[c] = p[1][c] - p[0][c]; e2[c] = p[2][c] - p[0][c]; }
  // [e1; e2] = [[du1, dv1], [du2, dv2]] [T; B]
  const double det = du1 * dv2 - dv1 * du2;
  for (int c = 0; c < 3; ++c) {
    T[c] = (dv2 * e1[c] - dv1 * e2[c]) / det;
    Bt[c] = (du1 * e2[c] - du2 * e1[c]) / det;
  }
  N[0] = e1[1] * e2[2] - e1[2] * e2[1];
  N[1] = e1[2] * e2[0] - e1[0] * e2[2];
  N[2] = e1[0] * e2[1] - e1[1] * e2[0];
  const double nl = sqrt(N[0] * N[0] + N[1] * N[1] + N[2] * N[2]);
  for (int c = 0; c < 3; ++c) N[c] /= nl;
  // Gram-Schmidt frame of [T B]
  double t[3], bb[3], nn[3];
  const double tl = sqrt(T[0] * T[0] + T[1] * T[1] + T[2] * T[2]);
  for (int c = 0; c < 3; ++c) t[c] = T[c] / tl;
  const double bt = Bt[0] * t[0] + Bt[1] * t[1] + Bt[2] * t[2];
  for (int c = 0; c < 3; ++c) bb[c] = Bt[c] - bt * t[c];
  const double bl = sqrt(bb[0] * bb[0] + bb[1] * bb[1] + bb[2] * bb[2]);
  for (int c = 0; c < 3; ++c) bb[c] /= bl;
  nn[0] = t[1] * bb[2] - t[2] * bb[1];
  nn[1] = t[2] * bb[0] - t[0] * bb[2];
  nn[2] = t[0] * bb[1] - t[1] * bb[0];
  const double G[9] = {t[0], bb[0], nn[0], t[1], bb[1], nn[1], t[2], bb[2], nn[2]};
  double q[4];
  quat_of_frame(G, q);
  float* out = frames + i * kFrameF;
  for (int r = 0; r < 3; ++r) {
    out[3 * r + 0] = (float)T[r];
    out[3 * r + 1] = (float)Bt[r];
    out[3 * r + 2] = (float)N[r];
  }
  for (int k = 0; k < 4; ++k) out[9 + k] = (float)q[k];
  out[13] = out[14] = out[15] = 0.0f;
}

__global__ __launch_bounds__(256) void tangent_fwd_kernel(const float* __restrict__ raw_t, TangentArgs tg, int B,
                                                          float* __restrict__ raw_d) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= (int64_t)B * tg.N) return;
  const int b = (int)(i / tg.N);
  const int64_t n = i % tg.N;
  const float4* src = reinterpret_cast<const float4*>(raw_t + i * kNF);
  float4* dst = reinterpret_cast<float4*>(raw_d + i * kNF);
  float4 d0, d1;
  tangent_deform(tg, b, n, src[0], src[1], d0, d1);
  dst[0] = d0;
  dst[1] = d1;
  dst[2] = src[2];
  dst[3] = src[3];
}

__global__ __launch_bounds__(256) void tangent_bwd_kernel(const float* __restrict__ draw_d, TangentArgs tg, int B,
                                                          float* __restrict__ draw_t) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= (int64_t)B * tg.N) return;
  const int b = (int)(i / tg.N);
  const int64_t n = i % tg.N;
  const float4* src = reinterpret_cast<const float4*>(draw_d + i * kNF);
  float4* dst = reinterpret_cast<float4*>(draw_t + i * kNF);
  float4 o0, o1;
  tangent_adjoint(tangent_frame(tg, b, n), src[0], src[1], o0, o1);
  dst[0] = o0;
  dst[1] = o1;
  dst[2] = src[2];
  dst[3] = src[3];
}

void launch_tangent_frames(const float* verts, const int32_t* faces, const float* face_uv, int B, int V, int F,
                           float* frames, hipStream_t s) {
  const int64_t n = (int64_t)B * F;
  if (n == 0) return;
  hipLaunchKernelGGL(tbn_kernel, dim3(div_up(n, 256)), dim3(256), 0, s, verts, faces, face_uv, B, V, F, frames);
}

void launch_tangent_fwd(const float* raw_t, const int32_t* tri, const float* bary, const float* verts,
                        const int32_t* faces, const float* frames, int B, int64_t N, int V, int F, float* raw_d,
                        hipStream_t s) {
  const int64_t n = (int64_t)B * N;
  if (n == 0) return;
  const TangentArgs tg{tri, bary, verts, faces, frames, N, V, F, 1, 0};
  hipLaunchKernelGGL(tangent_fwd_kernel, dim3(div_up(n, 256)), dim3(256), 0, s, raw_t, tg, B, raw_d);
}

void launch_tangent_bwd(const float* draw_d, const int32_t* tri, const float* frames, int B, int64_t N, int F,
                        float* draw_t, hipStream_t s) {
  const int64_t n = (int64_t)B * N;
  if (n == 0) return;
  const TangentArgs tg{tri, nullptr, nullptr, nullptr, frames, N, 0, F, 1, 0};
  hipLaunchKernelGGL(tangent_bwd_kernel, dim3(div_up(n, 256)), dim3(256), 0, s, draw_d, tg, B, draw_t);
}

}  // namespace gbr
