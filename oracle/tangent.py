"""Float64 reference for the tangent-space Gaussian transform (Sec. 3.1 and
the appendix's Gaussian Transformation: Eq. 4, Alg. 1).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Each Gaussian is bound to one mesh triangle with fixed barycentric (UV)
coordinates; its position and rotation are defined in that triangle's
tangent space and carried to the deformed mesh of every frame:

* TBN of a triangle (Alg. 1): with edges e1 = v1 - v0, e2 = v2 - v0 and UV
  differences (du1, dv1), (du2, dv2), the tangent T and bitangent B solve
  e1 = du1 T + dv1 B, e2 = du2 T + dv2 B (T follows increasing u, B
  increasing v), and N = e1 x e2 / |e1 x e2|; R = [T B N] (columns).
* position (Eq. 4): x_D = R x_T + t, t the barycentric point of the
  triangle;
* rotation (Eq. 4, q_D = R q_T): R is not orthonormal, so the rotation it
  stands for is its Gram-Schmidt frame [T^, B^, T^ x B^] (T^ = T / |T|,
  B^ = the unit part of B orthogonal to T^), as a unit quaternion q_R, and
  q_D = q_R (x) q_T (Hamilton product, (w, x, y, z)), so that
  rot(q_D) = rot(q_R) rot(q_T).  The raw quaternion keeps its norm, which the
  activation divides out.
* every other attribute is unchanged.

The transform is linear in the Gaussian's attributes; its adjoint is
dx_T = R^T dx_D, dq_T = conj(q_R) (x) dq_D, the rest passed through.
"""
from __future__ import annotations

import numpy as np


def tbn(v0, v1, v2, uv0, uv1, uv2) -> np.ndarray:
    """R = [T B N] (3x3, columns) of one triangle."""
    v0, v1, v2 = (np.asarray(v, dtype=np.float64) for v in (v0, v1, v2))
    uv0, uv1, uv2 = (np.asarray(u, dtype=np.float64) for u in (uv0, uv1, uv2))
    e1, e2 = v1 - v0, v2 - v0
    du1, dv1 = uv1 - uv0
    du2, dv2 = uv2 - uv0
    A = np.array([[du1, dv1], [du2, dv2]])          # [e1; e2] = A [T; B]
    TB = np.linalg.solve(A, np.vstack([e1, e2]))
    n = np.cross(e1, e2)
    n /= np.linalg.norm(n)
    return np.column_stack([TB[0], TB[1], n])


def gram_schmidt(R: np.ndarray) -> np.ndarray:
    t = R[:, 0] / np.linalg.norm(R[:, 0])
    b = R[:, 1] - np.dot(R[:, 1], t) * t
    b /= np.linalg.norm(b)
    return np.column_stack([t, b, np.cross(t, b)])


def quat_of_matrix(M: np.ndarray) -> np.ndarray:
    """Unit quaternion (w, x, y, z) of a rotation matrix, w >= 0."""
    tr = np.trace(M)
    if tr > 0:
        s = 2.0 * np.sqrt(1.0 + tr)
        q = np.array([0.25 * s, (M[2, 1] - M[1, 2]) / s, (M[0, 2] - M[2, 0]) / s, (M[1, 0] - M[0, 1]) / s])
    elif M[0, 0] > M[1, 1] and M[0, 0] > M[2, 2]:
        s = 2.0 * np.sqrt(1.0 + M[0, 0] - M[1, 1] - M[2, 2])
        q = np.array([(M[2, 1] - M[1, 2]) / s, 0.25 * s, (M[0, 1] + M[1, 0]) / s, (M[0, 2] + M[2, 0]) / s])
    elif M[1, 1] > M[2, 2]:
        s = 2.0 * np.sqrt(1.0 + M[1, 1] - M[0, 0] - M[2, 2])
        q = np.array([(M[0, 2] - M[2, 0]) / s, (M[0, 1] + M[1, 0]) / s, 0.25 * s, (M[1, 2] + M[2, 1]) / s])
    else:
        s = 2.0 * np.sqrt(1.0 + M[2, 2] - M[0, 0] - M[1, 1])
        q = np.array([(M[1, 0] - M[0, 1]) / s, (M[0, 2] + M[2, 0]) / s, (M[1, 2] + M[2, 1]) / s, 0.25 * s])
    q /= np.linalg.norm(q)
    return q if q[0] >= 0 else -q


def matrix_of_quat(q) -> np.ndarray:
    w, x, y, z = np.asarray(q, dtype=np.float64) / np.linalg.norm(q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def qmul(p, q) -> np.ndarray:
    """Hamilton product p (x) q, (w, x, y, z)."""
    pw, px, py, pz = p
    qw, qx, qy, qz = q
    return np.array([pw * qw - px * qx - py * qy - pz * qz,
                     pw * qx + px * qw + py * qz - pz * qy,
                     pw * qy - px * qz + py * qw + pz * qx,
                     pw * qz + px * qy - py * qx + pz * qw])


def frames(verts, faces, face_uv):
    """Per triangle: (R [F,3,3], q_R [F,4]) for one mesh."""
    verts = np.asarray(verts, dtype=np.float64)
    F = faces.shape[0]
    R = np.zeros((F, 3, 3))
    q = np.zeros((F, 4))
    for f in range(F):
        a, b, c = faces[f]
        R[f] = tbn(verts[a], verts[b], verts[c], face_uv[f, 0], face_uv[f, 1], face_uv[f, 2])
        q[f] = quat_of_matrix(gram_schmidt(R[f]))
    return R, q


def transform(raw_t, tri, bary, verts, faces, face_uv) -> np.ndarray:
    """raw_t [N,16] (tangent space) -> raw_d [N,16] (deformed space) for one frame."""
    raw_t = np.asarray(raw_t, dtype=np.float64)
    verts = np.asarray(verts, dtype=np.float64)
    R, qR = frames(verts, faces, face_uv)
    out = raw_t.copy()
    for n in range(raw_t.shape[0]):
        f = tri[n]
        a, b, c = faces[f]
        t = bary[n, 0] * verts[a] + bary[n, 1] * verts[b] + bary[n, 2] * verts[c]
        out[n, 0:3] = R[f] @ raw_t[n, 0:3] + t
        out[n, 3:7] = qmul(qR[f], raw_t[n, 3:7])
    return out


def transform_adjoint(draw_d, tri, verts, faces, face_uv) -> np.ndarray:
    """draw_d [N,16] -> draw_t [N,16] for one frame (the transform's transpose)."""
    draw_d = np.asarray(draw_d, dtype=np.float64)
    R, qR = frames(verts, faces, face_uv)
    out = draw_d.copy()
    for n in range(draw_d.shape[0]):
        f = tri[n]
        out[n, 0:3] = R[f].T @ draw_d[n, 0:3]
        conj = qR[f] * np.array([1.0, -1.0, -1.0, -1.0])
        out[n, 3:7] = qmul(conj, draw_d[n, 3:7])
    return out
