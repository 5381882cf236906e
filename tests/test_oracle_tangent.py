"""Pins of the tangent-space transform reference (Eq. 4, Alg. 1): a flat
triangle whose UVs are its own coordinates gives the identity frame; the
TBN solves its defining equations; a rigid motion of the mesh moves the
Gaussians rigidly; scaling the UVs scales the tangent offsets inversely; the
rotation is the Gram-Schmidt frame; the adjoint is the transpose."""
import numpy as np

from oracle import tangent
from paper_2503_12886_amd import synth


def test_flat_triangle_with_uv_equal_to_xy_is_the_identity_frame():
    v = np.array([[0.1, 0.2, 0.3], [0.6, 0.2, 0.3], [0.1, 0.9, 0.3]])
    uv = v[:, :2] - v[0, :2]
    R = tangent.tbn(v[0], v[1], v[2], uv[0], uv[1], uv[2])
    assert np.allclose(R, np.eye(3), atol=1e-14)
    faces = np.array([[0, 1, 2]])
    raw = np.zeros((1, 16)); raw[0, 0:3] = (0.01, -0.02, 0.005); raw[0, 3:7] = (0.5, 0.1, -0.3, 0.2); raw[0, 11] = 0.7
    bary = np.array([[0.2, 0.3, 0.5]])
    out = tangent.transform(raw, np.array([0]), bary, v, faces, uv[None])
    assert np.allclose(out[0, 0:3], raw[0, 0:3] + bary[0] @ v, atol=1e-15)
    assert np.allclose(out[0, 3:], raw[0, 3:], atol=1e-15)


def test_tbn_solves_its_defining_equations():
    rng = np.random.default_rng(0)
    for _ in range(20):
        v = rng.normal(size=(3, 3))
        uv = rng.uniform(size=(3, 2))
        R = tangent.tbn(v[0], v[1], v[2], uv[0], uv[1], uv[2])
        T, B, N = R[:, 0], R[:, 1], R[:, 2]
        d1, d2 = uv[1] - uv[0], uv[2] - uv[0]
        assert np.allclose(v[1] - v[0], d1[0] * T + d1[1] * B, atol=1e-12)
        assert np.allclose(v[2] - v[0], d2[0] * T + d2[1] * B, atol=1e-12)
        assert abs(np.linalg.norm(N) - 1) < 1e-14 and abs(N @ T) < 1e-12 and abs(N @ B) < 1e-12


def test_rigid_motion_of_the_mesh_moves_gaussians_rigidly():
    verts, faces, uv = synth.make_head_mesh(8, 12)
    tri, bary = synth.bind_gaussians(faces, verts, 50, seed=1)
    raw = synth.make_tangent_scene(50, 0, seed=2)[0].astype(np.float64)
    a = np.deg2rad(37.0)
    Q = tangent.matrix_of_quat([np.cos(a / 2), 0.3 * np.sin(a / 2), -0.9 * np.sin(a / 2), 0.3 * np.sin(a / 2)])
    tau = np.array([0.01, -0.03, 0.02])
    d0 = tangent.transform(raw, tri, bary, verts, faces, uv)
    d1 = tangent.transform(raw, tri, bary, verts.astype(np.float64) @ Q.T + tau, faces, uv)
    assert np.allclose(d1[:, 0:3], d0[:, 0:3] @ Q.T + tau, atol=1e-12)
    for n in range(50):
        assert np.allclose(tangent.matrix_of_quat(d1[n, 3:7]), Q @ tangent.matrix_of_quat(d0[n, 3:7]), atol=1e-12)
    assert np.allclose(d1[:, 7:], d0[:, 7:])


def test_uv_scale_scales_tangent_offsets_inversely():
    verts, faces, uv = synth.make_head_mesh(8, 12)
    tri, bary = synth.bind_gaussians(faces, verts, 30, seed=3)
    raw = np.zeros((30, 16)); raw[:, 0:2] = np.random.default_rng(4).normal(size=(30, 2)) * 1e-2
    raw[:, 3] = 1.0
    base = tangent.transform(raw * np.array([0] * 16), tri, bary, verts, faces, uv)[:, 0:3]
    d1 = tangent.transform(raw, tri, bary, verts, faces, uv)[:, 0:3] - base
    d2 = tangent.transform(raw, tri, bary, verts, faces, uv * 2.0)[:, 0:3] - base
    assert np.allclose(d2, 0.5 * d1, atol=1e-14)


def test_rotation_is_the_gram_schmidt_frame():
    verts, faces, uv = synth.make_head_mesh(8, 12)
    R, q = tangent.frames(verts, faces, uv)
    for f in range(len(faces)):
        G = tangent.matrix_of_quat(q[f])
        assert np.allclose(G.T @ G, np.eye(3), atol=1e-13) and np.linalg.det(G) > 0
        assert np.allclose(G[:, 0], R[f][:, 0] / np.linalg.norm(R[f][:, 0]), atol=1e-12)
        assert abs(G[:, 1] @ R[f][:, 2]) < 1e-12 and G[:, 2] @ R[f][:, 2] > 0.999


def test_adjoint_is_the_transpose():
    verts, faces, uv = synth.make_head_mesh(8, 12)
    tri, bary = synth.bind_gaussians(faces, verts, 40, seed=5)
    rng = np.random.default_rng(6)
    v, u = rng.normal(size=(40, 16)), rng.normal(size=(40, 16))
    zero = np.zeros((40, 16))
    Jv = tangent.transform(v, tri, bary, verts, faces, uv) - tangent.transform(zero, tri, bary, verts, faces, uv)
    JTu = tangent.transform_adjoint(u, tri, verts, faces, uv)
    assert abs((Jv * u).sum() - (v * JTu).sum()) < 1e-12 * np.abs(Jv * u).sum()
