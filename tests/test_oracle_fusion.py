"""Oracle pins for normals and fusion (Eq. (1)-(3)): planes give exact
closed forms, invariances hold, spheres stay within the point-to-plane
bound."""
import math

import numpy as np
import pytest

import oracle
from paper_2111_13652_amd import synth
from tests import scenes


def test_fals_normals_exact_on_fronto_parallel_plane():
    cam = scenes.SMALL_CAM
    depth = np.full((cam.height, cam.width), 2.0, np.float32)  # 1/z exact
    n, valid, cos = oracle.normals(depth, cam, 0.05)
    assert valid[2:-2, 2:-2].all() and not valid[:2].any() and not valid[:, -2:].any()
    np.testing.assert_allclose(n[valid], np.broadcast_to([0, 0, 1], n[valid].shape), atol=1e-12)
    # cosine of the viewing angle equals 1/|ray|
    rays = cam.rays()
    np.testing.assert_allclose(cos[valid], 1 / np.linalg.norm(rays, axis=-1)[valid], atol=1e-12)


@pytest.mark.parametrize("tilt_deg", [10.0, 40.0, 70.0])
def test_fals_normals_on_tilted_plane(tilt_deg):
    cam = scenes.SMALL_CAM
    a = math.radians(tilt_deg)
    nc = np.array([math.sin(a) * 0.6, math.sin(a) * 0.8, math.cos(a)])
    depth = scenes.depth_image(scenes.plane_depth(cam, nc, 1.5), cam)
    n, valid, cos = oracle.normals(depth, cam, 0.5)
    assert valid.sum() > 1000
    err = np.degrees(np.arccos(np.clip(n[valid] @ nc, -1, 1)))
    # only binary32 rounding of the depths separates the fit from the exact plane
    assert err.max() < 2e-3
    # the normal points away from the camera: n . ray > 0
    assert np.all(np.einsum("ij,ij->i", n[valid], cam.rays()[valid]) > 0)


def test_normals_reject_discontinuities_and_invalid_pixels():
    cam = scenes.SMALL_CAM
    depth = np.full((cam.height, cam.width), 2.0, np.float32)
    depth[:, 80:] = 2.2          # step of 0.2 m > T = 0.05
    depth[60, 30] = 0.0          # one invalid pixel
    _, valid, _ = oracle.normals(depth, cam, 0.05)
    assert not valid[:, 78:82].any()
    assert not valid[58:63, 28:33].any()
    assert valid[20, 20] and valid[20, 100]


def _fuse_plane(pose, n_cam, h, vs=0.01, T=0.05, eps=None, cam=scenes.SMALL_CAM):
    depth = scenes.depth_image(scenes.plane_depth(cam, n_cam, h), cam)
    M = oracle.OracleMap(vs, T)
    M.allocate(depth, cam, pose)
    M.integrate(depth, cam, pose, eps=eps)
    return M, depth


def test_fusion_fronto_parallel_plane_is_exact():
    M, _ = _fuse_plane(scenes.IDENTITY, [0, 0, 1], 2.0)
    keys = M.keys()
    psi, g, W, _ = M.voxels(keys)
    obs = W > 0
    assert obs.sum() > 1000
    lz = np.arange(512) // 64
    vz = 0.01 * (8 * keys[:, 2:3] + lz[None, :])
    # Eq. (1): every observation carries the same d = n.(v - p) = v_z - 2
    np.testing.assert_allclose(psi[obs], np.clip(vz - 2.0, -0.05, 0.05)[obs], atol=1e-12)
    gh = g[obs] / np.linalg.norm(g[obs], axis=1, keepdims=True)
    np.testing.assert_allclose(gh, np.broadcast_to([0, 0, 1], gh.shape), atol=1e-12)
    # free space in front of the surface is negative (Sec. 3.1 sign convention)
    assert np.all(psi[obs & (vz < 1.99)] < 0) and np.all(psi[obs & (vz > 2.01)] > 0)


def _plane_world(pose, n_cam, h):
    R, t = pose[:, :3], pose[:, 3]
    nw = R @ np.asarray(n_cam, float)
    return nw, h + nw @ t


def test_fusion_tilted_plane_at_general_pose():
    pose = synth.look_at([1.0, 0.5, 1.2], [1.3, 2.0, 0.7])
    n_cam = np.array([0.3, -0.2, 1.0])
    n_cam /= np.linalg.norm(n_cam)
    M, _ = _fuse_plane(pose, n_cam, 1.4)
    keys = M.keys()
    psi, g, W, _ = M.voxels(keys)
    obs = W > 0
    loc = np.stack([np.arange(512) % 8, (np.arange(512) // 8) % 8, np.arange(512) // 64], -1)
    v = 0.01 * (8 * keys[:, None, :] + loc[None])
    nw, hw = _plane_world(pose, n_cam, 1.4)
    exact = np.clip(v @ nw - hw, -0.05, 0.05)
    # binary32 depth rounding (~1e-7 relative) through the normal fit
    assert np.abs(psi[obs] - exact[obs]).max() < 2e-6
    gh = g[obs] / np.linalg.norm(g[obs], axis=1, keepdims=True)
    assert np.degrees(np.arccos(np.clip(gh @ nw, -1, 1))).max() < 2e-3


def test_single_plane_frame_does_not_depend_on_the_weight_function():
    pose = synth.look_at([1.0, 0.5, 1.2], [1.3, 2.0, 0.7])
    n_cam = np.array([0.1, -0.3, 1.0])
    n_cam /= np.linalg.norm(n_cam)
    A, _ = _fuse_plane(pose, n_cam, 1.3, eps=0.01)
    B, _ = _fuse_plane(pose, n_cam, 1.3, eps=0.03)
    pa, ga, Wa, _ = A.voxels()
    pb, gb, Wb, _ = B.voxels()
    both = (Wa > 0) & (Wb > 0)
    assert both.sum() > 1000 and not np.allclose(Wa[both], Wb[both])
    np.testing.assert_allclose(pa[both], pb[both], atol=1e-15)
    np.testing.assert_allclose(ga[both] / np.linalg.norm(ga[both], axis=1, keepdims=True),
                               gb[both] / np.linalg.norm(gb[both], axis=1, keepdims=True), atol=1e-14)


def test_fusion_is_order_independent():
    st = scenes.room_frames(scenes.SMALL_CAM, 3)
    A = oracle.OracleMap(0.02, 0.1)
    B = oracle.OracleMap(0.02, 0.1)
    for f in (0, 2):
        A.allocate(st.depth[f], st.cam, st.poses[f])
        A.integrate(st.depth[f], st.cam, st.poses[f])
    for f in (2, 0):
        B.allocate(st.depth[f], st.cam, st.poses[f])
        B.integrate(st.depth[f], st.cam, st.poses[f])
    np.testing.assert_array_equal(A.keys(), B.keys())
    pa, ga, Wa, _ = A.voxels()
    pb, gb, Wb, _ = B.voxels()
    np.testing.assert_allclose(Wa, Wb, rtol=1e-13, atol=0)
    np.testing.assert_allclose(pa, pb, rtol=0, atol=1e-15)
    np.testing.assert_allclose(ga, gb, rtol=0, atol=1e-12)


def test_running_average_is_the_weighted_mean():
    # two frames of parallel planes at different depths: each voxel's psi is
    # the W-weighted mean of the two exact distances (Eq. (1)-(2))
    cam = scenes.SMALL_CAM
    M = oracle.OracleMap(0.01, 0.05)
    for h in (2.0, 2.0078125):  # both 1/h exactly representable
        depth = np.full((cam.height, cam.width), h, np.float32)
        M.allocate(depth, cam, scenes.IDENTITY)
        M.integrate(depth, cam, scenes.IDENTITY, eps=0.01)
    keys = M.keys()
    psi, g, W, _ = M.voxels(keys)
    vz = 0.01 * (8 * keys[:, 2:3] + (np.arange(512) // 64)[None, :])
    d1 = np.clip(vz - 2.0, -0.05, 0.05)
    d2 = np.clip(vz - 2.0078125, -0.05, 0.05)
    w1 = np.array([[oracle.w_linear(x, 0.01, 0.05) for x in row] for row in d1])
    w2 = np.array([[oracle.w_linear(x, 0.01, 0.05) for x in row] for row in d2])
    obs = W > 0
    # Eq. (1)-(2) with k1 (k2) pixels observing the voxel in frame 1 (2):
    # W = k1 w1 + k2 w2 and W psi = k1 w1 d1 + k2 w2 d2.  Solving for the
    # counts must give non-negative integers.
    A11, A12, A21, A22 = w1[obs], w2[obs], (w1 * d1)[obs], (w2 * d2)[obs]
    b1, b2 = W[obs], (W * psi)[obs]
    det = A11 * A22 - A12 * A21
    ok = np.abs(det) > 1e-6
    k1 = (b1 * A22 - A12 * b2)[ok] / det[ok]
    k2 = (A11 * b2 - A21 * b1)[ok] / det[ok]
    assert ok.sum() > 1000
    np.testing.assert_allclose(k1, np.round(k1), atol=1e-6)
    np.testing.assert_allclose(k2, np.round(k2), atol=1e-6)
    assert k1.min() > -1e-6 and k2.min() > -1e-6 and (np.round(k1) + np.round(k2)).min() >= 1
    # where both frames give the same clamped distance, psi is that distance
    same = obs & (d1 == d2)
    np.testing.assert_allclose(psi[same], d1[same], atol=1e-15)


def test_linear_weight_and_huber_closed_forms():
    eps, T = 0.01, 0.05
    assert oracle.w_linear(-0.05, eps, T) == 1.0 and oracle.w_linear(eps, eps, T) == 1.0
    assert oracle.w_linear(0.03, eps, T) == pytest.approx(0.5, abs=1e-15)
    assert oracle.w_linear(T, eps, T) == 0.0
    d = 0.01
    for r in (-0.03, -0.01, -0.002, 0.0, 0.004, 0.01, 0.2):
        rho = oracle.huber_rho(r, d)
        assert rho == pytest.approx(0.5 * r * r if abs(r) <= d else d * abs(r) - d * d / 2, abs=1e-18)
        # rho'(r) = w r, continuous at |r| = delta
        h = 1e-7
        fd = (oracle.huber_rho(r + h, d) - oracle.huber_rho(r - h, d)) / (2 * h)
        assert oracle.huber_weight(r, d) * r == pytest.approx(fd, abs=1e-7)  # h/4 at the kink
    # delta -> infinity reduces to plain least squares
    assert oracle.huber_rho(0.3, 1e9) == pytest.approx(0.045, abs=1e-16)
    assert oracle.huber_weight(0.3, 1e9) == 1.0


def test_sphere_fusion_within_point_to_plane_bound():
    cfg = synth.CONFIG_SPHERE
    cam = cfg["cam"]
    c, R = np.array([0.0, 0.0, 1.5]), 0.5
    depth = synth.to_depth_image(synth.render_depth(synth.sphere_scene(), cam, scenes.IDENTITY), cam)
    M = oracle.OracleMap(0.02, 0.10, bounds=([-4, -4, 5], [4, 4, 13]))
    M.allocate(depth, cam, scenes.IDENTITY)
    M.integrate(depth, cam, scenes.IDENTITY)
    keys = M.keys()
    psi, g, W, _ = M.voxels(keys)
    loc = np.stack([np.arange(512) % 8, (np.arange(512) // 8) % 8, np.arange(512) // 64], -1)
    v = 0.02 * (8 * keys[:, None, :] + loc[None])
    obs = (W > 0) & (np.abs(psi) < 0.1 - 1e-9)
    true = R - np.linalg.norm(v - c, axis=-1)
    # point-to-plane distance to a tangent plane of a sphere differs from the
    # true SDF by at most (tangential offset)^2 / (2 (R - a)); offsets stay
    # below the band length T / cos(75 deg)
    b_max = 0.1 / math.cos(math.radians(75))
    bound = b_max ** 2 / (2 * (R - 0.1))
    err = np.abs(psi[obs] - true[obs])
    assert err.max() < bound
    assert np.median(err) < 0.1 * 0.02
    # stored gradients point into the sphere (Sec. 3.2: inward normal)
    gh = g[obs] / np.linalg.norm(g[obs], axis=-1, keepdims=True)
    gt = (c - v[obs]) / np.linalg.norm(c - v[obs], axis=-1, keepdims=True)
    ang = np.degrees(np.arccos(np.clip(np.einsum("ij,ij->i", gh, gt), -1, 1)))
    # normals of pixels whose rays cross a voxel a distance a off the surface
    # are taken a*tan(view angle) away on the sphere: small near the surface
    near = np.abs(true[obs]) < 0.01
    assert np.median(ang[near]) < 1.0 and np.median(ang) < 10.0
