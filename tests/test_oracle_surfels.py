"""Pins of the oracle's oriented point cloud (Sec. 4.3): on fused planes the
points lie on the plane and the selection is the brute-force set of cells
(subcells) whose centre is within half a cell of it; on a sphere the points
stay close to the surface with outward normals."""

import numpy as np

import oracle
from paper_2111_13652_amd import synth
from tests import scenes


def _fuse(depth, cam, pose, vs, T, bounds=None):
    M = oracle.OracleMap(vs, T, bounds=bounds)
    M.allocate(depth, cam, pose)
    M.integrate(depth, cam, pose)
    return M


def _voxel_centres(keys, vs):
    c = np.arange(512)
    loc = np.stack([c % 8, (c // 8) % 8, c // 64], -1)
    return vs * (8 * keys[:, None, :] + loc[None])


def test_plane_surfels_lie_on_the_plane_and_select_the_crossing_cells():
    cam = scenes.SMALL_CAM
    h = 2.0037   # not on a cell boundary
    depth = scenes.depth_image(scenes.plane_depth(cam, [0, 0, 1], h), cam)
    M = _fuse(depth, cam, scenes.IDENTITY, 0.01, 0.05)
    keys = M.keys()
    psi, g, W, _ = M.voxels(keys)
    v = _voxel_centres(keys, 0.01)
    obs = W > 0
    for level, half, offs in ((0, 0.005, [0.0]), (1, 0.0025, [-0.0025, 0.0025])):
        pts, nrm, ids = M.surfels(level, keys)
        np.testing.assert_allclose(pts[:, 2], h, atol=1e-12)
        np.testing.assert_allclose(nrm, np.broadcast_to([0, 0, -1], nrm.shape), atol=1e-11)
        # brute force: observed (sub)cells whose centre is within half a cell
        # of the plane; each of the four (x, y) subcell columns of a voxel has
        # its own centres, so a voxel contributes 4 points per z-layer hit
        want = 0
        for dz in offs:
            want += int(np.sum(obs & (np.abs(v[..., 2] + dz - h) <= half))) * (1 if level == 0 else 4)
        assert len(pts) == want > 100
        # each point sits at its (sub)cell's own x, y
        sub = ids[:, 3]
        sx = ids[:, 0] * 0.01 + (np.where(sub & 1, 0.0025, -0.0025) if level else 0.0)
        sy = ids[:, 1] * 0.01 + (np.where(sub & 2, 0.0025, -0.0025) if level else 0.0)
        np.testing.assert_allclose(pts[:, 0], sx, atol=1e-12)
        np.testing.assert_allclose(pts[:, 1], sy, atol=1e-12)


def test_tilted_plane_surfels_stay_on_the_plane():
    pose = synth.look_at([1.0, 0.5, 1.2], [1.3, 2.0, 0.7])
    n_cam = np.array([0.3, -0.2, 1.0])
    n_cam /= np.linalg.norm(n_cam)
    cam = scenes.SMALL_CAM
    depth = scenes.depth_image(scenes.plane_depth(cam, n_cam, 1.4), cam)
    M = _fuse(depth, cam, pose, 0.01, 0.05)
    nw = pose[:, :3] @ n_cam
    hw = 1.4 + nw @ pose[:, 3]
    for level in (0, 1):
        pts, nrm, _ = M.surfels(level)
        assert len(pts) > 100
        # psi carries the binary32 depth rounding through the normal fit
        assert np.abs(pts @ nw - hw).max() < 3e-6
        assert np.degrees(np.arccos(np.clip(-nrm @ nw, -1, 1))).max() < 2e-3


def test_sphere_surfels_near_the_surface_with_outward_normals():
    cfg = synth.CONFIG_SPHERE
    cam = cfg["cam"]
    c, R = np.array([0.0, 0.0, 1.5]), 0.5
    depth = synth.to_depth_image(synth.render_depth(synth.sphere_scene(), cam, scenes.IDENTITY), cam)
    M = _fuse(depth, cam, scenes.IDENTITY, 0.02, 0.10, bounds=([-4, -4, 5], [4, 4, 13]))
    pts0, nrm0, _ = M.surfels(0)
    pts1, nrm1, _ = M.surfels(1)
    for pts, nrm in ((pts0, nrm0), (pts1, nrm1)):
        r = np.linalg.norm(pts - c, axis=1)
        radial = (pts - c) / r[:, None]
        assert np.median(np.abs(r - R)) < 0.05 * 0.02
        ang = np.degrees(np.arccos(np.clip(np.einsum("ij,ij->i", nrm, radial), -1, 1)))
        assert np.median(ang) < 2.0 and np.all(np.einsum("ij,ij->i", nrm, radial) > 0)
    # twice the resolution in each surface direction: about four times the points
    assert 3.0 < len(pts1) / len(pts0) < 5.0
