"""Oracle pins: nearest voxel, block decomposition, ray-band voxels,
allocation.  Each is checked against brute force or geometry, not against
the oracle's own formulas."""
import os

import numpy as np
import pytest

import oracle
from paper_2111_13652_amd import synth
from tests import scenes

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    vals = {}
    for line in open(os.path.join(GOLDEN, name)):
        line = line.strip()
        if line and not line.startswith("#"):
            k, v = line.split()
            vals[k] = float(v)
    return vals


def test_nearest_voxel_is_bruteforce_argmin():
    # Sec. 4.1: j* = argmin_j |p - v_j| is found by rounding p / v_s
    rng = np.random.default_rng(5)
    vs = 0.02
    q = rng.uniform(-3, 3, size=(20000, 3))
    offs = np.array([[i, j, k] for i in (-1, 0, 1) for j in (-1, 0, 1) for k in (-1, 0, 1)])
    for p in q:
        m = oracle.nearest_voxel(p, vs)
        cand = m + offs
        d = np.linalg.norm(p - vs * cand, axis=1)
        assert d[13] <= d.min() + 1e-15  # index 13 is the centre offset (0,0,0)
    # exact ties break towards +inf (floor(x + 1/2))
    assert list(oracle.nearest_voxel(np.array([0.01, -0.01, 0.03]), vs)) == [1, 0, 2]


def test_floor_division_and_block_boundary_fraction():
    for m in range(-70, 70):
        assert oracle.floordiv8(m) == m // 8
    g = _golden("block_boundary_fraction.txt")
    # count voxels of one block with a 26-neighbour in another block
    b0 = np.array([-1, 2, 0])
    n_boundary = 0
    for lz in range(8):
        for ly in range(8):
            for lx in range(8):
                m = 8 * b0 + np.array([lx, ly, lz])
                outside = False
                for d in np.ndindex(3, 3, 3):
                    nb = m + np.array(d) - 1
                    if [oracle.floordiv8(int(c)) for c in nb] != list(b0):
                        outside = True
                        break
                n_boundary += outside
    frac = n_boundary / 512
    assert n_boundary == 8 ** 3 - int(g["interior_edge"]) ** 3
    assert round(100 * frac, 1) == g["fraction_percent"]


def _segment_cells(o, d, z0, z1, vs):
    """Exact (FP64) nearest-voxel cells crossed by o + z d, z in [z0, z1],
    with the z-length spent in each."""
    cells = []
    z = z0
    while z < z1:
        p = o + z * d
        m = np.floor(p / vs + 0.5).astype(int)
        zexit = z1
        for k in range(3):
            if d[k] > 0:
                zexit = min(zexit, ((m[k] + 0.5) * vs - o[k]) / d[k])
            elif d[k] < 0:
                zexit = min(zexit, ((m[k] - 0.5) * vs - o[k]) / d[k])
        cells.append((tuple(m), max(zexit, z) - z))
        z = max(zexit, z) + 1e-12
    return cells


def _cell_hits_segment(m, o, d, z0, z1, vs, tol):
    lo = vs * (np.asarray(m) - 0.5) - tol
    hi = vs * (np.asarray(m) + 0.5) + tol
    a, b = z0 - tol, z1 + tol
    for k in range(3):
        if d[k] == 0:
            if not (lo[k] <= o[k] <= hi[k]):
                return False
            continue
        t1, t2 = (lo[k] - o[k]) / d[k], (hi[k] - o[k]) / d[k]
        a, b = max(a, min(t1, t2)), min(b, max(t1, t2))
    return a <= b


@pytest.mark.parametrize("seed", [0, 1])
def test_band_voxels_match_ray_geometry(seed):
    """The voxels along the viewing ray within the truncation band (Sec. 5.3):
    each listed cell touches the band segment, and every cell the segment
    crosses for more than one sample spacing is listed."""
    rng = np.random.default_rng(seed)
    vs, T = 0.01, 0.05
    M = oracle.OracleMap(vs, T)
    cam = synth.CONFIG_ROOM["cam"]
    pose = synth.look_at(rng.uniform(1, 3, 3), rng.uniform(0, 4, 3))
    R, t = pose[:, :3], pose[:, 3]
    delta = vs / 2
    tol = 2e-5  # binary32 rounding of world coordinates up to ~5 m
    for _ in range(300):
        u, v = int(rng.integers(0, 640)), int(rng.integers(0, 480))
        D = float(np.float32(rng.uniform(0.4, 4.0)))
        band = M.band_voxels(cam, pose, u, v, D)
        assert len(band) >= 1 and len(band) <= 21
        assert np.all(np.any(band[1:] != band[:-1], axis=1))  # consecutive repeats removed
        ray = np.array([(u - cam.cx) / cam.fx, (v - cam.cy) / cam.fy, 1.0])
        d = R @ ray
        z0, z1 = D - T, D + T
        listed = {tuple(m) for m in band}
        for m in listed:
            assert _cell_hits_segment(m, t, d, z0, z1, vs, tol)
        for m, length in _segment_cells(t, d, z0, z1, vs):
            if length > delta + 1e-6:
                assert m in listed


def test_allocation_is_the_blocks_of_the_ray_bands():
    """Every block a valid pixel's band crosses by more than one sample
    spacing is allocated; every allocated block touches some band."""
    vs, T = 0.02, 0.10
    cam = synth.Camera(40.0, 40.0, 19.5, 14.5, 40, 30, 0.4, 4.0)
    poses = synth.smooth_trajectory(2, 3)
    sc = synth.room_scene(1, poses[:, :, 3])
    pose = poses[2]
    depth = synth.to_depth_image(synth.render_depth(sc, cam, pose), cam)
    M = oracle.OracleMap(vs, T)
    n = M.allocate(depth, cam, pose)
    keys = {tuple(k) for k in M.keys()}
    assert n == len(keys) > 0
    R, t = pose[:, :3], pose[:, 3]
    must, may = set(), set()
    tol = 2e-5
    for v in range(cam.height):
        for u in range(cam.width):
            D = float(depth[v, u])
            if D <= 0:
                continue
            d = R @ np.array([(u - cam.cx) / cam.fx, (v - cam.cy) / cam.fy, 1.0])
            for m, length in _segment_cells(t, d, D - T - tol, D + T + tol, vs):
                b = tuple(int(c) // 8 for c in m)
                may.add(b)
                if length > vs / 2 + 1e-6:
                    must.add(b)
    assert must <= keys <= may
    # allocating the same frame again creates nothing
    assert M.allocate(depth, cam, pose) == 0


def test_bounded_map_never_leaves_its_block_box():
    cfg = synth.CONFIG_SPHERE
    cam = cfg["cam"]
    depth = synth.to_depth_image(synth.render_depth(synth.sphere_scene(), cam, scenes.IDENTITY), cam)
    M = oracle.OracleMap(0.02, 0.10, bounds=([-4, -4, 5], [4, 4, 13]))
    M.allocate(depth, cam, scenes.IDENTITY)
    k = M.keys()
    assert np.all(k >= [-4, -4, 5]) and np.all(k < [4, 4, 13])
    U = oracle.OracleMap(0.02, 0.10)
    U.allocate(depth, cam, scenes.IDENTITY)
    # the 64^3 box covers the visible cap of the sphere: nothing is cut away
    assert len(U.keys()) == len(k)
