"""GPU <-> oracle parity of the plain FP32 path through the C ABI:
allocation keys bit-exact, voxel values, normal equations and poses within
the stated tolerances, and edge cases.  Needs an MI355X."""
import math

import numpy as np
import pytest

import oracle
from paper_2111_13652_amd import synth
from tests import scenes
from tests.gpu_helpers import (align_voxels, assert_same_keys, compare_voxels, dev, log,
                               marginal_voxels, pose_diff)

pytestmark = pytest.mark.gpu

ROOM = synth.CONFIG_ROOM
COS75 = math.cos(math.radians(75.0))


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    from paper_2111_13652_amd import gsdf  # noqa: F401  (loads libgsdf.so or fails)
    return torch


@pytest.fixture(scope="module")
def room_stream():
    return synth.make_stream(ROOM["cam"], 8, 1, 2, 3)


def _gpu_map(vs, T, max_blocks=60000, **kw):
    from paper_2111_13652_amd.gsdf import GsdfMap
    return GsdfMap(vs, T, max_blocks, **kw)


def test_sphere_config_keys_voxels_and_observable_pose(torch_mod):
    torch = torch_mod
    cfg = synth.CONFIG_SPHERE
    cam = cfg["cam"]
    log("case: sphere 160x120, bounded 64^3, fuse + track")
    sc = synth.sphere_scene()
    T0 = scenes.IDENTITY
    d0 = synth.to_depth_image(synth.render_depth(sc, cam, T0), cam)
    bounds = ([-4, -4, 5], [4, 4, 13])
    O = oracle.OracleMap(0.02, 0.10, bounds=bounds)
    O.allocate(d0, cam, T0)
    _, marg = O.integrate(d0, cam, T0, return_marginal=True)
    G = _gpu_map(0.02, 0.10, max_blocks=1024, bounds=bounds)
    D0 = dev(d0)
    P0 = dev(T0)
    G.allocate(D0, cam, P0)
    assert_same_keys(G.keys(), O.keys())
    G.integrate(D0, cam, P0)
    torch.cuda.synchronize()
    gpu, orc, keys = align_voxels(G, O)
    compare_voxels(gpu, orc, keys, 0.02, exclude=marginal_voxels(O, d0, cam, T0, marg))
    # tracking the perturbed render: the sphere centre in the camera frame is
    # the observable part of the pose
    T1 = synth.perturb_pose(T0, 0, 2.0, 0.02)
    d1 = synth.to_depth_image(synth.render_depth(sc, cam, T1), cam)
    To, _, _ = O.track(d1, cam, T0, 1, [10], 0.01)
    P = dev(T0.copy())
    stats = torch.zeros(20, dtype=torch.float32, device="cuda")
    G.track(dev(d1), cam, P, levels=1, iters=(10,), delta=0.01, stats=stats)
    Tg = P.cpu().numpy()
    c = np.array([0.0, 0.0, 1.5])
    cc = lambda T: T[:, :3].T @ (c - T[:, 3])
    err = np.linalg.norm(cc(Tg) - cc(To))
    log("sphere centre GPU vs oracle (m):", err, "energy", stats.cpu().numpy()[::2][-1])
    assert err < 1e-5
    assert G.status_flags() == []


def test_room_keys_bitexact_every_frame_and_voxels(torch_mod, room_stream):
    torch = torch_mod
    st = room_stream
    cam = st.cam
    O = oracle.OracleMap(0.01, 0.05)
    G = _gpu_map(0.01, 0.05)
    excl = set()
    for f in range(len(st.depth)):
        log(f"case: room 640x480 frame {f}: allocate + integrate at ground truth")
        D = dev(st.depth[f])
        P = dev(st.poses[f])
        O.allocate(st.depth[f], cam, st.poses[f])
        G.allocate(D, cam, P)
        assert_same_keys(G.keys(), O.keys())
        _, marg = O.integrate(st.depth[f], cam, st.poses[f], return_marginal=True)
        excl |= marginal_voxels(O, st.depth[f], cam, st.poses[f], marg)
        G.integrate(D, cam, P)
        if f in (0, len(st.depth) - 1):
            torch.cuda.synchronize()
            gpu, orc, keys = align_voxels(G, O)
            rep = compare_voxels(gpu, orc, keys, 0.01, exclude=excl)
            assert rep["excluded"] < 1e-4 * rep["n"] + 10
    assert G.status_flags() == []


def _oracle_room_map(st, frames):
    O = oracle.OracleMap(0.01, 0.05)
    for f in frames:
        O.allocate(st.depth[f], st.cam, st.poses[f])
        O.integrate(st.depth[f], st.cam, st.poses[f])
    return O


def _import(O, G):
    keys = O.keys()
    psi, g, W, _ = O.voxels(keys)
    G.import_blocks(keys, psi, g, W)


def test_normal_equations_parity(torch_mod, room_stream):
    st = room_stream
    O = _oracle_room_map(st, [0, 1, 2])
    G = _gpu_map(0.01, 0.05)
    _import(O, G)
    for f, pert in ((3, 0), (3, 1), (5, 2)):
        T = st.poses[f] if pert == 0 else synth.perturb_pose(st.poses[f], pert, 0.5, 0.005)
        log(f"case: normal equations frame {f} perturbation {pert}")
        ne_o = O.normal_equations(st.depth[f].astype(np.float64), st.cam, T, 0.01)
        ne_g = G.normal_equations(dev(st.depth[f]), st.cam, dev(T), 0.01).cpu().numpy()
        Ho, bo, Eo, no = oracle.unpack_upper(ne_o)
        Hg, bg, Eg, ng = oracle.unpack_upper(ne_g)
        relH = np.linalg.norm(Hg - Ho) / np.linalg.norm(Ho)
        relb = np.linalg.norm(bg - bo) / np.linalg.norm(bo)
        log(f"  n {ng} vs {no}; rel H {relH:.2e}; rel b {relb:.2e}; rel E {abs(Eg - Eo) / Eo:.2e}")
        assert abs(ng - no) <= 1e-5 * no
        assert relH < 1e-5 and relb < 1e-5 and abs(Eg - Eo) < 1e-5 * Eo


def test_track_frame_pose_parity(torch_mod, room_stream):
    torch = torch_mod
    st = room_stream
    O = _oracle_room_map(st, [0, 1, 2, 3])
    G = _gpu_map(0.01, 0.05)
    _import(O, G)
    for f in (4, 6):
        log(f"case: track frame {f} (3 levels, 4/5/10 iterations) from the previous pose")
        To, so, failed = O.track(st.depth[f], st.cam, st.poses[f - 1], 3, [4, 5, 10], 0.01)
        P = dev(st.poses[f - 1].copy())
        stats = torch.zeros(38, dtype=torch.float32, device="cuda")
        G.track(dev(st.depth[f]), st.cam, P, levels=3, iters=(4, 5, 10), delta=0.01, stats=stats)
        Tg = P.cpu().numpy()
        dr, dt = pose_diff(Tg, To)
        log(f"  GPU vs oracle: {dr:.2e} rad, {dt:.2e} m; oracle vs truth {pose_diff(To, st.poses[f])}")
        assert dr < 1e-5 and dt < 1e-5
        sg = stats.cpu().numpy().reshape(-1, 2)
        np.testing.assert_allclose(sg[:, 1], so[:, 1], rtol=1e-4)
        np.testing.assert_allclose(sg[:, 0], so[:, 0], rtol=1e-3)
    assert G.status_flags() == []


def test_exact_recovery_on_model_consistent_render(torch_mod):
    cam = synth.Camera(131.0, 131.0, 79.5, 59.5, 160, 120, 0.4, 4.0)
    sc = scenes.box_room_scene()
    T0 = scenes.box_room_pose()
    O = oracle.OracleMap(0.02, 0.1)
    for k in range(3):
        Tk = synth.perturb_pose(T0, 100 + k, 1.0, 0.01)
        d = synth.to_depth_image(synth.render_depth(sc, cam, Tk), cam)
        O.allocate(d, cam, Tk)
        O.integrate(d, cam, Tk)
    T1 = synth.perturb_pose(T0, 11, 2.0, 0.02)
    depth = O.render_taylor(cam, T1, 0.3, 6.0).astype(np.float32)
    G = _gpu_map(0.02, 0.1, max_blocks=4096)
    _import(O, G)
    log("case: model-consistent render, 20 GN iterations, one level")
    P = dev(T0.copy())
    G.track(dev(depth), cam, P, levels=1, iters=(20,), delta=0.01)
    dr, dt = pose_diff(P.cpu().numpy(), T1)
    log(f"  GPU vs truth: {dr:.2e} rad, {dt:.2e} m")
    assert dr < 1e-5 and dt < 1e-5


def test_empty_depth_and_capacity_edges(torch_mod, room_stream):
    torch = torch_mod
    st = room_stream
    cam = st.cam
    log("case: all-invalid depth")
    G = _gpu_map(0.01, 0.05)
    empty = torch.zeros((cam.height, cam.width), dtype=torch.float32, device="cuda")
    P = dev(st.poses[0])
    G.allocate(empty, cam, P)
    G.integrate(empty, cam, P)
    assert G.num_blocks() == 0
    P2 = dev(st.poses[0].copy())
    stats = torch.zeros(38, dtype=torch.float32, device="cuda")
    G.track(empty, cam, P2, stats=stats)
    np.testing.assert_array_equal(P2.cpu().numpy(), st.poses[0])  # every solve skipped
    assert "not_pd" in G.status_flags()
    assert np.all(stats.cpu().numpy()[1::2] == 0)
    log("case: pool capacity 64 blocks")
    S = _gpu_map(0.01, 0.05, max_blocks=64)
    S.allocate(dev(st.depth[0]), cam, P)
    O = oracle.OracleMap(0.01, 0.05)
    O.allocate(st.depth[0], cam, st.poses[0])
    k = S.keys()
    assert len(k) == 64 and "capacity" in S.status_flags()
    assert {tuple(x) for x in k} <= {tuple(x) for x in O.keys()}
    S.integrate(dev(st.depth[0]), cam, P)   # only allocated blocks receive updates
    torch.cuda.synchronize()


def test_ragged_image_and_repeat_allocation(torch_mod):
    torch = torch_mod
    cam = synth.Camera(100.0, 100.0, 78.0, 46.0, 157, 93, 0.4, 4.0)
    poses = synth.smooth_trajectory(2, 3)
    sc = synth.room_scene(1, poses[:, :, 3])
    d = synth.to_depth_image(synth.render_depth(sc, cam, poses[2]), cam)
    log("case: ragged 157x93 image, allocate twice, integrate, 3-level track")
    O = oracle.OracleMap(0.01, 0.05)
    O.allocate(d, cam, poses[2])
    _, marg = O.integrate(d, cam, poses[2], return_marginal=True)
    G = _gpu_map(0.01, 0.05, max_blocks=8192)
    D, P = dev(d), dev(poses[2])
    G.allocate(D, cam, P)
    n1 = G.num_blocks()
    G.allocate(D, cam, P)
    assert G.num_blocks() == n1
    assert_same_keys(G.keys(), O.keys())
    G.integrate(D, cam, P)
    torch.cuda.synchronize()
    gpu, orc, keys = align_voxels(G, O)
    compare_voxels(gpu, orc, keys, 0.01, exclude=marginal_voxels(O, d, cam, poses[2], marg))
    T1 = synth.perturb_pose(poses[2], 3, 0.5, 0.005)
    To, _, _ = O.track(d, cam, T1, 3, [4, 5, 10], 0.01)
    Pg = dev(T1.copy())
    Gi = _gpu_map(0.01, 0.05, max_blocks=8192)
    _import(O, Gi)
    Gi.track(D, cam, Pg, levels=3, iters=(4, 5, 10), delta=0.01)
    dr, dt = pose_diff(Pg.cpu().numpy(), To)
    log(f"  GPU vs oracle: {dr:.2e} rad, {dt:.2e} m")
    assert dr < 1e-5 and dt < 1e-5


@pytest.mark.parametrize("storage", ["fp32", "bf16"])
def test_fuse_frame_equals_allocate_then_integrate(torch_mod, room_stream, storage):
    """gsdf_fuse_frame (allocation and normals in one launch) leaves exactly
    the map that gsdf_allocate_blocks + gsdf_integrate_frame leave."""
    st = room_stream
    A = _gpu_map(0.01, 0.05, storage=storage)
    B = _gpu_map(0.01, 0.05, storage=storage)
    for f in range(len(st.depth)):
        log(f"case: fuse_frame vs allocate + integrate, room frame {f}, {storage}")
        D, P = dev(st.depth[f]), dev(st.poses[f])
        A.allocate(D, st.cam, P)
        A.integrate(D, st.cam, P)
        B.fuse(D, st.cam, P)
    ka, kb = A.keys(), B.keys()
    oa, ob = np.lexsort(ka.T[::-1]), np.lexsort(kb.T[::-1])
    np.testing.assert_array_equal(ka[oa], kb[ob])
    va, vb = A.voxels(len(ka)), B.voxels(len(kb))
    for xa, xb in zip(va, vb):
        np.testing.assert_array_equal(xa[oa], xb[ob])
    np.testing.assert_array_equal(A.counters(), B.counters())
    assert A.status_flags() == [] and B.status_flags() == []


def _tile_block_counts(depth, cam, vs, T):
    """Distinct blocks touched by the ray bands of each 16x16 pixel tile
    (the binary32 band rule of gsdf_allocate_blocks at the identity pose,
    every sample counted; a repeated voxel never adds a block)."""
    f32 = np.float32
    H, W = depth.shape
    ns = int(np.floor(2 * T / (vs / 2) + 0.5)) + 1
    v, u = np.mgrid[0:H, 0:W]
    xr = (u.astype(f32) - f32(cam.cx)) * f32(1 / cam.fx)
    yr = (v.astype(f32) - f32(cam.cy)) * f32(1 / cam.fy)
    D = depth.astype(f32)
    ty, tx = v // 16, u // 16
    seen = set()
    for k in range(ns):
        z = (D - f32(T)) + f32(k) * f32(vs / 2)
        m = [np.floor(q * f32(1 / vs) + f32(0.5)).astype(np.int64) >> 3 for q in (z * xr, z * yr, z)]
        seen.update(zip(ty.ravel(), tx.ravel(), m[0].ravel(), m[1].ravel(), m[2].ravel()))
    counts = {}
    for t in seen:
        counts[t[:2]] = counts.get(t[:2], 0) + 1
    return counts


def test_fuse_frame_when_tiles_touch_more_blocks_than_their_key_set(torch_mod):
    """A tilted plane seen through 0.5 mm voxels and a 15 mm band: every
    16x16 tile's bands cross about 3000 distinct blocks, more than the
    allocation's 1024-key LDS set per tile holds, so keys go to the global
    table directly; gsdf_fuse_frame still leaves the map that
    gsdf_allocate_blocks + gsdf_integrate_frame leave, bit for bit."""
    cam = synth.Camera(60.0, 60.0, 31.5, 31.5, 64, 64, 0.1, 4.0)
    v, u = np.mgrid[0:64, 0:64]
    depth = (0.5 / (1.0 - 0.3 * (u - cam.cx) / cam.fx)).astype(np.float32)
    vs, T = 0.0005, 0.015
    counts = _tile_block_counts(depth, cam, vs, T)
    log(f"case: tilted plane 64x64, 0.5 mm voxels, T 15 mm; blocks per tile {min(counts.values())}"
        f"-{max(counts.values())}")
    assert min(counts.values()) > 1024
    pose = np.hstack([np.eye(3), np.zeros((3, 1))])
    A = _gpu_map(vs, T, max_blocks=1 << 16)
    B = _gpu_map(vs, T, max_blocks=1 << 16)
    D, P = dev(depth), dev(pose)
    A.allocate(D, cam, P)
    A.integrate(D, cam, P)
    B.fuse(D, cam, P)
    ka, kb = A.keys(), B.keys()
    assert len(ka) > 40000
    oa, ob = np.lexsort(ka.T[::-1]), np.lexsort(kb.T[::-1])
    np.testing.assert_array_equal(ka[oa], kb[ob])
    va, vb = A.voxels(len(ka)), B.voxels(len(kb))
    for xa, xb in zip(va, vb):
        np.testing.assert_array_equal(xa[oa], xb[ob])
    c = A.counters()
    np.testing.assert_array_equal(c, B.counters())
    assert c[0] > 0
    assert A.status_flags() == [] and B.status_flags() == []


@pytest.mark.parametrize("levels,iters", [(3, (4, 0, 10)), (3, (0, 5, 10)), (3, (4, 5, 0)), (4, (2, 2, 3, 6))])
def test_track_level_schedules(torch_mod, room_stream, levels, iters):
    """Schedules with skipped or extra levels: work-groups join later levels
    from the pose published at a level boundary (or skip them); the pose and
    every iteration's energy must still match the oracle."""
    torch = torch_mod
    st = room_stream
    O = _oracle_room_map(st, [0, 1, 2, 3])
    G = _gpu_map(0.01, 0.05)
    _import(O, G)
    f = 5
    log(f"case: track frame {f}, {levels} levels, iterations {iters}, separate initial pose buffer")
    To, so, failed = O.track(st.depth[f], st.cam, st.poses[f - 1], levels, list(iters), 0.01)
    init = dev(st.poses[f - 1].copy())
    P = torch.zeros_like(init)
    stats = torch.zeros(2 * sum(iters), dtype=torch.float32, device="cuda")
    G.track(dev(st.depth[f]), st.cam, P, levels=levels, iters=iters, delta=0.01, stats=stats, init=init)
    assert torch.equal(init, dev(st.poses[f - 1].copy()))
    dr, dt = pose_diff(P.cpu().numpy(), To)
    log(f"  GPU vs oracle: {dr:.2e} rad, {dt:.2e} m")
    assert dr < 1e-5 and dt < 1e-5
    sg = stats.cpu().numpy().reshape(-1, 2)
    np.testing.assert_allclose(sg[:, 1], so[:, 1], rtol=1e-4)
    np.testing.assert_allclose(sg[:, 0], so[:, 0], rtol=1e-3)
    assert G.status_flags() == []


def test_track_ignores_words_left_in_its_scratch(torch_mod, room_stream):
    """The tracking reduction hands partials and leaf sums between
    work-groups as words tagged with their iteration, cleared before every
    call.  A scratch filled with words that carry every small tag (the
    value 1.0, tags 1..40) must give the same pose, bit for bit, as a new
    scratch, for schedules whose levels have different members and
    iteration numbers, run one after another on the same scratch."""
    torch = torch_mod
    from paper_2111_13652_amd.gsdf import camera
    st = room_stream
    O = _oracle_room_map(st, [0, 1, 2, 3])
    f = 5
    schedules = [(4, 5, 10), (0, 5, 10), (4, 0, 10), (4, 5, 10)]

    def run(G, iters):
        P = dev(st.poses[f - 1].copy())
        G.track(dev(st.depth[f]), st.cam, P, levels=3, iters=iters, delta=0.01)
        return P

    ref = {}
    for iters in schedules[:3]:
        G = _gpu_map(0.01, 0.05)
        _import(O, G)
        ref[iters] = run(G, iters)
        assert G.status_flags() == []
    G = _gpu_map(0.01, 0.05)
    _import(O, G)
    for iters in schedules:
        log(f"case: track frame {f}, iterations {iters}, scratch filled with tagged words")
        scratch = G._scratch_for(camera(st.cam), 3)
        words = scratch[: scratch.numel() // 8 * 8].view(torch.int64)
        tags = torch.arange(words.numel(), device=words.device, dtype=torch.int64) % 40 + 1
        words.copy_(tags | 0x3FF0000000000000)
        P = run(G, iters)
        assert torch.equal(P, ref[iters]), (iters, (P - ref[iters]).abs().max().item())
        assert G.status_flags() == []


def test_stream_closed_loop_matches_oracle(torch_mod):
    """The frame loop end to end on the 640x480 room stream: frame 0 fused at
    its true pose, every later frame tracked from the previous estimate and
    fused at the new one, on the GPU and in the FP64 oracle, each feeding on
    its own estimates.  Per-frame pose difference and both trajectories'
    errors against the truth are reported; the two loops stay together."""
    torch = torch_mod
    from paper_2111_13652_amd.gsdf import run_stream
    N = 16
    st = synth.make_stream(ROOM["cam"], N, 1, 2, 3)   # the room stream's first N frames
    log(f"case: closed loop, room 640x480, frames 0-{N - 1}, GPU and oracle each on their own estimates")
    _, po = oracle.track_stream(st.depth[:N], st.cam, st.poses[:N], 0.01, 0.05)
    po = np.asarray(po, np.float64)
    G = _gpu_map(0.01, 0.05)
    pg = run_stream(G, dev(st.depth[:N]), st.cam, dev(st.poses[0].copy())).cpu().numpy()
    assert G.status_flags() == []
    diffs = np.array([pose_diff(pg[f], po[f]) for f in range(N)])
    ate = lambda P: float(np.sqrt(np.mean(np.sum((P[:, :, 3] - st.poses[:N, :, 3]) ** 2, axis=1))))
    log(f"  per-frame GPU vs oracle: max {diffs[:, 0].max():.2e} rad, {diffs[:, 1].max():.2e} m "
        f"(last frame {diffs[-1, 0]:.2e} rad, {diffs[-1, 1]:.2e} m)")
    log(f"  ATE against the truth: GPU {ate(pg) * 1e3:.4f} mm, oracle {ate(po) * 1e3:.4f} mm")
    assert diffs[:, 0].max() < 1e-5 and diffs[:, 1].max() < 1e-5
    assert abs(ate(pg) - ate(po)) < 1e-6
