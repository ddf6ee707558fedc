"""Device-side status words forced from the host, and checkpoint/resume.

* GSDF_EHIP: tracking whose waits between work-groups are bounded to one
  poll gives up (every work-group still exits), and the next call on the
  same scratch tracks normally;
* GSDF_ELOST: a frame tracked from a pose that sees none of the map;
* GSDF_EINVAL on the device: a non-finite pose makes tracking, allocation
  and fusion do nothing;
* checkpoint: a map exported (keys, psi, g, W) and imported into a new map
  continues the stream like the original, within the parity tolerances.
Needs an MI355X."""
import numpy as np
import pytest

from paper_2111_13652_amd import synth
from tests.gpu_helpers import compare_voxels, dev, log, pose_diff

pytestmark = pytest.mark.gpu

ROOM = synth.CONFIG_ROOM


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    from paper_2111_13652_amd import gsdf  # noqa: F401  (loads libgsdf.so or fails)
    return torch


@pytest.fixture(scope="module")
def room_stream():
    return synth.make_stream(ROOM["cam"], 10, 1, 2, 3)


def _fused_map(st, frames, **kw):
    from paper_2111_13652_amd.gsdf import GsdfMap
    G = GsdfMap(ROOM["voxel_size"], ROOM["truncation"], 60000, **kw)
    for f in frames:
        G.fuse(dev(st.depth[f]), st.cam, dev(st.poses[f]))
    return G


def test_bounded_wait_gives_up_with_ehip_and_the_next_call_recovers(torch_mod, room_stream):
    torch = torch_mod
    st = room_stream
    G = _fused_map(st, [0, 1, 2])
    D = dev(st.depth[3])
    ref = dev(st.poses[2].copy())
    Gr = _fused_map(st, [0, 1, 2])
    Gr.track(D, st.cam, ref)
    torch.cuda.synchronize()
    log("case: tracking with every wait bounded to one poll")
    init = dev(st.poses[2].copy())
    out = torch.zeros_like(init)
    G.track(D, st.cam, out, init=init, max_polls=1)
    torch.cuda.synchronize()        # every work-group exited
    flags = G.status_flags()
    log("  status", flags)
    assert "gave_up" in flags
    log("case: the same map and scratch, default bounds")
    G.status.zero_()
    P = dev(st.poses[2].copy())
    G.track(D, st.cam, P)
    torch.cuda.synchronize()
    assert G.status_flags() == []
    assert torch.equal(P, ref)


def test_unrelated_pose_is_lost(torch_mod, room_stream):
    torch = torch_mod
    st = room_stream
    G = _fused_map(st, [0])
    # the first camera turned round by 180 degrees about the vertical: it
    # sees the half of the room frame 0 never observed
    T = st.poses[0].copy()
    T[:, :3] = synth.rotation_about([0.0, 0.0, 1.0], np.pi) @ T[:, :3]
    log("case: frame 0 tracked from the camera turned round")
    P = dev(T)
    G.track(dev(st.depth[0]), st.cam, P, min_inlier_frac=0.5)
    torch.cuda.synchronize()
    log("  status", G.status_flags())
    assert "lost" in G.status_flags()


def test_non_finite_pose_does_nothing(torch_mod, room_stream):
    torch = torch_mod
    st = room_stream
    G = _fused_map(st, [0])
    n0 = G.num_blocks()
    psi0, g0, W0 = G.voxels(n0)
    bad = st.poses[1].copy()
    bad[1, 3] = np.nan
    log("case: track, allocate and fuse at a pose with a NaN entry")
    init = dev(bad)
    out = torch.zeros_like(init)
    G.track(dev(st.depth[1]), st.cam, out, init=init)
    torch.cuda.synchronize()
    assert G.status_flags() == ["invalid"]
    assert torch.equal(torch.isnan(out), torch.isnan(init))
    assert torch.equal(torch.nan_to_num(out), torch.nan_to_num(init))
    G.status.zero_()
    G.allocate(dev(st.depth[1]), st.cam, init)
    G.integrate(dev(st.depth[1]), st.cam, init)
    G.fuse(dev(st.depth[1]), st.cam, init)
    torch.cuda.synchronize()
    assert G.status_flags() == ["invalid"]
    assert G.num_blocks() == n0
    psi1, g1, W1 = G.voxels(n0)
    assert np.array_equal(W0, W1) and np.array_equal(psi0, psi1) and np.array_equal(g0, g1)
    bad[1, 3] = np.inf
    G.status.zero_()
    G.track(dev(st.depth[1]), st.cam, dev(bad))
    torch.cuda.synchronize()
    assert G.status_flags() == ["invalid"]


def test_checkpoint_and_resume(torch_mod, room_stream):
    """Frames 0-4 fused, the map saved (keys, psi, g, W) and loaded into a
    new map; both maps then run frames 5-9.  Each tracks every frame from
    its own previous estimate, and the poses must agree within 1e-5 rad /
    1e-5 m.  Both fuse each frame at the uninterrupted run's estimate, and
    the maps must agree within the parity tolerances (psi is saved as the
    weighted mean, so the restored sum differs by a rounding).  Fusing each
    map at its own estimate would compare two fusions at poses that differ
    by rounding (about 1e-11), and the binary32 band rule places a band
    sample in a neighbouring voxel when it lies that close to a voxel face,
    which is no property of the checkpoint."""
    torch = torch_mod
    from paper_2111_13652_amd.gsdf import GsdfMap, run_stream
    st = room_stream
    cam = st.cam
    A = GsdfMap(ROOM["voxel_size"], ROOM["truncation"], 60000)
    D = dev(st.depth)
    est = run_stream(A, D, cam, dev(st.poses[0]), stop=5)
    keys = A.keys()
    psi, g, W = A.voxels(len(keys))
    log(f"case: checkpoint of {len(keys)} blocks after frame 4, resumed for frames 5-9")
    B = GsdfMap(ROOM["voxel_size"], ROOM["truncation"], 60000)
    B.import_blocks(keys, psi, g, W)
    ea, eb = est.clone(), est.clone()
    for f in range(5, 10):
        A.track(D[f], cam, ea[f], init=ea[f - 1])
        B.track(D[f], cam, eb[f], init=eb[f - 1])
        A.fuse(D[f], cam, ea[f])
        B.fuse(D[f], cam, ea[f])
    torch.cuda.synchronize()
    assert A.status_flags() == [] and B.status_flags() == []
    ea, eb = ea.cpu().numpy(), eb.cpu().numpy()
    worst = max(pose_diff(ea[f], eb[f]) for f in range(5, 10))
    log(f"  pose difference resumed vs uninterrupted: {worst[0]:.2e} rad, {worst[1]:.2e} m")
    assert worst[0] < 1e-5 and worst[1] < 1e-5
    ka, kb = A.keys(), B.keys()
    oa, ob = np.lexsort(ka.T[::-1]), np.lexsort(kb.T[::-1])
    assert np.array_equal(ka[oa], kb[ob])
    va = tuple(x[oa] for x in A.voxels(len(ka)))
    vb = tuple(x[ob] for x in B.voxels(len(kb)))
    compare_voxels(va, vb, ka[oa], ROOM["voxel_size"])
