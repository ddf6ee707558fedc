"""The map without stored gradients (GSDF_NOGRAD_FP32: distance and weight
only, Eq. (1)-(2)) tracked with the tri-linear model of Eq. (12)-(13): the
paper's baseline system (Sec. 5.3 runtime comparison), on the GPU through
the C ABI against the oracle's gradient-free mode.

* fusion: keys bit-exact, distances and weights within the voxel
  tolerances of the oracle, and bit-identical to the fp32 map's (the
  gradient sums feed neither);
* tracking: the tri-linear model on the gradient-free map gives the pose
  of the same model on the fp32 map bit for bit, and the oracle's pose
  within 1e-5 rad / 1e-5 m; the closed loop of the baseline system;
* calls that need the gradient reject the map.
Needs an MI355X."""
import numpy as np
import pytest

import oracle
from paper_2111_13652_amd import synth
from tests.gpu_helpers import (assert_same_keys, compare_voxels, dev, log, marginal_voxels, pack_coords,
                               pose_diff)

pytestmark = pytest.mark.gpu

ROOM = synth.CONFIG_ROOM


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    from paper_2111_13652_amd import gsdf  # noqa: F401  (loads libgsdf.so or fails)
    return torch


@pytest.fixture(scope="module")
def room_stream():
    return synth.make_stream(ROOM["cam"], 16, *ROOM["seeds"])


def _aligned(G, keys):
    gk = G.keys()
    psi, g, W = G.voxels(len(gk))
    order = np.argsort(pack_coords(gk))
    rows = order[np.searchsorted(pack_coords(gk)[order], pack_coords(keys))]
    assert np.array_equal(gk[rows], keys)
    return psi[rows], g[rows], W[rows]


def test_fusion_without_gradients(torch_mod, room_stream):
    torch = torch_mod
    from paper_2111_13652_amd.gsdf import GsdfMap
    st = room_stream
    cam = st.cam
    vs, T = ROOM["voxel_size"], ROOM["truncation"]
    O = oracle.OracleMap(vs, T)
    A = GsdfMap(vs, T, 60000, storage="nograd")
    B = GsdfMap(vs, T, 60000, storage="fp32")
    excl = set()
    for f in range(8):
        log(f"case: gradient-free fusion, room 640x480 frame {f} at ground truth")
        D, P = dev(st.depth[f]), dev(st.poses[f])
        O.allocate(st.depth[f], cam, st.poses[f])
        _, marg = O.integrate(st.depth[f], cam, st.poses[f], return_marginal=True, gradients=False)
        excl |= marginal_voxels(O, st.depth[f], cam, st.poses[f], marg)
        if f % 2:
            A.fuse(D, cam, P)
        else:
            A.allocate(D, cam, P)
            A.integrate(D, cam, P)
        B.fuse(D, cam, P)
        assert_same_keys(A.keys(), O.keys())
    torch.cuda.synchronize()
    keys = O.keys()
    pa, ga, Wa = _aligned(A, keys)
    pb, _, Wb = _aligned(B, keys)
    assert not ga.any()
    assert np.array_equal(pa, pb) and np.array_equal(Wa, Wb)
    po, go, Wo, _ = O.voxels(keys)
    assert not go.any()
    rep = compare_voxels((pa, ga, Wa), (po, go, Wo), keys, vs, exclude=excl, gradients=False)
    assert rep["n"] > 300000
    assert A.status_flags() == [] and B.status_flags() == []
    # the gradient-free record is a quarter of the fp32 one
    assert A.buffers[1].numel() * 4 == B.buffers[1].numel()


def test_trilinear_tracking_on_the_gradient_free_map(torch_mod, room_stream):
    torch = torch_mod
    from paper_2111_13652_amd import _lib
    from paper_2111_13652_amd.gsdf import GsdfMap
    st = room_stream
    cam = st.cam
    vs, T = ROOM["voxel_size"], ROOM["truncation"]
    O = oracle.OracleMap(vs, T)
    maps = {s: GsdfMap(vs, T, 60000, storage=s) for s in ("nograd", "fp32")}
    for f in range(4):
        O.allocate(st.depth[f], cam, st.poses[f])
        O.integrate(st.depth[f], cam, st.poses[f], gradients=False)
        for G in maps.values():
            G.fuse(dev(st.depth[f]), cam, dev(st.poses[f]))
    for f in (5, 7):
        log(f"case: tri-linear tracking of frame {f} on the gradient-free map (3 levels, 4/5/10)")
        To, so, _ = O.track(st.depth[f], cam, st.poses[f - 1], 3, [4, 5, 10], 0.01, model="trilinear")
        out = {}
        for s, G in maps.items():
            P = dev(st.poses[f - 1].copy())
            stats = torch.zeros(38, dtype=torch.float32, device="cuda")
            G.track(dev(st.depth[f]), cam, P, model="trilinear", stats=stats)
            out[s] = (P, stats)
        assert torch.equal(out["nograd"][0], out["fp32"][0])
        assert torch.equal(out["nograd"][1], out["fp32"][1])
        dr, dt = pose_diff(out["nograd"][0].cpu().numpy(), To)
        log(f"  GPU vs oracle: {dr:.2e} rad, {dt:.2e} m")
        assert dr < 1e-5 and dt < 1e-5
        sg = out["nograd"][1].cpu().numpy().reshape(-1, 2)
        np.testing.assert_allclose(sg[:, 1], so[:, 1], rtol=1e-4)
    G = maps["nograd"]
    assert G.status_flags() == []
    log("case: calls that need the stored gradient reject the gradient-free map")
    P = dev(st.poses[4].copy())
    with pytest.raises(_lib.GsdfError):
        G.track(dev(st.depth[5]), cam, P, model="taylor")
    with pytest.raises(_lib.GsdfError):
        G.normal_equations(dev(st.depth[5]), cam, P, 0.01)
    with pytest.raises(_lib.GsdfError):
        G.export_params()
    with pytest.raises(_lib.GsdfError):
        G.surfels()


def test_baseline_system_closed_loop(torch_mod, room_stream):
    """The baseline end to end: every frame tracked with the tri-linear model
    on the gradient-free map, then fused at the estimate; GPU and oracle each
    on their own estimates."""
    torch = torch_mod
    from paper_2111_13652_amd.gsdf import GsdfMap
    st = room_stream
    N = len(st.depth)
    vs, T = ROOM["voxel_size"], ROOM["truncation"]
    log(f"case: baseline closed loop (gradient-free map, tri-linear tracking), frames 0-{N - 1}")
    _, po = oracle.track_stream(st.depth, st.cam, st.poses, vs, T, model="trilinear", gradients=False)
    G = GsdfMap(vs, T, 60000, storage="nograd")
    D = dev(st.depth)
    P = torch.zeros((N, 3, 4), dtype=torch.float64, device="cuda")
    P[0].copy_(dev(st.poses[0]))
    G.fuse(D[0], st.cam, P[0])
    for f in range(1, N):
        G.track(D[f], st.cam, P[f], init=P[f - 1], model="trilinear")
        G.fuse(D[f], st.cam, P[f])
    pg = P.cpu().numpy()
    assert G.status_flags() == []
    diffs = np.array([pose_diff(pg[f], po[f]) for f in range(N)])
    ate = lambda E: float(np.sqrt(np.mean(np.sum((E[:, :, 3] - st.poses[:, :, 3]) ** 2, axis=1))))
    log(f"  per-frame GPU vs oracle: max {diffs[:, 0].max():.2e} rad, {diffs[:, 1].max():.2e} m; "
        f"ATE GPU {ate(pg) * 1e3:.4f} mm, oracle {ate(np.asarray(po)) * 1e3:.4f} mm")
    assert diffs[:, 0].max() < 1e-5 and diffs[:, 1].max() < 1e-5
