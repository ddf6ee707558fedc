"""The photometric term on the GPU through the C ABI (joint refinement with
colour): mean colour (Eq. (21)), loss and gradients against the FP64 oracle
on identical parameters, and the joint refinement driver on a BF16 map."""
import numpy as np
import pytest

import oracle
from paper_2111_13652_amd import synth
from tests.gpu_helpers import dev, log, pose_diff

pytestmark = pytest.mark.gpu

ROOM = synth.CONFIG_ROOM


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    from paper_2111_13652_amd import gsdf  # noqa: F401  (loads libgsdf.so or fails)
    return torch


@pytest.fixture(scope="module")
def rgbd_stream():
    return synth.make_rgbd_stream(ROOM["cam"], 10)


@pytest.fixture(scope="module")
def maps(torch_mod, rgbd_stream):
    """GPU map of frames 0-3 fused at the truth, and an oracle map holding
    exactly the GPU's float32 parameter values."""
    from paper_2111_13652_amd.gsdf import GsdfMap, voxel_order
    st = rgbd_stream
    G = GsdfMap(0.01, 0.05, 60000)
    for f in range(4):
        G.fuse(dev(st.depth[f]), st.cam, dev(st.poses[f]))
    keys = G.keys()
    params = G.export_params(len(keys))
    W = G.weight[: len(keys) * 512].view(len(keys), 512)
    inv = np.argsort(voxel_order())                       # Morton index -> lx + 8 ly + 64 lz
    p = params.cpu().numpy()[:, voxel_order(), :]         # -> (slot, lx + 8 ly + 64 lz, 4)
    Wl = W.cpu().numpy()[:, voxel_order()]
    O = oracle.OracleMap(0.01, 0.05)
    O.set_voxels(keys, p[..., 0].astype(np.float64), p[..., 1:].astype(np.float64), Wl.astype(np.float64))
    return G, O, keys, params, inv


def _to_gpu_order(x, order):
    """(n, 512, ...) in lx + 8 ly + 64 lz order -> Morton order."""
    out = np.empty_like(x)
    out[:, order] = x
    return out


def test_mean_colour_loss_and_gradients_match_the_oracle(torch_mod, rgbd_stream, maps):
    torch = torch_mod
    from paper_2111_13652_amd.gsdf import PhotometricLoss, mean_color, voxel_order
    st = rgbd_stream
    G, O, keys, params, _ = maps
    order = voxel_order()
    idx = [4, 6, 8]
    K = len(idx)
    T0 = np.stack([synth.perturb_pose(st.poses[f], 60 + i, 0.5, 0.005) for i, f in enumerate(idx)])
    xi = np.random.default_rng(5).standard_normal((K, 6)) * 1e-3
    D, I = st.depth[idx], st.rgb[idx]
    log(f"case: photometric term, {K} keyframes 640x480, 1 cm voxels")
    col_o, cnt_o = O.mean_color(D.astype(np.float64), I.astype(np.float64), st.cam, T0, xi, keys)
    col_g, cnt_g = mean_color(G, params, dev(xi), dev(D), dev(I), st.cam, dev(T0))
    col_g = col_g.cpu().numpy()[:, order]
    cnt_g = cnt_g.cpu().numpy()[:, order]
    log("  surface voxels seen:", int((cnt_o > 0).sum()), "views", int(cnt_o.sum()), "GPU views", int(cnt_g.sum()))
    np.testing.assert_array_equal(cnt_g, cnt_o)
    np.testing.assert_allclose(col_g, col_o, atol=2e-6)
    rho = (col_o + np.random.default_rng(6).standard_normal(col_o.shape) * 0.03).astype(np.float32)
    delta, lam = 0.05, 0.8
    L_o, dpsi_o, dcol_o, dxi_o, nvis = O.photo_loss_grad(D.astype(np.float64), I.astype(np.float64), st.cam, T0,
                                                         xi, rho.astype(np.float64), delta, lam, keys)
    P = params.clone().requires_grad_(True)
    R = dev(_to_gpu_order(rho, order)).requires_grad_(True)
    X = dev(xi).requires_grad_(True)
    L = PhotometricLoss.apply(P, R, X, G, dev(D), dev(I), st.cam, dev(T0), delta, lam)
    L.sum().backward()
    Lg = L.detach().cpu().numpy()
    log("  loss GPU", Lg, "oracle", L_o)
    np.testing.assert_allclose(Lg, L_o, rtol=1e-5)
    dxi_g = X.grad.cpu().numpy()
    for i in range(K):
        err = np.abs(dxi_g[i] - dxi_o[i]).max() / np.abs(dxi_o[i]).max()
        log(f"  dxi[{i}] rel err {err:.2e}")
        assert err < 1e-4
    gp = P.grad.cpu().numpy()[:, order]
    assert np.all(gp[..., 1:] == 0)
    gc = R.grad.cpu().numpy()[:, order]
    for name, gpu, orc in (("dpsi", gp[..., 0], dpsi_o), ("dcolor", gc, dcol_o)):
        scale = np.abs(orc).max()
        err = np.abs(gpu - orc)
        bad = err > 1e-4 * np.abs(orc) + 1e-6 * scale
        log(f"  {name}: nonzero {int((orc != 0).sum())}, max abs err {err.max():.2e} (scale {scale:.2e}), "
            f"outside bar {int(bad.sum())}")
        assert not bad.any()


def test_joint_refinement_on_a_bf16_map(torch_mod, rgbd_stream):
    """SDF + photometric refinement of 5 keyframes (poses perturbed by
    1 deg / 1 cm) on a BF16-stored map fused at the truth: 50 steps (Adam on
    psi/g and colours from both adjoints, one Gauss-Newton pose iteration per
    keyframe on the updated map) lower the joint loss and bring the poses
    back; the Adam pose variant gets most of the way."""
    torch = torch_mod
    import time
    from paper_2111_13652_amd.gsdf import GsdfMap, refine_joint
    st = rgbd_stream
    idx = [4, 5, 6, 7, 8]
    T0 = np.stack([synth.perturb_pose(st.poses[f], 80 + i, 1.0, 0.01) for i, f in enumerate(idx)])
    before = [pose_diff(T0[i], st.poses[f]) for i, f in enumerate(idx)]
    log("case: joint refinement, 5 keyframes, bf16 map; initial errors", before)
    for solver, rot_bar, t_bar in (("gn", np.deg2rad(0.05), 1e-3), ("adam", np.deg2rad(0.2), 4e-3)):
        G = GsdfMap(0.01, 0.05, 60000, storage="bf16")
        for f in range(4):
            G.fuse(dev(st.depth[f]), st.cam, dev(st.poses[f]))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        poses, params, colors, losses = refine_joint(G, dev(st.depth[idx]), dev(st.rgb[idx]), st.cam, dev(T0),
                                                     steps=50, pose_solver=solver)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        P = poses.cpu().numpy()
        after = [pose_diff(P[i], st.poses[f]) for i, f in enumerate(idx)]
        log(f"  {solver}: {dt * 1e3 / 50:.2f} ms per step; loss {losses[0]:.4f} -> {losses[-1]:.4f}; "
            f"final errors", after)
        assert losses[-1] < 0.3 * losses[0]
        for ra, ta in after:
            assert ra < rot_bar and ta < t_bar
        assert G.status_flags() == []
