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
        # wall time of the call, first launches and the optimiser's set-up included
        log(f"  {solver}: {dt * 1e3 / 50:.2f} ms of wall time per step; loss {losses[0]:.4f} -> {losses[-1]:.4f}; "
            f"final errors", after)
        assert losses[-1] < 0.3 * losses[0]
        for ra, ta in after:
            assert ra < rot_bar and ta < t_bar
        assert G.status_flags() == []


@pytest.mark.parametrize("coupled", [True, False])
def test_implicit_ba_energy_and_gradients_match_the_oracle(torch_mod, rgbd_stream, maps, coupled):
    """Bundle-adjustment energy without stored colour (Eq. (17) coupled through
    the mean colour, Eq. (20) decoupled) and its gradients in psi and the
    twists, GPU (autograd composition of the mean-colour and photometric
    kernels) against the FP64 oracle."""
    torch = torch_mod
    from paper_2111_13652_amd.gsdf import implicit_photometric_loss, voxel_order
    st = rgbd_stream
    G, O, keys, params, _ = maps
    order = voxel_order()
    idx = [4, 6, 8]
    K = len(idx)
    T0 = np.stack([synth.perturb_pose(st.poses[f], 90 + i, 0.5, 0.005) for i, f in enumerate(idx)])
    xi = np.random.default_rng(9).standard_normal((K, 6)) * 1e-3
    D, I = st.depth[idx], st.rgb[idx]
    delta = 0.02
    log(f"case: implicit BA energy, coupled={coupled}, {K} keyframes")
    L_o, dpsi_o, dxi_o = O.photo_energy(D.astype(np.float64), I.astype(np.float64), st.cam, T0, xi, delta, 1.0,
                                        coupled, keys)
    P = params.clone().requires_grad_(True)
    X = dev(xi).requires_grad_(True)
    L = implicit_photometric_loss(G, P, X, dev(D), dev(I), st.cam, dev(T0), delta, 1.0, coupled)
    L.sum().backward()
    Lg = L.detach().cpu().numpy()
    log("  energy GPU", Lg, "oracle", L_o)
    np.testing.assert_allclose(Lg, L_o, rtol=1e-5)
    dxi_g = X.grad.cpu().numpy()
    for i in range(K):
        err = np.abs(dxi_g[i] - dxi_o[i]).max() / np.abs(dxi_o[i]).max()
        log(f"  dxi[{i}] rel err {err:.2e}")
        assert err < 1e-4
    gp = P.grad.cpu().numpy()[:, order, 0]
    scale = np.abs(dpsi_o).max()
    err = np.abs(gp - dpsi_o)
    bad = err > 1e-4 * np.abs(dpsi_o) + 1e-5 * scale
    log(f"  dpsi: max abs err {err.max():.2e} (scale {scale:.2e}), outside bar {int(bad.sum())}")
    assert not bad.any()


def test_photometric_ba_recovers_keyframe_poses(torch_mod):
    """Implicit photometric BA (Eq. (17), no stored colour) of 5 keyframes 10
    frames apart, the first anchoring the gauge at its true pose and the
    other four perturbed by 1 deg / 1 cm, on a map fused at the truth.  The
    pose-only and the joint psi + pose variants (0.01 cm^-2 regulariser)
    descend to the energy's minimum (no higher than at the true poses) and
    pull the poses back.  The minimum itself lies a few millimetres from the
    truth: the surface points come from a map fused from noisy depth and the
    colours carry noise, so the translation bar is looser than the rotation
    bar."""
    torch = torch_mod
    from paper_2111_13652_amd.gsdf import GsdfMap, implicit_photometric_loss, photometric_ba
    st = synth.make_rgbd_stream(ROOM["cam"], 41)
    G = GsdfMap(0.01, 0.05, 60000)
    for f in range(0, 41, 4):
        G.fuse(dev(st.depth[f]), st.cam, dev(st.poses[f]))
    idx = [0, 10, 20, 30, 40]
    T0 = np.stack([st.poses[0]] + [synth.perturb_pose(st.poses[f], 120 + i, 1.0, 0.01)
                                   for i, f in enumerate(idx[1:])])
    D, I = dev(st.depth[idx]), dev(st.rgb[idx])
    z = torch.zeros((len(idx), 6), dtype=torch.float64, device="cuda")
    E_true = float(implicit_photometric_loss(G, G.export_params(), z, D, I, st.cam, dev(st.poses[idx])).sum())
    before = [pose_diff(T0[i], st.poses[f]) for i, f in enumerate(idx)]
    log("case: photometric BA, 5 keyframes (first anchored); energy at the truth", E_true,
        "; initial errors", before)
    for opt_psi in (False, True):
        poses, _, losses = photometric_ba(G, D, I, st.cam, dev(T0), steps=300, optimise_psi=opt_psi,
                                          lr_pose=4e-3)
        P = poses.cpu().numpy()
        after = [pose_diff(P[i], st.poses[f]) for i, f in enumerate(idx)]
        log(f"  optimise_psi={opt_psi}: energy {losses[0]:.4f} -> {losses[-1]:.4f}; final errors", after)
        assert losses[-1] < 0.05 * losses[0]
        if not opt_psi:
            assert losses[-1] <= 1.05 * E_true
        assert after[0] == before[0]
        for (ra, ta), (rb, tb) in zip(after[1:], before[1:]):
            assert ra < 0.3 * rb and ta < 0.6 * tb
    assert G.status_flags() == []


@pytest.mark.parametrize("solver", ["gn", "adam"])
def test_fused_joint_steps_are_the_autograd_steps(torch_mod, rgbd_stream, solver):
    """refine_joint with each step's loss and gradients from the two adjoint
    calls alone (fused) and with KeyframeLoss + PhotometricLoss composed
    through autograd: the same poses, parameters and colours, bit for bit,
    after 5 steps (the losses agree to rounding: each path sums them in its
    own pass)."""
    torch = torch_mod
    from paper_2111_13652_amd.gsdf import GsdfMap, refine_joint
    st = rgbd_stream
    idx = [4, 6, 8]
    T0 = dev(np.stack([synth.perturb_pose(st.poses[f], 90 + i, 1.0, 0.01) for i, f in enumerate(idx)]))
    out = []
    log(f"case: joint refinement, 3 keyframes, 5 steps, {solver} poses, fused and through autograd")
    for fused in (True, False):
        G = GsdfMap(0.01, 0.05, 60000, storage="bf16")
        for f in range(4):
            G.fuse(dev(st.depth[f]), st.cam, dev(st.poses[f]))
        P, p, c, losses = refine_joint(G, dev(st.depth[idx]), dev(st.rgb[idx]), st.cam, T0, steps=5,
                                       pose_solver=solver, fused=fused)
        torch.cuda.synchronize()
        assert G.status_flags() == []
        # parameter rows are in pool-slot order, which depends on the order
        # blocks were inserted: compare them by block key
        keys = G.keys()
        o = torch.as_tensor(np.lexsort(keys.T[::-1]), device=p.device)
        out.append((P, keys[o.cpu().numpy()], p[o], c[o], losses))
    (P1, k1, p1, c1, l1), (P2, k2, p2, c2, l2) = out
    np.testing.assert_array_equal(k1, k2)
    assert torch.equal(P1, P2) and torch.equal(p1, p2) and torch.equal(c1, c2)
    np.testing.assert_allclose(l1, l2, rtol=1e-9)
    log("  identical; losses", l1[0], "->", l1[-1])
