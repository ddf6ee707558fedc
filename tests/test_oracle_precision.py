"""Oracle pins for the reduced-precision (bf16 / fp16) storage emulation."""
import numpy as np
import torch

import oracle
from tests import scenes


def test_round_storage_matches_library_conversions():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.uniform(-1, 1, 3000), rng.standard_normal(3000) * 1e-3,
                        rng.standard_normal(100) * 1e-6, [0.0, 1.0, -1.0, 0.5]]).astype(np.float32)
    bf = torch.tensor(x).to(torch.bfloat16).to(torch.float64).numpy()
    f16 = x.astype(np.float16).astype(np.float64)
    for a, b, h in zip(x, bf, f16):
        assert oracle.round_storage(float(a), "bf16") == b
        assert oracle.round_storage(float(a), "fp16") == h


def test_rounded_fusion_of_a_plane_is_the_rounded_exact_distance():
    cam = scenes.SMALL_CAM
    depth = np.full((cam.height, cam.width), 2.0, np.float32)
    for storage in ("bf16", "fp16"):
        M = oracle.OracleMap(0.01, 0.05)
        M.allocate(depth, cam, scenes.IDENTITY)
        M.integrate_rounded(depth, cam, scenes.IDENTITY, storage)
        keys = M.keys()
        psi, g, W, _ = M.voxels(keys)
        obs = W > 0
        vz = 0.01 * (8 * keys[:, 2:3] + (np.arange(512) // 64)[None, :])
        exact = np.clip(vz - 2.0, -0.05, 0.05)
        want = np.vectorize(lambda e: 0.05 * oracle.round_storage(e / 0.05, storage))(exact[obs])
        np.testing.assert_array_equal(psi[obs], want)
        np.testing.assert_array_equal(g[obs], np.broadcast_to([0, 0, 1], g[obs].shape))
        # W is a binary32 sum of full weights (d <= eps) and linear ones
        assert np.all(W[obs] == W[obs].astype(np.float32))


def test_rounded_fusion_stays_within_storage_error_of_exact_fusion():
    st = scenes.room_frames(scenes.SMALL_CAM, 3)
    E = oracle.OracleMap(0.02, 0.1)
    B = oracle.OracleMap(0.02, 0.1)
    for f in range(3):
        for M in (E, B):
            M.allocate(st.depth[f], st.cam, st.poses[f])
        E.integrate(st.depth[f], st.cam, st.poses[f])
        B.integrate_rounded(st.depth[f], st.cam, st.poses[f], "bf16")
    keys = E.keys()
    pe, ge, We, _ = E.voxels(keys)
    pb, gb, Wb, _ = B.voxels(keys)
    obs = (We > 0) & (Wb > 0)
    np.testing.assert_array_equal(We > 0, Wb > 0)
    # bf16 keeps 8 significant bits: one rounding per frame of |psi/T| <= 1
    assert np.abs(pe[obs] - pb[obs]).max() <= 3 * 0.1 * 2.0 ** -8
    ghe = ge[obs] / np.linalg.norm(ge[obs], axis=-1, keepdims=True)
    ghb = gb[obs] / np.linalg.norm(gb[obs], axis=-1, keepdims=True)
    assert np.linalg.norm(ghe - ghb, axis=-1).max() < 3 * 2.0 ** -7
