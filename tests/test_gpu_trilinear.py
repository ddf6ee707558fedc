"""Tri-linear residual model (Sec. 4.1 Eq. (12)-(13), the comparison model)
on the GPU against the oracle: poses and per-iteration energies and counts
on identical maps, for float32 and bf16 storage."""
import numpy as np
import pytest

import oracle
from paper_2111_13652_amd import synth
from tests.gpu_helpers import dev, log, pose_diff

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    from paper_2111_13652_amd import gsdf  # noqa: F401  (loads libgsdf.so or fails)
    return torch


@pytest.fixture(scope="module")
def room_stream():
    return synth.make_stream(synth.CONFIG_ROOM["cam"], 8, 1, 2, 3)


@pytest.mark.parametrize("storage", ["fp32", "bf16"])
def test_trilinear_tracking_matches_the_oracle(torch_mod, room_stream, storage):
    from paper_2111_13652_amd.gsdf import GsdfMap
    torch = torch_mod
    st = room_stream
    G = GsdfMap(0.01, 0.05, 60000, storage=storage)
    for f in range(4):
        G.fuse(dev(st.depth[f]), st.cam, dev(st.poses[f]))
    keys = G.keys()
    psi, g, W = G.voxels(len(keys))
    O = oracle.OracleMap(0.01, 0.05)
    O.set_voxels(keys, psi.astype(np.float64), g.astype(np.float64), W.astype(np.float64))
    for f, (levels, iters) in ((5, (3, (4, 5, 10))), (6, (1, (6,)))):
        log(f"case: tri-linear tracking, room frame {f}, {storage}, {levels} levels {iters}")
        T0 = synth.perturb_pose(st.poses[f], 40 + f, 1.0, 0.01)
        To, so, failed = O.track(st.depth[f], st.cam, T0, levels, list(iters), 0.01, model="trilinear")
        P = dev(T0.copy())
        stats = torch.zeros(2 * sum(iters), dtype=torch.float32, device="cuda")
        G.track(dev(st.depth[f]), st.cam, P, levels=levels, iters=iters, delta=0.01, stats=stats,
                model="trilinear")
        dr, dt = pose_diff(P.cpu().numpy(), To)
        log(f"  GPU vs oracle {dr:.2e} rad {dt:.2e} m; oracle vs truth {pose_diff(To, st.poses[f])}")
        assert failed == 0
        assert dr < 1e-5 and dt < 1e-5
        sg = stats.cpu().numpy().reshape(-1, 2)
        np.testing.assert_allclose(sg[:, 1], so[:, 1], rtol=1e-4)
        np.testing.assert_allclose(sg[:, 0], so[:, 0], rtol=1e-3)
        assert sg[0, 1] > 1000
        # the comparison model reaches the truth about as well as the Taylor model
        Pt = dev(T0.copy())
        G.track(dev(st.depth[f]), st.cam, Pt, levels=levels, iters=iters, delta=0.01)
        e_tri = pose_diff(P.cpu().numpy(), st.poses[f])
        e_tay = pose_diff(Pt.cpu().numpy(), st.poses[f])
        log(f"  error vs truth: tri-linear {e_tri}, Taylor {e_tay}")
        assert e_tri[0] < 2e-3 and e_tri[1] < 5e-3
    assert G.status_flags() == []
