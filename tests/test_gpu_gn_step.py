"""The batched Gauss-Newton step of joint refinement (gsdf_gn_step_keyframes)
through the C ABI: for every keyframe the step gsdf_track_frame takes with
one level and one iteration, checked against those per-keyframe calls and
against the FP64 oracle's Gauss-Newton iteration on the same map values;
and its handling of a non-finite pose.  Needs an MI355X."""
import numpy as np
import pytest

import oracle
from paper_2111_13652_amd import synth
from tests.gpu_helpers import dev, log, pose_diff

pytestmark = pytest.mark.gpu

ROOM = synth.CONFIG_ROOM
DELTA = 0.01
DAMPING = 1e-6


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    from paper_2111_13652_amd import gsdf  # noqa: F401  (loads libgsdf.so or fails)
    return torch


@pytest.fixture(scope="module")
def room_stream():
    return synth.make_stream(ROOM["cam"], 10, 1, 2, 3)


def _fused_map(st, storage):
    from paper_2111_13652_amd.gsdf import GsdfMap
    G = GsdfMap(ROOM["voxel_size"], ROOM["truncation"], 60000, storage=storage)
    for f in range(6):
        G.fuse(dev(st.depth[f]), st.cam, dev(st.poses[f]))
    return G


@pytest.mark.parametrize("storage", ["fp32", "bf16"])
def test_batched_step_matches_per_keyframe_tracking_and_the_oracle(torch_mod, room_stream, storage):
    """Keyframes 6-9 at poses perturbed by 1 deg / 1 cm.  Against
    track(levels=1, iters=(1,)) per keyframe: the same step up to the
    float32 per-thread sums, which group the pixels differently (bar 1e-7
    rad / 1e-7 m, about 1e-5 of a step of 1 deg / 1 cm).  Against the
    oracle's iteration on the map's values: the tracking bar, 1e-5 rad /
    1e-5 m."""
    torch = torch_mod
    st = room_stream
    G = _fused_map(st, storage)
    idx = [6, 7, 8, 9]
    T0 = np.stack([synth.perturb_pose(st.poses[f], 30 + i, 1.0, 0.01) for i, f in enumerate(idx)])
    D = dev(st.depth[idx])
    log(f"case: batched Gauss-Newton step, {len(idx)} keyframes 640x480, {storage}")
    A = dev(T0)
    G.gn_step_keyframes(D, st.cam, A, delta=DELTA, damping=DAMPING)
    torch.cuda.synchronize()
    assert G.status_flags() == []
    A = A.cpu().numpy()
    B = []
    for i in range(len(idx)):
        P = dev(T0[i])
        G.track(D[i], st.cam, P, levels=1, iters=(1,), delta=DELTA, damping=DAMPING)
        B.append(P.cpu().numpy())
    torch.cuda.synchronize()
    assert G.status_flags() == []
    keys = G.keys()
    psi, g, W = G.voxels(len(keys))
    O = oracle.OracleMap(ROOM["voxel_size"], ROOM["truncation"])
    O.set_voxels(keys, psi.astype(np.float64), g.astype(np.float64), W.astype(np.float64))
    for i, f in enumerate(idx):
        step = pose_diff(A[i], T0[i])
        rb, tb = pose_diff(A[i], B[i])
        Tn, _, failed = O.gn_level(st.depth[f].astype(np.float64), st.cam, T0[i], 1, DELTA, DAMPING)
        ro, to = pose_diff(A[i], Tn)
        log(f"  keyframe {f}: step {np.rad2deg(step[0]):.3f} deg / {step[1] * 1e3:.2f} mm; "
            f"against the per-keyframe call {rb:.1e} rad / {tb:.1e} m; against the oracle {ro:.1e} rad / {to:.1e} m")
        assert failed == 0
        assert rb < 1e-7 and tb < 1e-7
        assert ro < 1e-5 and to < 1e-5


def test_batched_step_leaves_a_non_finite_pose_and_reports_it(torch_mod, room_stream):
    """One keyframe's pose holds a NaN: it is left as it is, the call
    reports GSDF_EINVAL, and the other keyframes take exactly the step they
    take without it (each keyframe's sums are its own)."""
    torch = torch_mod
    st = room_stream
    G = _fused_map(st, "fp32")
    idx = [6, 7, 8]
    T0 = np.stack([synth.perturb_pose(st.poses[f], 40 + i, 1.0, 0.01) for i, f in enumerate(idx)])
    bad = T0.copy()
    bad[1, 0, 3] = np.nan
    log("case: batched Gauss-Newton step with a NaN in keyframe 7's pose")
    A = dev(bad)
    G.gn_step_keyframes(dev(st.depth[idx]), st.cam, A)
    torch.cuda.synchronize()
    assert G.status_flags() == ["invalid"]
    A = A.cpu().numpy()
    assert np.array_equal(np.isnan(A[1]), np.isnan(bad[1]))
    assert np.array_equal(np.nan_to_num(A[1]), np.nan_to_num(bad[1]))
    G.status.zero_()
    ok = dev(T0[[0, 2]])
    G.gn_step_keyframes(dev(st.depth[[idx[0], idx[2]]]), st.cam, ok)
    torch.cuda.synchronize()
    assert G.status_flags() == []
    ok = ok.cpu().numpy()
    assert np.array_equal(A[0], ok[0]) and np.array_equal(A[2], ok[1])
