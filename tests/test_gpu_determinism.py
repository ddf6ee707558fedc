"""Run-to-run reproducibility of the frame path on the GPU: the same frames
tracked and fused twice from the same start give bit-identical poses and
bit-identical maps (fixed-point per-frame fusion sums, fixed-order tracking
reduction and solve), for every storage form."""
import numpy as np
import pytest

from paper_2111_13652_amd import synth
from tests.gpu_helpers import dev, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def stream():
    return synth.make_stream(synth.CONFIG_ROOM["cam"], 10, 1, 2, 3)


def _run(st, storage):
    import torch
    from paper_2111_13652_amd.gsdf import GsdfMap, run_stream
    G = GsdfMap(0.01, 0.05, 60000, storage=storage)
    D = dev(st.depth)
    poses = run_stream(G, D, st.cam, dev(st.poses[0].copy()))
    torch.cuda.synchronize()
    keys = G.keys()
    o = np.lexsort(keys.T[::-1])
    vox = G.voxels(len(keys))
    return poses.cpu().numpy(), keys[o], [v[o] for v in vox], G.status_flags()


@pytest.mark.parametrize("storage", ["fp32", "bf16", "fp16"])
def test_frame_path_is_bit_reproducible(stream, storage):
    log(f"case: determinism, room 640x480, 10 frames tracked + fused twice, {storage}")
    p1, k1, v1, s1 = _run(stream, storage)
    p2, k2, v2, s2 = _run(stream, storage)
    assert s1 == [] and s2 == []
    assert np.array_equal(p1, p2)
    assert np.array_equal(k1, k2)
    for a, b in zip(v1, v2):
        assert np.array_equal(a, b)
    err = np.linalg.norm(p1[:, :, 3] - stream.poses[:, :, 3], axis=1).max()
    log(f"  identical; largest position error against the truth {err:.2e} m")
    assert err < 5e-3
