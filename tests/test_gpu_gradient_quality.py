"""Gradient quality (Sec. 5.2, App. A) on the GPU: parity of the per-voxel
distances and angles with the oracle on identical stored values, and the
paper's finding in kind at its setup (five noisy spheres, 1 cm voxels,
truncation 10 voxels, true poses): stored gradients deviate far less from
the truth than finite differences of the stored distance."""
import numpy as np
import pytest

import oracle
from paper_2111_13652_amd import synth
from tests.gpu_helpers import dev, log

pytestmark = pytest.mark.gpu

CFG = synth.CONFIG_SPHERES


@pytest.fixture(scope="module")
def stream():
    return synth.make_spheres_stream(CFG["cam"], 40)


def _fuse(stream, storage, n):
    from paper_2111_13652_amd.gsdf import GsdfMap
    G = GsdfMap(CFG["voxel_size"], CFG["truncation"], 60000, storage=storage)
    for f in range(n):
        G.fuse(dev(stream.depth[f]), stream.cam, dev(stream.poses[f]))
    return G


@pytest.mark.parametrize("storage", ["fp32", "bf16"])
def test_gradient_quality_matches_the_oracle(stream, storage):
    log(f"case: gradient quality parity, five spheres 640x480, 12 frames, {storage}")
    G = _fuse(stream, storage, 12)
    keys = G.keys()
    psi, g, W = G.voxels(len(keys))
    O = oracle.OracleMap(CFG["voxel_size"], CFG["truncation"])
    O.set_voxels(keys, psi.astype(np.float64), g.astype(np.float64), W.astype(np.float64))
    q_gpu = G.gradient_quality(stream.scene.spheres).cpu().numpy().astype(np.float64)
    q_orc = O.gradient_quality(stream.scene.spheres, keys)
    assert q_gpu.shape == q_orc.shape
    np.testing.assert_array_equal(np.isnan(q_gpu), np.isnan(q_orc))
    ok = np.isfinite(q_orc)
    log(f"  {int(ok[1].sum())} voxels, {int(ok[4].sum())} with differences")
    assert ok[4].sum() > 100000
    np.testing.assert_allclose(q_gpu[0][ok[0]], q_orc[0][ok[0]], rtol=1e-6, atol=0)
    for k in range(1, 5):
        err = np.abs(q_gpu[k][ok[k]] - q_orc[k][ok[k]])
        assert err.max() < 3e-5, (k, err.max())


def test_gradient_quality_in_kind(stream):
    from paper_2111_13652_amd.gsdf import angle_statistics
    log("case: gradient quality experiment, five spheres 640x480, 40 frames, fp32")
    G = _fuse(stream, "fp32", 40)
    stats = angle_statistics(G.gradient_quality(stream.scene.spheres), CFG["voxel_size"], (1, 2, 5, 10))
    for x, row in stats.items():
        log(f"  within {x:2d} voxels (n={row['n']}): " +
            ", ".join(f"{k} {row[k][0]:.2f}/{row[k][1]:.2f}/{row[k][2]:.1f}"
                      for k in ("stored", "forward", "backward", "central")))
    r = stats[10]
    assert r["n"] > 200000
    assert r["stored"][0] < 0.7 * r["central"][0]
    assert r["central"][0] < r["forward"][0] and r["central"][0] < r["backward"][0]
    for x in (1, 2, 5, 10):
        assert stats[x]["stored"][2] < stats[x]["central"][2]
