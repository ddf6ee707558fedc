"""Helpers for GPU-vs-oracle parity tests (comparison logic only)."""
import sys

import numpy as np


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(x, dtype=None):
    import torch
    t = torch.as_tensor(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def sorted_keys(k):
    k = np.asarray(k, np.int32).reshape(-1, 3)
    return k[np.lexsort((k[:, 2], k[:, 1], k[:, 0]))]


def assert_same_keys(gpu_keys, orc_keys):
    g = sorted_keys(gpu_keys)
    o = sorted_keys(orc_keys)
    assert g.shape == o.shape, f"{len(g)} GPU blocks vs {len(o)} oracle blocks"
    np.testing.assert_array_equal(g, o)


def align_voxels(gpu_map, orc_map):
    """GPU (psi, g, W) re-ordered to the oracle's sorted key order."""
    gk = gpu_map.keys()
    psi, g, W = gpu_map.voxels(len(gk))
    ok = orc_map.keys()
    index = {tuple(k): i for i, k in enumerate(gk)}
    rows = np.array([index.get(tuple(k), -1) for k in ok])
    assert np.all(rows >= 0), "oracle block missing on the GPU"
    po, go, Wo, _ = orc_map.voxels(ok)
    return (psi[rows], g[rows], W[rows]), (po, go, Wo), ok


def marginal_voxels(orc_map, depth, cam, pose, marginal):
    """Voxel coordinates touched by pixels whose angle test was marginal."""
    out = set()
    for v, u in np.argwhere(marginal):
        for m in orc_map.band_voxels(cam, pose, int(u), int(v), float(depth[v, u])):
            out.add(tuple(int(c) for c in m))
    return out


def voxel_coords(keys):
    c = np.arange(512)
    loc = np.stack([c % 8, (c // 8) % 8, c // 64], -1)
    return 8 * np.asarray(keys)[:, None, :] + loc[None]


def compare_voxels(gpu, orc, keys, voxel_size, exclude=frozenset(), psi_tol=1e-4, g_tol=1e-5,
                   w_rtol=1e-5, w_atol=1e-4):
    """Parity of psi (in units of the voxel size), g-direction and W on voxels
    observed by both sides; returns a report dict.

    W is checked as |dW| <= w_rtol W + w_atol: the linear weight has slope
    1/(T - eps) in d, so a voxel whose observations all lie near d = T has a
    tiny W whose relative error is large while its absolute error (in units of
    one full-weight observation) stays ~1e-7 per observation."""
    pg, gg, Wg = gpu
    po, go, Wo = orc
    both = (Wg > 0) & (Wo > 0)
    if exclude:
        coords = voxel_coords(keys)
        ex = np.zeros_like(both)
        for b, j in np.argwhere(both):
            if tuple(coords[b, j]) in exclude:
                ex[b, j] = True
        both &= ~ex
        n_excluded = int(ex.sum())
    else:
        n_excluded = 0
    one_side = ((Wg > 0) != (Wo > 0)).sum()
    dpsi = np.abs(pg[both] - po[both]) / voxel_size
    ghg = gg[both] / np.linalg.norm(gg[both], axis=-1, keepdims=True)
    gho = go[both] / np.linalg.norm(go[both], axis=-1, keepdims=True)
    dg = np.linalg.norm(ghg - gho, axis=-1)
    dW = np.abs(Wg[both] - Wo[both]) / (Wo[both] + w_atol / w_rtol)
    rep = dict(n=int(both.sum()), excluded=n_excluded, one_side=int(one_side),
               psi_max=float(dpsi.max()), psi_p9999=float(np.quantile(dpsi, 0.9999)),
               g_max=float(dg.max()), w_max=float(dW.max()))
    log("voxel parity", rep)
    assert rep["n"] > 0
    assert rep["psi_max"] <= psi_tol, rep
    assert rep["g_max"] <= g_tol, rep
    assert rep["w_max"] <= w_rtol, rep
    return rep


def rot_angle(Ra, Rb):
    R = Ra @ Rb.T
    return float(np.linalg.norm([R[2, 1] - R[1, 2], R[0, 2] - R[2, 0], R[1, 0] - R[0, 1]]) / 2)


def pose_diff(Ta, Tb):
    return rot_angle(Ta[:, :3], Tb[:, :3]), float(np.linalg.norm(Ta[:, 3] - Tb[:, 3]))
