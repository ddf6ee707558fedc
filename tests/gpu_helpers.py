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


def pack_coords(c):
    """One int64 per integer (x, y, z) triple (|coordinate| < 2^20)."""
    c = np.asarray(c, np.int64) + (1 << 20)
    return (c[..., 0] << 42) | (c[..., 1] << 21) | c[..., 2]


def voxel_coords(keys):
    c = np.arange(512)
    loc = np.stack([c % 8, (c // 8) % 8, c // 64], -1)
    return 8 * np.asarray(keys)[:, None, :] + loc[None]


def compare_voxels(gpu, orc, keys, voxel_size, exclude=frozenset(), psi_tol=1e-4, g_tol=1e-5,
                   w_rtol=1e-5, w_atol=1e-4, gradients=True):
    """Parity of psi (in units of the voxel size), g-direction and W; returns
    a report dict.

    psi and g are compared on voxels observed by both sides.  W is compared
    on every voxel observed by either side, as |dW| <= w_rtol W + w_atol:
    W is a sum of observation weights, and the linear weight has slope
    1/(T - eps) in d, so each observation's weight carries an absolute error
    of that slope times the float32 error of d (about 25/m x 1e-8 m) however
    small the weight is.  A voxel whose only observations lie within that
    error of d = T has W ~ 1e-7 and may be observed by one side only; the
    same bound covers it (its W must stay below w_atol).  Voxels touched by
    a pixel whose angle test is within rounding of its threshold
    (``exclude``) are left out and counted.  gradients=False: maps without
    stored gradients (g is not compared)."""
    pg, gg, Wg = gpu
    po, go, Wo = orc
    either = (Wg > 0) | (Wo > 0)
    if len(exclude):
        ex = np.isin(pack_coords(voxel_coords(keys)), pack_coords(np.array(list(exclude)).reshape(-1, 3)))
        ex &= either
        either &= ~ex
        n_excluded = int(ex.sum())
    else:
        n_excluded = 0
    both = either & (Wg > 0) & (Wo > 0)
    one = either & ~both
    dpsi = np.abs(pg[both] - po[both]) / voxel_size
    if gradients:
        ghg = gg[both] / np.linalg.norm(gg[both], axis=-1, keepdims=True)
        gho = go[both] / np.linalg.norm(go[both], axis=-1, keepdims=True)
        dg = np.linalg.norm(ghg - gho, axis=-1)
    else:
        dg = np.zeros(1)
    dW = np.abs(Wg[either] - Wo[either]) / (Wo[either] + w_atol / w_rtol)
    rep = dict(n=int(both.sum()), excluded=n_excluded, one_side=int(one.sum()),
               one_side_w_max=float(np.maximum(Wg[one], Wo[one]).max()) if one.any() else 0.0,
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
