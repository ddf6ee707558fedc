"""Pins of the oracle's photometric term (joint refinement with colour):
the surface point v - psi g^ of Eq. (18) against the generator's analytic
colour, the mean colour of Eq. (21) as the minimiser of the quadratic
energy with the exact variance decomposition behind Eq. (19), invariance to
a common brightness offset, and the gradients against central differences."""
import numpy as np
import pytest

import oracle
from paper_2111_13652_amd import synth

CAM = synth.Camera(262.5, 262.5, 159.5, 119.5, 320, 240, 0.4, 4.0)
VS, TR = 0.02, 0.1


@pytest.fixture(scope="module")
def setup():
    """Noiseless colour stream; map fused from frames 0-2 at the truth."""
    st = synth.make_rgbd_stream(CAM, 6, noise_seed=None)
    M = oracle.OracleMap(VS, TR)
    for f in range(3):
        M.allocate(st.depth[f], CAM, st.poses[f])
        M.integrate(st.depth[f], CAM, st.poses[f])
    return st, M


def _object_of(scene, p):
    """Index (as synth.render_ids) of the surface nearest each point."""
    d = [np.min(np.abs(np.concatenate([p - scene.room[0], scene.room[1] - p], 1)), axis=1)]
    d += [np.abs(np.linalg.norm(p - s[:3], axis=1) - s[3]) for s in scene.spheres]
    d += [np.abs(synth._box_sdf_outside(p, b)) for b in scene.boxes]
    return np.argmin(np.stack(d, 1), axis=1)


def _surface_points(M, keys):
    psi, g, W, _ = M.voxels(keys)
    c = np.arange(512)
    m = 8 * keys[:, None, :] + np.stack([c % 8, (c // 8) % 8, c // 64], -1)[None]
    gh = g / np.maximum(np.linalg.norm(g, axis=-1, keepdims=True), 1e-300)
    return VS * m - psi[..., None] * gh, VS * m


def test_mean_colour_samples_the_surface_point_of_eq18(setup):
    st, M = setup
    keys = M.keys()
    K = 3
    idx = [3, 4, 5]
    xi = np.zeros((K, 6))
    col, cnt = M.mean_color(st.depth[idx].astype(np.float64), st.rgb[idx].astype(np.float64), CAM,
                            st.poses[idx], xi, keys)
    p, v = _surface_points(M, keys)
    psi = M.voxels(keys)[0]
    # the room's walls pass through voxel centres (psi ~ 0 there): assess the
    # voxels whose surface point is well away from the centre
    seen = (cnt > 0) & (np.abs(psi) > VS / 8)
    # and where the fused gradient agrees with the true normal: at concave
    # edges (two walls meeting) the averaged psi and g^ of Eq. (1)-(3) put
    # the surface point off both walls, which says nothing about sampling
    g = M.voxels(keys)[1]
    gh = g / np.maximum(np.linalg.norm(g, axis=-1, keepdims=True), 1e-300)
    n_true = np.zeros_like(p)
    n_true[seen] = -synth.surface_normal(st.scene, p[seen], _object_of(st.scene, p[seen]))
    seen &= np.linalg.norm(gh - n_true, axis=-1) < 0.05
    assert seen.sum() > 50
    ps, vs = p[seen], v[seen]
    truth_p = synth.shade(st.albedo, st.scene, ps, _object_of(st.scene, ps))
    truth_v = synth.shade(st.albedo, st.scene, vs, _object_of(st.scene, vs))
    err_p = np.abs(col[seen] - truth_p).max(axis=1)
    err_v = np.abs(col[seen] - truth_v).max(axis=1)
    # sampling at the surface point reproduces the analytic colour up to
    # bilinear interpolation and the fused distance error; the voxel centre
    # (more than v_s / 8 off the surface) does not
    assert np.median(err_p) < 0.002
    assert np.median(err_p) < 0.2 * np.median(err_v)


def test_mean_colour_minimises_the_quadratic_energy_with_exact_decomposition(setup):
    st, M = setup
    keys = M.keys()
    idx = [3, 4, 5]
    D, I = st.depth[idx].astype(np.float64), st.rgb[idx].astype(np.float64)
    xi = np.random.default_rng(1).standard_normal((3, 6)) * 1e-3
    mean, cnt = M.mean_color(D, I, CAM, st.poses[idx], xi, keys)
    big = 1e6   # Huber threshold far above any residual: rho(r) = r^2 / 2
    L0, _, dcol, _, nvis = M.photo_loss_grad(D, I, CAM, st.poses[idx], xi, mean, big, 1.0, keys)
    assert nvis == int(cnt.sum())
    assert np.abs(dcol).max() < 1e-12            # zero gradient in rho at the mean (Eq. (21))
    rng = np.random.default_rng(2)
    rho = mean + rng.standard_normal(mean.shape) * 0.05
    L1 = M.photo_loss_grad(D, I, CAM, st.poses[idx], xi, rho, big, 1.0, keys, want_grads=False)[0]
    # sum_i |I_ij - rho|^2 = sum_i |I_ij - mean|^2 + N_j |rho - mean|^2
    extra = 0.5 * np.sum(cnt[..., None] * (rho - mean) ** 2)
    assert L1.sum() == pytest.approx(L0.sum() + extra, rel=1e-10)


def test_common_brightness_offset_leaves_loss_and_gradients_unchanged(setup):
    st, M = setup
    keys = M.keys()
    idx = [3, 4]
    D, I = st.depth[idx].astype(np.float64), st.rgb[idx].astype(np.float64)
    xi = np.zeros((2, 6))
    col, _ = M.mean_color(D, I, CAM, st.poses[idx], xi, keys)
    col = col + np.random.default_rng(3).standard_normal(col.shape) * 0.02
    a = M.photo_loss_grad(D, I, CAM, st.poses[idx], xi, col, 0.1, 1.0, keys)
    b = M.photo_loss_grad(D, I + 0.25, CAM, st.poses[idx], xi, col + 0.25, 0.1, 1.0, keys)
    np.testing.assert_allclose(a[0], b[0], rtol=1e-9)
    for x, y in zip(a[1:4], b[1:4]):
        np.testing.assert_allclose(x, y, rtol=1e-7, atol=1e-9 * np.abs(x).max())


def test_photometric_gradients_match_central_differences(setup):
    st, M = setup
    keys = M.keys()
    idx = [3, 5]
    D, I = st.depth[idx].astype(np.float64), st.rgb[idx].astype(np.float64)
    rng = np.random.default_rng(4)
    xi = rng.standard_normal((2, 6)) * 1e-3
    col, _ = M.mean_color(D, I, CAM, st.poses[idx], np.zeros((2, 6)), keys)
    col = col + rng.standard_normal(col.shape) * 0.05
    delta, lam = 0.03, 0.7
    L, dpsi, dcol, dxi, _ = M.photo_loss_grad(D, I, CAM, st.poses[idx], xi, col, delta, lam, keys)
    f = lambda x=xi, c=col, mm=M: mm.photo_loss_grad(D, I, CAM, st.poses[idx], x, c, delta, lam, keys,
                                                     want_grads=False)[0].sum()
    # the bilinear sample is only piecewise smooth in (u, v) (its derivative
    # jumps at pixel boundaries) and the Huber loss at |r| = delta: a small
    # step keeps the share of samples crossing a kink negligible
    h = 1e-7
    for i in range(2):
        for k in range(6):
            e = np.zeros_like(xi)
            e[i, k] = h
            fd = (f(x=xi + e) - f(x=xi - e)) / (2 * h)
            assert dxi[i, k] == pytest.approx(fd, rel=1e-5, abs=1e-6 * np.abs(dxi).max())
    # colours enter piecewise quadratically (no bilinear kinks): a larger
    # step keeps the rounding of the summed loss out of the quotient
    h = 1e-5
    for b, j in np.argwhere(np.abs(dcol).max(axis=-1) > 1e-3)[:3]:
        for ch in range(3):
            e = np.zeros_like(col)
            e[b, j, ch] = h
            fd = (f(c=col + e) - f(c=col - e)) / (2 * h)
            assert dcol[b, j, ch] == pytest.approx(fd, rel=1e-5, abs=1e-9)
    psi, g, W, _ = M.voxels(keys)
    h = 1e-6
    for b, j in np.argwhere(np.abs(dpsi) > 1e-3 * np.abs(dpsi).max())[:4]:
        pp, pm = psi.copy(), psi.copy()
        pp[b, j] += h
        pm[b, j] -= h
        A = oracle.OracleMap(VS, TR)
        A.set_voxels(keys, pp, g, W)
        B = oracle.OracleMap(VS, TR)
        B.set_voxels(keys, pm, g, W)
        fd = (f(mm=A) - f(mm=B)) / (2 * h)
        assert dpsi[b, j] == pytest.approx(fd, rel=1e-5, abs=1e-9)


def test_implicit_energy_is_the_stored_colour_loss_at_the_mean(setup):
    """Eq. (17) against each voxel's mean (Eq. (21)) equals the stored-colour
    loss evaluated at the mean colours; for the quadratic penalty the
    coupled (Eq. (17)) and decoupled (Eq. (20)) gradients coincide, because
    a voxel's residuals about their own mean sum to zero."""
    st, M = setup
    keys = M.keys()
    idx = [3, 4, 5]
    D, I = st.depth[idx].astype(np.float64), st.rgb[idx].astype(np.float64)
    xi = np.random.default_rng(7).standard_normal((3, 6)) * 1e-3
    mean, _ = M.mean_color(D, I, CAM, st.poses[idx], xi, keys)
    for delta in (0.02, 1e6):
        Le, _, _ = M.photo_energy(D, I, CAM, st.poses[idx], xi, delta, 0.5, True, keys, want_grads=False)
        Ls = M.photo_loss_grad(D, I, CAM, st.poses[idx], xi, mean, delta, 0.5, keys, want_grads=False)[0]
        np.testing.assert_allclose(Le, Ls, rtol=1e-12)
    _, pc, xc = M.photo_energy(D, I, CAM, st.poses[idx], xi, 1e6, 1.0, True, keys)
    _, pd, xd = M.photo_energy(D, I, CAM, st.poses[idx], xi, 1e6, 1.0, False, keys)
    np.testing.assert_allclose(xc, xd, rtol=1e-9, atol=1e-12 * np.abs(xd).max())
    np.testing.assert_allclose(pc, pd, rtol=1e-9, atol=1e-12 * np.abs(pd).max())
    # with the Huber penalty the mean's own dependence matters
    _, pc, xc = M.photo_energy(D, I, CAM, st.poses[idx], xi, 0.005, 1.0, True, keys)
    _, pd, xd = M.photo_energy(D, I, CAM, st.poses[idx], xi, 0.005, 1.0, False, keys)
    assert np.abs(xc - xd).max() > 1e-6 * np.abs(xd).max()


def test_coupled_energy_gradients_match_central_differences(setup):
    st, M = setup
    keys = M.keys()
    idx = [3, 5]
    D, I = st.depth[idx].astype(np.float64), st.rgb[idx].astype(np.float64)
    xi = np.random.default_rng(8).standard_normal((2, 6)) * 1e-3
    delta = 0.005
    _, dpsi, dxi = M.photo_energy(D, I, CAM, st.poses[idx], xi, delta, 1.0, True, keys)
    f = lambda x=xi, mm=M: mm.photo_energy(D, I, CAM, st.poses[idx], x, delta, 1.0, True, keys,
                                           want_grads=False)[0].sum()
    h = 1e-7   # bilinear samples and the Huber penalty are only piecewise smooth
    for i in range(2):
        for k in range(6):
            e = np.zeros_like(xi)
            e[i, k] = h
            fd = (f(x=xi + e) - f(x=xi - e)) / (2 * h)
            assert dxi[i, k] == pytest.approx(fd, rel=1e-5, abs=1e-6 * np.abs(dxi).max())
    psi, g, W, _ = M.voxels(keys)
    h = 1e-6
    for b, j in np.argwhere(np.abs(dpsi) > 1e-3 * np.abs(dpsi).max())[:4]:
        pp, pm = psi.copy(), psi.copy()
        pp[b, j] += h
        pm[b, j] -= h
        A = oracle.OracleMap(VS, TR)
        A.set_voxels(keys, pp, g, W)
        B = oracle.OracleMap(VS, TR)
        B.set_voxels(keys, pm, g, W)
        fd = (f(mm=A) - f(mm=B)) / (2 * h)
        assert dpsi[b, j] == pytest.approx(fd, rel=1e-5, abs=1e-9)
