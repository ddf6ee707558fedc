"""Pins of the oracle's tri-linear distance (Sec. 4.1 Eq. (12)-(13)), the
direct SDF tracking the paper compares its Taylor model against.

Tri-linear interpolation reproduces linear fields exactly (value and
gradient), interpolates the voxel values, errs on a quadratic by the closed
form c v_s^2 f (1 - f) per axis, needs all eight voxels, and its gradient is
the derivative of the interpolant inside a cell.  Gauss-Newton with it
drives the residuals of a plane seen from a perturbed pose to the rounding
of the binary32 depths."""
import numpy as np

import oracle
from paper_2111_13652_amd import synth
from tests import scenes

VS = 0.02


def _coords(keys):
    c = np.arange(512)
    loc = np.stack([c % 8, (c // 8) % 8, c // 64], -1)
    return keys[:, None, :] * 8 + loc[None]


def _map(keys, field, W=None, vs=VS):
    m = _coords(keys)
    v = m * vs
    psi = field(v)
    W = np.ones(psi.shape) if W is None else W
    g = np.zeros(v.shape)
    g[..., 2] = 1.0
    O = oracle.OracleMap(vs, 0.1)
    O.set_voxels(keys, psi, g, W)
    return O, m


KEYS = np.array([[bx, by, bz] for bx in (-1, 0, 1) for by in (-1, 0) for bz in (0, 1)], np.int32)


def _inside_points(rng, n):
    # points whose 8 surrounding voxel centres lie in KEYS' voxel range
    lo = np.array([-8, -8, 0]) * VS
    hi = np.array([15, 7, 15]) * VS
    return rng.uniform(lo, hi, size=(n, 3))


def test_linear_field_is_exact():
    rng = np.random.default_rng(0)
    a, b = np.array([0.3, -0.7, 0.5]), 0.013
    O, _ = _map(KEYS, lambda v: v @ a + b)
    for q in _inside_points(rng, 500):
        r = O.trilinear(q)
        assert r is not None
        assert abs(r[0] - (a @ q + b)) < 1e-12
        np.testing.assert_allclose(r[1], a, atol=1e-9)


def test_interpolates_voxel_values_and_quadratic_error():
    rng = np.random.default_rng(1)
    O, m = _map(KEYS, lambda v: rng.standard_normal(v.shape[:-1]))
    psi, _, _, _ = O.voxels(KEYS)
    for i, j in zip(rng.integers(0, len(KEYS), 200), rng.integers(0, 512, 200)):
        q = m[i, j] * VS
        r = O.trilinear(q + 1e-13)
        if r is not None:
            assert abs(r[0] - psi[i, j]) < 1e-9
    c = np.array([3.0, -2.0, 5.0])
    O2, _ = _map(KEYS, lambda v: (c * v * v).sum(-1))
    for q in _inside_points(rng, 300):
        f = q / VS - np.floor(q / VS)
        r = O2.trilinear(q)
        want = (c * q * q).sum() + (c * VS * VS * f * (1 - f)).sum()
        assert abs(r[0] - want) < 1e-11


def test_needs_all_eight_voxels():
    rng = np.random.default_rng(2)
    W = (rng.random((len(KEYS), 512)) > 0.05).astype(np.float64)
    O, m = _map(KEYS, lambda v: v[..., 0], W=W)
    seen = {tuple(x) for x in m[W > 0]}
    n_none = 0
    for q in _inside_points(rng, 800):
        b = np.floor(q / VS).astype(int)
        want = all(tuple(b + np.array([i, j, k])) in seen for i in (0, 1) for j in (0, 1) for k in (0, 1))
        got = O.trilinear(q) is not None
        assert got == want
        n_none += not want
    assert 50 < n_none < 700


def test_gradient_is_the_derivative_of_the_interpolant():
    rng = np.random.default_rng(3)
    O, _ = _map(KEYS, lambda v: rng.standard_normal(v.shape[:-1]) * 0.01)
    h = 1e-6 * VS
    for q in _inside_points(rng, 200):
        f = q / VS - np.floor(q / VS)
        if np.any(f < 0.01) or np.any(f > 0.99):
            continue
        _, g = O.trilinear(q)
        num = [(O.trilinear(q + h * e)[0] - O.trilinear(q - h * e)[0]) / (2 * h) for e in np.eye(3)]
        np.testing.assert_allclose(num, g, rtol=1e-5, atol=1e-6)


def test_gauss_newton_with_trilinear_model_zeroes_plane_residuals():
    cam = scenes.SMALL_CAM
    n = np.array([0.2, -0.1, 1.0])
    n /= np.linalg.norm(n)
    h = 2.0
    vs = 0.05
    keys = np.array([[bx, by, bz] for bx in range(-5, 5) for by in range(-4, 4) for bz in range(3, 8)], np.int32)
    O, _ = _map(keys, lambda v: v @ n - h, vs=vs)      # psi > 0 behind the plane
    T1 = synth.perturb_pose(scenes.IDENTITY, 7, 1.5, 0.03)
    n_cam = T1[:, :3].T @ n
    h_cam = h - n @ T1[:, 3]
    depth = scenes.depth_image(scenes.plane_depth(cam, n_cam, h_cam), cam)
    Tn, stats, failed = O.track(depth, cam, scenes.IDENTITY, 1, [15], 0.01, model="trilinear")
    assert failed == 0
    assert stats[0, 1] > 0.9 * (depth > 0).sum()
    # down to the binary32 rounding of the depths (about 1e-7 m per pixel)
    assert stats[-1, 0] < 1e-9 and stats[-1, 0] < 1e-6 * stats[0, 0]
    # the estimate sees the same plane (the in-plane motion is unobservable)
    np.testing.assert_allclose(Tn[:, :3].T @ n, n_cam, atol=1e-6)
    assert abs((h - n @ Tn[:, 3]) - h_cam) < 1e-6


def test_map_without_gradients_fuses_the_same_distances():
    """Fusion without gradients applies Eq. (1)-(2) alone: the distances
    and weights are bit-identical to fusion with gradients (Eq. (3) feeds
    neither) and the gradients stay zero.  The tri-linear model reads only
    distances and weights, so tracking on either map ends at the same pose
    bit for bit: the gradient-free map with the tri-linear tracker is the
    paper's baseline system."""
    cam = scenes.SMALL_CAM
    sc = scenes.box_room_scene()
    T0 = scenes.box_room_pose()
    full = oracle.OracleMap(0.02, 0.1)
    plain = oracle.OracleMap(0.02, 0.1)
    for k in range(3):
        Tk = synth.perturb_pose(T0, 200 + k, 1.0, 0.01)
        d = scenes.depth_image(synth.render_depth(sc, cam, Tk), cam)
        for M, grad in ((full, True), (plain, False)):
            M.allocate(d, cam, Tk)
            n = M.integrate(d, cam, Tk, gradients=grad)
            assert n > 1000
    np.testing.assert_array_equal(full.keys(), plain.keys())
    pf, gf, Wf, _ = full.voxels()
    pp, gp, Wp, _ = plain.voxels()
    assert np.array_equal(pf, pp) and np.array_equal(Wf, Wp)
    assert not gp.any() and gf[Wf > 0].any()
    T1 = synth.perturb_pose(T0, 31, 1.0, 0.01)
    d1 = scenes.depth_image(synth.render_depth(sc, cam, T1), cam)
    Ta, sa, _ = full.track(d1, cam, T0, 1, [8], 0.01, model="trilinear")
    Tb, sb, _ = plain.track(d1, cam, T0, 1, [8], 0.01, model="trilinear")
    assert np.array_equal(Ta, Tb) and np.array_equal(sa, sb)
    # and the tri-linear tracker on it moves towards the truth
    assert np.linalg.norm(Tb[:, 3] - T1[:, 3]) < 0.5 * np.linalg.norm(T0[:, 3] - T1[:, 3])
