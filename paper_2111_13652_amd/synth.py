"""Seeded synthetic depth streams that stand in for the paper's Kinect data.

This module holds no arithmetic of the Gradient-SDF method.  It only makes
inputs: analytic scenes (spheres, yawed boxes, the inside of a room), exact
z-depth images ray-cast from them, the axial depth-noise model, and smooth
camera trajectories.  Both the HIP path and the FP64 oracle are fed from
here; neither depends on the other.

Conventions
-----------
* Camera frame: x right, y down, z forward (pinhole).  A pixel (u, v) has its
  centre at integer coordinates and the ray ``[(u-cx)/fx, (v-cy)/fy, 1]``.
* Depth images are float32 z-depth in metres, 0 where invalid (no hit, or out
  of the configured depth range).
* Poses are camera-to-world ``T_wc = (R, t)`` stored as 3x4 float64 row-major:
  a camera-frame point x maps to ``R x + t`` (Eq. (5) of the paper applies
  ``R p + t`` to camera points).
* Signed distance: positive inside objects / behind the visible surface,
  negative in free space (Sec. 3.1).  The analytic gradient therefore points
  into the object, away from the camera.

Random numbers come from ``numpy.random.Generator(PCG64(seed))``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

__all__ = [
    "Camera", "Scene", "sphere_scene", "room_scene", "render_depth",
    "depth_noise_sigma", "add_depth_noise", "smooth_trajectory",
    "look_at", "perturb_pose", "rotation_about", "Stream", "make_stream",
    "render_ids", "Albedo", "make_albedo", "surface_normal", "shade", "render_rgbd", "make_rgbd_stream",
    "CONFIG_SPHERE", "CONFIG_ROOM", "CONFIG_ROOM_HD", "spheres_scene", "orbit_views",
    "make_spheres_stream", "CONFIG_SPHERES",
]


# --------------------------------------------------------------------------
# Camera
# --------------------------------------------------------------------------
@dataclasses.dataclass(frozen=True)
class Camera:
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int
    zmin: float = 0.0
    zmax: float = float("inf")

    def rays(self) -> np.ndarray:
        """(H, W, 3) float64 camera-frame rays with unit z component."""
        u = np.arange(self.width, dtype=np.float64)
        v = np.arange(self.height, dtype=np.float64)
        uu, vv = np.meshgrid(u, v)
        d = np.empty((self.height, self.width, 3), np.float64)
        d[..., 0] = (uu - self.cx) / self.fx
        d[..., 1] = (vv - self.cy) / self.fy
        d[..., 2] = 1.0
        return d


# --------------------------------------------------------------------------
# Scenes
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Scene:
    """A union of solid primitives, optionally enclosed by a room AABB.

    ``spheres``: (Ns, 4) rows ``cx, cy, cz, r``.
    ``boxes``:   (Nb, 7) rows ``cx, cy, cz, hx, hy, hz, yaw`` (yaw about +z).
    ``room``:    (2, 3) ``[lo, hi]`` or None.  The room is seen from inside:
                 its walls are solid beyond the box.
    """
    spheres: np.ndarray
    boxes: np.ndarray
    room: Optional[np.ndarray] = None

    # ---- signed distance of the analytic scene (positive inside solids) ----
    def sdf(self, p: np.ndarray) -> np.ndarray:
        """Exact signed distance of points ``p`` (..., 3): >0 inside solid."""
        p = np.asarray(p, np.float64)
        best = np.full(p.shape[:-1], -np.inf)
        for s in self.spheres:
            best = np.maximum(best, s[3] - np.linalg.norm(p - s[:3], axis=-1))
        for b in self.boxes:
            best = np.maximum(best, -_box_sdf_outside(p, b))
        if self.room is not None:
            lo, hi = self.room
            # inside the room the wall is at distance min(p-lo, hi-p)
            dwall = np.minimum(p - lo, hi - p)
            inside = np.all(dwall > 0, axis=-1)
            d_in = -np.min(dwall, axis=-1)  # negative: free space
            d_out = np.linalg.norm(np.maximum(-dwall, 0.0), axis=-1)
            best = np.maximum(best, np.where(inside, d_in, d_out))
        return best


def _box_sdf_outside(p: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Standard signed distance to a yawed box, negative inside."""
    c, h, yaw = b[:3], b[3:6], b[6]
    cs, sn = math.cos(yaw), math.sin(yaw)
    d = p - c
    # rotate world offset into the box frame (rotation by -yaw about z)
    x = cs * d[..., 0] + sn * d[..., 1]
    y = -sn * d[..., 0] + cs * d[..., 1]
    q = np.stack([np.abs(x), np.abs(y), np.abs(d[..., 2])], -1) - h
    outside = np.linalg.norm(np.maximum(q, 0.0), axis=-1)
    inside = np.minimum(np.max(q, axis=-1), 0.0)
    return outside + inside


def sphere_scene(center=(0.0, 0.0, 1.5), radius=0.5) -> Scene:
    return Scene(spheres=np.array([[*center, radius]], np.float64),
                 boxes=np.zeros((0, 7)), room=None)


def room_scene(seed: int, cam_centres: np.ndarray, n_objects: int = 20,
               room=((0.0, 0.0, 0.0), (4.0, 4.0, 3.0)),
               size_range=(0.1, 0.5), clearance: float = 0.5) -> Scene:
    """A room with ``n_objects`` random spheres and yawed boxes.

    Half of the primitives are spheres, half boxes; radius / half-size is
    uniform in ``size_range``; boxes get a random yaw.  Centres are uniform in
    the room and kept so that every surface is at least ``clearance`` metres
    from every camera centre.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    lo, hi = np.asarray(room[0], float), np.asarray(room[1], float)
    spheres, boxes = [], []
    cam_centres = np.asarray(cam_centres, np.float64).reshape(-1, 3)
    kinds = [0, 1] * (n_objects // 2) + [0] * (n_objects % 2)
    for kind in kinds:
        for _ in range(10000):
            c = rng.uniform(lo, hi)
            if kind == 0:
                r = rng.uniform(*size_range)
                bound = r
                cand = np.array([*c, r])
            else:
                h = rng.uniform(size_range[0], size_range[1], size=3)
                yaw = rng.uniform(0.0, math.pi)
                bound = float(np.linalg.norm(h))
                cand = np.array([*c, *h, yaw])
            dmin = np.min(np.linalg.norm(cam_centres - c, axis=1))
            if dmin >= bound + clearance:
                (spheres if kind == 0 else boxes).append(cand)
                break
        else:  # pragma: no cover - generator parameters make this unreachable
            raise RuntimeError("could not place a primitive")
    return Scene(spheres=np.array(spheres, np.float64).reshape(-1, 4),
                 boxes=np.array(boxes, np.float64).reshape(-1, 7),
                 room=np.stack([lo, hi]))


# --------------------------------------------------------------------------
# Ray casting (exact)
# --------------------------------------------------------------------------
def spheres_scene(seed: int, n: int = 5, radius_range=(0.12, 0.35), half_extent: float = 0.8,
                  min_gap: float = 0.25) -> Scene:
    """``n`` spheres of random radii around the origin, no room: centres
    uniform in the cube of half-size ``half_extent``, radii uniform in
    ``radius_range``, every pair at least ``min_gap`` apart surface to
    surface (so each voxel's nearest surface is unambiguous within the
    truncation band)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out: List[np.ndarray] = []
    while len(out) < n:
        c = rng.uniform(-half_extent, half_extent, size=3)
        r = rng.uniform(*radius_range)
        if all(np.linalg.norm(c - o[:3]) >= r + o[3] + min_gap for o in out):
            out.append(np.array([*c, r]))
    return Scene(spheres=np.array(out, np.float64), boxes=np.zeros((0, 7)), room=None)


def orbit_views(seed: int, n_frames: int, distance=(1.8, 2.6), elevation_deg=(-40.0, 60.0),
                jitter: float = 0.1) -> np.ndarray:
    """Random viewpoints around the origin, each looking at the origin
    (plus a small random offset): (n_frames, 3, 4) camera-to-world poses.
    Azimuth uniform, elevation uniform in ``elevation_deg``, distance
    uniform in ``distance``."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(n_frames):
        az = rng.uniform(0.0, 2 * math.pi)
        el = math.radians(rng.uniform(*elevation_deg))
        d = rng.uniform(*distance)
        c = d * np.array([math.cos(el) * math.cos(az), math.cos(el) * math.sin(az), math.sin(el)])
        out.append(look_at(c, rng.uniform(-jitter, jitter, size=3)))
    return np.stack(out)


def _ray_sphere(o, d, s):
    """Nearest positive hit of rays ``o + t d`` (d: (N, 3)) with a sphere."""
    oc = o - s[:3]
    a = np.einsum("ij,ij->i", d, d)
    b = 2.0 * (d @ oc)
    c = float(oc @ oc) - s[3] ** 2
    disc = b * b - 4.0 * a * c
    hit = disc >= 0.0
    sq = np.sqrt(np.where(hit, disc, 0.0))
    t = (-b - sq) / (2.0 * a)
    return np.where(hit & (t > 0.0), t, np.inf)


def _ray_box(o, d, b):
    """Nearest positive hit with a box yawed about +z (slab method)."""
    c, h, yaw = b[:3], b[3:6], b[6]
    cs, sn = math.cos(yaw), math.sin(yaw)
    rot = np.array([[cs, sn, 0.0], [-sn, cs, 0.0], [0.0, 0.0, 1.0]])
    ol = rot @ (o - c)
    dl = d @ rot.T
    tn = np.full(len(d), -np.inf)
    tf = np.full(len(d), np.inf)
    with np.errstate(divide="ignore", invalid="ignore"):
        for k in range(3):
            inv = 1.0 / dl[:, k]
            t1 = (-h[k] - ol[k]) * inv
            t2 = (h[k] - ol[k]) * inv
            lo_k = np.minimum(t1, t2)
            hi_k = np.maximum(t1, t2)
            # a ray parallel to the slab: inside the slab -> no constraint
            par = dl[:, k] == 0.0
            inside = abs(ol[k]) <= h[k]
            lo_k = np.where(par, np.where(inside, -np.inf, np.inf), lo_k)
            hi_k = np.where(par, np.where(inside, np.inf, -np.inf), hi_k)
            tn = np.maximum(tn, lo_k)
            tf = np.minimum(tf, hi_k)
    hit = (tn <= tf) & (tn > 0.0)
    return np.where(hit, tn, np.inf)


def _ray_room_exit(o, d, room):
    lo, hi = room
    with np.errstate(divide="ignore", invalid="ignore"):
        tb = np.where(d > 0, (hi - o) / d, np.where(d < 0, (lo - o) / d, np.inf))
    return np.min(tb, axis=1)


def _screen_rect(cam: Camera, R, t, centre, radius):
    """Conservative pixel rectangle covering a bounding sphere, or None when
    it is behind the camera; the full image when it straddles the camera
    plane."""
    cc = R.T @ (np.asarray(centre) - t)
    if cc[2] + radius <= 0.0:
        return None
    if cc[2] - radius <= 1e-3:
        return 0, cam.width, 0, cam.height
    corners = cc[None, :] + radius * np.array(
        [[sx, sy, sz] for sx in (-1, 1) for sy in (-1, 1) for sz in (-1, 1)], float)
    u = cam.fx * corners[:, 0] / corners[:, 2] + cam.cx
    v = cam.fy * corners[:, 1] / corners[:, 2] + cam.cy
    u0 = max(0, int(math.floor(u.min())) - 1)
    u1 = min(cam.width, int(math.ceil(u.max())) + 2)
    v0 = max(0, int(math.floor(v.min())) - 1)
    v1 = min(cam.height, int(math.ceil(v.max())) + 2)
    if u0 >= u1 or v0 >= v1:
        return None
    return u0, u1, v0, v1


def render_ids(scene: Scene, cam: Camera, T_wc: np.ndarray):
    """Exact noiseless z-depth (float64, inf where nothing is hit) and the
    index of the surface hit: 0 the room, 1 + i sphere i, 1 + Ns + j box j,
    -1 nothing."""
    T = np.asarray(T_wc, np.float64).reshape(3, 4)
    R, t = T[:, :3], T[:, 3]
    rays = cam.rays()
    dirs = rays @ R.T  # world directions; the camera ray has z = 1
    best = np.full(dirs.shape[:-1], np.inf)
    obj = np.full(dirs.shape[:-1], -1, np.int32)
    if scene.room is not None:
        best = _ray_room_exit(t, dirs.reshape(-1, 3), scene.room).reshape(best.shape)
        obj[np.isfinite(best)] = 0
    prims = [(s, _ray_sphere, s[:3], s[3]) for s in scene.spheres]
    prims += [(b, _ray_box, b[:3], float(np.linalg.norm(b[3:6]))) for b in scene.boxes]
    for idx, (p, fn, c, r) in enumerate(prims):
        rect = _screen_rect(cam, R, t, c, r)
        if rect is None:
            continue
        u0, u1, v0, v1 = rect
        sub = dirs[v0:v1, u0:u1].reshape(-1, 3)
        hit = fn(t, sub, p).reshape(v1 - v0, u1 - u0)
        closer = hit < best[v0:v1, u0:u1]
        best[v0:v1, u0:u1] = np.where(closer, hit, best[v0:v1, u0:u1])
        obj[v0:v1, u0:u1] = np.where(closer, idx + 1, obj[v0:v1, u0:u1])
    return best, obj  # ray parameter == z-depth because the camera ray has z = 1


def render_depth(scene: Scene, cam: Camera, T_wc: np.ndarray) -> np.ndarray:
    """Exact noiseless z-depth (float64, inf where nothing is hit)."""
    return render_ids(scene, cam, T_wc)[0]


# --------------------------------------------------------------------------
# Colour: per-object smooth albedo fields with Lambertian shading
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Albedo:
    """Per-object albedo a_c(p) = base_c + amp * mean_m sin(k_m . p + phase_mc),
    clipped to [0, 1]; objects indexed as by ``render_ids``."""
    base: np.ndarray     # (n_obj, 3)
    amp: np.ndarray      # (n_obj,)
    k: np.ndarray        # (n_obj, 3 terms, 3) wave vectors, rad/m
    phase: np.ndarray    # (n_obj, 3 terms, 3 channels)
    light: np.ndarray    # (3,) unit direction towards the light
    ambient: float = 0.3


def make_albedo(scene: Scene, seed: int, k_range=(10.0, 40.0)) -> Albedo:
    rng = np.random.Generator(np.random.PCG64(seed))
    n = 1 + len(scene.spheres) + len(scene.boxes)
    dirs = rng.standard_normal((n, 3, 3))
    dirs /= np.linalg.norm(dirs, axis=-1, keepdims=True)
    k = dirs * rng.uniform(*k_range, size=(n, 3, 1))
    light = np.array([0.3, -0.5, 0.8])
    return Albedo(base=rng.uniform(0.3, 0.7, (n, 3)), amp=rng.uniform(0.1, 0.3, n), k=k,
                  phase=rng.uniform(0.0, 2 * math.pi, (n, 3, 3)), light=light / np.linalg.norm(light))


def surface_normal(scene: Scene, p: np.ndarray, obj: np.ndarray) -> np.ndarray:
    """Unit normal pointing into free space at surface points ``p`` (N, 3)
    of objects ``obj`` (N,) (0 = room wall, as ``render_ids``)."""
    n = np.zeros_like(p)
    ns = len(scene.spheres)
    room = obj == 0
    if room.any() and scene.room is not None:
        lo, hi = scene.room
        q = p[room]
        d = np.concatenate([q - lo, hi - q], axis=1)          # distances to the 6 walls
        w = np.argmin(np.abs(d), axis=1)
        nr = np.zeros_like(q)
        nr[np.arange(len(q)), w % 3] = np.where(w < 3, 1.0, -1.0)   # into the room
        n[room] = nr
    for i, sph in enumerate(scene.spheres):
        m = obj == 1 + i
        if m.any():
            d = p[m] - sph[:3]
            n[m] = d / np.linalg.norm(d, axis=1, keepdims=True)
    for j, b in enumerate(scene.boxes):
        m = obj == 1 + ns + j
        if m.any():
            c, h, yaw = b[:3], b[3:6], b[6]
            cs, sn = math.cos(yaw), math.sin(yaw)
            d = p[m] - c
            loc = np.stack([cs * d[:, 0] + sn * d[:, 1], -sn * d[:, 0] + cs * d[:, 1], d[:, 2]], 1)
            face = np.argmax(np.abs(loc) - h, axis=1)
            nl = np.zeros_like(loc)
            nl[np.arange(len(loc)), face] = np.sign(loc[np.arange(len(loc)), face])
            n[m] = np.stack([cs * nl[:, 0] - sn * nl[:, 1], sn * nl[:, 0] + cs * nl[:, 1], nl[:, 2]], 1)
    return n


def shade(alb: Albedo, scene: Scene, p: np.ndarray, obj: np.ndarray) -> np.ndarray:
    """Lambertian colour (N, 3) of surface points ``p`` on objects ``obj``."""
    k = alb.k[obj]                                             # (N, 3, 3)
    arg = np.einsum("nmd,nd->nm", k, p)[:, :, None] + alb.phase[obj]
    a = alb.base[obj] + alb.amp[obj, None] * np.mean(np.sin(arg), axis=1)
    n = surface_normal(scene, p, obj)
    lam = alb.ambient + (1.0 - alb.ambient) * np.maximum(0.0, n @ alb.light)
    return np.clip(a, 0.0, 1.0) * lam[:, None]


def render_rgbd(scene: Scene, cam: Camera, T_wc: np.ndarray, alb: Albedo):
    """Exact z-depth (float64, inf = no hit) and noiseless colour (H, W, 3)
    float32 in [0, 1] (0 where nothing is hit)."""
    z, obj = render_ids(scene, cam, T_wc)
    T = np.asarray(T_wc, np.float64).reshape(3, 4)
    hit = np.isfinite(z)
    rgb = np.zeros(z.shape + (3,), np.float64)
    if hit.any():
        x = cam.rays()[hit] * z[hit][:, None]                  # camera frame
        p = x @ T[:, :3].T + T[:, 3]
        rgb[hit] = shade(alb, scene, p, obj[hit])
    return z, rgb.astype(np.float32)


def depth_noise_sigma(z: np.ndarray) -> np.ndarray:
    """Axial noise model sigma(z) = 0.0012 + 0.0019 (z - 0.4)^2 metres."""
    return 0.0012 + 0.0019 * (z - 0.4) ** 2


def add_depth_noise(z: np.ndarray, rng: np.random.Generator) -> np.ndarray:
    z = np.asarray(z, np.float64)
    finite = np.isfinite(z)
    out = z.copy()
    out[finite] = z[finite] + rng.standard_normal(int(finite.sum())) * depth_noise_sigma(z[finite])
    return out


def to_depth_image(z: np.ndarray, cam: Camera) -> np.ndarray:
    """float32 depth with 0 outside ``[zmin, zmax]`` (or non-finite)."""
    z32 = np.where(np.isfinite(z), z, 0.0).astype(np.float32)
    ok = (z32 >= np.float32(cam.zmin)) & (z32 <= np.float32(cam.zmax))
    return np.where(ok, z32, np.float32(0.0)).astype(np.float32)


# --------------------------------------------------------------------------
# Poses and trajectories
# --------------------------------------------------------------------------
def rotation_about(axis: Sequence[float], angle: float) -> np.ndarray:
    """Rodrigues rotation (used only to build poses for the generator)."""
    a = np.asarray(axis, np.float64)
    a = a / np.linalg.norm(a)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + math.sin(angle) * K + (1 - math.cos(angle)) * K @ K


def look_at(centre, target, up=(0.0, 0.0, 1.0)) -> np.ndarray:
    """3x4 camera-to-world pose looking from ``centre`` at ``target``."""
    c = np.asarray(centre, np.float64)
    f = np.asarray(target, np.float64) - c
    f /= np.linalg.norm(f)
    x = np.cross(f, np.asarray(up, np.float64))
    x /= np.linalg.norm(x)
    y = np.cross(f, x)
    R = np.stack([x, y, f], axis=1)
    return np.concatenate([R, c[:, None]], axis=1)


def perturb_pose(T_wc: np.ndarray, seed: int, angle_deg: float, trans_m: float) -> np.ndarray:
    """Left-compose a rotation of exactly ``angle_deg`` about a random axis
    (about the camera centre) and a translation of exactly ``trans_m`` in a
    random direction.  Returns the new 3x4 pose."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ax = rng.standard_normal(3)
    dr = rng.standard_normal(3)
    dr /= np.linalg.norm(dr)
    T = np.asarray(T_wc, np.float64).reshape(3, 4)
    Rp = rotation_about(ax, math.radians(angle_deg))
    return np.concatenate([Rp @ T[:, :3], (T[:, 3] + trans_m * dr)[:, None]], axis=1)


def _rot_angle(Ra: np.ndarray, Rb: np.ndarray) -> float:
    c = (np.trace(Ra.T @ Rb) - 1.0) / 2.0
    return math.acos(max(-1.0, min(1.0, c)))


def smooth_trajectory(seed: int, n_frames: int, max_step_m: float = 0.02,
                      max_step_deg: float = 1.0,
                      centre_lo=(1.3, 1.3, 1.1), centre_hi=(2.7, 2.7, 1.9),
                      target_lo=(0.6, 0.6, 0.6), target_hi=(3.4, 3.4, 1.6)) -> np.ndarray:
    """Smooth random camera path: (n_frames, 3, 4) camera-to-world poses.

    Each axis of the camera centre and of the look-at target is a sum of
    three sinusoids with random frequencies and phases; the time step is
    chosen so that no frame-to-frame step exceeds ``max_step_m`` or
    ``max_step_deg``.
    """
    rng = np.random.Generator(np.random.PCG64(seed))

    def curve(lo, hi, slow):
        lo, hi = np.asarray(lo), np.asarray(hi)
        fr = rng.uniform(0.3, 1.0, size=(3, 3)) * (0.35 if slow else 1.0)
        ph = rng.uniform(0, 2 * math.pi, size=(3, 3))
        am = rng.uniform(0.5, 1.0, size=(3, 3))
        am /= am.sum(axis=1, keepdims=True)

        def f(s):
            s = np.atleast_1d(s)[:, None, None]
            w = (np.sin(fr[None] * s + ph[None]) * am[None]).sum(-1)  # in [-1,1]
            return (lo + hi) / 2 + (hi - lo) / 2 * w
        return f

    cpos = curve(centre_lo, centre_hi, slow=False)
    tpos = curve(target_lo, target_hi, slow=True)

    def poses(s):
        cs, ts = cpos(s), tpos(s)
        return np.stack([look_at(c, t) for c, t in zip(cs, ts)])

    # advance the curve parameter frame by frame; each step is the largest
    # one that keeps both the translation and the rotation within bounds
    out = [poses(0.0)[0]]
    s, h = 0.0, 1e-2
    for _ in range(n_frames - 1):
        prev = out[-1]
        while True:
            cand = poses(s + h)[0]
            dt = np.linalg.norm(cand[:, 3] - prev[:, 3]) / max_step_m
            dr = _rot_angle(prev[:, :3], cand[:, :3]) / math.radians(max_step_deg)
            worst = max(dt, dr)
            if worst <= 1.0:
                break
            h *= 0.9 / worst
        s += h
        out.append(cand)
        # aim the next step at 90% of the tighter bound
        h *= 0.9 / max(worst, 1e-3)
    return np.stack(out)


# --------------------------------------------------------------------------
# Streams
# --------------------------------------------------------------------------
CONFIG_SPHERE = dict(cam=Camera(131.0, 131.0, 79.5, 59.5, 160, 120, 0.0, float("inf")),
                     voxel_size=0.02, truncation=0.10)
# ``seeds``: (scene, trajectory, noise) of each stream.  The 1280x720
# stream uses trajectory 7: the trajectories of seeds 5 and 6 pass, after
# about 240 frames, through views of a single wall or the floor, where a
# plane leaves three degrees of freedom of the pose unobserved and every
# tracker slides; 7 is the first seed from 5 on whose 500 frames all keep
# the point-to-plane information of the view well conditioned (the check
# is tests/test_synth.py::test_hd_trajectory_keeps_the_pose_observable).
CONFIG_ROOM = dict(cam=Camera(525.0, 525.0, 319.5, 239.5, 640, 480, 0.4, 4.0),
                   voxel_size=0.01, truncation=0.05, seeds=(1, 2, 3))
CONFIG_ROOM_HD = dict(cam=Camera(920.0, 920.0, 639.5, 359.5, 1280, 720, 0.4, 4.0),
                      voxel_size=0.005, truncation=0.025, seeds=(1, 7, 6))

# Gradient-quality experiment: 1 cm voxels, truncation 10 voxels.
CONFIG_SPHERES = dict(cam=Camera(525.0, 525.0, 319.5, 239.5, 640, 480, 0.4, 4.0),
                      voxel_size=0.01, truncation=0.10)


@dataclasses.dataclass
class Stream:
    cam: Camera
    depth: np.ndarray      # (F, H, W) float32, 0 = invalid
    poses: np.ndarray      # (F, 3, 4) float64 ground-truth camera-to-world
    scene: Scene
    rgb: Optional[np.ndarray] = None      # (F, H, W, 3) float32 colour, when rendered
    albedo: Optional[Albedo] = None


def make_stream(cam: Camera, n_frames: int, scene_seed: int = 1, traj_seed: int = 2,
                noise_seed: Optional[int] = 3, n_objects: int = 20,
                frames: Optional[Sequence[int]] = None) -> Stream:
    """The seeded synthetic room stream (scene, trajectory, per-frame noise).

    Per-frame noise uses one child of ``SeedSequence(noise_seed)`` per frame,
    so any frame can be regenerated on its own: ``frames`` renders only
    those frames of the ``n_frames``-frame stream (the scene keeps its
    objects away from every camera centre of the whole trajectory, so it
    depends on ``n_frames``); ``depth`` then holds them in that order and
    ``poses`` is still the whole trajectory.
    """
    poses = smooth_trajectory(traj_seed, n_frames)
    scene = room_scene(scene_seed, poses[:, :, 3], n_objects=n_objects)
    kids = np.random.SeedSequence(noise_seed).spawn(n_frames) if noise_seed is not None else None
    which = list(range(n_frames)) if frames is None else [int(f) for f in frames]
    depth = np.empty((len(which), cam.height, cam.width), np.float32)
    for j, i in enumerate(which):
        z = render_depth(scene, cam, poses[i])
        if kids is not None:
            z = add_depth_noise(z, np.random.Generator(np.random.PCG64(kids[i])))
        depth[j] = to_depth_image(z, cam)
    return Stream(cam=cam, depth=depth, poses=poses, scene=scene)


def make_rgbd_stream(cam: Camera, n_frames: int, scene_seed: int = 1, traj_seed: int = 2,
                     noise_seed: Optional[int] = 3, albedo_seed: int = 4, color_noise: float = 0.005,
                     n_objects: int = 20, frames: Optional[Sequence[int]] = None) -> Stream:
    """The room stream with colour: the depth exactly as ``make_stream`` (same
    seeds give the same depth), plus Lambertian colour of seeded per-object
    albedo fields with Gaussian noise ``color_noise`` (second child seed of
    each frame), clipped to [0, 1].  ``frames`` as for ``make_stream``."""
    poses = smooth_trajectory(traj_seed, n_frames)
    scene = room_scene(scene_seed, poses[:, :, 3], n_objects=n_objects)
    alb = make_albedo(scene, albedo_seed)
    kids = np.random.SeedSequence(noise_seed).spawn(n_frames) if noise_seed is not None else None
    which = list(range(n_frames)) if frames is None else [int(f) for f in frames]
    depth = np.empty((len(which), cam.height, cam.width), np.float32)
    rgb = np.empty((len(which), cam.height, cam.width, 3), np.float32)
    for j, i in enumerate(which):
        z, col = render_rgbd(scene, cam, poses[i], alb)
        if kids is not None:
            z = add_depth_noise(z, np.random.Generator(np.random.PCG64(kids[i])))
            g = np.random.Generator(np.random.PCG64(kids[i].spawn(1)[0]))
            col = np.clip(col + g.standard_normal(col.shape).astype(np.float32) * np.float32(color_noise),
                          0.0, 1.0)
        depth[j] = to_depth_image(z, cam)
        rgb[j] = col
    return Stream(cam=cam, depth=depth, poses=poses, scene=scene, rgb=rgb, albedo=alb)


def make_spheres_stream(cam: Camera, n_frames: int, scene_seed: int = 11, view_seed: int = 12,
                        noise_seed: Optional[int] = 13) -> Stream:
    """Five random spheres seen from random viewpoints with axial depth
    noise (the synthetic setup of the gradient-quality experiment)."""
    scene = spheres_scene(scene_seed)
    poses = orbit_views(view_seed, n_frames)
    kids = np.random.SeedSequence(noise_seed).spawn(n_frames) if noise_seed is not None else None
    depth = np.empty((n_frames, cam.height, cam.width), np.float32)
    for i in range(n_frames):
        z = render_depth(scene, cam, poses[i])
        if kids is not None:
            z = add_depth_noise(z, np.random.Generator(np.random.PCG64(kids[i])))
        depth[i] = to_depth_image(z, cam)
    return Stream(cam=cam, depth=depth, poses=poses, scene=scene)
