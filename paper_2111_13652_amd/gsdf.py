"""Python front end of libgsdf: torch owns the device buffers, the library
does every step of the path.  Argument marshalling only.

    m = GsdfMap(voxel_size=0.01, truncation=0.05, max_blocks=40000)
    m.allocate(depth, cam, pose); m.integrate(depth, cam, pose)
    m.track(depth2, cam, pose2, levels=3, iters=(4, 5, 10))   # pose2 updated in place
"""
from __future__ import annotations

import ctypes as C
import math
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib

# "nograd": distance and weight only (no stored gradient), the plain SDF map
# of the paper's runtime comparison; it is tracked with model="trilinear".
STORAGE = {"fp32": _lib.FP32, "bf16": _lib.BF16, "fp16": _lib.FP16, "nograd": _lib.NOGRAD_FP32}
COS_75 = math.cos(math.radians(75.0))


def _stream() -> C.c_void_p:
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def camera(cam) -> _lib.Camera:
    """A ``_lib.Camera`` from any object with fx, fy, cx, cy, width, height,
    zmin, zmax attributes."""
    return _lib.Camera(float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy), int(cam.width),
                       int(cam.height), float(cam.zmin), float(min(cam.zmax, 3.0e38)))


def _need(t: torch.Tensor, dtype, shape=None, name="tensor"):
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise ValueError(f"{name} must be a CUDA tensor")
    if t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous {dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


class GsdfMap:
    """A sparse 8^3-block Gradient-SDF map living in device memory."""

    def __init__(self, voxel_size: float, truncation: float, max_blocks: int,
                 hash_slots: Optional[int] = None, storage: str = "fp32", bounds=None,
                 device: str = "cuda"):
        lib = _lib.load()
        if hash_slots is None:
            hash_slots = 1 << max(4, int(math.ceil(math.log2(4 * max_blocks))))
        d = _lib.MapDesc()
        d.voxel_size = float(voxel_size)
        d.truncation = float(truncation)
        d.storage = STORAGE[storage]
        d.hash_slots = int(hash_slots)
        d.max_blocks = int(max_blocks)
        if bounds is not None:
            d.bounded = 1
            for i in range(3):
                d.bmin[i] = int(bounds[0][i])
                d.bmax[i] = int(bounds[1][i])
        sizes = (C.c_size_t * 4)()
        _lib.check(lib.gsdf_map_buffer_sizes(C.byref(d), C.byref(sizes)), "map_buffer_sizes")
        self.device = torch.device(device)
        self.buffers = [torch.empty(int(s), dtype=torch.uint8, device=self.device) for s in sizes]
        self._map = _lib.Map(self.buffers[0].data_ptr(), self.buffers[1].data_ptr(),
                             self.buffers[2].data_ptr(), self.buffers[3].data_ptr(), d)
        self.voxel_size = float(voxel_size)
        self.truncation = float(truncation)
        self.max_blocks = int(max_blocks)
        self.storage = storage
        self.status = torch.zeros(1, dtype=torch.int32, device=self.device)
        self._scratch = {}
        self._timer = None
        self.reset()

    def __del__(self):
        t = getattr(self, "_timer", None)
        if t is not None and _lib._lib is not None:
            _lib._lib.gsdf_timer_destroy(t)
            self._timer = None

    # ---- per-kernel event timing (a gsdf_timer attached to this map) ----
    def timing(self, mask: int) -> None:
        """Record events around the launches of the kernel ids whose bits are
        set in ``mask`` (0: none) and clear the totals."""
        lib = _lib.load()
        if self._timer is None:
            h = C.c_void_p()
            _lib.check(lib.gsdf_timer_create(int(mask) & 0xffffffff, C.byref(h)), "timer_create")
            self._timer = h
            self._map.timer = h
        else:
            _lib.check(lib.gsdf_timer_select(self._timer, int(mask) & 0xffffffff), "timer_select")

    def timing_read(self, kernel_id: int):
        """(total ms, launches) recorded for one kernel id since the last
        ``timing`` call; synchronises the recorded events."""
        if self._timer is None:
            return 0.0, 0
        tot = C.c_double()
        n = C.c_int64()
        _lib.check(_lib.load().gsdf_timer_read(self._timer, int(kernel_id), C.byref(tot), C.byref(n)),
                   "timer_read")
        return tot.value, n.value

    # ---- buffers ----
    @property
    def weight(self) -> torch.Tensor:
        """Per-voxel accumulated weight W (max_blocks*512 float32, pool order)."""
        return self.buffers[2].view(torch.float32)

    def reset(self) -> None:
        _lib.check(_lib.load().gsdf_map_reset(C.byref(self._map), _stream()), "map_reset")
        self.status.zero_()

    def _scratch_for(self, cam: _lib.Camera, levels: int) -> torch.Tensor:
        key = (cam.width, cam.height, levels)
        if key not in self._scratch:
            n = _lib.load().gsdf_track_scratch_bytes(C.byref(cam), levels)
            if n == 0:
                raise ValueError("invalid camera / levels for tracking")
            self._scratch[key] = torch.empty(int(n), dtype=torch.uint8, device=self.device)
        return self._scratch[key]

    def _fuse_scratch_for(self, cam: _lib.Camera) -> torch.Tensor:
        key = ("fuse", cam.width, cam.height)
        if key not in self._scratch:
            n = _lib.load().gsdf_integrate_scratch_bytes(C.byref(cam))
            if n == 0:
                raise ValueError("invalid camera for fusion")
            self._scratch[key] = torch.empty(int(n), dtype=torch.uint8, device=self.device)
        return self._scratch[key]

    def counters(self) -> np.ndarray:
        """Work counters since the last reset (see gsdf_map_counters)."""
        out = torch.zeros(16, dtype=torch.int64, device=self.device)
        _lib.check(_lib.load().gsdf_map_counters(C.byref(self._map), _ptr(out), _stream()), "counters")
        return out.cpu().numpy().astype(np.uint64)

    # ---- the hot path ----
    def allocate(self, depth: torch.Tensor, cam, pose: torch.Tensor) -> None:
        c = camera(cam)
        _need(depth, torch.float32, (c.height, c.width), "depth")
        _need(pose, torch.float64, (3, 4), "pose")
        _lib.check(_lib.load().gsdf_allocate_blocks(C.byref(self._map), _ptr(depth), C.byref(c),
                                                     _ptr(pose), _ptr(self.status), _stream()),
                   "allocate_blocks")

    def integrate(self, depth: torch.Tensor, cam, pose: torch.Tensor, eps: Optional[float] = None,
                  cos_max_angle: float = COS_75) -> None:
        c = camera(cam)
        _need(depth, torch.float32, (c.height, c.width), "depth")
        _need(pose, torch.float64, (3, 4), "pose")
        p = _lib.FuseParams(float(self.voxel_size if eps is None else eps), float(cos_max_angle))
        scratch = self._fuse_scratch_for(c)
        _lib.check(_lib.load().gsdf_integrate_frame(C.byref(self._map), _ptr(depth), C.byref(c),
                                                     _ptr(pose), C.byref(p), _ptr(scratch),
                                                     scratch.numel(), _ptr(self.status), _stream()),
                   "integrate_frame")

    def fuse(self, depth: torch.Tensor, cam, pose: torch.Tensor, eps: Optional[float] = None,
             cos_max_angle: float = COS_75) -> None:
        """allocate + integrate in two launches (gsdf_fuse_frame); the same
        result as the two calls in sequence."""
        c = camera(cam)
        _need(depth, torch.float32, (c.height, c.width), "depth")
        _need(pose, torch.float64, (3, 4), "pose")
        p = _lib.FuseParams(float(self.voxel_size if eps is None else eps), float(cos_max_angle))
        scratch = self._fuse_scratch_for(c)
        _lib.check(_lib.load().gsdf_fuse_frame(C.byref(self._map), _ptr(depth), C.byref(c), _ptr(pose),
                                                C.byref(p), _ptr(scratch), scratch.numel(), _ptr(self.status),
                                                _stream()), "fuse_frame")

    def track(self, depth: torch.Tensor, cam, pose: torch.Tensor, levels: int = 3,
              iters: Sequence[int] = (4, 5, 10), delta: float = 0.01, damping: float = 1e-6,
              min_inlier_frac: float = 0.1, stats: Optional[torch.Tensor] = None,
              init: Optional[torch.Tensor] = None, model: str = "taylor", max_polls: int = 0,
              clocks: Optional[torch.Tensor] = None, device_scope: bool = False) -> None:
        """Coarse-to-fine tracking; ``pose`` (3x4 float64, device) receives
        the estimate, starting from ``init`` (default: ``pose`` itself, updated
        in place).  ``iters[l]`` iterations at level l (0 = finest).  ``model``:
        "taylor" (one voxel, Eq. (14)-(16)) or "trilinear" (eight voxels,
        Eq. (12)-(13), the comparison model).  ``max_polls`` bounds each
        wait between work-groups (0: the library default).  ``clocks``
        (int64, device, 4 per iteration): per-iteration wall-clock stamps of
        work-group 0 (see wall_clock_khz).  ``device_scope``: every
        per-iteration partial through device-scope memory rather than its
        XCD's L2 (same result bits, slower; for checking the exchange)."""
        c = camera(cam)
        _need(depth, torch.float32, (c.height, c.width), "depth")
        _need(pose, torch.float64, (3, 4), "pose")
        if init is None:
            init = pose
        _need(init, torch.float64, (3, 4), "init")
        it = list(iters) + [0] * (4 - len(iters))
        if stats is not None:
            _need(stats, torch.float32, None, "stats")
            if stats.numel() < 2 * sum(it[:levels]):
                raise ValueError("stats too small")
        if clocks is not None:
            _need(clocks, torch.int64, None, "clocks")
            if clocks.numel() < 4 * sum(it[:levels]):
                raise ValueError("clocks too small")
        p = _lib.TrackParams(int(levels), (C.c_int32 * 4)(*it[:4]), float(delta), float(damping),
                             float(min_inlier_frac), {"taylor": 0, "trilinear": 1}[model], int(max_polls),
                             _ptr(clocks), int(bool(device_scope)))
        scratch = self._scratch_for(c, levels)
        _lib.check(_lib.load().gsdf_track_frame(C.byref(self._map), _ptr(depth), C.byref(c),
                                                 C.byref(p), _ptr(init), _ptr(pose), _ptr(stats), _ptr(scratch),
                                                 scratch.numel(), _ptr(self.status), _stream()),
                   "track_frame")

    def gn_step_keyframes(self, depth: torch.Tensor, cam, poses: torch.Tensor, delta: float = 0.01,
                          damping: float = 1e-6, min_inlier_frac: float = 0.1) -> None:
        """One damped Gauss-Newton step at full resolution for each keyframe
        (``depth`` (K, H, W) float32, ``poses`` (K, 3, 4) float64, updated in
        place): the step of ``track(..., levels=1, iters=(1,))`` for all
        keyframes in two launches (sums in another fixed order, so equal to
        the per-keyframe calls to rounding)."""
        c = camera(cam)
        if depth.dim() != 3:
            raise ValueError("depth must be (K, H, W)")
        K = depth.shape[0]
        _need(depth, torch.float32, (K, c.height, c.width), "depth")
        _need(poses, torch.float64, (K, 3, 4), "poses")
        key = ("gn", c.width, c.height, K)
        if key not in self._scratch:
            n = _lib.load().gsdf_gn_scratch_bytes(C.byref(c), K)
            if n == 0:
                raise ValueError("invalid keyframe count for the Gauss-Newton step")
            self._scratch[key] = torch.empty(int(n), dtype=torch.uint8, device=self.device)
        scratch = self._scratch[key]
        _lib.check(_lib.load().gsdf_gn_step_keyframes(C.byref(self._map), _ptr(depth), K, C.byref(c), _ptr(poses),
                                                      float(delta), float(damping), float(min_inlier_frac),
                                                      _ptr(scratch), scratch.numel(), _ptr(self.status), _stream()),
                   "gn_step_keyframes")

    def normal_equations(self, depth: torch.Tensor, cam, pose: torch.Tensor, delta: float) -> torch.Tensor:
        c = camera(cam)
        _need(depth, torch.float32, (c.height, c.width), "depth")
        _need(pose, torch.float64, (3, 4), "pose")
        out = torch.zeros(29, dtype=torch.float64, device=self.device)
        scratch = self._scratch_for(c, 1)
        _lib.check(_lib.load().gsdf_normal_equations(C.byref(self._map), _ptr(depth), C.byref(c),
                                                      _ptr(pose), float(delta), _ptr(out),
                                                      _ptr(scratch), scratch.numel(), _stream()),
                   "normal_equations")
        return out

    # ---- differentiable form ----
    def export_params(self, n_blocks: Optional[int] = None) -> torch.Tensor:
        """Per-voxel parameters {psi, g} as a (n_blocks, 512, 4) float32 device
        tensor in pool order, voxel index = Morton order (see voxel_order)."""
        n = self.num_blocks() if n_blocks is None else int(n_blocks)
        out = torch.empty((max(n, 0), 512, 4), dtype=torch.float32, device=self.device)
        _lib.check(_lib.load().gsdf_export_params(C.byref(self._map), _ptr(out), n, _stream()),
                   "export_params")
        return out

    def import_params(self, params: torch.Tensor) -> None:
        """Write refined {psi, g} back into the observed voxels (W kept)."""
        _need(params, torch.float32, None, "params")
        if params.dim() != 3 or params.shape[1:] != (512, 4):
            raise ValueError("params must be (n_blocks, 512, 4)")
        _lib.check(_lib.load().gsdf_import_params(C.byref(self._map), _ptr(params), int(params.shape[0]),
                                                   _stream()), "import_params")

    def _keyframe_scratch(self, c: _lib.Camera, K: int) -> torch.Tensor:
        key = ("kf", c.width, c.height, K)
        if key not in self._scratch:
            n = _lib.load().gsdf_keyframe_scratch_bytes(C.byref(c), int(K), self.max_blocks)
            if n == 0:
                raise ValueError("invalid camera / keyframe count")
            self._scratch[key] = torch.empty(int(n), dtype=torch.uint8, device=self.device)
        return self._scratch[key]

    # ---- surface extraction ----
    def surfels(self, level: int = 0):
        """Oriented point cloud of Sec. 4.3 (level 1: 2x2x2 upsampled):
        (points (n,3), normals (n,3)) float32 and ids (n,4) int32 (voxel
        coordinates, subvoxel), device tensors."""
        lib = _lib.load()
        n_scr = lib.gsdf_surfel_scratch_bytes(C.byref(self._map))
        scratch = torch.empty(int(n_scr), dtype=torch.uint8, device=self.device)
        count = torch.zeros(1, dtype=torch.int64, device=self.device)
        _lib.check(lib.gsdf_extract_surfels(C.byref(self._map), int(level), None, None, None, 0, _ptr(count),
                                            _ptr(scratch), scratch.numel(), _stream()), "extract_surfels")
        n = int(count.item())
        pts = torch.empty((max(n, 1), 3), dtype=torch.float32, device=self.device)
        nrm = torch.empty((max(n, 1), 3), dtype=torch.float32, device=self.device)
        ids = torch.empty((max(n, 1), 4), dtype=torch.int32, device=self.device)
        if n:
            _lib.check(lib.gsdf_extract_surfels(C.byref(self._map), int(level), _ptr(pts), _ptr(nrm), _ptr(ids), n,
                                                _ptr(count), _ptr(scratch), scratch.numel(), _stream()),
                       "extract_surfels")
        return pts[:n], nrm[:n], ids[:n]

    def gradient_quality(self, spheres) -> "torch.Tensor":
        """Angles of the stored gradients and of forward / backward / central
        differences against a union of spheres (Sec. 5.2): (5, n_blocks, 512)
        float32 on the device, planes distance to the nearest surface, then
        angles in degrees (stored, forward, backward, central); NaN where
        undefined.  Voxel order lx + 8 ly + 64 lz."""
        sp = torch.as_tensor(np.ascontiguousarray(spheres, np.float64).reshape(-1, 4), device=self.device)
        n = self.num_blocks()
        out = torch.empty((5, max(n, 1), 512), dtype=torch.float32, device=self.device)
        _lib.check(_lib.load().gsdf_gradient_quality(C.byref(self._map), _ptr(sp), sp.shape[0], _ptr(out),
                                                     n * 512, _stream()), "gradient_quality")
        return out[:, :n]

    # ---- inspection ----
    def num_blocks(self) -> int:
        n = torch.zeros(1, dtype=torch.int32, device=self.device)
        _lib.check(_lib.load().gsdf_map_num_blocks(C.byref(self._map), _ptr(n), _stream()), "num_blocks")
        return int(n.item())

    def keys(self) -> np.ndarray:
        """Block keys (n, 3) int32 in pool order."""
        out = torch.zeros((self.max_blocks, 3), dtype=torch.int32, device=self.device)
        n = torch.zeros(1, dtype=torch.int32, device=self.device)
        _lib.check(_lib.load().gsdf_export_keys(C.byref(self._map), _ptr(out), _ptr(n), _stream()),
                   "export_keys")
        return out[: int(n.item())].cpu().numpy()

    def voxels(self, n_blocks: Optional[int] = None):
        """(psi, g, W) as numpy arrays (n, 512), (n, 512, 3), (n, 512) in pool
        order; voxel order lx + 8 ly + 64 lz."""
        n = self.num_blocks() if n_blocks is None else int(n_blocks)
        psi = torch.zeros((max(n, 1), 512), dtype=torch.float32, device=self.device)
        g = torch.zeros((max(n, 1), 512, 3), dtype=torch.float32, device=self.device)
        w = torch.zeros((max(n, 1), 512), dtype=torch.float32, device=self.device)
        _lib.check(_lib.load().gsdf_export_voxels(C.byref(self._map), n, _ptr(psi), _ptr(g), _ptr(w),
                                                   _stream()), "export_voxels")
        return psi[:n].cpu().numpy(), g[:n].cpu().numpy(), w[:n].cpu().numpy()

    def import_blocks(self, keys, psi, g, W) -> None:
        k = torch.as_tensor(np.ascontiguousarray(keys, np.int32), device=self.device)
        p = torch.as_tensor(np.ascontiguousarray(psi, np.float32), device=self.device)
        gg = torch.as_tensor(np.ascontiguousarray(g, np.float32), device=self.device)
        w = torch.as_tensor(np.ascontiguousarray(W, np.float32), device=self.device)
        _lib.check(_lib.load().gsdf_import_blocks(C.byref(self._map), _ptr(k), int(len(k)), _ptr(p),
                                                   _ptr(gg), _ptr(w), _ptr(self.status), _stream()),
                   "import_blocks")

    def status_flags(self):
        return _lib.status_bits(int(self.status.item()))


def voxel_order() -> np.ndarray:
    """order[lx + 8 ly + 64 lz] = index of that voxel inside a block of the
    map's (and the params') layout."""
    out = np.zeros(512, np.int32)
    _lib.check(_lib.load().gsdf_voxel_order(out.ctypes.data_as(C.c_void_p)), "voxel_order")
    return out


def _kf_args(gmap: GsdfMap, depth, cam, T0, xi, params, assoc):
    c = camera(cam)
    if depth.dim() != 3:
        raise ValueError("depth must be (K, H, W)")
    K = depth.shape[0]
    _need(depth, torch.float32, (K, c.height, c.width), "depth")
    _need(T0, torch.float64, (K, 3, 4), "T0")
    _need(xi, torch.float64, (K, 6), "xi")
    _need(params, torch.float32, None, "params")
    if params.dim() != 3 or params.shape[1:] != (512, 4):
        raise ValueError("params must be (n_blocks, 512, 4)")
    if assoc is not None:
        _need(assoc, torch.int32, (K, c.height, c.width, 3), "assoc")
    return c, K


def wall_clock_khz() -> int:
    """Rate of the device wall clock that the tracking stamps count, in kHz."""
    khz = C.c_int32(0)
    _lib.check(_lib.load().gsdf_wall_clock_khz(C.byref(khz)), "wall_clock_khz")
    return int(khz.value)


def keyframe_loss(gmap: GsdfMap, params: torch.Tensor, xi: torch.Tensor, depth: torch.Tensor, cam,
                  T0: torch.Tensor, delta: float = 0.01, assoc: Optional[torch.Tensor] = None,
                  freeze: bool = False, count: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Per-keyframe Huber loss (K float64), no gradient."""
    c, K = _kf_args(gmap, depth, cam, T0, xi, params, assoc)
    loss = torch.empty(K, dtype=torch.float64, device=depth.device)
    scratch = gmap._keyframe_scratch(c, K)
    _lib.check(_lib.load().gsdf_keyframe_loss(
        C.byref(gmap._map), _ptr(depth), K, C.byref(c), _ptr(T0), _ptr(xi), _ptr(params),
        int(params.shape[0]), float(delta), _ptr(assoc), 1 if freeze else 0, _ptr(loss), _ptr(count),
        _ptr(scratch), scratch.numel(), _stream()), "keyframe_loss")
    return loss


class KeyframeLoss(torch.autograd.Function):
    """L_i = sum_k rho_delta(psi_j + g^_j . (T_i x_k - v_j)), T_i = exp(xi_i^) T0_i,
    differentiable in the per-voxel parameters {psi, g} (scatter-added at the
    voxel's slot) and the twists xi.  The backward kernel recomputes the
    residuals; nothing per pixel is kept between the passes.

        loss = KeyframeLoss.apply(params, xi, gmap, depth, cam, T0, delta)
    """

    @staticmethod
    def forward(ctx, params, xi, gmap, depth, cam, T0, delta=0.01, assoc=None, freeze=False):
        loss = keyframe_loss(gmap, params, xi, depth, cam, T0, delta, assoc, freeze)
        ctx.save_for_backward(params, xi)
        ctx.rest = (gmap, depth, cam, T0, delta, assoc, freeze)
        return loss

    @staticmethod
    def backward(ctx, grad_loss):
        params, xi = ctx.saved_tensors
        gmap, depth, cam, T0, delta, assoc, freeze = ctx.rest
        c, K = _kf_args(gmap, depth, cam, T0, xi, params, assoc)
        gl = grad_loss.to(torch.float32).contiguous()
        dparams = torch.zeros_like(params)
        dxi = torch.empty_like(xi)
        scratch = gmap._keyframe_scratch(c, K)
        _lib.check(_lib.load().gsdf_backward(
            C.byref(gmap._map), _ptr(depth), K, C.byref(c), _ptr(T0), _ptr(xi), _ptr(params),
            int(params.shape[0]), float(delta), _ptr(assoc), 1 if freeze else 0, _ptr(gl), _ptr(dparams),
            _ptr(dxi), None, _ptr(scratch), scratch.numel(), _stream()), "keyframe_backward")
        return (dparams if ctx.needs_input_grad[0] else None, dxi if ctx.needs_input_grad[1] else None,
                None, None, None, None, None, None, None)


def adjoint_se3(T: torch.Tensor) -> torch.Tensor:
    """Adjoint matrices (K, 6, 6) of poses (K, 3, 4) for twists (rho, phi):
    exp((Ad(T) xi)^) = T exp(xi^) T^-1.  The refinement drivers take their
    pose variables in each camera's own frame (rotation about the camera
    centre) and hand Ad(T0) xi to the kernels, which compose on the left."""
    R = T[:, :, :3]
    t = T[:, :, 3]
    z = torch.zeros_like(t[:, 0])
    th = torch.stack([torch.stack([z, -t[:, 2], t[:, 1]], -1), torch.stack([t[:, 2], z, -t[:, 0]], -1),
                      torch.stack([-t[:, 1], t[:, 0], z], -1)], -2)
    A = torch.zeros((T.shape[0], 6, 6), dtype=T.dtype, device=T.device)
    A[:, :3, :3] = R
    A[:, :3, 3:] = th @ R
    A[:, 3:, 3:] = R
    return A


def refine_keyframes(gmap: GsdfMap, depth: torch.Tensor, cam, T0: torch.Tensor, steps: int = 50,
                     delta: float = 0.01, lr_pose: float = 4e-3, lr_geom: float = 0.0,
                     params: Optional[torch.Tensor] = None, write_back: bool = False):
    """Refinement of keyframe poses and (if lr_geom > 0) voxel parameters by
    Adam on the summed keyframe loss, the pose variables taken in each
    camera's frame, learning rates on a cosine schedule.  Returns (poses
    (K,3,4), params, losses per step).  With write_back the refined
    parameters are imported into the map."""
    K = depth.shape[0]
    if params is None:
        params = gmap.export_params()
    params = params.detach().clone().requires_grad_(lr_geom > 0)
    ad = adjoint_se3(T0)
    xc = torch.zeros((K, 6), dtype=torch.float64, device=depth.device, requires_grad=True)
    groups = [{"params": [xc], "lr": lr_pose}]
    if lr_geom > 0:
        groups.append({"params": [params], "lr": lr_geom})
    opt = torch.optim.Adam(groups, fused=depth.is_cuda)
    sched = torch.optim.lr_scheduler.CosineAnnealingLR(opt, steps)
    losses = []
    for _ in range(steps):
        opt.zero_grad(set_to_none=True)
        xi = (ad @ xc.unsqueeze(-1)).squeeze(-1)
        loss = KeyframeLoss.apply(params, xi, gmap, depth, cam, T0, delta).sum()
        loss.backward()
        opt.step()
        sched.step()
        losses.append(loss.detach())
    poses = compose_left((ad @ xc.detach().unsqueeze(-1)).squeeze(-1), T0)
    if write_back:
        gmap.import_params(params.detach())
    return poses, params.detach(), torch.stack(losses).cpu().numpy()


def _photo_args(gmap: GsdfMap, depth, rgb, cam, T0, xi, params, colors):
    c, K = _kf_args(gmap, depth, cam, T0, xi, params, None)
    _need(rgb, torch.float32, (K, c.height, c.width, 3), "rgb")
    if colors is not None:
        _need(colors, torch.float32, (params.shape[0], 512, 3), "colors")
    key = ("photo", int(params.shape[0]), K)
    if key not in gmap._scratch:
        n = _lib.load().gsdf_photometric_scratch_bytes(int(params.shape[0]), K)
        if n == 0:
            raise ValueError("invalid keyframe count for the photometric term")
        gmap._scratch[key] = torch.empty(int(n), dtype=torch.uint8, device=gmap.device)
    return c, K, gmap._scratch[key]


def mean_color(gmap: GsdfMap, params: torch.Tensor, xi: torch.Tensor, depth: torch.Tensor, rgb: torch.Tensor,
               cam, T0: torch.Tensor):
    """Mean colour of every surface voxel over the keyframes that see it
    (Eq. (21)) and its view count: ((n, 512, 3), (n, 512)) float32."""
    c, K, scratch = _photo_args(gmap, depth, rgb, cam, T0, xi, params, None)
    n = int(params.shape[0])
    col = torch.empty((n, 512, 3), dtype=torch.float32, device=depth.device)
    cnt = torch.empty((n, 512), dtype=torch.float32, device=depth.device)
    _lib.check(_lib.load().gsdf_mean_color(C.byref(gmap._map), _ptr(depth), _ptr(rgb), K, C.byref(c), _ptr(T0),
                                            _ptr(xi.detach().contiguous()), _ptr(params.detach().contiguous()), n,
                                            _ptr(col), _ptr(cnt), _ptr(scratch), scratch.numel(), _stream()),
               "mean_color")
    return col, cnt


class PhotometricLoss(torch.autograd.Function):
    """L_i = weight * sum_j sum_c huber_delta(I_i^c(pi(R_i^T (v_j - psi_j g^_j - t_i))) - rho_j^c)
    over the surface voxels keyframe i sees (Eq. (18) surface point, g^
    held fixed); differentiable in psi (params[..., 0]), the voxel colours
    rho and the twists xi.

        loss = PhotometricLoss.apply(params, colors, xi, gmap, depth, rgb, cam, T0, delta, weight)
    """

    @staticmethod
    def forward(ctx, params, colors, xi, gmap, depth, rgb, cam, T0, delta=0.1, weight=1.0):
        c, K, scratch = _photo_args(gmap, depth, rgb, cam, T0, xi, params, colors)
        loss = torch.empty(K, dtype=torch.float64, device=depth.device)
        _lib.check(_lib.load().gsdf_photometric_loss(
            C.byref(gmap._map), _ptr(depth), _ptr(rgb), K, C.byref(c), _ptr(T0), _ptr(xi), _ptr(params),
            _ptr(colors), int(params.shape[0]), float(delta), float(weight), _ptr(loss), None, _ptr(scratch),
            scratch.numel(), _stream()), "photometric_loss")
        ctx.save_for_backward(params, colors, xi)
        ctx.rest = (gmap, depth, rgb, cam, T0, delta, weight)
        return loss

    @staticmethod
    def backward(ctx, grad_loss):
        params, colors, xi = ctx.saved_tensors
        gmap, depth, rgb, cam, T0, delta, weight = ctx.rest
        c, K, scratch = _photo_args(gmap, depth, rgb, cam, T0, xi, params, colors)
        gl = grad_loss.to(torch.float32).contiguous()
        dparams = torch.zeros_like(params)
        dcolors = torch.zeros_like(colors)
        dxi = torch.empty_like(xi)
        _lib.check(_lib.load().gsdf_photometric_backward(
            C.byref(gmap._map), _ptr(depth), _ptr(rgb), K, C.byref(c), _ptr(T0), _ptr(xi), _ptr(params),
            _ptr(colors), int(params.shape[0]), float(delta), float(weight), _ptr(gl), _ptr(dparams),
            _ptr(dcolors), _ptr(dxi), None, _ptr(scratch), scratch.numel(), _stream()), "photometric_backward")
        return (dparams if ctx.needs_input_grad[0] else None, dcolors if ctx.needs_input_grad[1] else None,
                dxi if ctx.needs_input_grad[2] else None, None, None, None, None, None, None, None)


class MeanColor(torch.autograd.Function):
    """Mean colour of every surface voxel over the keyframes that see it
    (Eq. (21)), differentiable in psi (params[..., 0], g^ held fixed) and the
    twists xi; also returns the view counts N_j (not differentiable).

        colors, counts = MeanColor.apply(params, xi, gmap, depth, rgb, cam, T0)
    """

    @staticmethod
    def forward(ctx, params, xi, gmap, depth, rgb, cam, T0):
        col, cnt = mean_color(gmap, params, xi, depth, rgb, cam, T0)
        ctx.save_for_backward(params, xi, cnt)
        ctx.rest = (gmap, depth, rgb, cam, T0)
        ctx.mark_non_differentiable(cnt)
        return col, cnt

    @staticmethod
    def backward(ctx, grad_col, grad_cnt):
        params, xi, cnt = ctx.saved_tensors
        gmap, depth, rgb, cam, T0 = ctx.rest
        c, K, scratch = _photo_args(gmap, depth, rgb, cam, T0, xi, params, None)
        g = grad_col.to(torch.float32).contiguous() if grad_col is not None else torch.zeros(
            (params.shape[0], 512, 3), dtype=torch.float32, device=params.device)
        dparams = torch.zeros_like(params)
        dxi = torch.empty_like(xi)
        _lib.check(_lib.load().gsdf_mean_color_backward(
            C.byref(gmap._map), _ptr(depth), _ptr(rgb), K, C.byref(c), _ptr(T0), _ptr(xi.detach().contiguous()),
            _ptr(params.detach().contiguous()), int(params.shape[0]), _ptr(g), _ptr(cnt), _ptr(dparams), _ptr(dxi),
            _ptr(scratch), scratch.numel(), _stream()), "mean_color_backward")
        return (dparams if ctx.needs_input_grad[0] else None, dxi if ctx.needs_input_grad[1] else None,
                None, None, None, None, None)


def implicit_photometric_loss(gmap: GsdfMap, params: torch.Tensor, xi: torch.Tensor, depth: torch.Tensor,
                              rgb: torch.Tensor, cam, T0: torch.Tensor, delta: float = 0.1, weight: float = 1.0,
                              coupled: bool = True) -> torch.Tensor:
    """Bundle-adjustment energy of Sec. 4.2 without stored colour: every
    surface voxel's residuals are taken against its own mean colour.
    coupled=True differentiates through the mean (Eq. (17)); coupled=False
    holds it fixed (the decoupled per-pose energies of Eq. (20)).  Returns
    the per-keyframe shares (K float64)."""
    if coupled:
        col, _ = MeanColor.apply(params, xi, gmap, depth, rgb, cam, T0)
    else:
        col, _ = mean_color(gmap, params.detach(), xi.detach(), depth, rgb, cam, T0)
    return PhotometricLoss.apply(params, col, xi, gmap, depth, rgb, cam, T0, delta, weight)


class PsiRegulariser(torch.autograd.Function):
    """weight * sum_j (psi_j - psi0_j)^2 over observed voxels (scalar)."""

    @staticmethod
    def forward(ctx, params, params0, gmap, weight):
        n = int(params.shape[0])
        scratch = torch.empty(max(n, 1), dtype=torch.float64, device=params.device)
        loss = torch.empty((), dtype=torch.float64, device=params.device)
        _lib.check(_lib.load().gsdf_psi_regulariser(C.byref(gmap._map), _ptr(params.detach().contiguous()),
                                                     _ptr(params0), n, float(weight), _ptr(loss), None,
                                                     _ptr(scratch), scratch.numel() * 8, _stream()), "psi_regulariser")
        ctx.save_for_backward(params, params0)
        ctx.rest = (gmap, weight)
        return loss

    @staticmethod
    def backward(ctx, grad):
        params, params0 = ctx.saved_tensors
        gmap, weight = ctx.rest
        n = int(params.shape[0])
        scratch = torch.empty(max(n, 1), dtype=torch.float64, device=params.device)
        loss = torch.empty((), dtype=torch.float64, device=params.device)
        dparams = torch.zeros_like(params)
        _lib.check(_lib.load().gsdf_psi_regulariser(C.byref(gmap._map), _ptr(params.detach().contiguous()),
                                                     _ptr(params0), n, float(weight), _ptr(loss), _ptr(dparams),
                                                     _ptr(scratch), scratch.numel() * 8, _stream()), "psi_regulariser")
        return dparams * grad.to(torch.float32), None, None, None


def photometric_ba(gmap: GsdfMap, depth: torch.Tensor, rgb: torch.Tensor, cam, T0: torch.Tensor, steps: int = 50,
                   delta: float = 0.1, coupled: bool = True, optimise_psi: bool = True,
                   reg_weight: float = 100.0, lr_pose: float = 2e-3, lr_psi: float = 2e-5,
                   fix_first: bool = True, write_back: bool = False):
    """Implicit photometric bundle adjustment (Sec. 4.2): Adam on the
    keyframe poses (camera-frame variables) and, unless optimise_psi is
    False (the pose-only variant), on the distances psi, minimising the
    Eq. (17) (coupled) or Eq. (20) (decoupled) energy plus
    reg_weight sum_j (psi_j - psi0_j)^2 (100 m^-2 = 0.01 cm^-2).  The energy
    compares the keyframes with each other, so a motion common to all of
    them is (nearly) free: with fix_first the first keyframe anchors the
    gauge and keeps its pose.  Returns (poses (K,3,4), params, losses)."""
    K = depth.shape[0]
    params0 = gmap.export_params().detach()
    params = params0.clone().requires_grad_(optimise_psi)
    ad = adjoint_se3(T0)
    xc = torch.zeros((K, 6), dtype=torch.float64, device=depth.device, requires_grad=True)
    mask = torch.ones((K, 1), dtype=torch.float64, device=depth.device)
    if fix_first:
        mask[0] = 0.0
    groups = [{"params": [xc], "lr": lr_pose}]
    if optimise_psi:
        groups.append({"params": [params], "lr": lr_psi})
    opt = torch.optim.Adam(groups, fused=depth.is_cuda)
    sched = torch.optim.lr_scheduler.CosineAnnealingLR(opt, steps)
    losses = []
    for _ in range(steps):
        opt.zero_grad(set_to_none=True)
        xi = (ad @ (mask * xc).unsqueeze(-1)).squeeze(-1)
        loss = implicit_photometric_loss(gmap, params, xi, depth, rgb, cam, T0, delta, 1.0, coupled).sum()
        if optimise_psi and reg_weight > 0:
            loss = loss + PsiRegulariser.apply(params, params0, gmap, reg_weight)
        loss.backward()
        opt.step()
        sched.step()
        losses.append(loss.detach())
    poses = compose_left((ad @ (mask * xc.detach()).unsqueeze(-1)).squeeze(-1), T0)
    if write_back:
        gmap.import_params(params.detach())
    return poses, params.detach(), torch.stack(losses).cpu().numpy()


def joint_loss_and_grads(gmap: GsdfMap, params: torch.Tensor, colors: torch.Tensor, xi: torch.Tensor,
                         depth: torch.Tensor, rgb: torch.Tensor, cam, T0: torch.Tensor, delta: float = 0.01,
                         photo_delta: float = 0.1, photo_weight: float = 0.01):
    """The joint refinement objective sum_i (L_i + P_i), the SDF keyframe
    loss (KeyframeLoss) plus the photometric loss (PhotometricLoss), and its
    gradients in the voxel parameters, the voxel colours and the twists,
    from the two adjoint calls alone with unit upstream gradients (each also
    returns its loss, so no separate loss pass runs).  The gradients are
    those of (KeyframeLoss.apply(...).sum() + PhotometricLoss.apply(...).sum())
    through autograd, bit for bit.  Returns (loss (float64 scalar tensor),
    dparams, dcolors, dxi)."""
    params = params.detach()
    colors = colors.detach()
    xi = xi.detach()
    c, K = _kf_args(gmap, depth, cam, T0, xi, params, None)
    ones = torch.ones(K, dtype=torch.float32, device=depth.device)
    dparams = torch.zeros_like(params)
    dxi_s = torch.empty_like(xi)
    loss_s = torch.empty(K, dtype=torch.float64, device=depth.device)
    scratch = gmap._keyframe_scratch(c, K)
    _lib.check(_lib.load().gsdf_backward(
        C.byref(gmap._map), _ptr(depth), K, C.byref(c), _ptr(T0), _ptr(xi), _ptr(params),
        int(params.shape[0]), float(delta), None, 0, _ptr(ones), _ptr(dparams), _ptr(dxi_s), _ptr(loss_s),
        _ptr(scratch), scratch.numel(), _stream()), "keyframe_backward")
    cp, _, pscratch = _photo_args(gmap, depth, rgb, cam, T0, xi, params, colors)
    dcolors = torch.zeros_like(colors)
    dxi_p = torch.empty_like(xi)
    loss_p = torch.empty(K, dtype=torch.float64, device=depth.device)
    _lib.check(_lib.load().gsdf_photometric_backward(
        C.byref(gmap._map), _ptr(depth), _ptr(rgb), K, C.byref(cp), _ptr(T0), _ptr(xi), _ptr(params),
        _ptr(colors), int(params.shape[0]), float(photo_delta), float(photo_weight), _ptr(ones), _ptr(dparams),
        _ptr(dcolors), _ptr(dxi_p), _ptr(loss_p), _ptr(pscratch), pscratch.numel(), _stream()),
        "photometric_backward")
    return loss_s.sum() + loss_p.sum(), dparams, dcolors, dxi_s + dxi_p


def refine_joint(gmap: GsdfMap, depth: torch.Tensor, rgb: torch.Tensor, cam, T0: torch.Tensor,
                 steps: int = 50, delta: float = 0.01, photo_delta: float = 0.1, photo_weight: float = 0.01,
                 lr_psi: float = 2e-5, lr_color: float = 1e-2, pose_solver: str = "gn", lr_pose: float = 4e-3,
                 write_back: bool = True, fused: bool = True):
    """Joint refinement over keyframes of the voxel distances and gradients,
    the voxel colours and the keyframe poses on the sum of the SDF keyframe
    loss and the photometric loss.  Each step takes an Adam step on the
    voxel parameters and colours (gradients from both adjoint kernels), then
    updates the poses: ``pose_solver="gn"`` writes the parameters into the
    map (rounded to its storage format) and takes one Gauss-Newton
    iteration per keyframe on the updated map (gn_step_keyframes);
    ``"adam"`` moves camera-frame pose variables by Adam on the joint loss.
    Colours start from the Eq. (21) mean at the initial poses.  The default
    photometric weight (delta / photo_delta)^2 prices a residual at either
    Huber threshold equally; learning rates decay on a cosine schedule.
    ``fused`` takes each step's loss and gradients from the adjoint calls
    alone (joint_loss_and_grads); ``fused=False`` composes KeyframeLoss and
    PhotometricLoss through autograd (a loss pass, then the adjoints): the
    same gradients, so the same steps.
    Returns (poses (K,3,4), params, colours, losses)."""
    K = depth.shape[0]
    params = gmap.export_params().detach().clone()
    T = T0.detach().clone()
    ad = adjoint_se3(T0)
    xc = torch.zeros((K, 6), dtype=torch.float64, device=depth.device)
    colors, _ = mean_color(gmap, params, xc, depth, rgb, cam, T)
    params.requires_grad_(True)
    colors.requires_grad_(True)
    groups = [{"params": [params], "lr": lr_psi}, {"params": [colors], "lr": lr_color}]
    if pose_solver == "adam":
        xc.requires_grad_(True)
        groups.append({"params": [xc], "lr": lr_pose})
    elif pose_solver != "gn":
        raise ValueError("pose_solver must be 'gn' or 'adam'")
    # PyTorch's fused Adam: one kernel per parameter group and dtype a step
    opt = torch.optim.Adam(groups, fused=depth.is_cuda)
    sched = torch.optim.lr_scheduler.CosineAnnealingLR(opt, steps)
    losses = []
    for _ in range(steps):
        opt.zero_grad(set_to_none=True)
        xi = (ad @ xc.unsqueeze(-1)).squeeze(-1)
        if fused:
            loss, dparams, dcolors, dxi = joint_loss_and_grads(gmap, params, colors, xi, depth, rgb, cam, T,
                                                               delta, photo_delta, photo_weight)
            params.grad = dparams
            colors.grad = dcolors
            if pose_solver == "adam":
                xc.grad = (ad.transpose(1, 2) @ dxi.unsqueeze(-1)).squeeze(-1)
        else:
            loss = (KeyframeLoss.apply(params, xi, gmap, depth, cam, T, delta).sum()
                    + PhotometricLoss.apply(params, colors, xi, gmap, depth, rgb, cam, T, photo_delta,
                                            photo_weight).sum())
            loss.backward()
        opt.step()
        sched.step()
        losses.append(loss.detach())
        if pose_solver == "gn":
            gmap.import_params(params.detach())
            gmap.gn_step_keyframes(depth, cam, T, delta=delta)
    if pose_solver == "adam":
        T = compose_left((ad @ xc.detach().unsqueeze(-1)).squeeze(-1), T0)
    if write_back:
        gmap.import_params(params.detach())
    return T, params.detach(), colors.detach(), torch.stack(losses).cpu().numpy()


def compose_left(xi: torch.Tensor, T0: torch.Tensor) -> torch.Tensor:
    """exp(xi_i^) T0_i for (K, 6) / (K, 3, 4) float64 device tensors."""
    K = T0.shape[0]
    _need(T0, torch.float64, (K, 3, 4), "T0")
    xi = xi.detach().contiguous()
    _need(xi, torch.float64, (K, 6), "xi")
    out = torch.empty_like(T0)
    _lib.check(_lib.load().gsdf_compose_poses(K, _ptr(T0), _ptr(xi), _ptr(out), _stream()), "compose_poses")
    return out


def run_stream(m: GsdfMap, depth: torch.Tensor, cam, pose0: torch.Tensor, levels: int = 3,
               iters: Sequence[int] = (4, 5, 10), delta: float = 0.01, damping: float = 1e-6,
               poses_out: Optional[torch.Tensor] = None, start: int = 0, stop: Optional[int] = None):
    """The per-frame loop on the device: frame ``start`` is fused at
    ``pose0``; every later frame is tracked from the previous estimate and
    then fused at the new estimate.  ``depth`` is (F, H, W) float32 on the
    device; returns the (F, 3, 4) float64 device tensor of estimates."""
    F = depth.shape[0]
    stop = F if stop is None else stop
    if poses_out is None:
        poses_out = torch.zeros((F, 3, 4), dtype=torch.float64, device=depth.device)
    poses_out[start].copy_(pose0)
    m.fuse(depth[start], cam, poses_out[start])
    for f in range(start + 1, stop):
        m.track(depth[f], cam, poses_out[f], levels=levels, iters=iters, delta=delta, damping=damping,
                init=poses_out[f - 1])
        m.fuse(depth[f], cam, poses_out[f])
    return poses_out


def angle_statistics(quality, voxel_size: float, within=range(1, 11)):
    """Mean, median and 95th percentile of each angle plane of
    ``GsdfMap.gradient_quality`` over the voxels closer than x voxels to the
    surface, for each x in ``within``, on the voxels where all four angles
    are defined (a reporting helper on host copies).  Returns {x: {name:
    (mean, median, p95)}} with names stored / forward / backward / central,
    plus the voxel count under "n"."""
    q = quality.detach().float().cpu().numpy().reshape(5, -1) if hasattr(quality, "detach") else \
        np.asarray(quality, np.float64).reshape(5, -1)
    ok = np.isfinite(q).all(axis=0)
    out = {}
    for x in within:
        sel = ok & (q[0] < x * voxel_size)
        row = {"n": int(sel.sum())}
        for k, name in enumerate(("stored", "forward", "backward", "central")):
            a = q[1 + k][sel]
            row[name] = (float(a.mean()), float(np.median(a)), float(np.percentile(a, 95))) if a.size else None
        out[x] = row
    return out
