"""FP64 CPU reference of Gradient-SDF tracking and fusion -- TEST INFRASTRUCTURE.

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library and its Python
binding never touch it, and it shares no code with them.

The implementation lives in ``gsdf_oracle.cpp`` (single-threaded C++, FP64
values, binary32 only where a float decides an integer); this module is a
ctypes wrapper that takes and returns numpy arrays.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gsdf_oracle.cpp")
_LIB_PATH = os.path.join(_HERE, "libgsdf_oracle.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (strict IEEE: no FMA contraction)."""
    if force or not os.path.exists(_LIB_PATH):
        cmd = ["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared", "-o", _LIB_PATH + ".tmp", _SRC]
        subprocess.check_call(cmd)
        os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


class OrcCam(C.Structure):
    _fields_ = [("fx", C.c_double), ("fy", C.c_double), ("cx", C.c_double), ("cy", C.c_double),
                ("width", C.c_int32), ("height", C.c_int32), ("zmin", C.c_double),
                ("zmax", C.c_double)]


_P = C.c_void_p
_D = C.c_double
_I = C.c_int
_I64 = C.c_int64


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        build()
    lib = C.CDLL(_LIB_PATH)
    sig = {
        "orc_map_new": (_P, [_D, _D, _I, _P, _P]),
        "orc_map_free": (None, [_P]),
        "orc_map_clone": (_P, [_P]),
        "orc_num_blocks": (_I64, [_P]),
        "orc_export_keys": (None, [_P, _P]),
        "orc_export_voxels": (None, [_P, _P, _I64, _P, _P, _P, _P]),
        "orc_import_voxels": (None, [_P, _P, _I64, _P, _P, _P]),
        "orc_band_voxels": (_I, [_P, _P, _P, _I, _I, C.c_float, _P, _I]),
        "orc_allocate": (_I64, [_P, _P, _P, _P]),
        "orc_normals": (None, [_P, _P, _D, _P, _P, _P]),
        "orc_integrate": (_I64, [_P, _P, _P, _P, _D, _D, _D, _I, _P]),
        "orc_pyramid_down": (None, [_P, _P, _D, _P]),
        "orc_normal_equations": (None, [_P, _P, _P, _P, _D, _P]),
        "orc_gn_level": (_I, [_P, _P, _P, _I, _D, _D, _P, _P]),
        "orc_track": (_I, [_P, _P, _P, _I, _P, _D, _D, _P, _P]),
        "orc_track_model": (_I, [_P, _P, _P, _I, _P, _D, _D, _P, _P, _I]),
        "orc_trilinear": (_I, [_P, _P, _P, _P]),
        "orc_cholesky_solve6": (_I, [_P, _P, _P]),
        "orc_se3_exp": (None, [_P, _P]),
        "orc_se3_left_jacobian": (None, [_P, _P]),
        "orc_gn_step": (_I, [_P, _D, _P, _P]),
        "orc_huber_rho": (_D, [_D, _D]),
        "orc_huber_weight": (_D, [_D, _D]),
        "orc_w_linear": (_D, [_D, _D, _D]),
        "orc_nearest_voxel": (None, [_P, _D, _P]),
        "orc_floordiv8": (_I, [_I]),
        "orc_taylor": (_I, [_P, _P, _P, _P, _P]),
        "orc_loss_grad": (_D, [_P, _I, _P, _P, _P, _P, _D, _P, _I, _P, _I64, _P, _P, _P]),
        "orc_render_taylor": (None, [_P, _P, _P, _D, _D, _P]),
        "orc_integrate_rounded": (_I64, [_P, _P, _P, _P, _D, _D, _I]),
        "orc_round_storage": (_D, [_D, _I]),
        "orc_photo_loss_grad": (_D, [_P, _I, _P, _P, _P, _P, _P, _P, _I64, _P, _D, _D, _P, _P, _P, _P, _P]),
        "orc_mean_color": (None, [_P, _I, _P, _P, _P, _P, _P, _P, _I64, _P, _P]),
        "orc_extract_surfels": (_I64, [_P, _P, _I64, _I, _P, _P, _P, _I64]),
        "orc_fd_gradients": (None, [_P, _P, _I64, _P, _P, _P, _P]),
        "orc_gradient_quality": (None, [_P, _P, _I64, _P, _I, _P]),
        "orc_photo_energy": (_D, [_P, _I, _P, _P, _P, _P, _P, _P, _I64, _D, _D, _I, _P, _P, _P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def cam_struct(cam) -> OrcCam:
    return OrcCam(float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy), int(cam.width),
                  int(cam.height), float(cam.zmin), float(cam.zmax))


class OracleMap:
    """A sparse 8^3-block Gradient-SDF map held by the oracle (FP64)."""

    def __init__(self, voxel_size: float, truncation: float, bounds=None, _handle=None):
        lib = _load()
        self.voxel_size = float(voxel_size)
        self.truncation = float(truncation)
        self.bounds = bounds
        if _handle is not None:
            self._h = _handle
        elif bounds is None:
            self._h = lib.orc_map_new(self.voxel_size, self.truncation, 0, None, None)
        else:
            bmin = _c(bounds[0], np.int32)
            bmax = _c(bounds[1], np.int32)
            self._h = lib.orc_map_new(self.voxel_size, self.truncation, 1, _ptr(bmin), _ptr(bmax))

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.orc_map_free(self._h)
            self._h = None

    def clone(self) -> "OracleMap":
        return OracleMap(self.voxel_size, self.truncation, self.bounds,
                         _handle=_load().orc_map_clone(self._h))

    # ---- inspection ----
    def num_blocks(self) -> int:
        return int(_load().orc_num_blocks(self._h))

    def keys(self) -> np.ndarray:
        n = self.num_blocks()
        out = np.zeros((n, 3), np.int32)
        if n:
            _load().orc_export_keys(self._h, _ptr(out))
        return out

    def voxels(self, keys: Optional[np.ndarray] = None):
        """(psi, g, W, found) for blocks ``keys`` (default: all, sorted);
        voxel order within a block is lx + 8 ly + 64 lz."""
        keys = self.keys() if keys is None else _c(keys, np.int32).reshape(-1, 3)
        n = len(keys)
        psi = np.zeros((n, 512))
        g = np.zeros((n, 512, 3))
        W = np.zeros((n, 512))
        found = np.zeros(n, np.int32)
        if n:
            _load().orc_export_voxels(self._h, _ptr(keys), n, _ptr(psi), _ptr(g), _ptr(W), _ptr(found))
        return psi, g, W, found

    def set_voxels(self, keys, psi, g, W):
        keys = _c(keys, np.int32).reshape(-1, 3)
        n = len(keys)
        _load().orc_import_voxels(self._h, _ptr(keys), n, _ptr(_c(psi, np.float64)),
                                  _ptr(_c(g, np.float64)), _ptr(_c(W, np.float64)))

    # ---- the method ----
    def allocate(self, depth: np.ndarray, cam, T: np.ndarray) -> int:
        d = _c(depth, np.float32)
        c = cam_struct(cam)
        return int(_load().orc_allocate(self._h, _ptr(d), C.byref(c), _ptr(_c(T, np.float64))))

    def integrate(self, depth: np.ndarray, cam, T: np.ndarray, eps: Optional[float] = None,
                  cos_min: float = float(np.cos(np.deg2rad(75.0))), margin: float = 1e-5,
                  return_marginal: bool = False, gradients: bool = True):
        """Fusion of one frame (Eq. (1)-(3)); gradients=False fuses the
        distance and weight only (Eq. (1)-(2)), leaving g at zero."""
        d = _c(depth, np.float32)
        c = cam_struct(cam)
        eps = self.voxel_size if eps is None else float(eps)
        marg = np.zeros(depth.shape, np.int32) if return_marginal else None
        n = int(_load().orc_integrate(self._h, _ptr(d), C.byref(c), _ptr(_c(T, np.float64)),
                                      eps, float(cos_min), float(margin), 1 if gradients else 0, _ptr(marg)))
        return (n, marg) if return_marginal else n

    def integrate_rounded(self, depth: np.ndarray, cam, T: np.ndarray, storage: str,
                          eps: Optional[float] = None,
                          cos_min: float = float(np.cos(np.deg2rad(75.0)))) -> int:
        """Fusion with 16-bit storage emulated (psi/T and gbar rounded to
        bf16 / fp16 once per frame, W to binary32).  The map's g then holds
        the mean gradient gbar."""
        d = _c(depth, np.float32)
        c = cam_struct(cam)
        eps = self.voxel_size if eps is None else float(eps)
        return int(_load().orc_integrate_rounded(self._h, _ptr(d), C.byref(c), _ptr(_c(T, np.float64)),
                                                 eps, float(cos_min), STORAGE_CODES[storage]))

    def band_voxels(self, cam, T, u: int, v: int, D: float) -> np.ndarray:
        out = np.zeros((256, 3), np.int32)
        c = cam_struct(cam)
        n = _load().orc_band_voxels(self._h, C.byref(c), _ptr(_c(T, np.float64)), int(u), int(v),
                                    float(np.float32(D)), _ptr(out), 256)
        return out[:min(n, 256)].copy()

    def normal_equations(self, depth: np.ndarray, cam, T, delta: float) -> np.ndarray:
        out = np.zeros(29)
        c = cam_struct(cam)
        _load().orc_normal_equations(self._h, _ptr(_c(depth, np.float64)), C.byref(c),
                                     _ptr(_c(T, np.float64)), float(delta), _ptr(out))
        return out

    def gn_level(self, depth: np.ndarray, cam, T, iters: int, delta: float, damping: float = 1e-6):
        Tn = _c(T, np.float64).copy()
        stats = np.zeros((iters, 2))
        c = cam_struct(cam)
        failed = _load().orc_gn_level(self._h, _ptr(_c(depth, np.float64)), C.byref(c), int(iters),
                                      float(delta), float(damping), _ptr(Tn), _ptr(stats))
        return Tn, stats, int(failed)

    def track(self, depth: np.ndarray, cam, T, levels: int, iters: Sequence[int], delta: float,
              damping: float = 1e-6, model: str = "taylor"):
        """Coarse-to-fine tracking; model "taylor" (Eq. (14)-(16)) or
        "trilinear" (Eq. (12)-(13)).  Returns (pose, stats, failed solves)."""
        Tn = _c(T, np.float64).copy()
        it = _c(list(iters)[:levels], np.int32)
        stats = np.zeros((int(it.sum()), 2))
        c = cam_struct(cam)
        failed = _load().orc_track_model(self._h, _ptr(_c(depth, np.float32)), C.byref(c), int(levels),
                                         _ptr(it), float(delta), float(damping), _ptr(Tn), _ptr(stats),
                                         {"taylor": 0, "trilinear": 1}[model])
        return Tn, stats, int(failed)

    def trilinear(self, q) -> Optional[tuple]:
        """Tri-linear distance and gradient at world point q (Eq. (12)-(13)),
        or None when one of the eight voxels is missing or unobserved."""
        r = C.c_double()
        g = np.zeros(3)
        ok = _load().orc_trilinear(self._h, _ptr(_c(q, np.float64)), C.byref(r), _ptr(g))
        return (r.value, g) if ok else None

    def taylor(self, q) -> Optional[tuple]:
        r = C.c_double()
        gh = np.zeros(3)
        m = np.zeros(3, np.int32)
        ok = _load().orc_taylor(self._h, _ptr(_c(q, np.float64)), C.byref(r), _ptr(gh), _ptr(m))
        return (r.value, gh, m) if ok else None

    def loss_grad(self, depths: np.ndarray, cam, T0: np.ndarray, xi: np.ndarray, delta: float,
                  assoc: Optional[np.ndarray] = None, freeze: bool = False,
                  keys: Optional[np.ndarray] = None, want_voxel_grads: bool = True):
        """Keyframe Huber loss and its gradients (see orc_loss_grad)."""
        K = depths.shape[0]
        c = cam_struct(cam)
        keys = self.keys() if keys is None else _c(keys, np.int32).reshape(-1, 3)
        nk = len(keys)
        dpsi = np.zeros((nk, 512)) if want_voxel_grads else None
        dg = np.zeros((nk, 512, 3)) if want_voxel_grads else None
        dxi = np.zeros((K, 6))
        L = _load().orc_loss_grad(self._h, K, _ptr(_c(depths, np.float64)), C.byref(c),
                                  _ptr(_c(T0, np.float64)), _ptr(_c(xi, np.float64)), float(delta),
                                  _ptr(assoc), 1 if freeze else 0, _ptr(keys), nk, _ptr(dpsi),
                                  _ptr(dg), _ptr(dxi))
        return L, dpsi, dg, dxi

    def photo_loss_grad(self, depths: np.ndarray, rgb: np.ndarray, cam, T0, xi, colors, delta: float,
                        lam: float = 1.0, keys: Optional[np.ndarray] = None, want_grads: bool = True):
        """Photometric keyframe loss against stored voxel colours (see
        orc_photo_loss_grad).  Returns (loss per keyframe, dpsi, dcolor, dxi,
        number of visible (voxel, keyframe) pairs)."""
        K = depths.shape[0]
        c = cam_struct(cam)
        keys = self.keys() if keys is None else _c(keys, np.int32).reshape(-1, 3)
        nk = len(keys)
        loss = np.zeros(K)
        dpsi = np.zeros((nk, 512)) if want_grads else None
        dcol = np.zeros((nk, 512, 3)) if want_grads else None
        dxi = np.zeros((K, 6)) if want_grads else None
        nvis = C.c_int64()
        _load().orc_photo_loss_grad(self._h, K, _ptr(_c(depths, np.float64)), _ptr(_c(rgb, np.float64)),
                                    C.byref(c), _ptr(_c(T0, np.float64)), _ptr(_c(xi, np.float64)), _ptr(keys),
                                    nk, _ptr(_c(colors, np.float64)), float(delta), float(lam), _ptr(loss),
                                    _ptr(dpsi), _ptr(dcol), _ptr(dxi), C.byref(nvis))
        return loss, dpsi, dcol, dxi, int(nvis.value)

    def mean_color(self, depths: np.ndarray, rgb: np.ndarray, cam, T0, xi, keys: Optional[np.ndarray] = None):
        """Eq. (21) colour of every surface voxel and its view count N_j."""
        K = depths.shape[0]
        c = cam_struct(cam)
        keys = self.keys() if keys is None else _c(keys, np.int32).reshape(-1, 3)
        nk = len(keys)
        col = np.zeros((nk, 512, 3))
        cnt = np.zeros((nk, 512))
        _load().orc_mean_color(self._h, K, _ptr(_c(depths, np.float64)), _ptr(_c(rgb, np.float64)), C.byref(c),
                               _ptr(_c(T0, np.float64)), _ptr(_c(xi, np.float64)), _ptr(keys), nk, _ptr(col),
                               _ptr(cnt))
        return col, cnt

    def photo_energy(self, depths: np.ndarray, rgb: np.ndarray, cam, T0, xi, delta: float, lam: float = 1.0,
                     coupled: bool = True, keys: Optional[np.ndarray] = None, want_grads: bool = True):
        """Implicit photometric BA energy against each voxel's own mean colour
        (Eq. (17) coupled, Eq. (20) decoupled).  Returns (loss per keyframe,
        dpsi, dxi)."""
        K = depths.shape[0]
        c = cam_struct(cam)
        keys = self.keys() if keys is None else _c(keys, np.int32).reshape(-1, 3)
        nk = len(keys)
        loss = np.zeros(K)
        dpsi = np.zeros((nk, 512)) if want_grads else None
        dxi = np.zeros((K, 6)) if want_grads else None
        _load().orc_photo_energy(self._h, K, _ptr(_c(depths, np.float64)), _ptr(_c(rgb, np.float64)), C.byref(c),
                                 _ptr(_c(T0, np.float64)), _ptr(_c(xi, np.float64)), _ptr(keys), nk, float(delta),
                                 float(lam), 1 if coupled else 0, _ptr(loss), _ptr(dpsi), _ptr(dxi))
        return loss, dpsi, dxi

    def surfels(self, level: int = 0, keys: Optional[np.ndarray] = None):
        """Oriented point cloud of Sec. 4.3 (level 1: 2x2x2 upsampled).
        Returns (points (n,3), normals (n,3), ids (n,4): voxel + subvoxel)."""
        keys = self.keys() if keys is None else _c(keys, np.int32).reshape(-1, 3)
        lib = _load()
        n = int(lib.orc_extract_surfels(self._h, _ptr(keys), len(keys), int(level), None, None, None, 0))
        pts = np.zeros((n, 3))
        nrm = np.zeros((n, 3))
        ids = np.zeros((n, 4), np.int32)
        lib.orc_extract_surfels(self._h, _ptr(keys), len(keys), int(level), _ptr(pts), _ptr(nrm), _ptr(ids), n)
        return pts, nrm, ids

    def fd_gradients(self, keys: Optional[np.ndarray] = None):
        """Forward, backward and central differences of the stored distance
        (each (n, 512, 3)) and their validity (n, 512) bool, per voxel of
        ``keys``, voxel order lx + 8 ly + 64 lz."""
        keys = self.keys() if keys is None else _c(keys, np.int32).reshape(-1, 3)
        n = len(keys)
        f, b, c = (np.zeros((n, 512, 3)) for _ in range(3))
        ok = np.zeros((n, 512), np.uint8)
        _load().orc_fd_gradients(self._h, _ptr(keys), n, _ptr(f), _ptr(b), _ptr(c), _ptr(ok))
        return f, b, c, ok.astype(bool)

    def gradient_quality(self, spheres: np.ndarray, keys: Optional[np.ndarray] = None) -> np.ndarray:
        """(5, n, 512): distance to the nearest sphere surface, then the
        angles in degrees of the stored gradient and of the forward, backward
        and central differences against the true gradient; NaN where
        undefined."""
        keys = self.keys() if keys is None else _c(keys, np.int32).reshape(-1, 3)
        sp = _c(spheres, np.float64).reshape(-1, 4)
        out = np.zeros((5, len(keys), 512))
        _load().orc_gradient_quality(self._h, _ptr(keys), len(keys), _ptr(sp), len(sp), _ptr(out))
        return out

    def render_taylor(self, cam, T, smin: float = 0.05, smax: float = 10.0) -> np.ndarray:
        out = np.zeros((cam.height, cam.width))
        c = cam_struct(cam)
        _load().orc_render_taylor(self._h, C.byref(c), _ptr(_c(T, np.float64)), float(smin),
                                  float(smax), _ptr(out))
        return out


STORAGE_CODES = {"fp64": 0, "bf16": 1, "fp16": 2}


def round_storage(x: float, storage: str) -> float:
    """Round to bfloat16 / binary16 (ties to even), as the emulated store."""
    return float(_load().orc_round_storage(float(x), STORAGE_CODES[storage]))


# ---- free functions ----
def normals(depth: np.ndarray, cam, truncation: float):
    H, W = depth.shape
    n = np.zeros((H, W, 3))
    valid = np.zeros((H, W), np.int32)
    cos = np.zeros((H, W))
    c = cam_struct(cam)
    _load().orc_normals(_ptr(_c(depth, np.float32)), C.byref(c), float(truncation), _ptr(n),
                        _ptr(valid), _ptr(cos))
    return n, valid.astype(bool), cos


def pyramid_down(depth: np.ndarray, cam, truncation: float) -> np.ndarray:
    H, W = depth.shape
    out = np.zeros((H // 2, W // 2), np.float32)
    c = cam_struct(cam)
    _load().orc_pyramid_down(_ptr(_c(depth, np.float32)), C.byref(c), float(truncation), _ptr(out))
    return out


def cholesky_solve6(A, b):
    x = np.zeros(6)
    ok = _load().orc_cholesky_solve6(_ptr(_c(A, np.float64)), _ptr(_c(b, np.float64)), _ptr(x))
    return x if ok else None


def se3_exp(xi) -> np.ndarray:
    T = np.zeros((3, 4))
    _load().orc_se3_exp(_ptr(_c(xi, np.float64)), _ptr(T))
    return T


def se3_left_jacobian(xi) -> np.ndarray:
    J = np.zeros((6, 6))
    _load().orc_se3_left_jacobian(_ptr(_c(xi, np.float64)), _ptr(J))
    return J


def gn_step(ne, damping, T):
    Tn = _c(T, np.float64).copy()
    dxi = np.zeros(6)
    ok = _load().orc_gn_step(_ptr(_c(ne, np.float64)), float(damping), _ptr(Tn), _ptr(dxi))
    return (Tn, dxi) if ok else (None, None)


def huber_rho(r, delta):
    return _load().orc_huber_rho(float(r), float(delta))


def huber_weight(r, delta):
    return _load().orc_huber_weight(float(r), float(delta))


def w_linear(d, eps, T):
    return _load().orc_w_linear(float(d), float(eps), float(T))


def nearest_voxel(q, vs):
    m = np.zeros(3, np.int32)
    _load().orc_nearest_voxel(_ptr(_c(q, np.float64)), float(vs), _ptr(m))
    return m


def floordiv8(m: int) -> int:
    return int(_load().orc_floordiv8(int(m)))


def unpack_upper(ne: np.ndarray):
    """(H 6x6, b 6, E, n) from a 29-vector of packed normal equations."""
    H = np.zeros((6, 6))
    k = 0
    for i in range(6):
        for j in range(i, 6):
            H[i, j] = H[j, i] = ne[k]
            k += 1
    return H, np.asarray(ne[21:27]), float(ne[27]), float(ne[28])


def track_stream(depths: np.ndarray, cam, poses_gt: np.ndarray, voxel_size: float,
                 truncation: float, levels: int = 3, iters=(4, 5, 10), delta: float = 0.01,
                 damping: float = 1e-6, n_frames: Optional[int] = None, timings: Optional[list] = None,
                 model: str = "taylor", gradients: bool = True):
    """The per-frame loop: frame 0 fused at its ground-truth pose; every later
    frame is tracked from the previous estimate, then allocated and fused at
    the estimate.  ``iters`` is finest-first; ``model`` and ``gradients``
    select the residual model and whether fusion stores gradients (the
    paper's baseline: "trilinear" on a map without gradients).  Returns
    (map, poses)."""
    import time
    F = len(depths) if n_frames is None else n_frames
    M = OracleMap(voxel_size, truncation)
    T = np.asarray(poses_gt[0], np.float64).copy()
    est = [T.copy()]
    t0 = time.perf_counter()
    M.allocate(depths[0], cam, T)
    M.integrate(depths[0], cam, T, gradients=gradients)
    if timings is not None:
        timings.append(("fuse", time.perf_counter() - t0))
    for f in range(1, F):
        t0 = time.perf_counter()
        T, _, _ = M.track(depths[f], cam, T, levels, iters, delta, damping, model=model)
        t1 = time.perf_counter()
        M.allocate(depths[f], cam, T)
        M.integrate(depths[f], cam, T, gradients=gradients)
        t2 = time.perf_counter()
        if timings is not None:
            timings.append(("track", t1 - t0))
            timings.append(("fuse", t2 - t1))
        est.append(T.copy())
    return M, np.stack(est)
