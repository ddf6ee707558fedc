"""Small deterministic test inputs shared by the oracle pins and the GPU
parity tests.  Input generation only: no arithmetic of the method here."""
import math

import numpy as np

from paper_2111_13652_amd import synth

IDENTITY = np.hstack([np.eye(3), np.zeros((3, 1))])

SMALL_CAM = synth.Camera(131.0, 131.0, 79.5, 59.5, 160, 120, 0.4, 4.0)


def plane_depth(cam, n_cam, h):
    """Exact z-depth of the plane n . x = h (camera frame), float64."""
    rays = cam.rays()
    den = rays @ np.asarray(n_cam, np.float64)
    with np.errstate(divide="ignore"):
        z = h / den
    return np.where(den > 0, z, np.inf)


def depth_image(z, cam):
    return synth.to_depth_image(z, cam)


def box_room_scene():
    """A room with a few boxes and spheres: full-rank geometry for tracking."""
    spheres = np.array([[2.0, 2.6, 0.9, 0.35], [1.2, 2.9, 1.4, 0.25]])
    boxes = np.array([[2.6, 3.0, 0.6, 0.3, 0.25, 0.6, 0.4],
                      [1.5, 3.2, 0.4, 0.4, 0.3, 0.4, 1.1],
                      [3.1, 2.2, 1.5, 0.2, 0.3, 0.25, 0.2]])
    return synth.Scene(spheres=spheres, boxes=boxes,
                       room=np.array([[0.0, 0.0, 0.0], [4.0, 4.0, 3.0]]))


def box_room_pose():
    return synth.look_at([2.0, 1.0, 1.3], [2.2, 3.5, 0.9])


def room_frames(cam, n_frames, scene_seed=1, traj_seed=2, noise_seed=3):
    return synth.make_stream(cam, n_frames, scene_seed, traj_seed, noise_seed)


def cos75():
    return math.cos(math.radians(75.0))
