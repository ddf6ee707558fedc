"""Host-side logic of the Python binding that runs without a GPU."""
import numpy as np
import scipy.linalg as sl
import torch

from paper_2111_13652_amd import synth
from paper_2111_13652_amd.gsdf import adjoint_se3


def _hat6(x):
    r, p = x[:3], x[3:]
    M = np.zeros((4, 4))
    M[:3, :3] = [[0, -p[2], p[1]], [p[2], 0, -p[0]], [-p[1], p[0], 0]]
    M[:3, 3] = r
    return M


def test_adjoint_moves_a_camera_frame_twist_to_the_left():
    """exp((Ad(T) xi)^) T = T exp(xi^) (matrix exponential by scipy)."""
    rng = np.random.default_rng(0)
    T = np.stack([synth.look_at(rng.uniform(0, 4, 3), rng.uniform(0, 4, 3)) for _ in range(4)])
    A = adjoint_se3(torch.tensor(T)).numpy()
    for k in range(4):
        T4 = np.vstack([T[k], [0, 0, 0, 1]])
        x = rng.standard_normal(6) * 0.2
        np.testing.assert_allclose(sl.expm(_hat6(A[k] @ x)) @ T4, T4 @ sl.expm(_hat6(x)), atol=1e-12)
