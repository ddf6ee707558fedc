"""The C ABI: the built library loads without a GPU and exports every entry
point that include/gsdf.h declares; host-side argument checks work without
launching anything."""
import ctypes as C
import os
import re


ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gsdf.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gsdf_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_hot_path():
    names = _declared()
    for n in ("gsdf_allocate_blocks", "gsdf_integrate_frame", "gsdf_track_frame",
              "gsdf_normal_equations", "gsdf_export_keys", "gsdf_map_buffer_sizes"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2111_13652_amd import _lib
    lib = _lib.load()
    for n in _declared():
        assert hasattr(lib, n), n
    # the binding covers the same set
    assert set(_lib.exported_symbols()) == set(_declared())


def test_host_side_validation_without_gpu():
    from paper_2111_13652_amd import _lib
    lib = _lib.load()
    d = _lib.MapDesc()
    d.voxel_size, d.truncation, d.storage = 0.01, 0.05, 0
    d.hash_slots, d.max_blocks = 1 << 16, 20000
    sizes = (C.c_size_t * 4)()
    assert lib.gsdf_map_buffer_sizes(C.byref(d), C.byref(sizes)) == 0
    assert sizes[0] == (1 << 16) * 16 and sizes[1] == 20000 * 512 * 16 and sizes[2] == 20000 * 512 * 4
    d.storage = 1
    assert lib.gsdf_map_buffer_sizes(C.byref(d), C.byref(sizes)) == 0
    assert sizes[1] == 20000 * 512 * 8
    d.hash_slots = 3 * 10000  # not a power of two
    assert lib.gsdf_map_buffer_sizes(C.byref(d), C.byref(sizes)) == _lib.EINVAL
    d.hash_slots, d.truncation = 1 << 16, 0.001  # truncation below the voxel size
    assert lib.gsdf_map_buffer_sizes(C.byref(d), C.byref(sizes)) == _lib.EINVAL
    # null map / camera pointers are rejected before any launch
    cam = _lib.Camera(525.0, 525.0, 319.5, 239.5, 640, 480, 0.4, 4.0)
    assert lib.gsdf_allocate_blocks(None, None, C.byref(cam), None, None, None) == _lib.EINVAL
    assert lib.gsdf_track_scratch_bytes(C.byref(cam), 3) > 0
    assert lib.gsdf_track_scratch_bytes(C.byref(cam), 5) == 0
    assert lib.gsdf_integrate_scratch_bytes(C.byref(cam)) >= 640 * 480 * 16
    assert lib.gsdf_status_string(_lib.ECAPACITY) == b"hash table or block pool full"


def test_batched_gauss_newton_validates_without_gpu():
    """gsdf_gn_scratch_bytes: a float64 partial of 32 words per work-group
    and keyframe, a work-group per 4096 pixels (at least 1, at most 2048),
    rounded up to 256 bytes; 0 for K outside 1..65535.  gsdf_gn_step_keyframes
    refuses null buffers and bad parameters before any launch."""
    from paper_2111_13652_amd import _lib
    lib = _lib.load()
    cam = _lib.Camera(525.0, 525.0, 319.5, 239.5, 640, 480, 0.4, 4.0)
    groups = -(-640 * 480 // 4096)
    assert lib.gsdf_gn_scratch_bytes(C.byref(cam), 30) == -(-30 * groups * 32 * 8 // 256) * 256
    assert lib.gsdf_gn_scratch_bytes(C.byref(cam), 1) == -(-groups * 32 * 8 // 256) * 256
    assert lib.gsdf_gn_scratch_bytes(C.byref(cam), 0) == 0
    assert lib.gsdf_gn_scratch_bytes(C.byref(cam), 65536) == 0
    assert lib.gsdf_gn_scratch_bytes(None, 1) == 0
    tiny = _lib.Camera(100.0, 100.0, 3.5, 3.5, 8, 8, 0.4, 4.0)
    assert lib.gsdf_gn_scratch_bytes(C.byref(tiny), 2) == 2 * 1 * 32 * 8
    big = _lib.Camera(1000.0, 1000.0, 1023.5, 1023.5, 2048, 2048, 0.4, 4.0)
    assert lib.gsdf_gn_scratch_bytes(C.byref(big), 1) == 1024 * 32 * 8
    huge = _lib.Camera(1000.0, 1000.0, 2047.5, 2047.5, 4096, 4096, 0.4, 4.0)
    assert lib.gsdf_gn_scratch_bytes(C.byref(huge), 1) == 2048 * 32 * 8
    assert lib.gsdf_gn_step_keyframes(None, None, 1, C.byref(cam), None, 0.01, 1e-6, 0.1, None, 0, None,
                                      None) == _lib.EINVAL


def test_voxel_order_and_differentiable_calls_validate_without_gpu():
    import numpy as np
    from paper_2111_13652_amd import _lib
    lib = _lib.load()
    order = np.zeros(512, np.int32)
    assert lib.gsdf_voxel_order(order.ctypes.data_as(C.c_void_p)) == 0
    assert sorted(order.tolist()) == list(range(512))
    # every 2x2x2 sub-cube occupies 8 consecutive indices
    c = np.arange(512)
    lx, ly, lz = c % 8, (c // 8) % 8, c // 64
    cube = (lx // 2) + 4 * (ly // 2) + 16 * (lz // 2)
    for k in range(64):
        idx = np.sort(order[cube == k])
        assert idx[-1] - idx[0] == 7
    cam = _lib.Camera(525.0, 525.0, 319.5, 239.5, 640, 480, 0.4, 4.0)
    assert lib.gsdf_keyframe_scratch_bytes(C.byref(cam), 10, 40000) > lib.gsdf_keyframe_scratch_bytes(
        C.byref(cam), 10, 100) > 0
    assert lib.gsdf_keyframe_scratch_bytes(C.byref(cam), 0, 100) == 0
    assert lib.gsdf_keyframe_scratch_bytes(C.byref(cam), 10, -1) == 0
    # pixels are numbered in int32: K x W x H beyond INT32_MAX is refused
    assert lib.gsdf_keyframe_scratch_bytes(C.byref(cam), 7000, 100) == 0
    assert lib.gsdf_keyframe_loss(None, None, 1, C.byref(cam), None, None, None, 0, 0.01, None, 0, None,
                                  None, None, 0, None) == _lib.EINVAL
    assert lib.gsdf_backward(None, None, 1, C.byref(cam), None, None, None, 0, 0.01, None, 0, None,
                                      None, None, None, None, 0, None) == _lib.EINVAL
    assert lib.gsdf_compose_poses(-1, None, None, None, None) == _lib.EINVAL
    assert lib.gsdf_compose_poses(0, None, None, None, None) == _lib.OK
