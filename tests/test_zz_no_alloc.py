"""gsdf_track_frame_noalloc (tracking on the library's fixed scratch array,
for callers that cannot allocate) through the C ABI against
gsdf_track_frame with a caller scratch: two calls in a row, the second on a
smaller image, each bit-identical to the scratch-argument call.  Needs an
MI355X."""
import ctypes as C

import pytest

from paper_2111_13652_amd import synth
from tests.gpu_helpers import dev, log

pytestmark = pytest.mark.gpu

ROOM = synth.CONFIG_ROOM


def _noalloc(G, depth, cam, init, out, levels, iters):
    import torch
    from paper_2111_13652_amd import _lib
    from paper_2111_13652_amd.gsdf import camera
    c = camera(cam)
    it = list(iters) + [0] * (4 - len(iters))
    p = _lib.TrackParams(int(levels), (C.c_int32 * 4)(*it[:4]), 0.01, 1e-6, 0.1, 0, 0)
    stats = torch.zeros(2 * sum(it), dtype=torch.float32, device="cuda")
    rc = _lib.load().gsdf_track_frame_noalloc(
        C.byref(G._map), C.c_void_p(depth.data_ptr()), C.byref(c), C.byref(p), C.c_void_p(init.data_ptr()),
        C.c_void_p(out.data_ptr()), C.c_void_p(stats.data_ptr()), C.c_void_p(G.status.data_ptr()),
        C.c_void_p(torch.cuda.current_stream().cuda_stream))
    _lib.check(rc, "track_frame_noalloc")
    return stats


def test_noalloc_tracking_matches_scratch_tracking_twice():
    import torch
    from paper_2111_13652_amd import _lib
    from paper_2111_13652_amd.gsdf import GsdfMap
    st = synth.make_stream(ROOM["cam"], 4, 1, 2, 3)
    G = GsdfMap(ROOM["voxel_size"], ROOM["truncation"], 60000)
    for f in range(3):
        G.fuse(dev(st.depth[f]), st.cam, dev(st.poses[f]))
    small = synth.Camera(262.5, 262.5, 159.5, 119.5, 320, 240, 0.4, 4.0)
    d_small = synth.to_depth_image(synth.render_depth(st.scene, small, st.poses[3]), small)
    lib = _lib.load()
    cases = [("640x480, 3 levels", st.cam, st.depth[3], 3, (4, 5, 10)),
             ("320x240, 2 levels", small, d_small, 2, (5, 10))]
    for name, cam, d, levels, iters in cases:
        from paper_2111_13652_amd.gsdf import camera
        need = lib.gsdf_track_scratch_bytes(C.byref(camera(cam)), levels)
        assert 0 < need <= lib.gsdf_track_noalloc_max_bytes()
        log(f"case: no-alloc tracking, {name}")
        D = dev(d)
        init = dev(st.poses[2].copy())
        ref = torch.zeros_like(init)
        ref_stats = torch.zeros(2 * sum(iters), dtype=torch.float32, device="cuda")
        G.track(D, cam, ref, levels=levels, iters=iters, init=init, stats=ref_stats)
        out = torch.zeros_like(init)
        stats = _noalloc(G, D, cam, init, out, levels, iters)
        torch.cuda.synchronize()
        log(f"  max |pose difference| {(out - ref).abs().max().item():.3e}")
        assert G.status_flags() == []
        assert torch.equal(out, ref)
        assert torch.equal(stats, ref_stats)
    # a camera whose scratch exceeds the fixed array is rejected on the host
    huge = _lib.Camera(2000.0, 2000.0, 4095.5, 4095.5, 8192, 8192, 0.4, 4.0)
    p = _lib.TrackParams(3, (C.c_int32 * 4)(4, 5, 10, 0), 0.01, 1e-6, 0.1, 0, 0)
    assert lib.gsdf_track_frame_noalloc(C.byref(G._map), C.c_void_p(1), C.byref(huge), C.byref(p), C.c_void_p(1),
                                        C.c_void_p(1), None, None, None) == _lib.EINVAL
