"""MI355X-native Gradient-SDF tracking and fusion (Sommer et al., CVPR 2022).

The hot path runs in hand-written HIP kernels for gfx950 behind the C ABI
declared in ``include/gsdf.h``; ``gsdf`` is its thin torch-facing binding
and ``synth`` makes seeded synthetic depth streams.
"""
__all__ = ["gsdf", "synth", "build"]
