"""MI355X-native semi-discrete SE(2,N) hypoelliptic diffusion inpainting.

``paper_1304_2062_amd.se2n`` binds the gfx950 library (libse2n.so, built by
``python -m paper_1304_2062_amd.build``); ``paper_1304_2062_amd.synth`` draws
the seeded synthetic inputs.
"""
__all__ = ["se2n", "synth", "build"]
