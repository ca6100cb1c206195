"""MI355X-native hierarchical-simulation CVA path (HIP kernels behind a C ABI).

``hsim`` is the Python binding of libhsim.so; ``build`` compiles it for gfx950.
"""
__all__ = ["hsim", "build"]
