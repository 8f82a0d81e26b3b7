"""MI355X-native (gfx950) 3D Gaussian-splatting rasterizer.

The rendering pipeline runs in hand-written HIP kernels behind the C ABI
declared in ``include/cdnasplat.h``; this package is a thin binding over it.
Importing the package does not load the native library; the first render call
does, and fails loudly if it has not been built.
"""
__all__ = ["scenes"]
