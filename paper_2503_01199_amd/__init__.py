"""MI355X-native differentiable tile-based Gaussian rasterizer (LiteGS hot path).

Every step of the path runs in hand-written HIP kernels for gfx950 behind the C ABI
declared in ``include/gsr.h`` (``libgsr.so``). This package is the thin Python
binding: argument marshalling, the ``torch.autograd.Function`` and the render
server. Importing it does not load the library; the first call does, and fails
loudly if the library has not been built.
"""
__all__ = ["scenes"]
