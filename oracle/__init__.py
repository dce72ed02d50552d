"""FP64 CPU reference of the differentiable Gaussian rasterizer (test infrastructure).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. The GPU library does not and must not.
"""
from .oracle import *  # noqa: F401,F403
