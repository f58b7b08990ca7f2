"""FP64 CPU oracle of the textured 2D-Gaussian rasterizer (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import this package.
"""
from .gb_oracle import *  # noqa: F401,F403
from .gb_oracle import Options, RenderResult, Grads  # noqa: F401
