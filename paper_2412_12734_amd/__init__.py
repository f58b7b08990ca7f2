"""MI355X rasterizer for textured 2D Gaussian splats (Gaussian Billboards).

The compute path is the HIP library ``libgbb.so`` behind the C ABI in include/gbb.h; this
package only marshals arguments (``_lib``) and wires torch memory, streams and autograd to it
(``render``).
"""
from ._lib import GbbError, load  # noqa: F401
from .render import Options, Rasterizer, Splats, render  # noqa: F401
