"""MI355X (gfx950) hot path of the SVD-decomposed spatial-aware 2D-LUT image enhancer.

All computation runs in the HIP library libsvdlut.so (C ABI in include/svdlut.h); this
package only marshals torch device tensors and the current stream into it.  Importing the
package loads the library and fails if it has not been built.
"""
from ._lib import SvdlutError, load as _load_lib

_load_lib()

from .ops import apply, apply_autograd, deterministic, apply_loss_bwd, loss_bwd_workspace, apply_grid, apply_grid_bwd, apply_bwd, bwd_workspace, grid_bwd_workspace, loss, lut1d_apply, lut3d_apply, reconstruct, unfused_apply  # noqa: E402
from .plan import Plan, pack_offsets  # noqa: E402

__all__ = ["apply", "apply_autograd", "deterministic", "apply_loss_bwd", "loss_bwd_workspace", "apply_grid", "apply_grid_bwd", "apply_bwd", "bwd_workspace", "grid_bwd_workspace", "loss", "lut1d_apply", "lut3d_apply", "reconstruct", "unfused_apply", "Plan",
           "pack_offsets", "SvdlutError"]
