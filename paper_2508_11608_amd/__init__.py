"""CutFEM vertex-patch multigrid for AMD MI355X (gfx950).

The hot path (matrix-free Nitsche + ghost-penalty operator, coloured
multiplicative vertex-patch smoother, transfers, coarse solve, V-cycle, CG)
runs in hand-written HIP kernels behind the C ABI of include/cutmg.h; this
package is its thin Python binding.
"""
from .cutmg import EXPORTED, LIBRARY_PATH, CutmgError, Group, Problem, Server, footprint, load_library

__all__ = ["Problem", "Group", "Server", "CutmgError", "footprint", "load_library", "LIBRARY_PATH", "EXPORTED"]
