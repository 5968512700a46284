"""MI355X-native local noise filter for 3D CT volumes.

Tan Jerome et al., "Real-time Local Noise Filter in 3D Visualization of CT
Data": each voxel is replaced by the average of nine "average clusters" (cubic
sub-regions of side 2r+1 on the voxel and its eight diagonal neighbours), with
an Otsu-threshold noise gate.  The computation runs in hand-written HIP kernels
for gfx950 behind the C ABI of include/lnf.h; this package holds the ctypes
binding (`_lib`), a tensor-level convenience layer (`api`) and the seeded
phantom generator (`phantom`) used by tests and benchmarks.

Importing the package loads nothing; the library is loaded on first use.
"""
from ._lib import (LNF_MEAN9, LNF_MINVAR9, LNF_RADIUS_MAX, LNF_U8, LNF_U16,  # noqa: F401
                   LnfError)

__all__ = ["LNF_MEAN9", "LNF_MINVAR9", "LNF_RADIUS_MAX", "LNF_U8", "LNF_U16", "LnfError"]
