"""FP64 CPU oracle of the Voxel-GPR hot path: test infrastructure only.

Only the tests, the smoke check and the bench's CPU-baseline leg may import
this package; the HIP library never does.
"""
from .vgpr_oracle import *  # noqa: F401,F403
from .vgpr_oracle import Params, VoxelMap  # noqa: F401
