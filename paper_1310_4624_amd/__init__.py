"""MI355X (gfx950) particle-filter step with RNA / ARNA distributed resampling
(Demirel et al., arXiv:1310.4624), behind the C interface in include/arna.h.

The HIP library is loaded on first use; importing the package does not touch
the GPU.
"""
from ._native import (PF_INIT_INFOSHARE, PF_INIT_TRACKING, PF_LIK_PATCH, PF_LIK_POINT,  # noqa: F401
                      PF_LIK_POISSON,
                      PF_MODE_ARNA, PF_MODE_RNA, PF_DEBUG_LINEAGE, PF_DEBUG_TRACE, PFError,
                      PF_LAUNCH_AUTO, PF_LAUNCH_PERSISTENT, PF_LAUNCH_STEPWISE)
from .tracker import (TRAJ_RECORD_BYTES, Batch, Tracker, nex, philox, resample_q, ring,  # noqa: F401
                      trajectory)
