"""MI355X (gfx950) Abelian-Higgs lattice library: HIP kernels behind the C ABI
of include/ah.h, with a thin ctypes binding (``paper_1809_00995_amd.ah``)."""
from . import ah  # noqa: F401
from .ah import (AH_FP32, AH_FP64, AH_INIT_NONE, AH_INIT_RANDOM_PHASE,  # noqa: F401
                 AH_INIT_VACUUM, AH_KERNEL_AUTO, AH_KERNEL_PLAIN, AH_KERNEL_TILED,
                 AH_KERNEL_TILED2, AH_LAYOUT_15, AH_LAYOUT_20, AHError, Context, Obs, Params,
                 ObsRecords, alloc_planes, load_library, measure_noalloc, obs_from_bytes)
