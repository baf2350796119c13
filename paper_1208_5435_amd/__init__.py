"""MI355X-native matrix-free interior point solver for l1-regularised least
squares: HIP kernels for gfx950 behind a C ABI (include/mfipm.h), a ctypes
binding (`mfipm`) and an autograd wrapper (`autograd`)."""
from .mfipm import (OP_DENSE, OP_PDCT, OP_PDST, OP_WHT, STATUS, MfipmError, Solver, default_params,  # noqa: F401
                    load_library)
