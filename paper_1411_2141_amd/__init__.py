"""MI355X-native mesh-based image registration (arXiv:1411.2141).

The hot path lives in ``libmeshreg.so`` (HIP kernels for gfx950 plus the host
pre-computation behind the C ABI of ``include/meshreg.h``).  Importing this
package loads that library and fails if it has not been built
(``python -m paper_1411_2141_amd.build``); there is no fallback path.
"""
# torch first: it carries its own HIP runtime, and the library must bind to
# that same runtime (loaded first, the library would pull in the system's,
# and the process would hold two runtimes that do not share devices, streams
# or memory)
import torch  # noqa: F401,E402

from . import binding  # noqa: E402
from .binding import MeshRegError, load_library  # noqa: E402

load_library()

from .registration import MeshReg  # noqa: E402
from .autograd import MeshRegUnrolled, unrolled_msd  # noqa: E402

__all__ = ["binding", "MeshReg", "MeshRegError", "MeshRegUnrolled", "load_library",
           "unrolled_msd"]
