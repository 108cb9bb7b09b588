"""MI355X-native CB-ESSFM digital backpropagation (hand-written HIP for gfx950).

The operation and its C ABI are described in ``include/cbessfm.h``.  This
package is a thin binding: PyTorch provides device memory and streams, the
library ``libcbessfm.so`` (built in-tree by ``paper_2409_14489_amd.build``)
does all of the arithmetic.
"""
from .plan import LinkSpec, Plan, analytic_coeffs, plan_check  # noqa: F401
from ._lib import CbessfmError, EXPORTED, LIB_PATH  # noqa: F401
