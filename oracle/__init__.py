"""CPU oracle of the CB-ESSFM hot path (FP64).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py``, never by the product package.
It shares no code with the HIP path.
"""
from .cbessfm import OraclePlan, run, run_blocks, process_block, dft_bruteforce, zero_coeffs  # noqa: F401
from .coeffs import Link, dbp_coefficients, physical_coefficients, kernel, kernel_eq22  # noqa: F401
from .tied import expand as tied_expand, expand_adjoint as tied_expand_adjoint  # noqa: F401
from .tied import step_weights, tied_half_taps, ssfm_start  # noqa: F401
from . import complexity  # noqa: F401
