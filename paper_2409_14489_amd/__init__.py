"""MI355X-native CB-ESSFM digital backpropagation (hand-written HIP for gfx950).

The operation and its C ABI are described in ``include/cbessfm.h``.  This
package is a thin binding: PyTorch provides device memory and streams, the
library ``libcbessfm.so`` (built in-tree by ``paper_2409_14489_amd.build``)
does all of the arithmetic.  The public names are resolved on first use, so
the build module can be imported before the library exists; using any of
them without the library raises ImportError.
"""
_PUBLIC = {
    "LinkSpec": "plan", "Plan": "plan", "analytic_coeffs": "plan", "plan_check": "plan",
    "CbessfmError": "_lib", "EXPORTED": "_lib", "LIB_PATH": "_lib",
    "CBESSFMFunction": "autograd", "cbessfm": "autograd", "cbessfm_steps": "autograd",
    "Batch": "batch", "schedule": "batch", "autotune": "batch",
    "tie": "tied", "tie_expand": "tied", "tie_reduce": "tied", "fit_tied": "tied", "step_weights": "tied",
    "tied_half_taps": "tied", "ssfm_start": "tied", "analytic_rows": "tied", "tied_coeffs": "tied",
    "complexity": "baselines", "run_method": "baselines",
}

__all__ = sorted(_PUBLIC)


def __getattr__(name):
    mod = _PUBLIC.get(name)
    if mod is None:
        raise AttributeError(f"module {__name__!r} has no attribute {name!r}")
    import importlib
    return getattr(importlib.import_module(f"{__name__}.{mod}"), name)
