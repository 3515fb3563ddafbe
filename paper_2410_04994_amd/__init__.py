"""MI355X-native split-step Fourier march of the coupled SHG equations.

The compute path is the HIP library libshg.so (C ABI: include/shg.h); this
package holds its build script, a ctypes binding, the GPU input-beam builder,
the autograd wrapper of the hand-written adjoint, and the batch autotuner.
"""
from .binding import (Plan, ShgError, load_library, propagate_batch, batch_workspace_bytes,  # noqa: F401
                      SHG_UNDEPLETED, SHG_NO_GRAPH)

__all__ = ["Plan", "ShgError", "load_library", "propagate_batch", "batch_workspace_bytes",
           "SHG_UNDEPLETED", "SHG_NO_GRAPH"]
