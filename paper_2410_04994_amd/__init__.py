"""MI355X-native split-step Fourier march of the coupled SHG equations.

The compute path is the HIP library libshg.so (C ABI: include/shg.h); this
package holds its build script, a ctypes binding (march, adjoint, batch, heat
equation and the self-consistent loop), the GPU input-beam builder, the
autograd wrapper of the hand-written adjoint, and the batch autotuner.
"""
from .binding import (Plan, ShgError, Thermal, load_library, propagate_batch,  # noqa: F401
                      batch_workspace_bytes, self_consistent, SHG_UNDEPLETED, SHG_NO_GRAPH)

__all__ = ["Plan", "ShgError", "Thermal", "load_library", "propagate_batch", "batch_workspace_bytes",
           "self_consistent", "SHG_UNDEPLETED", "SHG_NO_GRAPH"]
