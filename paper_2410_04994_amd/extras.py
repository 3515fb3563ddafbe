"""Secondary benchmark lines (batched sweep, forward + adjoint) reported
beside the single-instance forward march.  Each entry is filled in once the
corresponding path exists in the library."""
from __future__ import annotations


def run_all(device) -> dict:
    return {}
