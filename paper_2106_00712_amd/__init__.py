"""MI355X-native batched DQMC sweeps (the data-parallel hot path of network-initialised MC).

The product is libdqmc.so (HIP kernels for gfx950 behind the C ABI of include/dqmc.h); this
package holds its sources (csrc/), the in-tree build (build.py), the ctypes binding (dqmc.py)
and the host-side tools around it (autotune.py, serving.py).
"""
from . import dqmc
from .dqmc import Batch, DqmcError, make_model, sweep_multi, workspace_bytes, chain_bytes

__all__ = ["dqmc", "Batch", "DqmcError", "make_model", "sweep_multi", "workspace_bytes",
           "chain_bytes"]
