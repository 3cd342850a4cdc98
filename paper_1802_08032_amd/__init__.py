"""MI355X (gfx950) state-vector / density-matrix gate engine for the method of
"QuEST and High Performance Simulation of Quantum Computers" (arXiv:1802.08032).

The compute path is libqstate.so (HIP, C ABI in include/qstate.h); this
package is its thin Python binding.
"""
from .qstate import (  # noqa: F401
    C64, C128, DAMPING, DENSITY, DEPHASING, DEPOLARISING, STATEVEC, Batch, Circuit, Env,
    QStateError, Register, lib, philox_draws, prob_noalloc, reg_bytes,
)
