"""MI355X-native stochastic proximal-gradient (SPGM) near-field MIMO imaging projector.

The compute path is the HIP library ``libspgm.so`` (built from ``csrc/``) behind the C-ABI
declared in ``include/spgm.h``; :mod:`.binding` marshals arguments to it and raises if the
library is missing.  :mod:`.workloads` holds the seeded synthetic input generators.
"""
__all__ = ["binding", "workloads"]
