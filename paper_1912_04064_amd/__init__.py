"""MI355X-native SDMD particle-in-cell step (Derouillat & Beck, "Single Domain
Multiple Decompositions for Particle-in-Cell simulations").

The compute path is the HIP library ``libsdmd.so`` built from ``csrc/`` for
gfx950, reached through the C ABI declared in ``include/sdmd_pic.h``;
:mod:`.binding` is its thin Python binding.  :mod:`.workloads` draws seeded
synthetic initial states.  Importing this package loads nothing: the library
is opened on first use of the binding.
"""

__all__ = ["binding", "workloads"]
