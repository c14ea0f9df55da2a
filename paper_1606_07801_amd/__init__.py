"""MI355X-native fluctuating lattice Boltzmann for the diffusion equation.

The time step runs in hand-written HIP kernels for gfx950 behind the C-ABI
library ``libflb.so`` (declared in ``include/flb.h``); this package holds the
thin ctypes binding (:mod:`.flb`), the batched ensemble engine and tuner, the
serving loop, and the seeded input generators (:mod:`.inputs`).  Importing
the package loads nothing native; the library is loaded on first use and
its absence is an error.
"""
