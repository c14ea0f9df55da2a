"""Plain FP64 CPU oracle of the fluctuating lattice Boltzmann method for the
diffusion equation (Wagner & Strand, "A Fluctuating Lattice Boltzmann Method
for the Diffusion Equation", arXiv:1606.07801).

THIS PACKAGE IS TEST INFRASTRUCTURE. Only the test suite, the smoke check of
the package entry point and the CPU-baseline leg of the benchmark may import,
call or execute anything in it. The product path (the HIP library and its
Python binding) never reaches it, and it shares no code, constant, table or
helper with that path: every constant here (velocity sets, weights, moment
basis, Philox round constants, uniform/normal mappings) is derived or typed
independently.

The oracle is written for clarity, not speed: numpy arrays in float64, the
paper's steps in the paper's order and notation, one lattice at a time.

Modules
-------
lattice  velocity sets, weights and the orthonormal moment basis
         (Sec. II: equilibrium moments, D2Q5 weights, Gram-Schmidt basis)
philox   Philox4x32-10 counter-based generator (Salmon et al., SC'11) and the
         mapping of its words to uniform and Gaussian variates
step     one collision + streaming step: eq. (LB), eq. (collision) with the
         moment-space relaxation and the local / global noise variance
         eq. (xilocal) / eq. (xiglobal), negative-density rule of Sec. IV;
         lattices whose theta and rates vary by region (Sec. IV,
         non-homogeneous systems)
stats    lattice sums (mass, <f_i>, <f_i f_j>), the density structure
         factor S(k), the populations' Fourier sums, their structure factor
         S_ij(k) and the density time correlator (Sec. IV)

Parity status of each function is stated in its docstring; functions without
an independent pin say "parity unpinned".
"""

from .lattice import Lattice, make_lattice  # noqa: F401
from .philox import philox4x32_10, words_to_uniform, box_muller  # noqa: F401
from .step import (Params, collide, stream, step, run, noise_draws, step_sites, run_sites, run_box,  # noqa: F401
                   step_regions, run_regions)
from .stats import (lattice_sums, structure_factor, density, population_amplitudes, correlate,  # noqa: F401
                    profile)
