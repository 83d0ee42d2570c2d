"""Plain FP64 CPU oracle of the D2Q9 pseudopotential MRT lattice Boltzmann
timestep of Shan et al. (arXiv:1605.01800), plus the coexistence solvers of
Eqs. 9 and 11.

TEST INFRASTRUCTURE ONLY: the slow, obviously correct reference that the GPU
library is checked against.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import it.  It shares no code with the GPU
library, and nothing in the library imports it.

Modules:
  stepper     -- ctypes binding of lbm_oracle.c (Eqs. 3-8, 13-16, streaming)
  coexist     -- critical point of Eq. 15, Maxwell rule (Eq. 11), mechanical
                 stability condition (Eq. 9), in mpmath
  diagnostics -- bubble radius, pressure jump, slab densities from rho fields

Parity unpinned: the bubble-radius definition and the wall-pressure peak have
no value in the paper to check against; only their agreement with the GPU path
is tested.  The mirror reading of the pseudopotential at solid wall sites is
likewise not in the paper; it is pinned only through the symmetry it implies
(for states uniform in x and at rest, each wall is a plane of mirror symmetry
of the periodic channel twice as tall).
"""
