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

The paper defines neither a bubble radius nor a wall-pressure peak, so these
two outputs follow readings of this project (area-equivalent radius, maximum of
Eq. 15's pressure on the wall rows); the functions that compute them are pinned
to geometry and exact arithmetic (squares of known area, fractional sites,
clipping, nearest-centre ownership, compensated sums), while the readings
themselves have no value in the paper to check against.  The mirror reading of the pseudopotential at solid wall sites is
likewise not in the paper; it is pinned only through the symmetry it implies
(for states uniform in x and at rest, each wall is a plane of mirror symmetry
of the periodic channel twice as tall).
"""
