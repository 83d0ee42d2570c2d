"""gfx950 (MI355X) implementation of the D2Q9 pseudopotential multi-relaxation-
time lattice Boltzmann timestep of Shan et al. (arXiv:1605.01800).

  lbm      -- Python binding of liblbm.so (include/lbm.h): Sim, Batch, host helpers
  serving  -- continuous-batching request server on top of lbm.Batch
  inputs   -- the workload configurations (configs/c1 ... c5) and seeded
              synthetic inputs (bubble layouts, request traces)
  studies  -- the paper's experiments run on the GPU path
  build    -- hipcc build of liblbm.so

Submodules are imported on demand so that `inputs` and `build` work without a
GPU or a built library.
"""
