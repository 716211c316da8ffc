"""MI355X (gfx950) implementation of the ionization-seeded direct laser
acceleration Monte Carlo of arXiv 2509.01741: neon atoms sampled over the
focal volume of a radially polarized focus, field-ionized state by state with
a tunnelling rate, every electron pushed from rest by the Newton-Lorentz
equations, final energies and angles binned forward / backward.

Modules:
  binding    -- ctypes binding of the C ABI (include/rpdla.h); torch tensors
                carry device memory and streams.  Importing it loads
                librpdla.so and fails loudly if it is not built.
  pipeline   -- the whole hot path for one workload on the GPU.
  workloads  -- seeded synthetic workload parameters.
  build      -- hipcc build of librpdla.so.
"""
__version__ = "0.1.0"
