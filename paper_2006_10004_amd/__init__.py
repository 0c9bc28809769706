"""MI355X-native spectral total-variation decomposition (arXiv 2006.10004).

The decomposition runs in the HIP library libtvspec.so behind the C ABI of
include/tvspec.h and include/tvspec_nn.h.  Submodules:

  paper_2006_10004_amd.tvspec     ctypes binding of include/tvspec.h (loads the library)
  paper_2006_10004_amd.nn         ctypes binding of include/tvspec_nn.h (the surrogate network)
  paper_2006_10004_amd.surrogate  surrogate training data, training loop and serving
  paper_2006_10004_amd.synth      seeded synthetic shape images (pure numpy)
  paper_2006_10004_amd.build      builds libtvspec.so for gfx950

Nothing is imported here, so ``synth`` can be used without loading the
library.
"""
