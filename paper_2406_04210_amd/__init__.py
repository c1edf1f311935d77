"""MI355X-native truncated Lennard-Jones MD hot path.

Submodules (imported explicitly, so that the input generators can be used
without loading the GPU library):
  * ``paper_2406_04210_amd.ljmd``      -- ctypes binding of the HIP/gfx950 C-ABI
                                          library ``libljmd.so``
  * ``paper_2406_04210_amd.workloads`` -- seeded synthetic inputs (no method
                                          arithmetic)
"""
