"""MI355X (gfx950) Kadanoff-Baym propagation step (arXiv 2505.19467).

Submodules:
  inputs  -- seeded synthetic workloads (parameters and random arrays only)
  build   -- hipcc build of the in-tree HIP library libkbe.so
  kbe     -- ctypes binding of the C ABI in include/kbe.h (loads libkbe.so on import)
"""
