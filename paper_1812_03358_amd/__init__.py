"""MI355X-native light-transport camera model (arXiv 1812.03358).

Submodules:
  ltm        -- ctypes binding of libltm.so (project, backproject, solver)
  workloads  -- seeded synthetic volumes, noise and camera descriptions
  build      -- compiles libltm.so for gfx950
Nothing is imported eagerly, so the generators can be used without a GPU.
"""
