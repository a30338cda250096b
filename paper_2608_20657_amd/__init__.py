"""MI355X-native symmetry-adapted HEOM (hot path of arXiv 2608.20657).

Submodules:
  workloads -- seeded synthetic inputs (shared with the test oracle)
  heom      -- ctypes binding of libheom.so (imported on demand; raises
               ImportError if the library has not been built)
  build     -- compiles libheom.so for gfx950
"""
