"""MI355X-native topology-free immersed boundary time step (arXiv:2002.06206).

  include/ibm.h          C ABI (the boundary)
  csrc/*.hip             gfx950 kernels and the ABI implementation (libibm.so)
  ibm.py                 ctypes binding with the same names as the C ABI
  inputs.py              seeded synthetic geometries and grids
  build.py               in-tree hipcc build of libibm.so

Import ``paper_2002_06206_amd.ibm`` for the binding; it refuses to load without
the compiled library.
"""
