"""Oracle for the immersed-boundary hot path: plain, slow, obviously correct.

TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the CPU-baseline
leg of the benchmark may import, call, link or execute anything under this
directory.  It shares no code with the HIP path and never imports it.

  tag_exact.c  - exact-predicate fluid/ghost tagging (C, built with gcc)
  tagging.py   - ctypes wrapper of tag_exact.c
  flow.py      - FP64 numpy time step: stencils, CSM, predictor, Poisson, projection, forces
  cnn.py       - FP64 3-D convolution network forward/backward, flexible CG

Parity pins for every function live in tests/ (marked "not gpu").
"""
