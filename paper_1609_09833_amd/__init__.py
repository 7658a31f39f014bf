"""MI355X (gfx950) library for the bias-force hot path of adaptive biasing
potentials (arXiv:1609.09833): collective variables, direct and gridded hill
sums, the mABP transform and chain-rule forces, and a continuous-batching
server of bias-force requests.

Submodules:
  abp        - Python binding of libabp.so (C-ABI in include/abp.h), including
               the server (abp.Server); loading it requires the built library
               and raises if it is missing.
  workloads  - seeded synthetic inputs (no arithmetic of the method).
  build      - in-tree build of libabp.so (hipcc) and of the example serving
               load generator (g++).
  examples   - clients of the C-ABI that are not part of the library: a plain
               C client and the serving load generator with its binding.
"""
