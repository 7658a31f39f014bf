"""MI355X (gfx950) library for the bias-force hot path of adaptive biasing
potentials (arXiv:1609.09833): collective variables, direct and gridded hill
sums, the mABP transform and chain-rule forces.

Submodules:
  abp        - Python binding of libabp.so (C-ABI in include/abp.h); loading it
               requires the built library and raises if it is missing.
  workloads  - seeded synthetic inputs (no arithmetic of the method).
  build      - in-tree hipcc build of libabp.so.
  serving    - binding of the continuous-batching server in libabp.so.
"""
