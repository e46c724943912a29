"""MI355X-native exponential time differencing with embedded boundaries and a
level-set free boundary (HIP, gfx950, FP64).

The compute path is libetdfb.so (include/etdfb.h), built in-tree by
``paper_2209_15095_amd.build``; ``paper_2209_15095_amd.api`` is its thin
Python binding.  ``paper_2209_15095_amd.inputs`` generates seeded workloads.
Importing the package does not load the library; the first call that needs
it does, and fails loudly if it has not been built.
"""

__all__ = ["api", "inputs", "build"]
