"""MI355X (gfx950) randomized unpivoted QLP: the HIP library and its binding.

The compute path lives in librqlp.so (csrc/, C ABI in include/rqlp.h); the
Python module `rqlp` only marshals arguments.  Build with
`python -m paper_2209_12464_amd.build`.
"""
