"""Open-rectangular-pipe Poisson solver (Ryne, arXiv:1111.4971) for AMD MI355X.

The solver itself lives in libpipe.so (HIP kernels for gfx950 behind the C ABI
of include/pipe_poisson.h); ``paper_1111_4971_amd.pipe`` is its Python binding
and ``paper_1111_4971_amd.workloads`` holds the seeded synthetic inputs.
Importing the package loads nothing; the binding loads the library on first use.
"""
