"""MI355X (gfx950) library for the p-multigrid solvers of the Riesz maps of the L2
de Rham complex.  The compute path is ``librz.so`` (HIP kernels behind the C ABI
of ``include/rz.h``); ``paper_2211_14284_amd.rz`` is its ctypes binding and
``paper_2211_14284_amd.build`` compiles it.
"""
