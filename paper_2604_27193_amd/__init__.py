"""MI355X-native Monte Carlo evaluation of emergency braking under uncertainty.

The compute path is a C-ABI shared library of hand-written HIP kernels for
gfx950 (``csrc/``, declared in ``include/aeb.h``); ``binding`` marshals
arguments to it.  ``workloads`` builds seeded synthetic scenario inputs.
"""
