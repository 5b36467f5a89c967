"""MI355X (gfx950) Parareal / projection Navier-Stokes hot path.

Submodules: ``nsp`` (binding of libnsp.so, the C ABI in include/nsp.h),
``inputs`` (seeded synthetic workloads), ``build`` (hipcc build of libnsp.so).
Importing the package loads nothing; ``nsp.lib()`` loads the HIP library.
"""
