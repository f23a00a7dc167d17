"""MI355X (gfx950) CP-APR MU: the Phi(n) hot path as hand-written HIP behind a C ABI.

Submodules: ``cpapr`` (ctypes binding of libcpapr.so, same names as the C
entry points), ``synth`` (seeded synthetic inputs), ``build`` (hipcc build of
the library). Importing the package loads nothing; the library is loaded on
first use and its absence is an error.
"""
__all__ = ["cpapr", "synth", "build"]
