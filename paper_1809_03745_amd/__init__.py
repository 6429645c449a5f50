"""MI355X-native embedded-boundary geometric-multigrid elliptic solver.

The library (libebmg.so: host C++ setup + HIP kernels for gfx950) is reached
through ``paper_1809_03745_amd.ebmg`` (ctypes). Importing the package itself
loads nothing; import ``ebmg`` to load the library.
"""
