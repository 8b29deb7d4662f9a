"""AIRG reduction multigrid on MI355X (gfx950): HIP kernels behind a C ABI
(libairg.so, include/airg.h) and a thin ctypes binding (airg.py)."""
