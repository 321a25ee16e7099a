"""GLS map-making on MI355X: P, P^T, N^-1 and the PCG solve of
(P^T N^-1 P) m = P^T N^-1 d as hand-written HIP kernels behind a C ABI.

The C library (``libmapmaker.so``) is loaded lazily by ``binding``; importing
this package does not touch the GPU.
"""
__all__ = ["synth", "binding"]
