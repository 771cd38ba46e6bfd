"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This package holds workload recipes (scan geometry, voxel grid) and the phantom
model (random ellipsoids / Gaussian blobs with closed-form line integrals).  It
contains none of the reconstruction method's arithmetic: no derivative, rebinning,
Hilbert filter, PI-line or backprojection code lives here.
"""
