"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package draws inputs only: Gaussian-blob images and densities, smooth
random-Fourier velocity fields, random directions, and the workload
descriptions (grid sizes, step counts, regularisation weights, seeds).  It
holds none of the registration method's arithmetic, so both the FP64 oracle
and the GPU path can take their inputs from here without sharing any of the
computation that is being checked.
"""

from .generators import blob_image, fourier_velocity, random_direction, cell_centres
from .workloads import Workload, WORKLOADS, workload

__all__ = [
    "blob_image",
    "fourier_velocity",
    "random_direction",
    "cell_centres",
    "Workload",
    "WORKLOADS",
    "workload",
]
