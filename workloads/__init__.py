"""Seeded synthetic inputs for SP2 purification runs.

This module only draws random numbers and assembles input matrices. It holds
none of the purification arithmetic, so the CPU oracle and the GPU path can
both consume the same inputs without sharing any of the method's code.

Construction (Kruchinina, Rudberg, Rubensson, sec. 5 and sec. 4.1, the dense
experiments): eigenvectors come from the QR factorisation of a matrix with
independent standard-normal entries, and a prescribed spectrum with a gap
around the Fermi level is placed on them, F = Q diag(lambda) Q^T.
"""
from .dense import (  # noqa: F401
    DenseInstance,
    random_orthogonal,
    two_band_spectrum,
    dense_instance,
    config_small,
    config_mid,
    config_metric,
    e5_instance,
    e6_instance,
    symmetric_gaussian_perturbation,
    diagonal_instance,
)
from .batch import batch_instances  # noqa: F401
