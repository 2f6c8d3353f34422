"""Seeded synthetic inputs for the L-ACE exchange path.

This package only draws inputs: plane-wave Miller indices, orbital
coefficients, localized-orbital centres and widths, arrival times.  It holds
none of the exchange arithmetic, and both the CPU oracle and the GPU path
consume what it produces.
"""
from .generators import (  # noqa: F401
    WORKLOADS,
    BATCH_CLASSES,
    rng_for,
    miller_sphere,
    random_orbitals,
    gaussian_orbitals,
    virtual_orbitals,
    make_inputs,
    make_batch_cells,
    perturb_gaussian_params,
    gaussian_params,
    orbitals_from_params,
    poisson_arrivals,
    serving_classes,
    serving_stream,
    SERVE_RATE,
    SERVE_STEPS,
)
