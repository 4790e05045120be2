"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package holds only inputs: geometries, species, molecule ids, model
hyper-parameters and random weights.  It contains none of the potential's
arithmetic (no switching function, no basis, no network), so that the FP64
oracle and the GPU path can both consume the same inputs while sharing no code
that computes the method.

Units: Angstrom, femtosecond, amu, eV.  Species are indices 0..6 in the order
H, C, N, O, F, S, Cl.
"""
from .params import ModelSpec, ani2x_like_spec, ani2x_like_ensemble, SPECIES, SPECIES_INDEX, MASSES
from .geometry import (
    Workload,
    water_cluster,
    water_box,
    organic_box,
    serving_molecule,
    serving_stream,
    workload,
    adversarial_cases,
)
from .weights import glorot_weights

__all__ = [
    "ModelSpec", "ani2x_like_spec", "ani2x_like_ensemble", "SPECIES", "SPECIES_INDEX", "MASSES",
    "Workload", "water_cluster", "water_box", "organic_box", "serving_molecule",
    "serving_stream", "workload", "adversarial_cases", "glorot_weights",
]
