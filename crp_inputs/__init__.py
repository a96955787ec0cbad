"""Seeded synthetic inputs shared by the GPU path, the oracle and the benchmark.

This package holds input generation only: turbulent field realisations,
particle lists and the workload table.  It contains none of the propagation
arithmetic (no integrator, interpolation, step control or stop logic), so the
oracle and the HIP path can both consume its arrays without sharing method code.

Workloads follow the example application of the paper (section 4): a regular
vector grid filled with a random Kolmogorov turbulent realisation, and a
mixed composition of H, He, N and Fe nuclei (section 4, text after Eq. (1)).
"""
from .configs import CONFIGS, Workload, get_config, mass_number
from .kolmogorov import kolmogorov_field, coherence_length, spectral_mask
from .modulation import lognormal_modulation
from .particles import box_positions, isotropic_particles, realisation_table, realisation_particles
from .quantize import round_to_bf16, round_to_f16
from .seeds import config_seeds, position_seed

__all__ = [
    "CONFIGS", "Workload", "get_config", "mass_number",
    "kolmogorov_field", "coherence_length", "spectral_mask", "lognormal_modulation",
    "box_positions", "isotropic_particles", "realisation_table", "realisation_particles",
    "config_seeds", "position_seed", "round_to_f16", "round_to_bf16",
]
