"""Seed tree for every synthetic input.

One root ``SeedSequence(14105323)`` (the arXiv number of the paper) spawns one
child per workload; each child spawns three streams: field, particles and
realisation parameters (the modulated workload draws its modulation grid from
the third).  A child depends only on its index, not on how many children are
spawned.  ``SeedSequence.spawn`` is stateful, so the tree is rebuilt from the
root on every call to keep results reproducible.
"""
import numpy as np

ROOT_SEED = 14105323
N_WORKLOADS = 6


def config_seeds(index: int):
    """Return (field, particles, realisations) seed sequences for workload ``index``."""
    if not 0 <= index < N_WORKLOADS:
        raise ValueError(f"workload index {index} out of range")
    child = np.random.SeedSequence(ROOT_SEED).spawn(N_WORKLOADS)[index]
    field_ss, particle_ss, real_ss = child.spawn(3)
    return field_ss, particle_ss, real_ss
