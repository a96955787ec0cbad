"""Seed tree for every synthetic input.

One root ``SeedSequence(14105323)`` (the arXiv number of the paper) spawns one
child per workload; each child spawns four streams: field, particles, realisation parameters
(the modulated workloads draw their modulation grid from the third) and start
positions (workloads whose particles start spread over a box).  A child depends only on its index, not on how many children are
spawned.  ``SeedSequence.spawn`` is stateful, so the tree is rebuilt from the
root on every call to keep results reproducible.
"""
import numpy as np

ROOT_SEED = 14105323
N_WORKLOADS = 8


def config_seeds(index: int):
    """Return (field, particles, realisations) seed sequences for workload ``index``."""
    if not 0 <= index < N_WORKLOADS:
        raise ValueError(f"workload index {index} out of range")
    child = np.random.SeedSequence(ROOT_SEED).spawn(N_WORKLOADS)[index]
    field_ss, particle_ss, real_ss = child.spawn(3)
    return field_ss, particle_ss, real_ss


def position_seed(index: int):
    """Seed sequence of the start positions of workload ``index`` (the fourth
    stream of its child; the first three are those of ``config_seeds``)."""
    if not 0 <= index < N_WORKLOADS:
        raise ValueError(f"workload index {index} out of range")
    return np.random.SeedSequence(ROOT_SEED).spawn(N_WORKLOADS)[index].spawn(4)[3]
