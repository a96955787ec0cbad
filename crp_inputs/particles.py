"""Seeded particle lists: all start at the origin with isotropic directions.

The paper's sources emit isotropically (section 4) and the cosmic-ray particle
carries position, direction, energy, charge and mass (section 3.1).  Energies
are log-uniform over each workload's range; charges are drawn uniformly from
the workload's set of nuclei (H, He, N, Fe as in section 4).
"""
from __future__ import annotations

import numpy as np

from .configs import Workload


def _draw(rng: np.random.Generator, n: int, e_min: float, e_max: float, charges):
    u1 = rng.random(n)
    u2 = rng.random(n)
    ue = rng.random(n)
    zi = rng.integers(0, len(charges), size=n)
    cz = 2.0 * u1 - 1.0
    phi = 2.0 * np.pi * u2
    s = np.sqrt(np.maximum(0.0, 1.0 - cz * cz))
    u = np.stack([s * np.cos(phi), s * np.sin(phi), cz], axis=1)
    a = np.log10(e_min)
    b = np.log10(e_max)
    energy = 10.0 ** (a + (b - a) * ue)
    if e_min == e_max:
        energy[:] = e_min
    charge = np.asarray(charges, dtype=np.int32)[zi]
    return u, energy, charge


def isotropic_particles(n: int, e_min: float, e_max: float, charges, seed,
                        charge_rule: str = "uniform") -> dict:
    """Return a dict of numpy arrays for n particles starting at the origin.

    Keys: pos (n,3) float64 Mpc, dir (n,3) unit vectors, energy (n,) eV,
    charge (n,) int32, mass (n,) int32.
    ``charge_rule='alternate'`` sets charges[i] = charges[i % len(charges)].
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    u, energy, charge = _draw(rng, n, e_min, e_max, charges)
    if charge_rule == "alternate":
        charge = np.asarray(charges, dtype=np.int32)[np.arange(n) % len(charges)]
    elif charge_rule != "uniform":
        raise ValueError(charge_rule)
    return {
        "pos": np.zeros((n, 3), dtype=np.float64),
        "dir": u,
        "energy": energy,
        "charge": charge.astype(np.int32),
        "mass": _mass_vec(charge),
    }


def box_positions(n: int, lo, hi, seed) -> np.ndarray:
    """n start positions (Mpc) drawn uniformly in the box [lo, hi] (per axis)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    return lo + (hi - lo) * rng.random((n, 3))


def _mass_vec(charge: np.ndarray) -> np.ndarray:
    """Vectorised ``mass_number``: A = 1 for |Z| = 1, else A = 2|Z|."""
    z = np.abs(charge)
    return np.where(z == 1, 1, 2 * z).astype(np.int32)


def realisation_table(w: Workload, seed) -> dict:
    """Per-realisation parameters for a batched workload.

    B_rms = 10^(log10(b_lo) + (log10(b_hi)-log10(b_lo)) U), particle count
    round(10^(log10(c_lo) + ... U)), observer radius r_lo + (r_hi - r_lo) U.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    m = w.n_realisations
    ub = rng.random(m)
    uc = rng.random(m)
    ur = rng.random(m)
    lb0, lb1 = np.log10(w.b_rms_range)
    lc0, lc1 = np.log10(w.count_range)
    return {
        "b_rms": 10.0 ** (lb0 + (lb1 - lb0) * ub),
        "count": np.rint(10.0 ** (lc0 + (lc1 - lc0) * uc)).astype(np.int64),
        "radius": w.radius_range[0] + (w.radius_range[1] - w.radius_range[0]) * ur,
    }


def realisation_particles(w: Workload, table: dict, seed) -> dict:
    """Concatenated particle list of all realisations, with param_index per particle."""
    counts = table["count"]
    n = int(counts.sum())
    p = isotropic_particles(n, w.e_min, w.e_max, w.charges, seed)
    p["param_index"] = np.repeat(np.arange(len(counts), dtype=np.int32), counts)
    return p
