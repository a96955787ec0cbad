"""The workloads: sizes, field parameters, step limits and stops.

Values follow the workload descriptions of this project; entries marked
"chosen" fill parameters those descriptions leave open.  Lengths are in Mpc,
energies in eV, fields in nG.  A workload with ``n_realisations > 0`` is a
batch of independent field realisations, each with its own B_rms, particle
count and observer radius.
"""
from __future__ import annotations

import dataclasses
import math


def mass_number(z: int) -> int:
    """Mass number used for a charge number: A = 1 for protons, else A = 2Z.

    The mass number is carried through the state but does not enter the
    dynamics at these energies (beta = 1 to better than 1e-13).
    """
    z = abs(int(z))
    return 1 if z == 1 else 2 * z


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    index: int
    n_particles: int
    charges: tuple
    e_min: float
    e_max: float
    grid_n: int
    spacing: float
    l_min: float
    l_max: float
    b_rms: float
    grid_dtype: str          # storage dtype of the device grid: f64 | f32 | f16 | bf16
    tol: float
    h_min: float
    h_max: float
    obs_radius: float        # <= 0: no observer sphere
    max_length: float        # math.inf: no length limit
    charge_rule: str = "uniform"
    n_realisations: int = 0
    b_rms_range: tuple = (0.0, 0.0)
    count_range: tuple = (0, 0)
    radius_range: tuple = (0.0, 0.0)
    checkpoint_every: int = 0
    mod_n: int = 0               # modulation grid nodes per axis (0: no modulation)
    mod_spacing: float = 0.0     # Mpc
    mod_l_corr: float = 0.0      # correlation length of the log-normal modulation, Mpc
    mod_sigma: float = 0.0       # standard deviation of log m
    reflect_half: float = 0.0    # > 0: reflective box [-h, h]^3 (Mpc); the particles start uniformly in it
    lens_nside: int = 0          # > 0: a lens workload (backtracking from the origin, HEALPix nside)

    @property
    def mod_origin(self) -> float:
        """The modulation grid is centred on the origin (where the particles start)."""
        return -0.5 * self.mod_n * self.mod_spacing

    @property
    def reflect_box(self):
        """((lo x, y, z), (hi x, y, z)) of the reflective box, or None."""
        if self.reflect_half <= 0.0:
            return None
        h = self.reflect_half
        return ((-h, -h, -h), (h, h, h))

    @property
    def box(self) -> float:
        return self.grid_n * self.spacing


MIXED = (1, 2, 7, 26)

CONFIGS = (
    # 1,000 protons at 1 EeV in a 32^3 FP64 grid; stop at 50 Mpc of path.
    Workload("small_fp64_32cube", 0, 1000, (1,), 1e18, 1e18, 32, 0.1, 0.2, 1.6, 1.0, "f64",
             1e-4, 0.01, 1.0, 0.0, 50.0),
    # 1e6 mixed nuclei, 256^3 FP32 grid; stop at r = 20 Mpc or 1 Gpc of path.
    Workload("production_256cube", 1, 1_000_000, MIXED, 1e18, 1e20, 256, 0.05, 0.1, 5.0, 1.0, "f32",
             1e-4, 0.001, 1.0, 20.0, 1000.0),
    # 64 realisations of 64^3 FP32 grids; spacing, band, tol, step limits and L_max chosen
    # (L_max = 100 Mpc keeps the longest, h_min-limited trajectory at 1e5 steps).
    Workload("batched_64x64cube", 2, 0, MIXED, 1e17, 1e20, 64, 0.05, 0.1, 1.6, 1.0, "f32",
             1e-4, 0.001, 1.0, 0.0, 100.0, n_realisations=64, b_rms_range=(0.1, 10.0),
             count_range=(100, 100_000), radius_range=(1.0, 50.0)),
    # 4e6 mixed nuclei, 1024^3 grid stored FP16/BF16 (or FP32); tol, step limits and L_max chosen.
    Workload("precision_1024cube", 3, 4_000_000, MIXED, 1e18, 1e20, 1024, 0.01, 0.02, 2.0, 1.0, "f16",
             1e-4, 0.001, 1.0, 10.0, 1000.0),
    # 1e5 protons and iron, 128^3 FP32 grid; band, tol, step limits and L_max chosen.
    Workload("adjoint_128cube", 4, 100_000, (1, 26), 1e18, 1e19, 128, 0.05, 0.1, 3.2, 1.0, "f32",
             1e-4, 0.001, 1.0, 10.0, 1000.0, charge_rule="alternate", checkpoint_every=64),
    # Modulated field as in the paper's example: the production vector grid (256^3 at 50 kpc,
    # periodic every 12.8 Mpc) times a 132 Mpc modulation grid at 300 kpc (440^3); the
    # log-normal modulation (correlation length 2 Mpc, sigma 1) is chosen.
    Workload("modulated_256cube", 5, 1_000_000, MIXED, 1e18, 1e20, 256, 0.05, 0.1, 5.0, 1.0, "f32",
             1e-4, 0.001, 1.0, 20.0, 1000.0, mod_n=440, mod_spacing=0.3, mod_l_corr=2.0, mod_sigma=1.0),
    # The paper's example with its reflective boundaries: the modulated field above inside a
    # reflective box over the modulation grid's 132 Mpc; 1e6 nuclei start uniformly in the box
    # (uniform sources and the 100 Mpc length limit per call are chosen; no observer sphere).
    Workload("reflective_132box", 6, 1_000_000, MIXED, 1e18, 1e20, 256, 0.05, 0.1, 5.0, 1.0, "f32",
             1e-4, 0.001, 1.0, 0.0, 100.0, mod_n=440, mod_spacing=0.3, mod_l_corr=2.0, mod_sigma=1.0,
             reflect_half=66.0),
    # A lens of one rigidity (section 3.3, lensing): protons at 10 EeV observed at the origin in
    # directions spread uniformly over the sky are traced back through the production field to a
    # sphere of 20 Mpc standing for the galactic border (r_g = 10.8 Mpc in 1 nG, as 10 EeV
    # protons in a 1 uG galaxy of 20 kpc); HEALPix nside 64 (49,152 pixels, < 1 degree) with 64
    # launches per pixel on average (all chosen).
    Workload("lens_nside64", 7, 12 * 64 * 64 * 64, (1,), 1e19, 1e19, 256, 0.05, 0.1, 5.0, 1.0, "f32",
             1e-4, 0.001, 1.0, 20.0, 1000.0, lens_nside=64),
)


def get_config(key) -> Workload:
    """Look a workload up by index or by name."""
    if isinstance(key, int):
        return CONFIGS[key]
    for w in CONFIGS:
        if w.name == key:
            return w
    raise KeyError(key)


assert all(math.isfinite(w.max_length) for w in CONFIGS)
