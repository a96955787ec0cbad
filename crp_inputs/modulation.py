"""Scalar modulation grid for modulated fields.

The paper combines a small high-resolution vector grid, repeated
periodically, with a large low-resolution scalar grid that carries the
large-scale structure (section 3.2, modulated grids); its example derives
that scalar from a simulated matter distribution through a density-field
relation (section 4).  Those simulations are not available, so the stand-in
here is a log-normal field, the usual model of a density contrast:

1. white Gaussian noise on an n^3 periodic grid (PCG64 from the seed);
2. low-pass filtered in Fourier space by exp(-(k l)^2 / 4), so the power goes
   as exp(-(k l)^2 / 2): a smooth field with correlation length ~ l;
3. normalised to zero mean and unit variance over the nodes: g;
4. m = exp(sigma g), divided by sqrt(<m^2>) so that the mean square of the
   modulated field equals that of the vector grid.

Output layout: ``[ix][iy][iz]``, float64 (cast once to ``dtype``), node
(i, j, k) at origin + spacing*(i, j, k), periodic with period n*spacing.
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft


def lognormal_modulation(n: int, spacing: float, l_corr: float, sigma: float, seed,
                         dtype=np.float64) -> np.ndarray:
    if n < 4 or n % 2:
        raise ValueError("grid size must be even and >= 4")
    ss = seed if isinstance(seed, np.random.SeedSequence) else np.random.SeedSequence(seed)
    rng = np.random.Generator(np.random.PCG64(ss))
    noise = rng.standard_normal((n, n, n))
    spec = sfft.rfftn(noise, workers=-1)
    del noise
    k = 2.0 * np.pi * np.fft.fftfreq(n, spacing)
    kz = 2.0 * np.pi * np.fft.rfftfreq(n, spacing)
    k2 = k[:, None, None] ** 2 + k[None, :, None] ** 2 + kz[None, None, :] ** 2
    spec *= np.exp(-k2 * (l_corr * l_corr / 4.0))
    del k2
    g = sfft.irfftn(spec, s=(n, n, n), workers=-1)
    del spec
    g -= g.mean()
    g /= np.sqrt(np.mean(g * g))
    m = np.exp(sigma * g)
    m /= np.sqrt(np.mean(m * m))
    return m.astype(dtype, copy=False)
