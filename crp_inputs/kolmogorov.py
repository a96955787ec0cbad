"""Gaussian random Kolmogorov turbulence on a periodic regular grid.

The paper fills its high-resolution vector grid with "a random turbulent
realization of Kolmogorov power spectrum" with a stated coherence length
(section 4, structured-universe example; the grid technique is section 3.2).
It does not say how the realisation is built, so the construction here is:

1. wave vectors k = 2*pi*fftfreq(N, spacing) on x and y, 2*pi*rfftfreq on z;
2. modes kept for 2*pi/l_max <= |k| <= 2*pi/l_min, k != 0, and no Nyquist index
   on any axis (a Nyquist mode has no distinct partner -k, so it could not be
   kept both real and divergence-free);
3. complex Gaussian amplitudes (a + i b)/sqrt(2), drawn slab by slab along the
   kx index, each slab from its own PCG64 stream spawned from the seed (slab i
   uses child i): a of shape (3, N, N/2+1), then b of that shape; slabs are
   independent, so they are drawn concurrently;
4. projection onto the plane normal to k (divergence-free field), and on the
   kz = 0 plane xi(k) <- (xi(k) + conj(xi(-k)))/sqrt(2) so that the half
   spectrum is Hermitian there and keeps its full power;
5. amplitude |k|^(-11/6), so that the 3D power spectrum goes as k^(-11/3)
   (the shell spectrum as k^(-5/3));
6. real inverse FFT per component in FP64, rescaled so that the
   root-mean-square of |B| over the nodes equals B_rms (the mean square is
   taken from the spectrum by Parseval's theorem, exact up to rounding), then
   rounded once into the storage dtype.

Output layout: ``[ix][iy][iz][component]`` (iz fastest), float64, nanogauss.
Node (i, j, k) sits at origin + spacing*(i, j, k); the field repeats with
period N*spacing along each axis.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import scipy.fft as sfft

_SLACK = 1e-12  # relative slack on the |k| band edges, in units of (N*spacing/l)^2


def _workers() -> int:
    try:
        return max(1, min(16, len(os.sched_getaffinity(0))))
    except AttributeError:  # pragma: no cover
        return max(1, min(16, os.cpu_count() or 1))


def spectral_mask(n: int, spacing: float, l_min: float, l_max: float):
    """Integer mode vectors and the kept-mode mask on the rfft half-spectrum grid.

    Returns (nx, ny, nz, mask) where n* are integer mode indices (signed on x
    and y, non-negative on z) broadcastable to shape (N, N, N//2+1).
    """
    if n < 4 or n % 2:
        raise ValueError("grid size must be even and >= 4")
    box = n * spacing
    ix = np.fft.fftfreq(n, 1.0 / n).astype(np.int64)
    iz = np.fft.rfftfreq(n, 1.0 / n).astype(np.int64)
    nx = ix[:, None, None]
    ny = ix[None, :, None]
    nz = iz[None, None, :]
    n2 = nx * nx + ny * ny + nz * nz
    lo = (box / l_max) ** 2 * (1.0 - _SLACK)
    hi = (box / l_min) ** 2 * (1.0 + _SLACK)
    nyq = n // 2
    not_nyq = (np.abs(nx) != nyq) & (np.abs(ny) != nyq) & (nz != nyq)
    mask = (n2 > 0) & (n2 >= lo) & (n2 <= hi) & not_nyq
    return nx, ny, nz, mask


def kolmogorov_field(n: int, spacing: float, l_min: float, l_max: float,
                     b_rms: float, seed, dtype=np.float64) -> np.ndarray:
    """Return an (N, N, N, 3) array, in nG, of one seeded realisation.

    ``seed`` is a ``numpy.random.SeedSequence`` (or anything PCG64 accepts).
    ``dtype`` is the storage dtype of the returned array; the synthesis is
    always FP64 and the cast (if any) rounds to nearest even.
    """
    ss = seed if isinstance(seed, np.random.SeedSequence) else np.random.SeedSequence(seed)
    slab_seeds = ss.spawn(n)
    nx, ny, nz, mask = spectral_mask(n, spacing, l_min, l_max)
    nzh = n // 2 + 1
    kx = nx.astype(np.float64)
    ky = ny.astype(np.float64)
    kz = nz.astype(np.float64)

    spec = [np.empty((n, n, nzh), dtype=np.complex128) for _ in range(3)]
    inv_sqrt2 = 1.0 / np.sqrt(2.0)

    def slab(i):
        rng = np.random.Generator(np.random.PCG64(slab_seeds[i]))
        a = rng.standard_normal((3, n, nzh))
        b = rng.standard_normal((3, n, nzh))
        xi = (a + 1j * b) * inv_sqrt2
        kxi = kx[i, 0, 0]
        kyi = ky[0, :, :]
        kzi = kz[0, :, :]
        k2 = kxi * kxi + kyi * kyi + kzi * kzi
        m = mask[i]
        k2s = np.where(m, k2, 1.0)
        kdot = kxi * xi[0] + kyi * xi[1] + kzi * xi[2]
        proj = kdot / k2s
        xi[0] -= kxi * proj
        xi[1] -= kyi * proj
        xi[2] -= kzi * proj
        amp = np.where(m, k2s ** (-11.0 / 12.0), 0.0)  # |k|^(-11/6)
        for c in range(3):
            spec[c][i] = xi[c] * amp

    with ThreadPoolExecutor(max_workers=_workers()) as ex:
        list(ex.map(slab, range(n)))

    # The real inverse transform keeps only the Hermitian part of the kz = 0
    # plane, which would halve its power; make that plane Hermitian here,
    # (xi(k) + conj(xi(-k)))/sqrt(2), which keeps both the power and k.xi = 0.
    neg = (-np.arange(n)) % n
    for c in range(3):
        p0 = spec[c][:, :, 0]
        spec[c][:, :, 0] = (p0 + np.conj(p0[neg][:, neg])) * inv_sqrt2

    # Mean of |B|^2 over the nodes from the spectrum (Parseval): every kz > 0
    # column stands for itself and its conjugate partner.
    w = np.full(nzh, 2.0)
    w[0] = 1.0
    ms = 0.0
    for c in range(3):
        ms += float(np.sum(np.sum(spec[c].real ** 2 + spec[c].imag ** 2, axis=(0, 1)) * w))
    ms /= float(n) ** 6
    scale = b_rms / np.sqrt(ms)

    out = np.empty((n, n, n, 3), dtype=dtype)
    for c in range(3):
        comp = sfft.irfftn(spec[c], s=(n, n, n), workers=_workers())
        spec[c] = None
        comp *= scale
        out[..., c] = comp  # rounds to nearest even when dtype is narrower
        del comp
    return out


def coherence_length(l_min: float, l_max: float, alpha: float = 5.0 / 3.0) -> float:
    """Coherence length of a power-law turbulence band (Harari, Mollerach & Roulet 2002).

    L_c = (l_max/2) * ((alpha-1)/alpha) * (1 - r^alpha) / (1 - r^(alpha-1)),
    r = l_min/l_max, alpha = 5/3 for Kolmogorov.  This equals twice the
    one-sided integral of the normalised correlation <B(0).B(r)>/<B^2>.
    """
    r = l_min / l_max
    return 0.5 * l_max * (alpha - 1.0) / alpha * (1.0 - r ** alpha) / (1.0 - r ** (alpha - 1.0))
