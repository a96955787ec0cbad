"""Lens oracle: HEALPix binning, lens matrices and their application (numpy, FP64).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline may use this module; the GPU library shares nothing with it.

The lensing technique of section 3.3 (the PARSEC method): for one rigidity,
particles are traced back from Earth (backtracking) in directions spread over
the sky to the galactic border.  A matrix over sky pixels then maps the
cosmic-ray directions at the border to the directions observed at Earth, and
whole arrival distributions are transformed by matrix-vector products.  The
sky is pixelised with HEALPix (Gorski et al. 2005, ApJ 622:759), here in its
RING numbering, and the matrices are held sparse (CSR).

Readings (the paper gives the technique, not its formulas):
  * a direction is binned as the direction the particle comes from, i.e. the
    reverse of its velocity;
  * row i of the lens is the observed pixel, column j the pixel at the border:
    L[i, j] = (launches from observed pixel i that reach the border from
    pixel j) / (all launches from observed pixel i); launches that do not
    reach the border count in the denominator only, so a row sums to the
    fraction of its launches that escaped;
  * the value is that ratio computed in FP64 and rounded once to FP32;
  * the application y = L x maps a flux map at the border to the observed
    one (flux is constant along a trajectory), summed in FP64.

The clamps below change nothing in exact arithmetic (the ring index and q
stay in range there); they only keep a direction that rounding puts exactly
on the belt's edge inside the valid pixel range.

Pixel decision (FP64 throughout, in this order):
    r = sqrt(ux*ux + uy*uy + uz*uz), z = uz / r, za = |z|
    phi = atan2(uy, ux), plus 2 pi if negative; tt = phi / (pi/2), 0 if tt >= 4
    za <= 2/3 (equatorial belt):
        t1 = nside * (0.5 + tt), t2 = nside * (z * 0.75)
        jp = floor(t1 - t2), jm = floor(t1 + t2)       (edge-line indices)
        ir = nside + 1 + jp - jm, clamped to 1 .. 2 nside + 1 (belt rings)
        q = jp + jm - nside + (1 - ir mod 2) + 1, clamped to >= 0
        ip = (q / 2, rounded down) mod 4 nside
        pix = 2 nside (nside - 1) + 4 nside (ir - 1) + ip
    za > 2/3 (polar caps):
        tp = tt - floor(tt), s = nside * sqrt(3 * (1 - za))
        jp = floor(tp * s), jm = floor((1 - tp) * s), ir = jp + jm + 1 clamped to 1 .. nside
        ip = floor(tt * ir) mod 4 ir
        pix = 2 ir (ir - 1) + ip (north), 12 nside^2 - 2 ir (ir + 1) + ip (south)
"""
from __future__ import annotations

import math

import numpy as np

HALF_PI = math.pi / 2.0
TWO_PI = 2.0 * math.pi


def npix(nside: int) -> int:
    return 12 * nside * nside


def pix_ring(nside: int, ux, uy, uz) -> np.ndarray:
    """RING-scheme pixel of each direction (any non-zero finite length), int64;
    -1 for a zero or non-finite direction."""
    ux = np.asarray(ux, dtype=np.float64)
    uy = np.asarray(uy, dtype=np.float64)
    uz = np.asarray(uz, dtype=np.float64)
    ns = float(nside)
    r = np.sqrt(ux * ux + uy * uy + uz * uz)
    bad = ~((r > 0.0) & np.isfinite(r))
    r = np.where(bad, 1.0, r)
    z = np.where(bad, 0.0, uz / r)
    ux = np.where(bad, 1.0, ux)
    uy = np.where(bad, 0.0, uy)
    za = np.abs(z)
    phi = np.arctan2(uy, ux)
    phi = np.where(phi < 0.0, phi + TWO_PI, phi)
    tt = phi / HALF_PI
    tt = np.where(tt >= 4.0, 0.0, tt)
    out = np.empty(z.shape, dtype=np.int64)

    eq = za <= 2.0 / 3.0
    t1 = ns * (0.5 + tt[eq])
    t2 = ns * (z[eq] * 0.75)
    jp = np.floor(t1 - t2).astype(np.int64)
    jm = np.floor(t1 + t2).astype(np.int64)
    ir = np.clip(nside + 1 + jp - jm, 1, 2 * nside + 1)
    kshift = 1 - (ir & 1)
    q = np.maximum(jp + jm - nside + kshift + 1, 0)
    ip = np.mod(q // 2, 4 * nside)
    out[eq] = 2 * nside * (nside - 1) + 4 * nside * (ir - 1) + ip

    po = ~eq
    ttp = tt[po]
    tp = ttp - np.floor(ttp)
    s = ns * np.sqrt(3.0 * (1.0 - za[po]))
    jp = np.floor(tp * s).astype(np.int64)
    jm = np.floor((1.0 - tp) * s).astype(np.int64)
    ir = np.clip(jp + jm + 1, 1, nside)
    ip = np.mod(np.floor(ttp * ir).astype(np.int64), 4 * ir)
    out[po] = np.where(z[po] > 0.0, 2 * ir * (ir - 1) + ip, npix(nside) - 2 * ir * (ir + 1) + ip)
    out[bad] = -1
    return out


def pix_centres(nside: int):
    """(z, phi) of every pixel centre in RING order, from the ring geometry:
    ring i = 1 .. 4 nside - 1 from the north pole; polar rings i < nside hold
    4 i pixels at z = 1 - i^2 / (3 nside^2), phi = pi / (2 i) (j + 1/2); belt
    rings hold 4 nside pixels at z = 4/3 - 2 i / (3 nside), phi = pi / (2 nside)
    (j + s / 2) with s = 1 when i - nside is even, else 0; the south cap
    mirrors the north one."""
    zs, ph = [], []
    for i in range(1, 4 * nside):
        if i < nside:
            m = 4 * i
            z = 1.0 - i * i / (3.0 * nside * nside)
            phis = math.pi / (2 * i) * (np.arange(m) + 0.5)
        elif i <= 3 * nside:
            m = 4 * nside
            z = 4.0 / 3.0 - 2.0 * i / (3.0 * nside)
            s = 1 if (i - nside) % 2 == 0 else 0
            phis = math.pi / (2 * nside) * (np.arange(m) + 0.5 * s)
        else:
            k = 4 * nside - i
            m = 4 * k
            z = -(1.0 - k * k / (3.0 * nside * nside))
            phis = math.pi / (2 * k) * (np.arange(m) + 0.5)
        zs.append(np.full(m, z))
        ph.append(phis)
    return np.concatenate(zs), np.concatenate(ph)


def lens_matrix(nside: int, rows, ux, uy, uz, arrived):
    """CSR lens (row_ptr int64, col int32, val float32) from the observed pixel
    of each launch (rows), the velocity directions reached and the mask of the
    launches that reached the border."""
    rows = np.asarray(rows, dtype=np.int64)
    arrived = np.asarray(arrived, dtype=bool)
    n_pix = npix(nside)
    launches = np.bincount(rows, minlength=n_pix)
    cols = pix_ring(nside, -np.asarray(ux)[arrived], -np.asarray(uy)[arrived], -np.asarray(uz)[arrived])
    keep = cols >= 0  # a direction that cannot be binned counts as not arrived
    arrived = arrived.copy()
    arrived[np.nonzero(arrived)[0][~keep]] = False
    cols = cols[keep]
    keys, counts = np.unique(rows[arrived] * n_pix + cols, return_counts=True)
    r = keys // n_pix
    c = keys % n_pix
    val = (counts.astype(np.float64) / launches[r].astype(np.float64)).astype(np.float32)
    row_ptr = np.zeros(n_pix + 1, dtype=np.int64)
    row_ptr[1:] = np.cumsum(np.bincount(r, minlength=n_pix))
    return row_ptr, c.astype(np.int32), val


def lens_apply(row_ptr, col, val, x) -> np.ndarray:
    """y = L x for x of shape (npix,) or (npix, nvec), summed in FP64."""
    x = np.asarray(x, dtype=np.float64)
    v = np.asarray(val, dtype=np.float64)
    n = len(row_ptr) - 1
    contrib = v[:, None] * x.reshape(x.shape[0], -1)[np.asarray(col)]
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    y = np.zeros((n, contrib.shape[1]))
    np.add.at(y, rows, contrib)
    return y.reshape((n,) + x.shape[1:])
