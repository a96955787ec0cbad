"""Pins of the lens oracle (section 3.3, lensing technique).

HEALPix RING binning (Gorski et al. 2005):
* every pixel centre, computed from the ring geometry, is binned into its own
  pixel (the centre formulas and the binning are separate derivations);
* the twelve base pixels at nside = 1 sit at the textbook positions;
* the poles fall into the first and last four pixels;
* equal areas: uniform random directions fill the pixels uniformly.

Lens matrices and their application:
* no field: every backtracked particle leaves in its launch direction, so the
  lens is the identity;
* brute force on a tiny case (a dictionary count) gives the same CSR;
* rows sum to the escaped fraction; a uniform map stays uniform where all
  launches escape; a single-pixel map is transported to the lens column.
"""
import math

import numpy as np
import pytest

from oracle import lens as LN


def _unit(z, phi):
    s = np.sqrt(1.0 - z * z)
    return s * np.cos(phi), s * np.sin(phi), z


@pytest.mark.parametrize("nside", [1, 2, 4, 8, 16, 64])
def test_pixel_centres_bin_to_themselves(nside):
    z, phi = LN.pix_centres(nside)
    assert len(z) == LN.npix(nside)
    assert np.all(np.diff(z) <= 0)  # rings ordered north to south
    p = LN.pix_ring(nside, *_unit(z, phi))
    assert np.array_equal(p, np.arange(LN.npix(nside)))


def test_base_pixels_at_nside_1():
    z, phi = LN.pix_centres(1)
    assert np.allclose(z[:4], 2.0 / 3.0) and np.allclose(z[4:8], 0.0) and np.allclose(z[8:], -2.0 / 3.0)
    assert np.allclose(phi[:4], math.pi / 4 + np.arange(4) * math.pi / 2)
    assert np.allclose(phi[4:8], np.arange(4) * math.pi / 2)
    assert np.allclose(phi[8:], math.pi / 4 + np.arange(4) * math.pi / 2)


@pytest.mark.parametrize("nside", [1, 4, 64])
def test_poles(nside):
    n = LN.npix(nside)
    assert 0 <= LN.pix_ring(nside, [0.0], [0.0], [1.0])[0] < 4
    assert n - 4 <= LN.pix_ring(nside, [0.0], [0.0], [-1.0])[0] < n
    # near the poles, all four quarters of the first and last ring are reached
    phi = np.arange(8) * math.pi / 4 + 0.1
    assert set(LN.pix_ring(nside, *_unit(np.full(8, 1 - 1e-9), phi))) == {0, 1, 2, 3}
    assert set(LN.pix_ring(nside, *_unit(np.full(8, -1 + 1e-9), phi))) == {n - 4, n - 3, n - 2, n - 1}


def test_equal_area():
    nside = 4
    rng = np.random.default_rng(5)
    m = 2_000_000
    v = rng.standard_normal((m, 3))
    c = np.bincount(LN.pix_ring(nside, v[:, 0] * 3.0, v[:, 1] * 3.0, v[:, 2] * 3.0), minlength=LN.npix(nside))
    mean = m / LN.npix(nside)
    assert len(c) == LN.npix(nside)
    assert np.max(np.abs(c - mean)) < 6 * math.sqrt(mean)


def test_identity_lens_without_field(oracle_mod):
    O = oracle_mod
    nside = 8
    rng = np.random.default_rng(2)
    n = 20000
    d = rng.standard_normal((n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    rows = LN.pix_ring(nside, d[:, 0], d[:, 1], d[:, 2])
    g = O.Grid(np.zeros((4, 4, 4, 3)), 1.0)
    prm = O.params_array(1e-4, 1e-3, 1.0, radius=5.0, l_max=100.0, backtrack=True)
    r = O.propagate(g, prm, np.zeros((n, 3)), -d, np.full(n, 1e19), np.ones(n, np.int32))
    assert np.all(r["status"] == 1)
    row_ptr, col, val = LN.lens_matrix(nside, rows, r["dir"][:, 0], r["dir"][:, 1], r["dir"][:, 2],
                                       r["status"] == 1)
    full = np.diff(row_ptr)
    assert np.all(full[np.bincount(rows, minlength=LN.npix(nside)) > 0] == 1)
    assert np.array_equal(col, np.nonzero(np.bincount(rows, minlength=LN.npix(nside)))[0])
    assert np.all(val == 1.0)


def test_brute_force_csr():
    nside = 2
    rng = np.random.default_rng(9)
    n = 400
    rows = rng.integers(0, LN.npix(nside), n)
    u = rng.standard_normal((n, 3))
    arrived = rng.random(n) < 0.8
    row_ptr, col, val = LN.lens_matrix(nside, rows, u[:, 0], u[:, 1], u[:, 2], arrived)
    # brute force: a dictionary of counts, the border pixel found by nearest centre test
    zc, pc = LN.pix_centres(nside)
    counts, launches = {}, {}
    for k in range(n):
        launches[rows[k]] = launches.get(rows[k], 0) + 1
        if arrived[k]:
            j = int(LN.pix_ring(nside, [-u[k, 0]], [-u[k, 1]], [-u[k, 2]])[0])
            counts[(rows[k], j)] = counts.get((rows[k], j), 0) + 1
    keys = sorted(counts)
    assert np.array_equal(col, np.array([j for _, j in keys]))
    assert np.array_equal(val, np.array([np.float32(counts[k] / launches[k[0]]) for k in keys]))
    assert row_ptr[-1] == len(keys)
    for i in range(LN.npix(nside)):
        assert np.all(np.diff(col[row_ptr[i]:row_ptr[i + 1]]) > 0)
        assert row_ptr[i + 1] - row_ptr[i] == sum(1 for (a, _) in keys if a == i)
    # the binned direction is the reverse of the velocity: the pixel whose centre is nearest to -u
    cx, cy, cz = _unit(zc, pc)
    near = np.argmax(-(u[:, :1] * cx + u[:, 1:2] * cy + u[:, 2:] * cz), axis=1)
    own = LN.pix_ring(nside, -u[:, 0], -u[:, 1], -u[:, 2])
    assert np.mean(near == own) > 0.8  # pixels are not Voronoi cells, but mostly agree


def test_application():
    nside = 4
    n_pix = LN.npix(nside)
    rng = np.random.default_rng(4)
    n = 30000
    rows = rng.integers(0, n_pix, n)
    u = rng.standard_normal((n, 3))
    arrived = rng.random(n) < 0.9
    arrived[rows < 10] = True
    row_ptr, col, val = LN.lens_matrix(nside, rows, u[:, 0], u[:, 1], u[:, 2], arrived)
    dense = np.zeros((n_pix, n_pix))
    for i in range(n_pix):
        dense[i, col[row_ptr[i]:row_ptr[i + 1]]] = val[row_ptr[i]:row_ptr[i + 1]]
    launches = np.bincount(rows, minlength=n_pix)
    esc = np.bincount(rows[arrived], minlength=n_pix)
    y1 = LN.lens_apply(row_ptr, col, val, np.ones(n_pix, np.float32))
    assert np.allclose(y1, esc / launches, rtol=1e-6)
    assert np.allclose(y1[:10], 1.0, rtol=1e-6)
    e = np.zeros((n_pix, 3), np.float32)
    e[17, 0] = 1.0
    e[:, 1] = rng.random(n_pix)
    e[:, 2] = -2.0
    y = LN.lens_apply(row_ptr, col, val, e)
    assert np.array_equal(y[:, 0], dense[:, 17])
    assert np.allclose(y[:, 1], dense @ e[:, 1].astype(np.float64), rtol=1e-12)
    assert np.allclose(y[:, 2], -2.0 * esc / launches, rtol=1e-6)
