"""Pins of the oracle's modulated field (section 3.2, modulated grids) and of
the log-normal modulation generator.

* a modulation of 1 leaves every result bitwise unchanged;
* a modulation of 2 doubles the field exactly, which for the Lorentz force
  is the same as halving the energy: trajectories are bitwise equal;
* an affine modulation is reproduced exactly by trilinear interpolation, so
  the field is scipy's interpolant of the vector grid times the affine
  function (to rounding);
* the modulation repeats with its own period;
* the generator's output has unit mean square and log m has standard
  deviation sigma, with a Gaussian power spectrum of the stated length.
"""
import numpy as np
import pytest
from scipy.interpolate import RegularGridInterpolator

import crp_inputs as ci


@pytest.fixture(scope="module")
def small(oracle_mod):
    w = ci.get_config(0)
    fs, ps, _ = ci.config_seeds(0)
    B = ci.kolmogorov_field(w.grid_n, w.spacing, w.l_min, w.l_max, w.b_rms, fs)
    P = ci.isotropic_particles(64, 3e18, 3e19, (1, 26), ps)
    return w, B, P


def _run(O, grid, P, energy=None):
    prm = O.params_array(1e-5, 1e-6, 0.2, radius=1.5, l_max=20.0)
    return O.propagate(grid, prm, P["pos"], P["dir"], P["energy"] if energy is None else energy, P["charge"])


def _same(a, b):
    for k in ("pos", "dir", "length", "status", "n_acc", "n_rej"):
        assert np.array_equal(a[k], b[k]), k


def test_unit_modulation_changes_nothing(oracle_mod, small):
    O = oracle_mod
    w, B, P = small
    ones = np.ones((10, 12, 14))
    plain = _run(O, O.Grid(B, w.spacing), P)
    mod = _run(O, O.Grid(B, w.spacing, modulation=O.Modulation(ones, 0.37, (-1.0, 0.5, 2.0))), P)
    _same(plain, mod)


def test_modulation_two_equals_half_energy(oracle_mod, small):
    O = oracle_mod
    w, B, P = small
    twos = np.full((8, 8, 8), 2.0, dtype=np.float32)
    mod = _run(O, O.Grid(B, w.spacing, modulation=O.Modulation(twos, 0.5)), P)
    half = _run(O, O.Grid(B, w.spacing), P, energy=P["energy"] * 0.5)
    _same(mod, half)


def test_affine_modulation_times_vector_interpolant(oracle_mod, small):
    O = oracle_mod
    w, B, _ = small
    nm, dm, om = 24, 0.25, np.array([-3.0, -3.0, -3.0])
    x = om[0] + dm * np.arange(nm)
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    a, g = 1.5, np.array([0.11, -0.07, 0.05])
    m = a + g[0] * X + g[1] * Y + g[2] * Z
    grid = O.Grid(B, w.spacing, modulation=O.Modulation(m, dm, om))
    rng = np.random.default_rng(5)
    pts = rng.uniform(-2.5, 2.5, size=(500, 3))  # inside the modulation grid, away from its seam
    got = O.field_at(grid, pts)
    n = w.grid_n
    pad = np.concatenate([B, B[:1]], axis=0)
    pad = np.concatenate([pad, pad[:, :1]], axis=1)
    pad = np.concatenate([pad, pad[:, :, :1]], axis=2)
    ax = w.spacing * np.arange(n + 1)
    ref_b = RegularGridInterpolator((ax, ax, ax), pad)(np.mod(pts, n * w.spacing))
    ref = ref_b * (a + pts @ g)[:, None]
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_modulation_repeats_with_its_period(oracle_mod, small):
    O = oracle_mod
    w, B, _ = small
    m = ci.lognormal_modulation(16, 0.4, 1.0, 0.8, 3)  # period 6.4 Mpc = 2 x the vector grid's 3.2
    grid = O.Grid(B, w.spacing, modulation=O.Modulation(m, 0.4))
    rng = np.random.default_rng(6)
    pts = rng.uniform(0.0, 6.4, size=(200, 3))
    base = O.field_at(grid, pts)
    for a in range(3):
        sh = pts.copy()
        sh[:, a] += 6.4
        assert np.max(np.abs(O.field_at(grid, sh) - base)) <= 1e-12 * np.max(np.abs(base))


def test_lognormal_generator_statistics():
    n, dx, l, sigma = 64, 0.3, 1.2, 0.9
    m = ci.lognormal_modulation(n, dx, l, sigma, 11)
    assert m.shape == (n, n, n) and np.all(m > 0)
    assert abs(np.mean(m * m) - 1.0) < 1e-12
    g = np.log(m)
    assert abs(np.std(g) - sigma) < 1e-12
    # power spectrum of g: log P falls linearly in k^2 with slope -l^2/2
    p = np.abs(np.fft.rfftn(g - g.mean())) ** 2
    k = 2 * np.pi * np.fft.fftfreq(n, dx)
    kz = 2 * np.pi * np.fft.rfftfreq(n, dx)
    k2 = k[:, None, None] ** 2 + k[None, :, None] ** 2 + kz[None, None, :] ** 2
    sel = (k2 > 0) & (k2 < (3.0 / l) ** 2)
    slope = np.polyfit(k2[sel], np.log(p[sel]), 1)[0]
    assert abs(slope / (-l * l / 2.0) - 1.0) < 0.1
    # the same seed gives the same grid; FP32 output is the rounded FP64 one
    assert np.array_equal(ci.lognormal_modulation(n, dx, l, sigma, 11, dtype=np.float32), m.astype(np.float32))
