"""Pins of the oracle's reflective box (the example of section 4 uses
reflective boundaries).

* at B = 0 the motion is a billiard: the final position is the straight line
  folded back into the box (a triangle wave per axis) and each direction
  component is negated once per reflection on its axis;
* in a field, every state stays in the box and the direction stays a unit vector;
* a box the particles never reach leaves every result bitwise unchanged;
* a taped run (for the adjoint) in a box is the untaped run.
"""
import math

import numpy as np
import pytest

import crp_inputs as ci


def _fold(x, lo, hi):
    w = hi - lo
    r = np.mod(x - lo, 2 * w)
    pos = np.where(r <= w, lo + r, lo + 2 * w - r)
    flips = np.floor((x - lo) / w)
    return pos, np.where(np.mod(flips, 2) == 0, 1.0, -1.0)


def test_billiard_at_zero_field(oracle_mod):
    O = oracle_mod
    g = O.Grid(np.zeros((4, 4, 4, 3)), 1.0)
    rng = np.random.default_rng(3)
    n = 64
    u0 = rng.standard_normal((n, 3))
    u0 /= np.linalg.norm(u0, axis=1, keepdims=True)
    x0 = rng.uniform(-0.5, 0.5, size=(n, 3))
    lo, hi, L = np.array([-1.0, -0.75, -1.25]), np.array([1.0, 1.25, 0.5]), 7.3
    prm = O.params_array(1e-6, 1e-9, 0.2, l_max=L, box=(lo, hi))
    o = O.propagate(g, prm, x0, u0, np.full(n, 1e18), np.ones(n, np.int32))
    assert np.all(o["status"] == 2) and np.all(o["length"] == L)
    pos, sign = _fold(x0 + L * u0, lo, hi)
    assert np.max(np.abs(o["pos"] - pos)) < 1e-12
    assert np.max(np.abs(o["dir"] - sign * u0)) < 1e-13
    assert np.all((o["pos"] >= lo) & (o["pos"] <= hi))


def test_field_keeps_particles_in_the_box(oracle_mod):
    O = oracle_mod
    w = ci.get_config(0)
    fs, ps, _ = ci.config_seeds(0)
    B = ci.kolmogorov_field(w.grid_n, w.spacing, w.l_min, w.l_max, w.b_rms, fs)
    P = ci.isotropic_particles(200, 1e18, 1e20, (1, 26), ps)
    lo, hi = np.array([-1.0, -1.0, -1.0]), np.array([1.0, 1.0, 1.0])
    prm = O.params_array(1e-5, 1e-6, 0.3, l_max=15.0, box=(lo, hi))
    o = O.propagate(O.Grid(B, w.spacing), prm, P["pos"], P["dir"], P["energy"], P["charge"])
    assert np.all(o["status"] == 2)
    assert np.all((o["pos"] >= lo) & (o["pos"] <= hi))
    assert np.max(np.abs(np.linalg.norm(o["dir"], axis=1) - 1.0)) < 1e-14


def test_unreached_box_changes_nothing(oracle_mod):
    O = oracle_mod
    w = ci.get_config(0)
    fs, ps, _ = ci.config_seeds(0)
    B = ci.kolmogorov_field(w.grid_n, w.spacing, w.l_min, w.l_max, w.b_rms, fs)
    P = ci.isotropic_particles(100, 3e18, 3e19, (1, 26), ps)
    a = O.propagate(O.Grid(B, w.spacing), O.params_array(1e-5, 1e-6, 0.3, radius=2.0, l_max=10.0),
                    P["pos"], P["dir"], P["energy"], P["charge"])
    far = (np.full(3, -1e6), np.full(3, 1e6))
    b = O.propagate(O.Grid(B, w.spacing), O.params_array(1e-5, 1e-6, 0.3, radius=2.0, l_max=10.0, box=far),
                    P["pos"], P["dir"], P["energy"], P["charge"])
    for k in ("pos", "dir", "length", "status", "n_acc", "n_rej"):
        assert np.array_equal(a[k], b[k]), k


def test_taped_runs_in_a_box_match_untaped(oracle_mod):
    """Recording the tape (for the adjoint) does not change a reflective run."""
    O = oracle_mod
    w = ci.get_config(0)
    fs, ps, _ = ci.config_seeds(0)
    g = O.Grid(ci.kolmogorov_field(w.grid_n, w.spacing, w.l_min, w.l_max, w.b_rms, fs), w.spacing)
    P = ci.isotropic_particles(6, 3e18, 3e19, (1, 26), ps)
    prm = O.params_array(1e-6, 1e-7, 0.2, radius=1.3, l_max=6.0, box=((-1, -1, -1), (1, 1, 1)))
    ref = O.propagate(g, prm, np.zeros((6, 3)), P["dir"], P["energy"], P["charge"])
    for i in range(6):
        t = O.propagate_taped(g, prm, np.zeros(3), P["dir"][i], P["energy"][i], P["charge"][i])
        assert np.array_equal(t["y"], np.concatenate([ref["pos"][i], ref["dir"][i]]))
        assert t["status"] == ref["status"][i] and t["n_steps"] == ref["n_acc"][i]
