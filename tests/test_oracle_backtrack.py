"""Pins of the oracle's backtracking mode (section 3.3: a particle observed at
one place is traced back to where it came from).

* at B = 0 the particle is traced back along a straight line: x0 - L u, with
  its direction unchanged;
* in a uniform field the result is the closed-form helix at path length -L
  (the physical particle's state L earlier), converging with the tolerance;
* forward propagation followed by backtracking from the end state returns to
  the start (time reversal), to the accuracy of the two runs;
* with the observer sphere the backtracked particle leaves through it.
"""
import math

import numpy as np

import crp_inputs as ci


def helix(u0, x0, kb, s):
    """Closed-form trajectory for B = B zhat, kb = kappa*B (1/Mpc), path length s."""
    w0 = u0[0] + 1j * u0[1]
    rot = np.exp(-1j * kb * s)
    w = w0 * rot
    p = (x0[0] + 1j * x0[1]) + 1j * w0 * (rot - 1.0) / kb
    return np.array([p.real, p.imag, x0[2] + u0[2] * s]), np.array([w.real, w.imag, u0[2]])


def _uniform(O, b):
    v = np.empty((4, 4, 4, 3))
    v[...] = b
    return O.Grid(v, 1.0)


def test_straight_line_back_at_zero_field(oracle_mod):
    O = oracle_mod
    rng = np.random.default_rng(21)
    n = 40
    u = rng.standard_normal((n, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    x0 = rng.uniform(-1, 1, (n, 3))
    L = 13.7
    prm = O.params_array(1e-4, 0.01, 1.0, l_max=L, backtrack=True)
    r = O.propagate(_uniform(O, [0.0, 0.0, 0.0]), prm, x0, u, np.full(n, 1e18), np.full(n, 7, np.int32))
    assert np.all(r["status"] == 2) and np.all(r["length"] == L)
    assert np.max(np.abs(r["pos"] - (x0 - L * u))) < 1e-12 * L
    assert np.max(np.abs(r["dir"] - u)) < 1e-15


def test_uniform_field_gives_the_earlier_helix_state(oracle_mod):
    O = oracle_mod
    B = 2.0
    g = _uniform(O, [0.0, 0.0, B])
    E, Z = 3e18, 2
    kb = O.kappa(Z, E) * B
    rg = 1.0 / abs(kb)
    u0 = np.array([0.48, -0.6, 0.64])
    x0 = np.array([0.3, -0.2, 0.1])
    L = 2.5 * 2 * math.pi * rg
    xr, ur = helix(u0, x0, kb, -L)
    xf, _ = helix(u0, x0, kb, L)
    assert np.linalg.norm(xr - xf) > 0.1 * rg  # backwards and forwards differ
    errs = []
    for tol in (1e-4, 1e-6, 1e-8, 1e-10):
        prm = O.params_array(tol, 1e-9, 10.0, l_max=L, backtrack=True)
        r = O.propagate(g, prm, x0[None], u0[None], [E], [Z])
        assert r["status"][0] == 2 and r["length"][0] == L
        e = max(np.linalg.norm(r["pos"][0] - xr) / rg, float(np.linalg.norm(r["dir"][0] - ur)))
        errs.append(e)
    assert errs[-1] < 1e-8
    assert all(errs[i + 1] < errs[i] * 0.2 for i in range(len(errs) - 1)), errs


def test_forward_then_back_returns_to_the_start(oracle_mod):
    O = oracle_mod
    w = ci.get_config(0)
    fs, ps, _ = ci.config_seeds(0)
    Bv = ci.kolmogorov_field(w.grid_n, w.spacing, w.l_min, w.l_max, w.b_rms, fs)
    g = O.Grid(Bv, w.spacing)
    P = ci.isotropic_particles(64, 1e19, 1e20, (1, 2), ps)
    x0 = np.tile([0.2, -0.4, 0.7], (64, 1))
    L = 5.0
    fwd = O.propagate(g, O.params_array(1e-10, 1e-9, 0.2, l_max=L), x0, P["dir"], P["energy"], P["charge"])
    back = O.propagate(g, O.params_array(1e-10, 1e-9, 0.2, l_max=L, backtrack=True), fwd["pos"], fwd["dir"],
                       P["energy"], P["charge"])
    assert np.all(back["status"] == 2)
    assert np.max(np.linalg.norm(fwd["pos"] - x0, axis=1)) > 1.0  # they moved
    assert np.max(np.linalg.norm(back["pos"] - x0, axis=1)) < 1e-7
    assert np.max(np.linalg.norm(back["dir"] - P["dir"], axis=1)) < 1e-7
    # the same runs with the charge left as it is do not return
    wrong = O.propagate(g, O.params_array(1e-10, 1e-9, 0.2, l_max=L), fwd["pos"], -fwd["dir"], P["energy"],
                        P["charge"])
    assert np.median(np.linalg.norm(wrong["pos"] - x0, axis=1)) > 1e-3


def test_backtracked_particles_leave_through_the_sphere(oracle_mod):
    O = oracle_mod
    w = ci.get_config(0)
    fs, ps, _ = ci.config_seeds(0)
    Bv = ci.kolmogorov_field(w.grid_n, w.spacing, w.l_min, w.l_max, w.b_rms, fs)
    P = ci.isotropic_particles(200, 1e18, 1e20, (1, 26), ps)
    R = 2.0
    r = O.propagate(O.Grid(Bv, w.spacing), O.params_array(1e-4, 1e-4, 0.5, radius=R, l_max=200.0, backtrack=True),
                    P["pos"], P["dir"], P["energy"], P["charge"])
    assert np.all(r["status"] == 1)
    d = np.linalg.norm(r["pos"], axis=1)
    assert np.all(d >= R) and np.max(d - R) < 1e-10
