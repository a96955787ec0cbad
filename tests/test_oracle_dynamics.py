"""Pins of the oracle's equation of motion, integrator and step control.

Closed forms: straight lines at B = 0 and the helix in a uniform field
(gyroradius r = E/(Z e c B), path period 2 pi r); fixed-step convergence
orders; brute-force integration with an independent integrator (scipy DOP853
on scipy's trilinear interpolant); invariants (direction norm, rigidity
scaling, time reversal, which the paper's backtracking relies on).
"""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp
from scipy.interpolate import RegularGridInterpolator

import crp_inputs as ci


def uniform_grid(O, b, n=4, h=1.0):
    v = np.empty((n, n, n, 3))
    v[...] = b
    return O.Grid(v, h)


def helix(u0, x0, kb, s):
    """Closed-form trajectory for B = B zhat, kb = kappa*B (1/Mpc), path length s."""
    w0 = u0[0] + 1j * u0[1]
    rot = np.exp(-1j * kb * s)
    w = w0 * rot
    p = (x0[0] + 1j * x0[1]) + 1j * w0 * (rot - 1.0) / kb
    return np.array([p.real, p.imag, x0[2] + u0[2] * s]), np.array([w.real, w.imag, u0[2]])


def ang(a, b):
    return math.atan2(np.linalg.norm(np.cross(a, b)), float(np.dot(a, b)))


def test_straight_line_at_zero_field(oracle_mod):
    O = oracle_mod
    g = uniform_grid(O, [0.0, 0.0, 0.0])
    rng = np.random.default_rng(10)
    u = rng.standard_normal((50, 3))
    u /= np.linalg.norm(u, axis=1)[:, None]
    prm = O.params_array(1e-4, 0.01, 1.0, radius=20.0, l_max=1000.0)
    r = O.propagate(g, prm, np.zeros((50, 3)), u, np.full(50, 1e18), np.ones(50, np.int32))
    assert np.all(r["status"] == 1)
    assert np.max(np.abs(r["length"] - 20.0)) <= 1e-13 * 20
    assert np.max(np.abs(r["pos"] - 20.0 * u)) <= 1e-13 * 20
    assert np.max(np.abs(r["time"] - 20.0 * O.constants()["MPC_OVER_C"])) <= 1e-13 * r["time"].max()
    assert set(np.unique(r["n_acc"])) <= {20, 21}
    assert np.all(r["n_rej"] == 0)
    # zero error: every bid grows by the maximum factor 5, capped at h_max
    assert np.all((r["h_next"] == 1.0) | (r["h_next"] >= 5 * 0.01))


def test_uniform_field_helix_and_sense_of_rotation(oracle_mod):
    O = oracle_mod
    B = 1.0
    g = uniform_grid(O, [0.0, 0.0, B])
    E = 1e18
    kb = O.kappa(1, E) * B
    rg = 1.0 / kb
    # quarter gyration: a positive charge moving along +x turns towards -y
    L = 0.5 * math.pi * rg
    prm = O.params_array(1e-10, 1e-6, 1.0, l_max=L)
    r = O.propagate(g, prm, np.zeros((1, 3)), np.array([[1.0, 0.0, 0.0]]), [E], [1])
    assert r["status"][0] == 2 and r["length"][0] == L
    assert np.allclose(r["dir"][0], [0.0, -1.0, 0.0], atol=1e-8)
    assert np.allclose(r["pos"][0], [rg, -rg, 0.0], atol=1e-8)
    # a negative charge turns the other way
    r = O.propagate(g, prm, np.zeros((1, 3)), np.array([[1.0, 0.0, 0.0]]), [E], [-1])
    assert np.allclose(r["dir"][0], [0.0, 1.0, 0.0], atol=1e-8)


@pytest.mark.parametrize("pitch_deg", [90.0, 35.0])
def test_helix_error_falls_with_tolerance(oracle_mod, pitch_deg):
    O = oracle_mod
    B = 2.0
    g = uniform_grid(O, [0.0, 0.0, B])
    E = 3e18
    kb = O.kappa(2, E) * B
    rg = 1.0 / kb
    L = 3 * 2 * math.pi * rg  # three gyration periods of path
    p = math.radians(pitch_deg)
    u0 = np.array([math.sin(p), 0.0, math.cos(p)])
    x0 = np.array([0.3, -0.2, 0.1])
    xr, ur = helix(u0, x0, kb, L)
    errs = []
    for tol in (1e-4, 1e-6, 1e-8, 1e-10):
        prm = O.params_array(tol, 1e-9, 10.0, l_max=L)
        r = O.propagate(g, prm, x0[None], u0[None], [E], [2])
        assert r["status"][0] == 2 and r["length"][0] == L
        errs.append(max(np.linalg.norm(r["pos"][0] - xr) / rg, ang(r["dir"][0], ur)))
    assert errs[-1] < 1e-8
    assert all(errs[i + 1] < errs[i] * 0.2 for i in range(len(errs) - 1)), errs
    # direction norm conserved to a few ulp after normalisation
    assert abs(np.linalg.norm(r["dir"][0]) - 1.0) < 4e-16


def test_fixed_step_convergence_orders(oracle_mod):
    """Global error of the 5th-order solution ~ h^5; embedded estimate ~ h^5 per step."""
    O = oracle_mod
    g = uniform_grid(O, [0.0, 0.0, 1.0])
    E = 1e18
    kb = O.kappa(1, E)
    u0 = np.array([0.6, 0.0, 0.8])
    y0 = np.concatenate([np.zeros(3), u0])
    L = 2.0
    xr, ur = helix(u0, np.zeros(3), kb, L)
    errs = []
    for m in (8, 16, 32, 64):
        y = O.fixed_steps(g, kb, y0, L / m, m)
        errs.append(np.linalg.norm(y[:3] - xr) + np.linalg.norm(y[3:] - ur))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(3)]
    assert all(4.8 < q < 5.3 for q in rates), rates
    dl = []
    for h in (0.4, 0.2, 0.1):
        _, d = O.ck_eval(g, kb, y0, h)
        dl.append(np.linalg.norm(d))
    r1 = math.log2(dl[0] / dl[1])
    r2 = math.log2(dl[1] / dl[2])
    assert 4.7 < r1 < 5.3 and 4.7 < r2 < 5.3, (r1, r2)


def test_steps_shrink_where_deflection_is_strong(oracle_mod):
    """Smaller rigidity (stronger deflection) -> more, smaller steps (paper, section 3.1)."""
    O = oracle_mod
    w = ci.get_config(0)
    fs, _, _ = ci.config_seeds(0)
    B = ci.kolmogorov_field(w.grid_n, w.spacing, w.l_min, w.l_max, w.b_rms, fs)
    g = O.Grid(B, w.spacing)
    u = np.tile([[0.48, 0.6, 0.64]], (4, 1))
    E = np.array([1e20, 1e19, 1e18, 1e17])
    prm = O.params_array(1e-4, 0.001, 1.0, l_max=20.0)
    r = O.propagate(g, prm, np.zeros((4, 3)), u, E, np.ones(4, np.int32))
    assert np.all(np.diff(r["n_acc"]) > 0), r["n_acc"]


def test_rigidity_scaling_is_bitwise(oracle_mod):
    """Trajectories depend on (Z, E) only through E/Z (paper, section 3.3);
    power-of-two rescalings of kappa and of kappa*B are exact in FP64."""
    O = oracle_mod
    w = ci.get_config(0)
    fs, ps, _ = ci.config_seeds(0)
    B = ci.kolmogorov_field(w.grid_n, w.spacing, w.l_min, w.l_max, w.b_rms, fs)
    P = ci.isotropic_particles(40, 1e17, 1e19, (1,), ps)
    prm = O.params_array(1e-4, 0.01, 1.0, radius=2.0, l_max=30.0)
    base = O.propagate(O.Grid(B, w.spacing), prm, P["pos"], P["dir"], P["energy"], P["charge"])
    dbl = O.propagate(O.Grid(B, w.spacing), prm, P["pos"], P["dir"], 2 * P["energy"], 2 * P["charge"])
    fld = O.propagate(O.Grid(2 * B, w.spacing), prm, P["pos"], P["dir"], 2 * P["energy"], P["charge"])
    for k in ("pos", "dir", "length", "n_acc", "n_rej", "status", "h_next"):
        assert np.array_equal(base[k], dbl[k]), k
        assert np.array_equal(base[k], fld[k]), k


def test_time_reversal_retraces_path(oracle_mod):
    """Backtracking (paper, section 3.3): reverse u and Z, propagate the same length."""
    O = oracle_mod
    w = ci.get_config(0)
    fs, ps, _ = ci.config_seeds(0)
    B = ci.kolmogorov_field(w.grid_n, w.spacing, w.l_min, w.l_max, w.b_rms, fs)
    g = O.Grid(B, w.spacing)
    P = ci.isotropic_particles(20, 2e19, 1e20, (1,), ps)  # r_g >> L_c: not chaotic
    L = 10.0
    miss = []
    for tol in (1e-9, 1e-12):
        prm = O.params_array(tol, 1e-9, 0.2, l_max=L)
        f = O.propagate(g, prm, P["pos"], P["dir"], P["energy"], P["charge"])
        b = O.propagate(g, prm, f["pos"], -f["dir"], P["energy"], -P["charge"])
        miss.append(np.max(np.linalg.norm(b["pos"] - P["pos"], axis=1)))
        # the return error is of order (tol x path) times the number of cell faces crossed
        assert miss[-1] < 1e4 * tol * L, miss
        dots = np.sum(-b["dir"] * P["dir"], axis=1)
        assert np.min(dots) > 1 - 1e3 * tol
    assert miss[1] < 1e-2 * miss[0]


def _brute_force(Bgrid, h, kap, y0, L):
    n = Bgrid.shape[:3]
    vp = np.pad(Bgrid, ((0, 1), (0, 1), (0, 1), (0, 0)), mode="wrap")
    axes = [np.arange(k + 1) * h for k in n]
    interp = [RegularGridInterpolator(axes, vp[..., c]) for c in range(3)]
    box = np.array(n) * h

    def f(s, y):
        xr = np.mod(y[:3], box)[None]
        Bv = np.array([interp[c](xr)[0] for c in range(3)])
        u = y[3:]
        return np.concatenate([u, kap * np.cross(u, Bv)])

    sol = solve_ivp(f, (0.0, L), y0, method="DOP853", rtol=1e-12, atol=1e-13)
    return sol.y[:, -1]


def test_brute_force_convergence(oracle_mod):
    """Adaptive result approaches an independent tight-tolerance integration as tol -> 0."""
    O = oracle_mod
    w = ci.get_config(0)
    fs, _, _ = ci.config_seeds(0)
    B = ci.kolmogorov_field(w.grid_n, w.spacing, w.l_min, w.l_max, w.b_rms, fs)
    g = O.Grid(B, w.spacing)
    E, Z = 5e18, 1
    kap = O.kappa(Z, E)
    u0 = np.array([0.36, -0.48, 0.8])
    L = 3.0
    ref = _brute_force(B, w.spacing, kap, np.concatenate([np.zeros(3), u0]), L)
    diffs = []
    for tol in (1e-4, 1e-6, 1e-8, 1e-10):
        prm = O.params_array(tol, 1e-7, 1.0, l_max=L)
        r = O.propagate(g, prm, np.zeros((1, 3)), u0[None], [E], [Z])
        diffs.append(np.linalg.norm(r["pos"][0] - ref[:3]) / L)
    assert diffs[-1] < 1e-8, diffs
    assert all(diffs[i + 1] < diffs[i] for i in range(3)), diffs
