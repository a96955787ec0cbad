"""Pins of the oracle's rigidity derivative (the kappa cotangent of the
replayed map; kappa = Z K / E, so d/dE = -kappa/E d/dkappa).  It is the
sensitivity of a lens to the rigidity of its particles (section 3.3).

* scaling: the equation of motion holds kappa and the field only as the
  product kappa B, and B is linear in the grid values G, so
  kappa * kappa-bar = <G, G-bar> (the grid gradient is pinned separately);
* central finite differences of the replay map in kappa, where the map is
  smooth at the difference scale;
* a uniform field with a length stop: the direction is rotated by -kappa |B| L
  about B, so d u_N / d kappa = -|B| L (b x u_N), and the path length does not
  depend on kappa.
"""
import math

import numpy as np
import pytest

import crp_inputs as ci


@pytest.fixture(scope="module")
def kolmo(oracle_mod):
    w = ci.get_config(0)
    fs, ps, _ = ci.config_seeds(0)
    B = ci.kolmogorov_field(w.grid_n, w.spacing, w.l_min, w.l_max, w.b_rms, fs)
    return w, oracle_mod.Grid(B, w.spacing), B, ps


def _cases(O, g, ps, n, R=2.0):
    P = ci.isotropic_particles(n, 3e18, 3e19, (1, 26), ps)
    prm = O.params_array(1e-6, 1e-7, 0.2, radius=R, l_max=30.0)
    out = []
    for i in range(n):
        t = O.propagate_taped(g, prm, P["pos"][i], P["dir"][i], P["energy"][i], P["charge"][i])
        assert t["status"] in (1, 2)
        out.append((P["pos"][i], P["dir"][i], O.kappa(P["charge"][i], P["energy"][i]), t))
    return out, R


def test_scaling_identity(oracle_mod, kolmo):
    O = oracle_mod
    w, g, B, ps = kolmo
    cases, R = _cases(O, g, ps, 8)
    rng = np.random.default_rng(4)
    events = 0
    for x0, u0, kap, t in cases:
        events += bool(t["event"])
        ub, lb = rng.standard_normal(3), rng.standard_normal()
        gbar = np.zeros_like(B)
        adj = O.replay_adjoint(g, kap, x0, u0, t["tape"], t["event"], ub, lb, radius=R, gbar=gbar)
        lhs = kap * adj["kappabar"]
        rhs = float(np.sum(B * gbar))
        assert abs(lhs - rhs) <= 1e-10 * (abs(rhs) + np.sqrt(np.sum((B * gbar) ** 2))), (lhs, rhs)
    assert events >= 2


def test_central_differences_in_kappa(oracle_mod, kolmo):
    O = oracle_mod
    w, g, B, ps = kolmo
    cases, R = _cases(O, g, ps, 16)
    rng = np.random.default_rng(6)
    used = 0
    for x0, u0, kap, t in cases:
        ub, lb = rng.standard_normal(3), rng.standard_normal()
        adj = O.replay_adjoint(g, kap, x0, u0, t["tape"], t["event"], ub, lb, radius=R)

        def f(k):
            r = O.replay_tangent(g, k, x0, u0, t["tape"], t["event"], radius=R)
            return ub @ r["u"] + lb * r["length"]

        try:
            d1 = (f(kap * (1 + 1e-7)) - f(kap * (1 - 1e-7))) / (2e-7 * kap)
            d2 = (f(kap * (1 + 2e-7)) - f(kap * (1 - 2e-7))) / (4e-7 * kap)
        except ValueError:
            continue  # the perturbed crossing left the frozen last step
        if abs(d1 - d2) > 1e-5 * abs(d1):
            continue  # a cell face inside the difference interval
        used += 1
        assert abs(d1 - adj["kappabar"]) <= 1e-4 * abs(d1), (d1, adj["kappabar"])
    assert used >= 5


def test_uniform_field_rotation_rate(oracle_mod):
    O = oracle_mod
    Bv = np.array([0.3, -0.5, 0.8])
    grid = np.empty((4, 4, 4, 3))
    grid[...] = Bv
    g = O.Grid(grid, 1.0)
    E, Z = 2e18, 2
    kap = O.kappa(Z, E)
    L = 3.0
    u0 = np.array([0.6, 0.0, 0.8])
    t = O.propagate_taped(g, O.params_array(1e-10, 1e-8, 0.05, l_max=L), np.zeros(3), u0, E, Z)
    assert t["status"] == 2 and not t["event"]
    uN = t["y"][3:]
    bh = Bv / np.linalg.norm(Bv)
    du = -np.linalg.norm(Bv) * L * np.cross(bh, uN)
    for ub in np.eye(3):
        adj = O.replay_adjoint(g, kap, np.zeros(3), u0, t["tape"], False, ub, 0.0)
        assert abs(adj["kappabar"] - ub @ du) < 1e-6 * np.linalg.norm(du)
    adj = O.replay_adjoint(g, kap, np.zeros(3), u0, t["tape"], False, np.zeros(3), 1.0)
    assert adj["kappabar"] == 0.0
