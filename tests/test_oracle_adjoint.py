"""Pins of the oracle's derivatives of the replayed (frozen-step) map.

* the replay reproduces the forward run bitwise;
* forward mode (dual numbers) and reverse mode (full tape) agree through the
  dot-product identity <w, J v> = <J^T w, v>, for initial-direction,
  initial-position and grid directions;
* central finite differences of the replay map agree with forward mode (and
  with the reverse sweep's position and kappa gradients) where the map is
  smooth at the difference scale (trilinear fields are only C0);
* in a uniform field with a length stop the direction map is the rotation by
  -kappa B L about B, and the time gradient is zero;
* the grid gradient is supported on the cells the trajectory visits.
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


def _taped(O, g, prm, x0, u0, E, Z):
    t = O.propagate_taped(g, prm, x0, u0, E, Z)
    assert t["status"] in (1, 2)
    return t


def _cases(O, g, ps, n=6, E=(3e18, 3e19), R=2.0):
    P = ci.isotropic_particles(n, E[0], E[1], (1, 26), ps)
    prm = O.params_array(1e-6, 1e-7, 0.2, radius=R, l_max=30.0)
    out = []
    for i in range(n):
        t = _taped(O, g, prm, P["pos"][i], P["dir"][i], P["energy"][i], P["charge"][i])
        out.append((P["pos"][i], P["dir"][i], O.kappa(P["charge"][i], P["energy"][i]), t))
    return out, R


def test_replay_reproduces_forward(oracle_mod, kolmo):
    O = oracle_mod
    w, g, B, ps = kolmo
    cases, R = _cases(O, g, ps)
    for x0, u0, kap, t in cases:
        r = O.replay_tangent(g, kap, x0, u0, t["tape"], t["event"], radius=R)
        assert np.array_equal(r["u"], t["y"][3:]) and np.array_equal(r["x"], t["y"][:3])
        assert r["length"] == t["length"]


def test_dot_product_identity_direction_and_grid(oracle_mod, kolmo):
    O = oracle_mod
    w, g, B, ps = kolmo
    cases, R = _cases(O, g, ps)
    rng = np.random.default_rng(11)
    for x0, u0, kap, t in cases:
        ub = rng.standard_normal(3)
        lb = rng.standard_normal()
        gbar = np.zeros_like(B)
        adj = O.replay_adjoint(g, kap, x0, u0, t["tape"], t["event"], ub, lb, radius=R, gbar=gbar)
        v = rng.standard_normal(3)
        tan = O.replay_tangent(g, kap, x0, u0, t["tape"], t["event"], radius=R, du0=v)
        lhs = ub @ tan["du"] + lb * tan["dlength"]
        rhs = adj["u0bar"] @ v
        assert abs(lhs - rhs) <= 1e-11 * (abs(lhs) + np.linalg.norm(adj["u0bar"]) * np.linalg.norm(v) + 1e-300)
        vg = rng.standard_normal(B.shape)
        tan = O.replay_tangent(g, kap, x0, u0, t["tape"], t["event"], radius=R, vgrid=vg)
        lhs = ub @ tan["du"] + lb * tan["dlength"]
        rhs = float(np.sum(gbar * vg))
        assert abs(lhs - rhs) <= 1e-11 * (abs(lhs) + np.sqrt(np.sum(gbar ** 2) * np.sum(vg ** 2)))


def test_dot_product_identity_position(oracle_mod, kolmo):
    """The reverse sweep's position cotangent against forward mode in the
    initial position.  Forward mode forms (dB/dX) X-dot component by
    component, sum over corners of (grad w . X-dot) G; the reverse sweep
    forms (dB/dX)^T B-bar as the sum over corners of grad w (G . B-bar).  The
    two orders differ only in rounding, so the identity holds to rounding
    whatever grouping either side uses."""
    O = oracle_mod
    w, g, B, ps = kolmo
    P = ci.isotropic_particles(8, 3e18, 3e19, (1, 26), ps)
    R = 2.0
    prm = O.params_array(1e-6, 1e-7, 0.2, radius=R, l_max=30.0)
    rng = np.random.default_rng(14)
    for i in range(8):
        x0 = rng.uniform(-0.05, 0.05, 3)
        t = _taped(O, g, prm, x0, P["dir"][i], P["energy"][i], P["charge"][i])
        u0, kap = P["dir"][i], O.kappa(P["charge"][i], P["energy"][i])
        ub, lb = rng.standard_normal(3), rng.standard_normal()
        adj = O.replay_adjoint(g, kap, x0, u0, t["tape"], t["event"], ub, lb, radius=R)
        v = rng.standard_normal(3)
        tan = O.replay_tangent(g, kap, x0, u0, t["tape"], t["event"], radius=R, dx0=v)
        lhs = ub @ tan["du"] + lb * tan["dlength"]
        rhs = adj["x0bar"] @ v
        assert abs(lhs - rhs) <= 1e-11 * (abs(lhs) + np.linalg.norm(adj["x0bar"]) * np.linalg.norm(v)), (lhs, rhs)
        # the position tangent alone moves nothing else: du0 = 0 gives the same
        tan0 = O.replay_tangent(g, kap, x0, u0, t["tape"], t["event"], radius=R)
        assert np.all(tan0["du"] == 0.0) and tan0["dlength"] == 0.0


def test_central_differences(oracle_mod, kolmo):
    O = oracle_mod
    w, g, B, ps = kolmo
    cases, R = _cases(O, g, ps, n=16)
    rng = np.random.default_rng(12)
    used = 0
    for x0, u0, kap, t in cases:
        v = np.cross(u0, rng.standard_normal(3))
        v /= np.linalg.norm(v)
        tan = O.replay_tangent(g, kap, x0, u0, t["tape"], t["event"], radius=R, du0=v)
        jv = np.concatenate([tan["du"], [tan["dlength"]]])

        def fd(eps):
            a = O.replay_tangent(g, kap, x0, u0 + eps * v, t["tape"], t["event"], radius=R)
            b = O.replay_tangent(g, kap, x0, u0 - eps * v, t["tape"], t["event"], radius=R)
            return (np.concatenate([a["u"], [a["length"]]]) - np.concatenate([b["u"], [b["length"]]])) / (2 * eps)

        try:
            d1, d2 = fd(1e-6), fd(2e-6)
        except ValueError:
            continue  # the perturbed crossing left the frozen last step: outside the map's domain
        if np.linalg.norm(d1 - d2) > 1e-6 * np.linalg.norm(d1):
            continue  # a cell face inside the difference interval: the map is only C0 there
        used += 1
        assert np.linalg.norm(d1 - jv) <= 1e-4 * np.linalg.norm(jv), (d1, jv)
    assert used >= 5


def test_central_differences_position_and_kappa(oracle_mod, kolmo):
    """The position and kappa gradients of the reverse sweep against central
    differences of the replay map, from starts off the grid's nodes (at a node
    the trilinear field has a kink and a central difference averages the
    one-sided slopes); used where steps of 1e-7 and 1e-8 agree to 2e-6."""
    O = oracle_mod
    w, g, B, ps = kolmo
    P = ci.isotropic_particles(12, 3e18, 3e19, (1, 26), ps)
    R = 2.0
    prm = O.params_array(1e-6, 1e-7, 0.2, radius=R, l_max=30.0)
    rng = np.random.default_rng(13)
    used = {"x": 0, "kappa": 0}
    for i in range(12):
        x0 = rng.uniform(-0.05, 0.05, 3)
        t = _taped(O, g, prm, x0, P["dir"][i], P["energy"][i], P["charge"][i])
        u0, kap = P["dir"][i], O.kappa(P["charge"][i], P["energy"][i])
        ub, lb = rng.standard_normal(3), rng.standard_normal()
        adj = O.replay_adjoint(g, kap, x0, u0, t["tape"], t["event"], ub, lb, radius=R)

        def J(x=x0, k=kap):
            r = O.replay_tangent(g, k, x, u0, t["tape"], t["event"], radius=R)
            return ub @ r["u"] + lb * r["length"]

        e = rng.standard_normal(3)
        e /= np.linalg.norm(e)
        for name, f, want in (("x", lambda s: J(x=x0 + s * e), adj["x0bar"] @ e),
                              ("kappa", lambda s: J(k=kap * (1.0 + s)) / kap, adj["kappabar"])):
            try:
                d1 = (f(1e-7) - f(-1e-7)) / 2e-7
                d2 = (f(1e-8) - f(-1e-8)) / 2e-8
            except ValueError:
                continue  # the perturbed crossing left the frozen last step
            if abs(d1 - d2) > 2e-6 * max(abs(d2), 1e-3):
                continue  # a cell face inside the difference interval
            used[name] += 1
            assert abs(d2 - want) <= 1e-5 * max(abs(d2), 1e-3), (name, d2, want)
    assert min(used.values()) >= 6, used


def test_uniform_field_rotation_and_zero_time_gradient(oracle_mod):
    O = oracle_mod
    Bv = np.array([0.3, -0.5, 0.8])
    grid = np.empty((4, 4, 4, 3))
    grid[...] = Bv
    g = O.Grid(grid, 1.0)
    E, Z = 2e18, 1
    kap = O.kappa(Z, E)
    L = 3.0
    u0 = np.array([0.6, 0.0, 0.8])
    prm = O.params_array(1e-10, 1e-8, 0.05, l_max=L)
    t = _taped(O, g, prm, np.zeros(3), u0, E, Z)
    assert t["status"] == 2 and not t["event"]
    J = np.zeros((3, 3))
    for a in range(3):
        e = np.zeros(3)
        e[a] = 1.0
        J[:, a] = O.replay_tangent(g, kap, np.zeros(3), u0, t["tape"], False, du0=e)["du"]
    bh = Bv / np.linalg.norm(Bv)
    ang = -kap * np.linalg.norm(Bv) * L
    K = np.array([[0, -bh[2], bh[1]], [bh[2], 0, -bh[0]], [-bh[1], bh[0], 0]])
    Rm = np.eye(3) + math.sin(ang) * K + (1 - math.cos(ang)) * K @ K
    Pt = np.eye(3) - np.outer(u0, u0)  # input direction is normalised first
    assert np.max(np.abs(J - Rm @ Pt)) < 1e-7
    adj = O.replay_adjoint(g, kap, np.zeros(3), u0, t["tape"], False, np.zeros(3), 1.0)
    assert np.all(adj["u0bar"] == 0.0)


def test_grid_gradient_support_follows_path(oracle_mod, kolmo):
    O = oracle_mod
    w, g, B, ps = kolmo
    u0 = np.array([0.48, 0.6, 0.64])
    E, Z = 1e20, 1  # nearly straight over 1.5 Mpc
    prm = O.params_array(1e-6, 1e-7, 0.05, l_max=1.5)
    t = _taped(O, g, prm, np.zeros(3), u0, E, Z)
    gbar = np.zeros_like(B)
    O.replay_adjoint(g, O.kappa(Z, E), np.zeros(3), u0, t["tape"], False, np.array([1.0, -2.0, 0.5]), 0.0,
                     gbar=gbar)
    nz = np.argwhere(np.any(gbar != 0.0, axis=-1))
    assert 0 < len(nz) < 0.05 * np.prod(B.shape[:3])
    pos = nz * w.spacing
    # distance of each supporting node from the straight segment 0 -> 1.5 u0 (wrapped box)
    box = w.grid_n * w.spacing
    best = np.full(len(pos), np.inf)
    for shift in np.array(np.meshgrid([-box, 0, box], [-box, 0, box], [-box, 0, box])).T.reshape(-1, 3):
        p = pos + shift
        s = np.clip(p @ u0, 0, 1.5)
        best = np.minimum(best, np.linalg.norm(p - s[:, None] * u0, axis=1))
    assert best.max() < 2.0 * math.sqrt(3) * w.spacing
