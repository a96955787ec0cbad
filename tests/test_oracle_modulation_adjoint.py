"""Pins of the oracle's derivatives of the replayed map for modulated fields
(section 3.2, modulated grids: B = b m).

The vector grid's value b takes the cotangent m B-bar; the position takes
(db/dX)^T m B-bar + (b . B-bar) dm/dX; the modulation grid's own values get
no gradient.

* the replay reproduces the modulated forward run bitwise;
* forward mode and reverse mode agree through the dot-product identity, for
  initial-direction, initial-position and grid directions;
* central differences of the replay map agree with the adjoint's direction,
  position and kappa gradients where the map is smooth at the difference
  scale (starts off both grids' nodes);
* kappa and the vector grid enter only as kappa b(G) m with b linear in G, so
  kappa kappa-bar = <G, G-bar>;
* a constant modulation c is the grid c G: on the same frozen steps the
  gradients agree, with G-bar (modulated) = c G-bar (scaled grid).
"""
import numpy as np
import pytest

import crp_inputs as ci

MOD_ORIGIN = (-0.13, 0.07, 0.21)  # modulation nodes off the vector grid's


@pytest.fixture(scope="module")
def modf(oracle_mod):
    O = oracle_mod
    w = ci.get_config(0)
    fs, ps, _ = ci.config_seeds(0)
    B = ci.kolmogorov_field(w.grid_n, w.spacing, w.l_min, w.l_max, w.b_rms, fs)
    M = ci.lognormal_modulation(8, 0.4, 0.8, 0.6, 77)
    g = O.Grid(B, w.spacing, modulation=O.Modulation(M, 0.4, MOD_ORIGIN))
    return w, g, B, M, ps


def _cases(O, g, ps, n=12):
    """Starts off both grids' nodes; a sphere of radius 2 with a long length
    limit (arrivals) for even i, a length stop at 3 Mpc for odd i."""
    P = ci.isotropic_particles(n, 3e18, 3e19, (1, 26), ps)
    starts = np.random.default_rng(60).uniform(-0.05, 0.05, (n, 3))
    out = []
    for i in range(n):
        R, lmax = (2.0, 30.0) if i % 2 == 0 else (0.0, 3.0)
        prm = O.params_array(1e-6, 1e-7, 0.2, radius=R, l_max=lmax)
        t = O.propagate_taped(g, prm, starts[i], P["dir"][i], P["energy"][i], P["charge"][i])
        assert t["status"] in (1, 2)
        out.append((starts[i], P["dir"][i], O.kappa(P["charge"][i], P["energy"][i]), t, R))
    return out


def test_replay_reproduces_modulated_forward(oracle_mod, modf):
    O = oracle_mod
    w, g, B, M, ps = modf
    events = 0
    for x0, u0, kap, t, R in _cases(O, g, ps):
        r = O.replay_tangent(g, kap, x0, u0, t["tape"], t["event"], radius=R)
        assert np.array_equal(r["u"], t["y"][3:]) and np.array_equal(r["x"], t["y"][:3])
        assert r["length"] == t["length"]
        events += t["event"]
    assert events >= 4


def test_dot_product_identity_modulated(oracle_mod, modf):
    O = oracle_mod
    w, g, B, M, ps = modf
    rng = np.random.default_rng(61)
    for x0, u0, kap, t, R in _cases(O, g, ps):
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
        # the position cotangent against forward mode in the initial position
        v = rng.standard_normal(3)
        tan = O.replay_tangent(g, kap, x0, u0, t["tape"], t["event"], radius=R, dx0=v)
        lhs = ub @ tan["du"] + lb * tan["dlength"]
        rhs = adj["x0bar"] @ v
        assert abs(lhs - rhs) <= 1e-11 * (abs(lhs) + np.linalg.norm(adj["x0bar"]) * np.linalg.norm(v) + 1e-300)


def test_central_differences_modulated(oracle_mod, modf):
    """Differences of 1e-7 and 1e-8 used where they agree to 2e-6 (no cell face
    of either grid inside the larger one)."""
    O = oracle_mod
    w, g, B, M, ps = modf
    rng = np.random.default_rng(62)
    used = {"u": 0, "x": 0, "kappa": 0}
    for x0, u0, kap, t, R in _cases(O, g, ps, n=16):
        ub = rng.standard_normal(3)
        lb = rng.standard_normal() * (1.0 if t["event"] else 0.0)
        adj = O.replay_adjoint(g, kap, x0, u0, t["tape"], t["event"], ub, lb, radius=R)

        def J(x=x0, u=u0, k=kap):
            r = O.replay_tangent(g, k, x, u, t["tape"], t["event"], radius=R)
            return ub @ r["u"] + lb * r["length"]

        v = np.cross(u0, rng.standard_normal(3))
        v /= np.linalg.norm(v)
        e = rng.standard_normal(3)
        e /= np.linalg.norm(e)
        for name, f, want in (("u", lambda s: J(u=u0 + s * v), adj["u0bar"] @ v),
                              ("x", lambda s: J(x=x0 + s * e), adj["x0bar"] @ e),
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


def test_scaling_identity_modulated(oracle_mod, modf):
    O = oracle_mod
    w, g, B, M, ps = modf
    rng = np.random.default_rng(63)
    for x0, u0, kap, t, R in _cases(O, g, ps, n=8):
        ub, lb = rng.standard_normal(3), rng.standard_normal()
        gbar = np.zeros_like(B)
        adj = O.replay_adjoint(g, kap, x0, u0, t["tape"], t["event"], ub, lb, radius=R, gbar=gbar)
        lhs = kap * adj["kappabar"]
        rhs = float(np.sum(B * gbar))
        assert abs(lhs - rhs) <= 1e-10 * (abs(rhs) + np.sqrt(np.sum((B * gbar) ** 2))), (lhs, rhs)


def test_constant_modulation_is_a_scaled_grid(oracle_mod, modf):
    O = oracle_mod
    w, g, B, M, ps = modf
    c = 1.7
    gm = O.Grid(B, w.spacing, modulation=O.Modulation(np.full((6, 6, 6), c), 0.55, MOD_ORIGIN))
    gs = O.Grid(B * c, w.spacing)
    rng = np.random.default_rng(64)
    P = ci.isotropic_particles(8, 3e18, 3e19, (1, 26), ps)
    prm = O.params_array(1e-6, 1e-7, 0.2, radius=2.0, l_max=3.0)
    for i in range(8):
        x0 = rng.uniform(-0.05, 0.05, 3)
        t = O.propagate_taped(gm, prm, x0, P["dir"][i], P["energy"][i], P["charge"][i])
        kap = O.kappa(P["charge"][i], P["energy"][i])
        ub, lb = rng.standard_normal(3), rng.standard_normal()
        gbm, gbs = np.zeros_like(B), np.zeros_like(B)
        am = O.replay_adjoint(gm, kap, x0, P["dir"][i], t["tape"], t["event"], ub, lb, radius=2.0, gbar=gbm)
        a_s = O.replay_adjoint(gs, kap, x0, P["dir"][i], t["tape"], t["event"], ub, lb, radius=2.0, gbar=gbs)
        for k in ("u0bar", "x0bar"):
            assert np.linalg.norm(am[k] - a_s[k]) <= 1e-9 * (np.linalg.norm(a_s[k]) + 1e-12), k
        assert abs(am["kappabar"] - a_s["kappabar"]) <= 1e-9 * abs(a_s["kappabar"])
        assert np.linalg.norm(gbm - c * gbs) <= 1e-9 * np.linalg.norm(c * gbs)
