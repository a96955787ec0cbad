"""Pins of the oracle's step controller, stop conditions and failure handling.

The fifth root of the controller is compared with mpmath; stops are checked
against their exact definitions (length stop lands on L_max bitwise, sphere
crossing lies on the sphere); a run interrupted by the step budget and
resumed is bitwise identical to an uninterrupted run; bad inputs and
non-finite fields give their status without disturbing other particles.
"""
import math

import mpmath
import numpy as np
import pytest

import crp_inputs as ci


@pytest.fixture(scope="module")
def c1(oracle_mod):
    w = ci.get_config(0)
    fs, ps, _ = ci.config_seeds(0)
    B = ci.kolmogorov_field(w.grid_n, w.spacing, w.l_min, w.l_max, w.b_rms, fs)
    P = ci.isotropic_particles(w.n_particles, w.e_min, w.e_max, w.charges, ps)
    return w, oracle_mod.Grid(B, w.spacing), P, B


def test_inv_fifth_root_against_mpmath(oracle_mod):
    mpmath.mp.dps = 40
    rng = np.random.default_rng(20)
    xs = np.concatenate([10.0 ** rng.uniform(-12, 6, 20000), 2.0 ** np.arange(-40, 21),
                         [1.0, 0.5, 0.9999999999999999, 1e-300, 5e-324, 1.7e308]])
    worst = 0
    for x in xs:
        got = oracle_mod.inv_fifth_root(float(x))
        ref = mpmath.power(mpmath.mpf(float(x)), mpmath.mpf(-1) / 5)
        ulp = math.ulp(float(ref))
        worst = max(worst, abs(float((mpmath.mpf(got) - ref) / ulp)))
    assert worst <= 4.0, worst
    assert oracle_mod.inv_fifth_root(1.0) == 1.0
    assert oracle_mod.inv_fifth_root(32.0) == 0.5


def test_length_stop_lands_exactly(oracle_mod, c1):
    w, g, P, _ = c1
    prm = oracle_mod.params_array(w.tol, w.h_min, w.h_max, l_max=7.3)
    r = oracle_mod.propagate(g, prm, P["pos"][:100], P["dir"][:100], P["energy"][:100],
                             P["charge"][:100])
    assert np.all(r["status"] == 2)
    assert np.all(r["length"] == 7.3)


def test_sphere_arrival_on_the_sphere(oracle_mod, c1):
    w, g, P, _ = c1
    R = 2.5
    c = np.array([0.01, -0.02, 0.03])
    prm = oracle_mod.params_array(w.tol, w.h_min, w.h_max, center=c, radius=R, l_max=100.0)
    r = oracle_mod.propagate(g, prm, P["pos"][:200], P["dir"][:200], P["energy"][:200],
                             P["charge"][:200])
    assert np.all(r["status"] == 1)
    d = np.linalg.norm(r["pos"] - c, axis=1)
    assert np.max(np.abs(d - R)) <= 1e-13 * R
    assert np.all(d >= R * (1 - 1e-15))
    assert r["counters"]["event_evals"] > 0
    # arrival time is the path length at the speed of light
    assert np.array_equal(r["time"], r["length"] * oracle_mod.constants()["MPC_OVER_C"])


def test_event_point_is_on_the_trajectory(oracle_mod, c1):
    """The located crossing equals a propagation stopped by length at that L."""
    w, g, P, _ = c1
    prm = oracle_mod.params_array(1e-9, 1e-9, 0.05, radius=1.5, l_max=100.0)
    sel = slice(0, 10)
    r = oracle_mod.propagate(g, prm, P["pos"][sel], P["dir"][sel], P["energy"][sel], P["charge"][sel])
    prm2 = oracle_mod.params_array(1e-9, 1e-9, 0.05, l_max=100.0)
    for i in range(10):
        p2 = prm2.copy()
        p2[7] = r["length"][i]
        q = oracle_mod.propagate(g, p2, P["pos"][i:i + 1], P["dir"][i:i + 1], P["energy"][i:i + 1],
                                 P["charge"][i:i + 1])
        assert np.linalg.norm(q["pos"][0] - r["pos"][i]) < 1e-7


def test_start_outside_sphere_arrives_without_step(oracle_mod, c1):
    w, g, P, _ = c1
    prm = oracle_mod.params_array(w.tol, w.h_min, w.h_max, radius=1.0, l_max=100.0)
    pos = np.array([[1.5, 0.0, 0.0], [0.0, 1.0, 0.0]])
    r = oracle_mod.propagate(g, prm, pos, P["dir"][:2], P["energy"][:2], P["charge"][:2])
    assert np.all(r["status"] == 1) and np.all(r["n_acc"] == 0)
    assert np.array_equal(r["pos"], pos)


def test_resume_after_step_budget_is_bitwise(oracle_mod, c1):
    w, g, P, _ = c1
    n = 64
    prm = oracle_mod.params_array(w.tol, w.h_min, w.h_max, radius=3.0, l_max=w.max_length)
    full = oracle_mod.propagate(g, prm, P["pos"][:n], P["dir"][:n], P["energy"][:n], P["charge"][:n])
    st = oracle_mod.propagate(g, prm, P["pos"][:n], P["dir"][:n], P["energy"][:n], P["charge"][:n],
                              max_steps=7)
    rounds = 0
    while np.any(st["status"] == 3):
        assert np.all(st["n_acc"][st["status"] == 3] % 7 == 0)
        status = np.where(st["status"] == 3, 0, st["status"]).astype(np.int32)
        st = oracle_mod.propagate(g, prm, st["pos"], st["dir"], P["energy"][:n], P["charge"][:n],
                                  length=st["length"], h_next=st["h_next"], status=status,
                                  n_acc=st["n_acc"], n_rej=st["n_rej"], max_steps=7)
        rounds += 1
    assert rounds > 2
    for k in ("pos", "dir", "length", "h_next", "status", "n_acc", "n_rej"):
        assert np.array_equal(full[k], st[k]), k


def test_inactive_particles_untouched(oracle_mod, c1):
    w, g, P, _ = c1
    prm = oracle_mod.params_array(w.tol, w.h_min, w.h_max, l_max=5.0)
    status = np.array([2, 1, 4, 0], np.int32)
    r = oracle_mod.propagate(g, prm, P["pos"][:4], P["dir"][:4], P["energy"][:4], P["charge"][:4],
                             status=status)
    assert list(r["status"]) == [2, 1, 4, 2]
    assert np.all(r["n_acc"][:3] == 0) and np.array_equal(r["dir"][:3], P["dir"][:3])


def test_bad_inputs_get_status(oracle_mod, c1):
    w, g, P, _ = c1
    prm = oracle_mod.params_array(w.tol, w.h_min, w.h_max, l_max=5.0)
    pos = np.zeros((5, 3))
    pos[3, 1] = np.nan
    d = np.tile([[1.0, 0.0, 0.0]], (5, 1))
    d[1] = 0.0
    E = np.array([1e18, 1e18, -1.0, 1e18, 1e18])
    r = oracle_mod.propagate(g, prm, pos, d, E, np.ones(5, np.int32))
    assert list(r["status"]) == [2, 6, 6, 6, 2]


def test_zero_charge_is_a_straight_line(oracle_mod, c1):
    w, g, P, _ = c1
    prm = oracle_mod.params_array(w.tol, w.h_min, w.h_max, l_max=12.0)
    r = oracle_mod.propagate(g, prm, P["pos"][:5], P["dir"][:5], P["energy"][:5], np.zeros(5, np.int32))
    assert np.allclose(r["pos"], 12.0 * P["dir"][:5], rtol=0, atol=1e-13 * 12)
    assert np.all(r["n_rej"] == 0)


def test_nonfinite_field_flags_only_affected(oracle_mod, c1):
    w, _, P, B = c1
    Bn = B.copy()
    Bn[0, 0, 0, :] = np.nan
    g = oracle_mod.Grid(Bn, w.spacing)
    prm = oracle_mod.params_array(w.tol, w.h_min, w.h_max, l_max=5.0)
    pos = np.array([[0.05, 0.05, 0.05], [1.6, 1.6, 1.6]])
    r = oracle_mod.propagate(g, prm, pos, P["dir"][:2], P["energy"][:2], P["charge"][:2])
    assert list(r["status"]) == [4, 2]


@pytest.mark.parametrize("prm", [
    [0.0, 0.01, 1.0, 0, 0, 0, 0, 10.0],          # tol <= 0
    [1e-4, 0.0, 1.0, 0, 0, 0, 0, 10.0],          # h_min <= 0
    [1e-4, 2.0, 1.0, 0, 0, 0, 0, 10.0],          # h_min > h_max
    [1e-4, 0.01, 1.0, 0, 0, 0, 5.0, math.inf],   # no length limit, no budget
    [1e-4, 0.01, 1.0, 0, 0, 0, 0, -1.0],         # negative length limit
])
def test_invalid_parameters_rejected(oracle_mod, c1, prm):
    w, g, P, _ = c1
    with pytest.raises(ValueError):
        oracle_mod.propagate(g, np.array(prm, np.float64), P["pos"][:1], P["dir"][:1],
                             P["energy"][:1], P["charge"][:1])


def test_counters_add_up(oracle_mod, c1):
    w, g, P, _ = c1
    prm = oracle_mod.params_array(w.tol, w.h_min, w.h_max, radius=2.0, l_max=w.max_length)
    r = oracle_mod.propagate(g, prm, P["pos"], P["dir"], P["energy"], P["charge"])
    c = r["counters"]
    assert c["accepted"] == r["n_acc"].sum() and c["rejected"] == r["n_rej"].sum()
    assert c["evals"] == c["accepted"] + c["rejected"] + c["event_evals"]
