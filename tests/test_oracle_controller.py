"""Pins of the oracle's step controller and error norm against closed forms.

The paper asks for the largest step that still keeps the accuracy the user
set (section 3.1, bidding system); the oracle reads this as an embedded
Cash-Karp 5(4) error estimate with err = max(|delta_u|, |delta_x| / h) / tol,
rejection shrink max(0.1, 0.9 err^-1/4), growth min(5, 0.9 err^-1/5).

In a uniform field with the direction normal to B, the direction moves on a
circle, w' = -i omega w (w = u_x + i u_y, omega = kappa B), and the position
follows p' = w.  Both are linear, so every Cash-Karp stage is a polynomial in
z = -i omega h applied to the current state, and the error estimate's norms
are functions of h alone (the rotation leaves them unchanged).  They are
computed here in 40-digit arithmetic from the tableau as exact rationals
(the tableau itself is pinned by the order conditions in
test_oracle_tableau.py).  From that function:

* the controller's fixed point h* solves 0.9 err(h*)^(-1/5) = 1, i.e.
  err(h*) = 0.9^5, and the oracle's accepted steps must settle on it;
* a fresh start at h_max is rejected and shrunk along the chain
  h <- h max(0.1, 0.9 err(h)^(-1/4)) until err(h) <= 1;
* with no field the estimate vanishes and each bid grows by exactly 5.

A different safety factor, growth cap, shrink floor or exponent, or |delta_x|
in place of |delta_x| / h, changes these numbers far beyond the tolerances
used (checked below on the 40-digit side as well).
"""
from fractions import Fraction

import mpmath
import numpy as np
import pytest

mpmath.mp.dps = 40


def _rat(x: float) -> Fraction:
    r = Fraction(x).limit_denominator(10 ** 7)
    assert float(r) == x
    return r


@pytest.fixture(scope="module")
def tab(oracle_mod):
    c = oracle_mod.constants()
    A = [[_rat(v) for v in row] for row in c["A"]]
    e = [_rat(v) for v in c["e"]]
    return A, e


def _mpf(q: Fraction):
    return mpmath.mpf(q.numerator) / q.denominator


def error_norms(tab, h, omega):
    """(|delta_u|, |delta_x|) of one Cash-Karp attempt of size h for the
    circular motion w' = -i omega w, p' = w from |w| = 1, at 40 digits."""
    A, e = tab
    h = mpmath.mpf(h)
    lam = mpmath.mpc(0, -1) * mpmath.mpf(omega)
    W = []
    for i in range(6):
        acc = mpmath.mpc(0)
        for j in range(i):
            acc += _mpf(A[i][j]) * lam * W[j]
        W.append(mpmath.mpc(1) + h * acc)
    du = abs(h * sum(_mpf(e[i]) * lam * W[i] for i in range(6)))
    dx = abs(h * sum(_mpf(e[i]) * W[i] for i in range(6)))
    return du, dx


def err_of(tab, h, omega, tol, norm="max"):
    du, dx = error_norms(tab, h, omega)
    h = mpmath.mpf(h)
    if norm == "max":
        v = max(du, dx / h)
    elif norm == "no_h":          # |delta_x| not divided by h
        v = max(du, dx)
    elif norm == "sum":
        v = du + dx / h
    else:                         # direction part only
        v = du
    return v / mpmath.mpf(tol)


def steady_step(tab, omega, tol, h0, safety="0.9", expo=5, norm="max"):
    target = mpmath.mpf(safety) ** expo
    return mpmath.findroot(lambda x: err_of(tab, x, omega, tol, norm) - target, h0)


def uniform_grid(O, b):
    v = np.empty((4, 4, 4, 3))
    v[...] = b
    return O.Grid(v, 1.0)


@pytest.mark.parametrize("tol, dominant", [(1e-4, "position"), (1e-2, "direction")])
def test_steady_step_in_uniform_field(oracle_mod, tab, tol, dominant):
    O = oracle_mod
    E, B = 1e18, 1.0
    omega = O.kappa(1, E) * B
    g = uniform_grid(O, [0.0, 0.0, B])
    prm = O.params_array(tol, 1e-6, 20.0, l_max=200.0 if tol > 1e-3 else 30.0)
    r = O.propagate_taped(g, prm, [0.0, 0.0, 0.0], [1.0, 0.0, 0.0], E, 1)
    h = r["tape"]
    assert r["length_bound"] and len(h) > 30
    late = h[-6:-1]                      # settled steps before the final length step
    hs = steady_step(tab, omega, tol, float(late[-1]))
    # which part of the error norm decides at h*: |delta_x|/h while h omega < 1
    du, dx = error_norms(tab, hs, omega)
    assert (dx / hs > du) == (dominant == "position")
    assert mpmath.almosteq(err_of(tab, hs, omega, tol), mpmath.mpf("0.9") ** 5, 1e-30)
    # the oracle's err carries the rounding of a cancelling sum (sum e_i = 0),
    # about 1e-16 / tol relative, and h* moves by a quarter of that
    rel = np.abs(late / float(hs) - 1.0)
    assert rel.max() <= 1e-11, (late, hs)
    # the readings this pins: each alternative moves h* by far more than that
    alts = [dict(safety="0.8"), dict(expo=4), dict(norm="no_h"), dict(norm="sum")]
    if dominant == "position":
        alts.append(dict(norm="u"))
    for alt in alts:
        ha = steady_step(tab, omega, tol, float(hs), **alt)
        assert abs(ha / hs - 1) > 1e-3, alt


def _shrink_chain(tab, h_max, omega, tol):
    """Attempt sizes of a fresh start: h_max, shrunk by max(0.1, 0.9 err^-1/4)
    until err <= 1.  Returns (accepted h, rejections, floor-limited shrinks)."""
    h = mpmath.mpf(h_max)
    rej = floor = 0
    while True:
        err = err_of(tab, h, omega, tol)
        assert abs(err - 1) > 1e-6, "decision too close to call"
        if err <= 1:
            return h, rej, floor
        fac = mpmath.mpf("0.9") * err ** mpmath.mpf("-0.25")
        if fac < mpmath.mpf("0.1"):
            fac = mpmath.mpf("0.1")
            floor += 1
        h = h * fac
        rej += 1


@pytest.mark.parametrize("B, h_max, want_floor", [(3.0, 1.0, False), (40.0, 1.0, True), (2.0, 5.0, True)])
def test_first_attempt_shrink_chain(oracle_mod, tab, B, h_max, want_floor):
    O = oracle_mod
    E = 1e18
    omega = O.kappa(1, E) * B
    tol = 1e-4
    g = uniform_grid(O, [0.0, 0.0, B])
    prm = O.params_array(tol, 1e-9, h_max, l_max=1e3)
    r = O.propagate(g, prm, np.zeros((1, 3)), np.array([[1.0, 0.0, 0.0]]), [E], [1], max_steps=1)
    h_acc, rej, floor = _shrink_chain(tab, h_max, omega, tol)
    assert rej >= 1 and (floor > 0) == want_floor
    assert r["n_rej"][0] == rej and r["n_acc"][0] == 1
    # the first accepted step is the path length after one step
    # (each shrink factor carries the rounding of the cancelling error sum,
    # about 1e-16 / tol relative, divided by four)
    assert abs(r["length"][0] / float(h_acc) - 1.0) <= 1e-11
    # and the bid after it is min(5, 0.9 err^-1/5) times it
    err = err_of(tab, h_acc, omega, tol)
    g_next = min(mpmath.mpf(5), mpmath.mpf("0.9") * err ** mpmath.mpf("-0.2"))
    assert abs(r["h_next"][0] / float(h_acc * g_next) - 1.0) <= 1e-11


def test_growth_is_capped_at_five_without_field(oracle_mod):
    """No field: the error estimate vanishes (to rounding) and every bid is
    exactly five times the step just taken, until h_max caps it."""
    O = oracle_mod
    g = uniform_grid(O, [0.0, 0.0, 0.0])
    h_min, h_max = 1e-3, 2.0
    prm = O.params_array(1e-4, h_min, h_max, l_max=1e3)
    pos = np.zeros((1, 3))
    u = np.array([[0.48, 0.6, 0.64]])
    st = {"length": np.zeros(1), "h_next": np.array([h_min]), "n_acc": np.zeros(1, np.int64)}
    seq = []
    for _ in range(8):
        r = O.propagate(g, prm, pos, u, [1e18], [1], length=st["length"], h_next=st["h_next"],
                        status=np.zeros(1, np.int32), n_acc=st["n_acc"], max_steps=1)
        assert r["status"][0] == 3 and r["n_rej"][0] == 0
        seq.append((r["length"][0] - st["length"][0], r["h_next"][0]))
        pos, u = r["pos"], r["dir"]
        st = {"length": r["length"], "h_next": r["h_next"], "n_acc": r["n_acc"]}
    h = h_min
    for taken, bid in seq:
        assert taken == pytest.approx(h, rel=1e-12)
        h = min(h * 5.0, h_max)
        assert bid == h
    assert seq[-1][1] == h_max
