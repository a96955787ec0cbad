"""Pins of the oracle's Cash-Karp tableau and constants, independent of retyping.

The coefficients are read back from the oracle library, recovered as exact
rationals and checked against the Runge-Kutta order conditions (Butcher
trees up to order 5).  A transposed, mistyped or dropped coefficient breaks
at least one condition.  Physical constants are recomputed from their SI/IAU
definitions at 50 digits.
"""
from fractions import Fraction

import mpmath
import numpy as np
import pytest


def _rat(x: float) -> Fraction:
    r = Fraction(x).limit_denominator(10 ** 7)
    assert float(r) == x, "coefficient is not the FP64 rounding of a small rational"
    return r


@pytest.fixture(scope="module")
def tab(oracle_mod):
    c = oracle_mod.constants()
    A = [[_rat(v) for v in row] for row in c["A"]]
    return {
        "A": A,
        "c": [_rat(v) for v in c["c"]],
        "b5": [_rat(v) for v in c["b5"]],
        "b4": [_rat(v) for v in c["b4"]],
        "e": [_rat(v) for v in c["e"]],
        "raw": c,
    }


def _conditions(A, b, c):
    """Residuals of the order conditions for orders 1..5 (17 trees)."""
    s = 6
    Ac = [sum(A[i][j] * c[j] for j in range(min(i, 5))) for i in range(s)]
    Ac2 = [sum(A[i][j] * c[j] ** 2 for j in range(min(i, 5))) for i in range(s)]
    Ac3 = [sum(A[i][j] * c[j] ** 3 for j in range(min(i, 5))) for i in range(s)]
    AAc = [sum(A[i][j] * Ac[j] for j in range(min(i, 5))) for i in range(s)]
    AcAc = [sum(A[i][j] * c[j] * Ac[j] for j in range(min(i, 5))) for i in range(s)]
    AAc2 = [sum(A[i][j] * Ac2[j] for j in range(min(i, 5))) for i in range(s)]
    AAAc = [sum(A[i][j] * AAc[j] for j in range(min(i, 5))) for i in range(s)]
    S = lambda v: sum(b[i] * v[i] for i in range(s))  # noqa: E731
    one = [Fraction(1)] * s
    conds = {
        1: [S(one) - 1],
        2: [S(c) - Fraction(1, 2)],
        3: [S([x ** 2 for x in c]) - Fraction(1, 3), S(Ac) - Fraction(1, 6)],
        4: [S([x ** 3 for x in c]) - Fraction(1, 4), S([c[i] * Ac[i] for i in range(s)]) - Fraction(1, 8),
            S(Ac2) - Fraction(1, 12), S(AAc) - Fraction(1, 24)],
        5: [S([x ** 4 for x in c]) - Fraction(1, 5),
            S([c[i] ** 2 * Ac[i] for i in range(s)]) - Fraction(1, 10),
            S([Ac[i] ** 2 for i in range(s)]) - Fraction(1, 20),
            S([c[i] * Ac2[i] for i in range(s)]) - Fraction(1, 15),
            S(Ac3) - Fraction(1, 20),
            S([c[i] * AAc[i] for i in range(s)]) - Fraction(1, 30),
            S(AcAc) - Fraction(1, 40),
            S(AAc2) - Fraction(1, 60),
            S(AAAc) - Fraction(1, 120)],
    }
    return conds


def test_row_sums_equal_nodes(tab):
    for i in range(6):
        assert sum(tab["A"][i]) == tab["c"][i]


def test_fifth_order_weights_meet_all_conditions_to_order_5(tab):
    conds = _conditions(tab["A"], tab["b5"], tab["c"])
    for order in range(1, 6):
        assert all(r == 0 for r in conds[order]), f"b5 fails order {order}: {conds[order]}"


def test_fourth_order_weights_are_exactly_order_4(tab):
    conds = _conditions(tab["A"], tab["b4"], tab["c"])
    for order in range(1, 5):
        assert all(r == 0 for r in conds[order]), f"b4 fails order {order}"
    assert any(r != 0 for r in conds[5]), "embedded weights should not be fifth order"


def test_error_weights_are_exact_difference(tab):
    for i in range(6):
        assert tab["e"][i] == tab["b5"][i] - tab["b4"][i]


def test_tableau_is_explicit(tab):
    for i in range(6):
        for j in range(i, 5):
            assert tab["A"][i][j] == 0


def test_physical_constants_from_definitions(oracle_mod):
    mpmath.mp.dps = 50
    c = mpmath.mpf(299792458)
    au = mpmath.mpf(149597870700)
    mpc = mpmath.mpf(10) ** 6 * 648000 / mpmath.pi * au
    K = c * mpmath.mpf("1e-13") * mpc
    cst = oracle_mod.constants()
    assert cst["K"] == float(K)
    assert cst["MPC_OVER_C"] == float(mpc / c)


def test_fifth_root_table_correctly_rounded(oracle_mod):
    mpmath.mp.dps = 50
    T = oracle_mod.constants()["two_pow_neg_fifths"]
    for j in range(5):
        assert T[j] == float(mpmath.power(2, -mpmath.mpf(j) / 5))


def test_gyroradius_of_eev_proton(oracle_mod):
    """r_g = E/(Z e c B): 1 EeV proton in 1 nG -> 1.0810 Mpc (kappa*B = 1/r_g)."""
    mpmath.mp.dps = 30
    r_m = mpmath.mpf("1e18") / (mpmath.mpf(299792458) * mpmath.mpf("1e-13"))
    mpc = mpmath.mpf(10) ** 6 * 648000 / mpmath.pi * mpmath.mpf(149597870700)
    r_mpc = float(r_m / mpc)
    kap = oracle_mod.kappa(1, 1e18)
    assert abs(1.0 / kap - r_mpc) <= 1e-15 * r_mpc
    assert abs(r_mpc - 1.0810) < 1e-4
