"""Pins of the oracle's periodic trilinear field lookup.

Trilinear interpolation reproduces every function in span{1, x, y, z, xy, yz,
xz, xyz} exactly, so a multilinear field sampled on the nodes must come back
at any interior point up to rounding; swapped axes, a wrong lerp order or a
wrong corner index all break this.  A random field is compared against
scipy's RegularGridInterpolator on a periodically padded copy (an independent
library implementation), which also pins the wrap-around.
"""
import numpy as np
import pytest
from scipy.interpolate import RegularGridInterpolator


def _grid(O, vals, spacing, origin=(0.0, 0.0, 0.0)):
    return O.Grid(vals, spacing, origin)


def test_constant_field_bitwise(oracle_mod):
    O = oracle_mod
    v = np.empty((8, 6, 5, 3))
    v[...] = [0.3, -1.7, 2.5]
    g = _grid(O, v, 0.13, origin=(-0.4, 0.2, 1.0))
    X = np.random.default_rng(1).uniform(-5, 5, size=(500, 3))
    B = O.field_at(g, X)
    assert np.array_equal(B, np.broadcast_to([0.3, -1.7, 2.5], B.shape))


def test_node_values_bitwise(oracle_mod):
    O = oracle_mod
    rng = np.random.default_rng(2)
    v = rng.standard_normal((6, 7, 8, 3))
    g = _grid(O, v, 0.125)  # power-of-two spacing: node positions are exact
    idx = np.stack(np.meshgrid(np.arange(6), np.arange(7), np.arange(8), indexing="ij"), -1).reshape(-1, 3)
    B = O.field_at(g, idx * 0.125)
    assert np.array_equal(B, v.reshape(-1, 3))


def test_multilinear_field_reproduced(oracle_mod):
    O = oracle_mod
    rng = np.random.default_rng(3)
    n = (9, 10, 11)
    h = 0.37
    coef = rng.standard_normal((3, 8))  # per component: 1, x, y, z, xy, yz, xz, xyz

    def f(P):
        x, y, z = P[..., 0], P[..., 1], P[..., 2]
        basis = np.stack([np.ones_like(x), x, y, z, x * y, y * z, x * z, x * y * z], -1)
        return basis @ coef.T

    nodes = np.stack(np.meshgrid(*[np.arange(k) * h for k in n], indexing="ij"), -1)
    g = _grid(O, f(nodes), h)
    # interior points: cells 0 .. n-2 (the last cell wraps to node 0)
    X = rng.uniform(0, 1, size=(2000, 3)) * (np.array(n) - 1) * h
    B = O.field_at(g, X)
    ref = f(X)
    scale = np.abs(coef).sum(1) * (1 + np.max(n) * h) ** 3
    assert np.max(np.abs(B - ref) / scale) < 1e-14


def test_affine_field_with_origin_offset(oracle_mod):
    O = oracle_mod
    rng = np.random.default_rng(4)
    M = rng.standard_normal((3, 3))
    B0 = rng.standard_normal(3)
    origin = np.array([-1.3, 0.7, 2.1])
    h = 0.05
    n = 16
    nodes = origin + np.stack(np.meshgrid(*[np.arange(n) * h] * 3, indexing="ij"), -1)
    g = _grid(O, B0 + nodes @ M.T, h, origin)
    X = origin + rng.uniform(0, (n - 1) * h, size=(3000, 3))
    B = O.field_at(g, X)
    ref = B0 + X @ M.T
    assert np.max(np.abs(B - ref)) < 1e-13 * (1 + np.abs(ref).max())


def test_random_field_matches_scipy_with_periodic_wrap(oracle_mod):
    O = oracle_mod
    rng = np.random.default_rng(5)
    n = (7, 9, 6)
    h = 0.2
    v = rng.standard_normal(n + (3,))
    g = _grid(O, v, h)
    vp = np.pad(v, ((0, 1), (0, 1), (0, 1), (0, 0)), mode="wrap")
    axes = [np.arange(k + 1) * h for k in n]
    X = rng.uniform(-30, 30, size=(4000, 3))
    box = np.array(n) * h
    Xr = np.mod(X, box)
    ref = np.stack([RegularGridInterpolator(axes, vp[..., c])(Xr) for c in range(3)], -1)
    B = O.field_at(g, X)
    assert np.max(np.abs(B - ref)) < 1e-12


def test_periodicity(oracle_mod):
    O = oracle_mod
    rng = np.random.default_rng(6)
    v = rng.standard_normal((8, 8, 8, 3))
    h = 0.1
    g = _grid(O, v, h)
    X = rng.uniform(0, 0.8, size=(1000, 3))
    B0 = O.field_at(g, X)
    for shift in ([0.8, 0, 0], [0, -1.6, 0], [0, 0, 8.0], [-0.8, 2.4, -4.0]):
        B1 = O.field_at(g, X + np.array(shift))
        assert np.max(np.abs(B1 - B0)) < 1e-12


def test_float32_grid_reads_exact_values(oracle_mod):
    O = oracle_mod
    rng = np.random.default_rng(7)
    v = rng.standard_normal((5, 5, 5, 3)).astype(np.float32)
    X = rng.uniform(-2, 2, size=(300, 3))
    B32 = O.field_at(O.Grid(v, 0.3), X)
    B64 = O.field_at(O.Grid(v.astype(np.float64), 0.3), X)
    assert np.array_equal(B32, B64)


def test_nan_cell_propagates(oracle_mod):
    O = oracle_mod
    v = np.ones((4, 4, 4, 3))
    v[2, 2, 2, 0] = np.nan
    B = O.field_at(O.Grid(v, 1.0), np.array([[1.5, 1.5, 1.5], [2.5, 2.5, 2.5], [0.2, 0.2, 0.2]]))
    assert np.isnan(B[0, 0]) and np.isnan(B[1, 0]) and np.all(np.isfinite(B[2]))


@pytest.mark.parametrize("bad", [np.zeros((1, 4, 4, 3)), np.zeros((4, 4, 4, 2))])
def test_bad_grid_rejected(oracle_mod, bad):
    with pytest.raises(ValueError):
        g = oracle_mod.Grid(bad, 1.0)
        oracle_mod.field_at(g, np.zeros((1, 3)))
