"""ctypes wrapper of the FP64 CPU oracle (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
module.  It imports nothing from the GPU package; inputs come as numpy arrays
from the shared seeded input generators.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(HERE, "liboracle.so")
_lib = None

STATUS = {"ACTIVE": 0, "ARRIVED": 1, "MAX_LENGTH": 2, "MAX_STEPS": 3, "NONFINITE": 4,
          "CANCELLED": 5, "BAD_INPUT": 6}

_pd = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_pi32 = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_pi64 = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_GRID_ARGS = [C.c_void_p, C.c_int, C.c_int64, C.c_int64, C.c_int64, _pd, C.c_double, C.c_void_p, C.c_void_p]


def lib():
    global _lib
    if _lib is None:
        src = os.path.join(HERE, "crp_oracle.c")
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
            from . import build_oracle  # noqa: F401  (package-relative when imported as oracle.oracle)
            build_oracle.build()
        L = C.CDLL(_LIB_PATH)
        L.oracle_constants.argtypes = [_pd]
        L.oracle_inv_fifth_root.argtypes = [C.c_double]
        L.oracle_inv_fifth_root.restype = C.c_double
        L.oracle_field_at.argtypes = _GRID_ARGS + [_pd, _pd, C.c_int64]
        L.oracle_ck_eval.argtypes = _GRID_ARGS + [C.c_double, _pd, C.c_double, _pd, _pd]
        L.oracle_fixed_steps.argtypes = _GRID_ARGS + [C.c_double, _pd, C.c_double, C.c_int64]
        L.oracle_propagate.argtypes = _GRID_ARGS + [_pd, C.c_int64, C.c_int64, _pd, _pd, _pd,
                                                    _pi32, _pd, _pd, _pi32, _pi64, _pi64,
                                                    C.c_void_p, C.c_int]
        L.oracle_propagate_taped.argtypes = _GRID_ARGS + [_pd, _pd, C.c_double, C.c_int32, _pd,
                                                          _pd, _pd, C.c_int64, _pd]
        L.oracle_propagate_taped.restype = C.c_int64
        _pdn = C.c_void_p  # optional double arrays (NULL allowed)
        L.oracle_replay_tangent.argtypes = _GRID_ARGS + [C.c_double, _pd, _pd, _pdn, _pdn, _pdn, _pd, C.c_int64,
                                                         C.c_int, _pd, C.c_double, _pdn, _pd]
        L.oracle_replay_tangent.restype = C.c_int
        L.oracle_replay_adjoint.argtypes = _GRID_ARGS + [C.c_double, _pd, _pd, _pd, C.c_int64, C.c_int, _pd,
                                                         C.c_double, _pdn, _pd, C.c_double, _pd, _pd, _pdn, _pd]
        L.oracle_replay_adjoint.restype = C.c_int
        for f in (L.oracle_field_at, L.oracle_ck_eval, L.oracle_fixed_steps, L.oracle_propagate):
            f.restype = C.c_int
        _lib = L
    return _lib


class Modulation:
    """A periodic scalar modulation grid (section 3.2, modulated grids): values
    [n0][n1][n2], float64 or float32, node (0, 0, 0) at ``origin``."""

    def __init__(self, values: np.ndarray, spacing: float, origin=(0.0, 0.0, 0.0)):
        v = np.ascontiguousarray(values)
        if v.dtype not in (np.float64, np.float32) or v.ndim != 3:
            raise ValueError("modulation must be float64/float32 of shape (n0, n1, n2)")
        self.values = v
        self.desc = np.array([v.shape[0], v.shape[1], v.shape[2], 0 if v.dtype == np.float64 else 1,
                              origin[0], origin[1], origin[2], spacing], dtype=np.float64)


class Grid:
    """A periodic vector grid as the oracle reads it: values [n0][n1][n2][3] in nG,
    optionally multiplied by a Modulation.

    Accepts float64 or float32 values (each read exactly as FP64)."""

    def __init__(self, values: np.ndarray, spacing: float, origin=(0.0, 0.0, 0.0), modulation=None):
        v = np.ascontiguousarray(values)
        if v.dtype not in (np.float64, np.float32) or v.ndim != 4 or v.shape[3] != 3:
            raise ValueError("grid must be float64/float32 of shape (n0, n1, n2, 3)")
        self.values = v
        self.dtype_code = 0 if v.dtype == np.float64 else 1
        self.shape = v.shape[:3]
        self.spacing = float(spacing)
        self.origin = np.asarray(origin, dtype=np.float64).copy()
        self.modulation = modulation

    def args(self):
        m = self.modulation
        return (self.values.ctypes.data, self.dtype_code, self.shape[0], self.shape[1],
                self.shape[2], self.origin, self.spacing, None if m is None else m.values.ctypes.data,
                None if m is None else m.desc.ctypes.data)


def constants() -> dict:
    out = np.zeros(67)
    lib().oracle_constants(out)
    return {"K": out[0], "MPC_OVER_C": out[1], "A": out[2:38].reshape(6, 6)[:, :5],
            "c": out[38:44], "b5": out[44:50], "b4": out[50:56], "e": out[56:62],
            "two_pow_neg_fifths": out[62:67]}


def inv_fifth_root(err: float) -> float:
    return lib().oracle_inv_fifth_root(float(err))


def field_at(grid: Grid, X: np.ndarray) -> np.ndarray:
    X = np.ascontiguousarray(X, dtype=np.float64).reshape(-1, 3)
    B = np.empty_like(X)
    if lib().oracle_field_at(*grid.args(), X, B, X.shape[0]):
        raise ValueError("oracle_field_at: bad arguments")
    return B


def kappa(charge: int, energy: float) -> float:
    """kappa = Z*K/E (per Mpc per nG), evaluated exactly as the propagator does."""
    return (float(charge) * constants()["K"]) / float(energy)


def ck_eval(grid: Grid, kap: float, y, h: float):
    y = np.ascontiguousarray(y, dtype=np.float64)
    y5 = np.empty(6)
    d = np.empty(6)
    if lib().oracle_ck_eval(*grid.args(), float(kap), y, float(h), y5, d):
        raise ValueError("oracle_ck_eval: bad arguments")
    return y5, d


def fixed_steps(grid: Grid, kap: float, y, h: float, nsteps: int) -> np.ndarray:
    y = np.array(y, dtype=np.float64)
    if lib().oracle_fixed_steps(*grid.args(), float(kap), y, float(h), int(nsteps)):
        raise ValueError("oracle_fixed_steps: bad arguments")
    return y


def params_array(tol, h_min, h_max, center=(0.0, 0.0, 0.0), radius=0.0, l_max=math.inf, box=None,
                 backtrack=False):
    """Parameter block of the oracle: tolerance, step limits, observer sphere,
    length limit, an optional reflective box ((lo x, y, z), (hi x, y, z)) and
    the backtracking flag."""
    lo, hi, on = ((0.0,) * 3, (0.0,) * 3, 0.0) if box is None else (box[0], box[1], 1.0)
    return np.array([tol, h_min, h_max, center[0], center[1], center[2], radius, l_max,
                     lo[0], lo[1], lo[2], hi[0], hi[1], hi[2], on, 1.0 if backtrack else 0.0], dtype=np.float64)


def _prm(prm) -> np.ndarray:
    a = np.ascontiguousarray(prm, dtype=np.float64)
    if a.shape != (16,):
        raise ValueError("the parameter block has 16 entries (params_array)")
    return a


def propagate(grid: Grid, prm: np.ndarray, pos, dir, energy, charge, length=None, h_next=None,
              status=None, n_acc=None, n_rej=None, max_steps: int = 0, nthreads: int = 0) -> dict:
    """Propagate particles; returns a dict of new arrays (inputs are not modified)."""
    n = len(energy)
    st = {
        "pos": np.array(pos, dtype=np.float64).reshape(n, 3).copy(),
        "dir": np.array(dir, dtype=np.float64).reshape(n, 3).copy(),
        "energy": np.ascontiguousarray(energy, dtype=np.float64),
        "charge": np.ascontiguousarray(charge, dtype=np.int32),
        "length": np.zeros(n) if length is None else np.array(length, dtype=np.float64),
        "h_next": np.zeros(n) if h_next is None else np.array(h_next, dtype=np.float64),
        "status": np.zeros(n, np.int32) if status is None else np.array(status, dtype=np.int32),
        "n_acc": np.zeros(n, np.int64) if n_acc is None else np.array(n_acc, dtype=np.int64),
        "n_rej": np.zeros(n, np.int64) if n_rej is None else np.array(n_rej, dtype=np.int64),
    }
    counters = np.zeros(5, dtype=np.int64)
    rc = lib().oracle_propagate(*grid.args(), _prm(prm),
                                int(max_steps), n, st["pos"], st["dir"], st["energy"],
                                st["charge"], st["length"], st["h_next"], st["status"],
                                st["n_acc"], st["n_rej"], counters.ctypes.data, int(nthreads))
    if rc:
        raise ValueError("oracle_propagate: bad arguments")
    st["time"] = st["length"] * constants()["MPC_OVER_C"]
    st["counters"] = dict(zip(["evals", "accepted", "rejected", "event_evals", "floor_hits"],
                              counters.tolist()))
    return st


def propagate_taped(grid: Grid, prm: np.ndarray, pos, dir, energy, charge, cap: int = 1 << 20):
    """One particle from a fresh start, recording accepted step sizes."""
    y = np.concatenate([np.asarray(pos, np.float64), np.asarray(dir, np.float64)]).copy()
    L = np.zeros(1)
    hn = np.zeros(1)
    tape = np.zeros(cap)
    info = np.zeros(4)
    m = lib().oracle_propagate_taped(*grid.args(), _prm(prm), y,
                                     float(energy), int(charge), L, hn, tape, cap, info)
    if m < 0:
        raise ValueError("oracle_propagate_taped: bad arguments")
    return {"y": y, "length": L[0], "h_next": hn[0], "tape": tape[:min(m, cap)].copy(),
            "n_steps": int(m), "status": int(info[0]), "event": bool(info[1]),
            "s_event": info[2], "length_bound": bool(info[3])}


def _opt(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64).ctypes.data


def _box(box):
    """Reflective box ((lo x, y, z), (hi x, y, z)) as the 6 doubles the
    replays take, or None."""
    if box is None:
        return None
    b = np.ascontiguousarray(np.concatenate([np.asarray(box[0], np.float64), np.asarray(box[1], np.float64)]))
    if b.shape != (6,):
        raise ValueError("box: ((lo x, y, z), (hi x, y, z))")
    return b


def replay_tangent(grid: Grid, kap: float, x0, u0, h, event: bool, center=(0.0, 0.0, 0.0), radius=0.0,
                   du0=None, vgrid=None, box=None, dx0=None) -> dict:
    """Frozen-step replay with forward-mode derivatives (tangents du0 of the
    raw initial direction, dx0 of the initial position and vgrid of the grid
    values), in the reflective box ((lo), (hi)) if one is given."""
    out = np.zeros(12)
    du = None if du0 is None else np.ascontiguousarray(du0, dtype=np.float64)
    dx = None if dx0 is None else np.ascontiguousarray(dx0, dtype=np.float64)
    vg = None if vgrid is None else np.ascontiguousarray(vgrid, dtype=np.float64)
    bx = _box(box)
    rc = lib().oracle_replay_tangent(*grid.args(), float(kap), np.ascontiguousarray(x0, np.float64),
                                     np.ascontiguousarray(u0, np.float64), None if du is None else du.ctypes.data,
                                     None if dx is None else dx.ctypes.data,
                                     None if vg is None else vg.ctypes.data, np.ascontiguousarray(h, np.float64),
                                     len(h), int(bool(event)), np.asarray(center, np.float64), float(radius),
                                     None if bx is None else bx.ctypes.data, out)
    if rc:
        raise ValueError("oracle_replay_tangent: no crossing bracketed or bad arguments")
    return {"u": out[0:3].copy(), "length": out[3], "du": out[4:7].copy(), "dlength": out[7],
            "x": out[8:11].copy(), "s_event": out[11]}


def replay_adjoint(grid: Grid, kap: float, x0, u0, h, event: bool, ubar, lbar: float, center=(0.0, 0.0, 0.0),
                   radius=0.0, gbar=None, box=None) -> dict:
    """Full-tape reverse sweep of the frozen-step replay (in the reflective
    box ((lo), (hi)) if one is given).  gbar (FP64 array of the grid's shape)
    is accumulated in place when given.  kappabar: the cotangent of kappa (the
    energy gradient is kappabar * (-kappa / E))."""
    u0b = np.zeros(3)
    x0b = np.zeros(3)
    kb = np.zeros(1)
    if gbar is not None:
        assert gbar.dtype == np.float64 and gbar.flags.c_contiguous
    bx = _box(box)
    rc = lib().oracle_replay_adjoint(*grid.args(), float(kap), np.ascontiguousarray(x0, np.float64),
                                     np.ascontiguousarray(u0, np.float64), np.ascontiguousarray(h, np.float64),
                                     len(h), int(bool(event)), np.asarray(center, np.float64), float(radius),
                                     None if bx is None else bx.ctypes.data,
                                     np.ascontiguousarray(ubar, np.float64), float(lbar), u0b, x0b,
                                     None if gbar is None else gbar.ctypes.data, kb)
    if rc:
        raise ValueError("oracle_replay_adjoint: no crossing bracketed or bad arguments")
    return {"u0bar": u0b, "x0bar": x0b, "kappabar": float(kb[0])}
