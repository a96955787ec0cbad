"""Helpers shared by the GPU tests: device availability, workload builders and the
parity comparison against the oracle (bitwise goal, stated tolerances as the gate)."""
from __future__ import annotations

import math

import numpy as np
import pytest

import crp_inputs as ci

# Tolerances of the FP64-state path against the FP64 oracle, per particle with
# equal accepted-step counts: arrival direction <= 1e-6 rad, position relative
# to max(|x|, 1 Mpc) <= 1e-9, length relative <= 1e-9.
ANGLE_TOL = 1e-6
POS_TOL = 1e-9
LEN_TOL = 1e-9


def require_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1410_5323_amd import crp
    crp.lib()
    return torch, crp


def angle(a, b):
    c = np.linalg.norm(np.cross(a, b), axis=-1)
    d = np.sum(a * b, axis=-1)
    return np.arctan2(c, d)


def compare(gpu: dict, ora: dict, label: str = "", require_bitwise: bool = True) -> dict:
    """Compare GPU and oracle results particle by particle; asserts the gate."""
    st_eq = gpu["status"] == ora["status"]
    assert np.all(st_eq), f"{label}: status differs for {np.count_nonzero(~st_eq)} particles"
    nacc_eq = gpu["n_accepted"] == ora["n_acc"]
    nrej_eq = gpu["n_rejected"] == ora["n_rej"]
    assert np.all(nacc_eq), f"{label}: accepted-step count differs for {np.count_nonzero(~nacc_eq)}"
    ang = angle(gpu["dir"], ora["dir"])
    dpos = np.linalg.norm(gpu["pos"] - ora["pos"], axis=1) / np.maximum(np.linalg.norm(ora["pos"], axis=1), 1.0)
    dlen = np.abs(gpu["length"] - ora["length"]) / np.maximum(ora["length"], 1e-300)
    assert np.max(ang, initial=0) <= ANGLE_TOL, f"{label}: max angle {np.max(ang)}"
    assert np.max(dpos, initial=0) <= POS_TOL, f"{label}: max rel position {np.max(dpos)}"
    assert np.max(dlen, initial=0) <= LEN_TOL, f"{label}: max rel length {np.max(dlen)}"
    bit = (np.all(gpu["pos"] == ora["pos"], axis=1) & np.all(gpu["dir"] == ora["dir"], axis=1)
           & (gpu["length"] == ora["length"]) & nacc_eq & nrej_eq & (gpu["h_next"] == ora["h_next"]))
    frac = float(np.mean(bit)) if len(bit) else 1.0
    if require_bitwise:
        assert frac == 1.0, f"{label}: bitwise equal for {frac:.6f} of particles"
    return {"bitwise_fraction": frac, "max_angle": float(np.max(ang, initial=0)),
            "max_rel_pos": float(np.max(dpos, initial=0))}


def workload(index: int, n: int | None = None, grid_dtype=None):
    """Field (numpy, the storage dtype), particles and the params array of a workload."""
    w = ci.get_config(index)
    fs, ps, _ = ci.config_seeds(index)
    dt = {"f64": np.float64, "f32": np.float32}.get(grid_dtype or w.grid_dtype, np.float32)
    B = ci.kolmogorov_field(w.grid_n, w.spacing, w.l_min, w.l_max, w.b_rms, fs, dtype=dt)
    npart = w.n_particles if n is None else n
    P = ci.isotropic_particles(npart, w.e_min, w.e_max, w.charges, ps, charge_rule=w.charge_rule)
    return w, B, P


def run_gpu(crp, torch, B, spacing, w, P, layout="linear", dtype=None, tuning=None, sel=None,
            max_steps=0, radius=None, l_max=None, center=(0.0, 0.0, 0.0), state=None, counters=None):
    dtype = dtype or ("f64" if B.dtype == np.float64 else "f32")
    f = crp.make_field(B, spacing, dtype=dtype, layout=layout)
    prm = crp.make_params(w.tol, w.h_min, w.h_max,
                          obs_radius=w.obs_radius if radius is None else radius,
                          l_max=w.max_length if l_max is None else l_max, obs_center=center,
                          max_steps=max_steps)
    if state is None:
        idx = slice(None) if sel is None else sel
        state = crp.particles_to_device(P["pos"][idx], P["dir"][idx], P["energy"][idx], P["charge"][idx],
                                        mass=P["mass"][idx])
    crp.crp_propagate([f], [prm], state, tuning=tuning, counters=counters)
    torch.cuda.synchronize()
    return crp.particles_to_host(state), state, f


def run_oracle(O, B, spacing, w, P, sel=None, max_steps=0, radius=None, l_max=None,
               center=(0.0, 0.0, 0.0), nthreads=0):
    idx = slice(None) if sel is None else sel
    g = O.Grid(B, spacing)
    prm = O.params_array(w.tol, w.h_min, w.h_max, center=center,
                         radius=w.obs_radius if radius is None else radius,
                         l_max=w.max_length if l_max is None else l_max)
    return O.propagate(g, prm, P["pos"][idx], P["dir"][idx], P["energy"][idx], P["charge"][idx],
                       max_steps=max_steps, nthreads=nthreads)


def finite_or_inf(x):
    return x if math.isfinite(x) else math.inf
