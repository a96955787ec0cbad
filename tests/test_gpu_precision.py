"""Mixed precision at the stated error on the precision workload (1024^3
Kolmogorov grid at 10 kpc, nuclei from the origin to a 10 Mpc sphere), on
the first 10,000 particles of its seeded list.

A particle is non-chaotic when the oracle's arrival direction moves by at
most 1e-6 rad as its initial direction is rotated by 1e-15 rad (a Lyapunov
probe).  On those particles the mixed kernel (FP16 grid, FP32 stages, FP64
accumulation) must stay within 1e-4 rad of the oracle on the FP32 grid at the
95th percentile.  At the workloads' tolerance 1e-4 no tolerance-limited
implementation other than a bit-identical one can (the FP64 path itself moves
by 1e-3 .. 1 rad under such perturbations); the loosest tolerance at which the
bound holds is 1e-8 (1e-4 and 1e-6 miss it), which is where this test runs.
The FP64 path runs the same particles and must equal the oracle bit for bit.
"""
import sys

import numpy as np
import pytest

import crp_inputs as ci
from gpu_common import angle, require_gpu

pytestmark = pytest.mark.gpu

SUBSET = 10000
TOL = 1e-8
BOUND = 1e-4


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _rotate(u, eps):
    ax = np.cross(u, np.array([0.3, 0.5, 0.81]))
    ax /= np.linalg.norm(ax, axis=1)[:, None]
    return u * np.cos(eps) + np.cross(ax, u) * np.sin(eps)


@pytest.fixture(scope="module")
def c4(oracle_mod):
    torch, crp = require_gpu()
    w = ci.get_config("precision_1024cube")
    fs, ps, _ = ci.config_seeds(w.index)
    _say(f"case: precision workload {w.grid_n}^3 grid, first {SUBSET} of {w.n_particles} particles, tol {TOL}")
    B32 = ci.kolmogorov_field(w.grid_n, w.spacing, w.l_min, w.l_max, w.b_rms, fs, dtype=np.float32)
    P = ci.isotropic_particles(w.n_particles, w.e_min, w.e_max, w.charges, ps)
    P = {k: v[:SUBSET] for k, v in P.items()}
    O = oracle_mod
    prm = O.params_array(TOL, w.h_min, w.h_max, radius=w.obs_radius, l_max=w.max_length)
    g = O.Grid(B32, w.spacing)
    ref = O.propagate(g, prm, P["pos"], P["dir"], P["energy"], P["charge"])
    probe = O.propagate(g, prm, P["pos"], _rotate(P["dir"], 1e-15), P["energy"], P["charge"])
    calm = angle(probe["dir"], ref["dir"]) <= 1e-6
    _say(f"  oracle done: {int(calm.sum())} non-chaotic particles")
    src = torch.from_numpy(B32).cuda()
    fields = {dt: crp.make_field(src, w.spacing, dtype=dt, layout="linear") for dt in ("f16", "bf16", "f32")}
    del src
    torch.cuda.empty_cache()
    return torch, crp, w, P, ref, calm, fields


def _gpu(torch, crp, w, P, field, precision):
    prm = crp.make_params(TOL, w.h_min, w.h_max, obs_radius=w.obs_radius, l_max=w.max_length)
    st = crp.particles_to_device(P["pos"], P["dir"], P["energy"], P["charge"])
    crp.crp_propagate([field], [prm], st, precision=precision)
    torch.cuda.synchronize()
    return crp.particles_to_host(st)


def test_fp64_path_bitwise_on_the_subset(c4):
    torch, crp, w, P, ref, calm, fields = c4
    g = _gpu(torch, crp, w, P, fields["f32"], crp.CRP_PREC_FP64)
    for k, ko in (("pos", "pos"), ("dir", "dir"), ("length", "length"), ("status", "status"),
                  ("n_accepted", "n_acc"), ("n_rejected", "n_rej")):
        assert np.array_equal(g[k], ref[ko]), k


@pytest.mark.parametrize("dtype, prec", [("f16", "f64acc"), ("f16", "dfacc"), ("bf16", "f64acc")])
def test_mixed_error_bound_on_non_chaotic_particles(c4, dtype, prec):
    torch, crp, w, P, ref, calm, fields = c4
    pv = crp.CRP_PREC_MIXED_F64ACC if prec == "f64acc" else crp.CRP_PREC_MIXED_DFACC
    g = _gpu(torch, crp, w, P, fields[dtype], pv)
    assert calm.sum() >= 100, "too few non-chaotic particles to estimate a 95th percentile"
    a = angle(g["dir"], ref["dir"])[calm]
    p95 = float(np.percentile(a, 95))
    dl = np.abs(g["length"] - ref["length"])[calm] / ref["length"][calm]
    _say(f"  {dtype}/{prec}: non-chaotic {int(calm.sum())}, angle p50 {np.median(a):.2e} p95 {p95:.2e} "
         f"max {a.max():.2e} rad; length p95 {np.percentile(dl, 95):.2e}")
    assert p95 <= BOUND, p95
    # length: FP64 or double-float accumulation of FP32 increments
    assert np.percentile(dl, 95) <= 1e-5
