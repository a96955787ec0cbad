"""Backtracking on the GPU (section 3.3): particles are traced back from where
they were observed, as antiparticles with reversed direction, and the
direction written back is the physical one.  Compared with the oracle bit for
bit; the mixed-precision kernel against its own forward run of the
antiparticles."""
import sys

import numpy as np
import pytest

import crp_inputs as ci
from gpu_common import compare, require_gpu

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    return require_gpu()


@pytest.fixture(scope="module")
def small():
    w = ci.get_config(0)
    fs, ps, _ = ci.config_seeds(0)
    B = ci.kolmogorov_field(w.grid_n, w.spacing, w.l_min, w.l_max, w.b_rms, fs)
    P = ci.isotropic_particles(3000, 1e18, 3e19, (1, 2, 7, 26), ps)
    return w, B, P


PRM = dict(tol=1e-4, h_min=1e-4, h_max=0.5, obs_radius=2.0, l_max=30.0)


def _gpu(crp, torch, B, spacing, kw, pos, dirs, energy, charge, layout="linear", dtype="f64", precision=0,
         backtrack=True):
    f = crp.make_field(B, spacing, dtype=dtype, layout=layout)
    prm = crp.make_params(**kw, backtrack=backtrack)
    st = crp.particles_to_device(pos, dirs, energy, charge)
    crp.crp_propagate([f], [prm], st, precision=precision)
    torch.cuda.synchronize()
    return crp.particles_to_host(st)


@pytest.mark.parametrize("layout,dtype", [("linear", "f64"), ("cell8", "f32")])
def test_backtracking_matches_oracle(dev, oracle_mod, small, layout, dtype):
    torch, crp = dev
    w, B, P = small
    _say(f"case: backtracking, {layout} {dtype}")
    Bs = B if dtype == "f64" else B.astype(np.float32)
    g = _gpu(crp, torch, Bs, w.spacing, PRM, P["pos"], P["dir"], P["energy"], P["charge"], layout=layout, dtype=dtype)
    O = oracle_mod
    prm = O.params_array(PRM["tol"], PRM["h_min"], PRM["h_max"], radius=PRM["obs_radius"], l_max=PRM["l_max"],
                         backtrack=True)
    o = O.propagate(O.Grid(Bs, w.spacing), prm, P["pos"], P["dir"], P["energy"], P["charge"])
    compare(g, o, "backtracking")
    assert set(np.unique(g["status"])) == {1, 2}


def test_backtracking_is_the_reversed_antiparticle(dev, small):
    torch, crp = dev
    w, B, P = small
    _say("case: backtracking = forward antiparticle with reversed direction")
    b = _gpu(crp, torch, B, w.spacing, PRM, P["pos"], P["dir"], P["energy"], P["charge"])
    f = _gpu(crp, torch, B, w.spacing, PRM, P["pos"], -P["dir"], P["energy"], -P["charge"], backtrack=False)
    for k in ("pos", "length", "status", "n_accepted", "n_rejected", "h_next"):
        assert np.array_equal(b[k], f[k]), k
    assert np.array_equal(b["dir"], -f["dir"])


def test_forward_then_back_returns(dev, small):
    torch, crp = dev
    w, B, P = small
    _say("case: forward, then backtracking from the end state")
    n = 500
    E = np.full(n, 5e19)
    Z = np.ones(n, np.int32)
    x0 = np.tile([0.2, -0.4, 0.7], (n, 1))
    kw = dict(tol=1e-10, h_min=1e-9, h_max=0.2, obs_radius=0.0, l_max=5.0)
    fw = _gpu(crp, torch, B, w.spacing, kw, x0, P["dir"][:n], E, Z, backtrack=False)
    bk = _gpu(crp, torch, B, w.spacing, kw, fw["pos"], fw["dir"], E, Z)
    assert np.max(np.linalg.norm(bk["pos"] - x0, axis=1)) < 1e-6
    assert np.max(np.linalg.norm(bk["dir"] - P["dir"][:n], axis=1)) < 1e-6


def test_two_groups_forward_and_back(dev, oracle_mod, small):
    torch, crp = dev
    w, B, P = small
    _say("case: two parameter groups, forward and backtracking")
    f = crp.make_field(B, w.spacing, dtype="f64")
    prms = [crp.make_params(**PRM), crp.make_params(**PRM, backtrack=True)]
    pidx = np.arange(len(P["energy"])) % 2
    st = crp.particles_to_device(P["pos"], P["dir"], P["energy"], P["charge"], param_index=pidx)
    crp.crp_propagate([f], prms, st)
    torch.cuda.synchronize()
    g = crp.particles_to_host(st)
    O = oracle_mod
    for gi in (0, 1):
        sel = np.nonzero(pidx == gi)[0]
        prm = O.params_array(PRM["tol"], PRM["h_min"], PRM["h_max"], radius=PRM["obs_radius"], l_max=PRM["l_max"],
                             backtrack=gi == 1)
        o = O.propagate(O.Grid(B, w.spacing), prm, P["pos"][sel], P["dir"][sel], P["energy"][sel], P["charge"][sel])
        compare({k: v[sel] for k, v in g.items()}, o, f"group {gi}")


def test_mixed_kernel_backtracks(dev, small):
    """The mixed-precision kernel's backtracking equals its own forward run of
    the reversed antiparticles, bit for bit (same arithmetic, signs flipped)."""
    torch, crp = dev
    w, B, P = small
    _say("case: mixed-precision backtracking")
    B32 = B.astype(np.float32)
    for prec in (crp.CRP_PREC_MIXED_F64ACC, crp.CRP_PREC_MIXED_DFACC):
        b = _gpu(crp, torch, B32, w.spacing, PRM, P["pos"], P["dir"], P["energy"], P["charge"], dtype="f16",
                 precision=prec)
        f = _gpu(crp, torch, B32, w.spacing, PRM, P["pos"], -P["dir"], P["energy"], -P["charge"], dtype="f16",
                 precision=prec, backtrack=False)
        for k in ("pos", "length", "status", "n_accepted", "n_rejected", "h_next"):
            assert np.array_equal(b[k], f[k]), (prec, k)
        assert np.array_equal(b["dir"], -f["dir"])
        assert set(np.unique(b["status"])) == {1, 2}
