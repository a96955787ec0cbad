"""Modulated fields on the GPU (section 3.2, modulated grids): the vector grid
times a periodic scalar modulation grid, against the oracle bit for bit."""
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
    fs, ps, rs = ci.config_seeds(0)
    B = ci.kolmogorov_field(w.grid_n, w.spacing, w.l_min, w.l_max, w.b_rms, fs)
    M = ci.lognormal_modulation(24, 0.25, 1.0, 1.0, rs)
    P = ci.isotropic_particles(3000, 1e18, 3e19, (1, 2, 7, 26), ps)
    return w, B, M, P


def _gpu(crp, torch, B, spacing, prm_kw, P, modulation=None, layout="linear", dtype="f64", tuning=None, sel=None):
    f = crp.make_field(B, spacing, dtype=dtype, layout=layout, modulation=modulation)
    prm = crp.make_params(**prm_kw)
    idx = slice(None) if sel is None else sel
    st = crp.particles_to_device(P["pos"][idx], P["dir"][idx], P["energy"][idx], P["charge"][idx])
    crp.crp_propagate([f], [prm], st, tuning=tuning)
    torch.cuda.synchronize()
    return crp.particles_to_host(st)


def _oracle(O, B, spacing, prm_kw, P, M=None, mspacing=None, morigin=None, sel=None):
    g = O.Grid(B, spacing, modulation=None if M is None else O.Modulation(M, mspacing, morigin))
    prm = O.params_array(prm_kw["tol"], prm_kw["h_min"], prm_kw["h_max"], radius=prm_kw["obs_radius"],
                         l_max=prm_kw["l_max"])
    idx = slice(None) if sel is None else sel
    return O.propagate(g, prm, P["pos"][idx], P["dir"][idx], P["energy"][idx], P["charge"][idx])


PRM = dict(tol=1e-4, h_min=1e-4, h_max=0.5, obs_radius=2.5, l_max=30.0)


def test_unit_modulation_is_bitwise_neutral(dev, small):
    torch, crp = dev
    w, B, M, P = small
    _say("case: modulation of ones")
    mod = crp.make_modulation(np.ones((7, 9, 11)), 0.31, origin=(-1.0, 0.2, 0.4))
    a = _gpu(crp, torch, B, w.spacing, PRM, P)
    b = _gpu(crp, torch, B, w.spacing, PRM, P, modulation=mod)
    for k in ("pos", "dir", "length", "status", "n_accepted", "n_rejected", "h_next"):
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("layout,mdtype,cache", [("linear", "f64", 0), ("cell8", "f32", 0), ("cell8", "f64", 1),
                                                 ("linear", "f32", -1), ("cell8", "f32", 1), ("linear", "f32", 1)])
def test_modulated_small_grid_matches_oracle(dev, oracle_mod, small, layout, mdtype, cache):
    torch, crp = dev
    w, B, M, P = small
    _say(f"case: modulated small grid, {layout}, modulation {mdtype}, cache {cache}")
    Mv = M if mdtype == "f64" else M.astype(np.float32)
    mod = crp.make_modulation(Mv, 0.25, origin=(-3.0, -3.0, -3.0), dtype=mdtype)
    g = _gpu(crp, torch, B, w.spacing, PRM, P, modulation=mod, layout=layout,
             tuning=crp.make_tuning(cache_cells=cache))
    o = _oracle(oracle_mod, B, w.spacing, PRM, P, Mv, 0.25, (-3.0, -3.0, -3.0))
    r = compare(g, o, "modulated small grid")
    _say(f"  bitwise fraction {r['bitwise_fraction']}")
    assert set(np.unique(g["status"])) <= {1, 2}


def test_two_fields_one_modulated(dev, oracle_mod, small):
    torch, crp = dev
    w, B, M, P = small
    _say("case: two fields, one modulated, per-particle parameter groups")
    mod = crp.make_modulation(M, 0.25, origin=(-3.0, -3.0, -3.0), dtype="f64")
    f0 = crp.make_field(B, w.spacing, dtype="f64")
    f1 = crp.make_field(B, w.spacing, dtype="f64", modulation=mod)
    prms = [crp.make_params(**PRM, field_index=0), crp.make_params(**PRM, field_index=1)]
    pidx = np.arange(len(P["energy"])) % 2
    st = crp.particles_to_device(P["pos"], P["dir"], P["energy"], P["charge"], param_index=pidx)
    crp.crp_propagate([f0, f1], prms, st)
    torch.cuda.synchronize()
    g = crp.particles_to_host(st)
    for fi, Mi in ((0, None), (1, M)):
        sel = np.nonzero(pidx == fi)[0]
        o = _oracle(oracle_mod, B, w.spacing, PRM, P, Mi, 0.25, (-3.0, -3.0, -3.0), sel=sel)
        compare({k: v[sel] for k, v in g.items()}, o, f"field {fi}")


def test_modulated_workload_sample(dev, oracle_mod):
    """The modulated workload at full size (256^3 FP32 vector grid, 440^3 FP32
    modulation, 1e6 nuclei) in one launch; a sample against the oracle."""
    torch, crp = dev
    w = ci.get_config(5)
    fs, ps, rs = ci.config_seeds(5)
    B = ci.kolmogorov_field(w.grid_n, w.spacing, w.l_min, w.l_max, w.b_rms, fs, dtype=np.float32)
    M = ci.lognormal_modulation(w.mod_n, w.mod_spacing, w.mod_l_corr, w.mod_sigma, rs, dtype=np.float32)
    P = ci.isotropic_particles(w.n_particles, w.e_min, w.e_max, w.charges, ps)
    o0 = (w.mod_origin,) * 3
    _say(f"case: modulated workload, {w.n_particles} particles, grid {w.grid_n}^3 x modulation {w.mod_n}^3")
    mod = crp.make_modulation(M, w.mod_spacing, origin=o0)
    prm_kw = dict(tol=w.tol, h_min=w.h_min, h_max=w.h_max, obs_radius=w.obs_radius, l_max=w.max_length)
    g = _gpu(crp, torch, B, w.spacing, prm_kw, P, modulation=mod, layout="cell8", dtype="f32")
    assert set(np.unique(g["status"])) <= {1, 2}
    rng = np.random.default_rng(8)
    sel = np.sort(rng.choice(w.n_particles, 400, replace=False))
    o = _oracle(oracle_mod, B, w.spacing, prm_kw, P, M, w.mod_spacing, o0, sel=sel)
    r = compare({k: v[sel] for k, v in g.items()}, o, "modulated workload sample")
    _say(f"  bitwise fraction {r['bitwise_fraction']}")


@pytest.mark.parametrize("prec", ["mixed_f64acc", "mixed_dfacc"])
def test_mixed_kernel_modulation(dev, oracle_mod, small, prec):
    """The mixed-precision kernel (FP16 grid, FP32 stages) with a modulation:
    a modulation of ones changes nothing, bit for bit; with the log-normal
    modulation the deflections follow the FP64 path's distribution."""
    from scipy.stats import ks_2samp
    torch, crp = dev
    w, B, M, P = small
    pv = {"mixed_f64acc": crp.CRP_PREC_MIXED_F64ACC, "mixed_dfacc": crp.CRP_PREC_MIXED_DFACC}[prec]
    _say(f"case: mixed kernel ({prec}) with a modulation")
    B32 = B.astype(np.float32)

    def run(mod, precision, dtype):
        f = crp.make_field(B32, w.spacing, dtype=dtype, modulation=mod)
        st = crp.particles_to_device(P["pos"], P["dir"], P["energy"], P["charge"])
        crp.crp_propagate([f], [crp.make_params(**PRM)], st, precision=precision)
        torch.cuda.synchronize()
        return crp.particles_to_host(st)

    ones = crp.make_modulation(np.ones((7, 9, 11), np.float32), 0.31, origin=(-1.0, 0.2, 0.4))
    a, b = run(None, pv, "f16"), run(ones, pv, "f16")
    for k in ("pos", "dir", "length", "status", "n_accepted", "n_rejected", "h_next"):
        assert np.array_equal(a[k], b[k]), k
    mod = crp.make_modulation(M.astype(np.float32), 0.25, origin=(-3.0, -3.0, -3.0))
    g = run(mod, pv, "f16")
    # the cell cache (vector cell and FP32 modulation cell) holds stored
    # values: the same results bit for bit with it forced on and off
    for cache in (1, -1):
        f = crp.make_field(B32, w.spacing, dtype="f16", layout="cell8", modulation=mod)
        st = crp.particles_to_device(P["pos"], P["dir"], P["energy"], P["charge"])
        crp.crp_propagate([f], [crp.make_params(**PRM)], st, precision=pv, tuning=crp.make_tuning(cache_cells=cache))
        torch.cuda.synchronize()
        r = crp.particles_to_host(st)
        if cache == 1:
            c_on = r
    for k in ("pos", "dir", "length", "status", "n_accepted", "n_rejected", "h_next"):
        assert np.array_equal(c_on[k], r[k]), k
    ref = run(mod, crp.CRP_PREC_FP64, "f32")
    assert set(np.unique(g["status"])) <= {1, 2}
    defl = lambda r: np.arccos(np.clip(np.sum(r["dir"] * P["dir"], axis=1), -1, 1))  # noqa: E731
    ks = ks_2samp(defl(g), defl(ref))
    _say(f"  KS deflection p = {ks.pvalue:.3f}; arrived {np.mean(g['status'] == 1):.3f} vs {np.mean(ref['status'] == 1):.3f}")
    assert ks.pvalue > 0.01
    assert abs(np.mean(g["status"] == 1) - np.mean(ref["status"] == 1)) < 0.02
    # unmodulated versus modulated: the modulation does change the result
    assert not np.array_equal(g["dir"], a["dir"])
