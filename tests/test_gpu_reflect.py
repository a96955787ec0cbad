"""Reflective box on the GPU (the example of section 4 has reflective
boundaries): the distance to the nearest face bids for the step, and an
accepted step that ends outside the box is mirrored on that face.  Compared
with the oracle bit for bit; the zero-field billiard also against its closed
form."""
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
    P = ci.isotropic_particles(3000, 1e18, 3e19, (1, 2, 7, 26), ps)
    return w, B, P


BOX = ((-1.2, -0.9, -1.5), (1.3, 1.1, 1.0))


def _in_box(P, box, seed=11):
    Q = dict(P)
    Q["pos"] = ci.box_positions(len(P["energy"]), box[0], box[1], np.random.SeedSequence(seed))
    return Q


def _gpu(crp, torch, B, spacing, prm_kw, P, box, layout="linear", dtype="f64", tuning=None, modulation=None,
         sel=None, max_steps=0, state=None):
    f = crp.make_field(B, spacing, dtype=dtype, layout=layout, modulation=modulation)
    prm = crp.make_params(**prm_kw, box=box, max_steps=max_steps)
    idx = slice(None) if sel is None else sel
    st = state if state is not None else crp.particles_to_device(P["pos"][idx], P["dir"][idx], P["energy"][idx],
                                                                 P["charge"][idx])
    crp.crp_propagate([f], [prm], st, tuning=tuning)
    torch.cuda.synchronize()
    return crp.particles_to_host(st), st


def _oracle(O, B, spacing, prm_kw, P, box, modulation=None, sel=None):
    g = O.Grid(B, spacing, modulation=modulation)
    prm = O.params_array(prm_kw["tol"], prm_kw["h_min"], prm_kw["h_max"], radius=prm_kw["obs_radius"],
                         l_max=prm_kw["l_max"], box=box)
    idx = slice(None) if sel is None else sel
    return O.propagate(g, prm, P["pos"][idx], P["dir"][idx], P["energy"][idx], P["charge"][idx])


def _inside(pos, box):
    return np.all((pos >= np.asarray(box[0])) & (pos <= np.asarray(box[1])))


PRM = dict(tol=1e-4, h_min=1e-4, h_max=0.5, obs_radius=0.0, l_max=20.0)


def test_billiard_at_zero_field(dev, oracle_mod):
    torch, crp = dev
    _say("case: zero-field billiard")
    B = np.zeros((4, 4, 4, 3))
    rng = np.random.default_rng(5)
    n = 2000
    u0 = rng.standard_normal((n, 3))
    u0 /= np.linalg.norm(u0, axis=1, keepdims=True)
    P = {"pos": rng.uniform(-0.5, 0.5, size=(n, 3)), "dir": u0, "energy": np.full(n, 1e18),
         "charge": np.ones(n, np.int32)}
    lo, hi, L = np.array([-1.0, -0.75, -1.25]), np.array([1.0, 1.25, 0.5]), 7.3
    kw = dict(tol=1e-6, h_min=1e-9, h_max=0.2, obs_radius=0.0, l_max=L)
    g, _ = _gpu(crp, torch, B, 1.0, kw, P, (lo, hi))
    o = _oracle(oracle_mod, B, 1.0, kw, P, (lo, hi))
    compare(g, o, "billiard")
    wdt = hi - lo
    r = np.mod(P["pos"] + L * u0 - lo, 2 * wdt)
    fold = np.where(r <= wdt, lo + r, lo + 2 * wdt - r)
    sign = np.where(np.mod(np.floor((P["pos"] + L * u0 - lo) / wdt), 2) == 0, 1.0, -1.0)
    assert np.max(np.abs(g["pos"] - fold)) < 1e-12
    assert np.max(np.abs(g["dir"] - sign * u0)) < 1e-13


@pytest.mark.parametrize("layout,dtype,cache", [("linear", "f64", 0), ("cell8", "f32", 0), ("linear", "f32", 1)])
def test_turbulent_box_matches_oracle(dev, oracle_mod, small, layout, dtype, cache):
    torch, crp = dev
    w, B, P = small
    _say(f"case: reflective box in the 32^3 grid, {layout} {dtype}, cache {cache}")
    Bs = B if dtype == "f64" else B.astype(np.float32)
    Q = _in_box(P, BOX)
    g, _ = _gpu(crp, torch, Bs, w.spacing, PRM, Q, BOX, layout=layout, dtype=dtype,
                tuning=crp.make_tuning(cache_cells=cache))
    o = _oracle(oracle_mod, Bs, w.spacing, PRM, Q, BOX)
    r = compare(g, o, "reflective box")
    _say(f"  bitwise fraction {r['bitwise_fraction']}")
    assert np.all(g["status"] == 2)
    assert _inside(g["pos"], BOX)
    assert np.max(np.abs(np.linalg.norm(g["dir"], axis=1) - 1.0)) < 1e-14


def test_box_and_sphere_together(dev, oracle_mod, small):
    """Particles from the origin, the observer sphere (r = 2.5) and the box
    (+-2 Mpc, corners outside the sphere): both stops occur."""
    torch, crp = dev
    w, B, P = small
    _say("case: box and observer sphere")
    box = ((-2.0, -2.0, -2.0), (2.0, 2.0, 2.0))
    kw = dict(PRM, obs_radius=2.5, l_max=40.0)
    g, _ = _gpu(crp, torch, B, w.spacing, kw, P, box)
    o = _oracle(oracle_mod, B, w.spacing, kw, P, box)
    compare(g, o, "box and sphere")
    st = set(np.unique(g["status"]))
    _say(f"  statuses {sorted(st)}")
    assert st == {1, 2}


def test_far_box_changes_nothing(dev, small):
    torch, crp = dev
    w, B, P = small
    _say("case: a box the particles never reach")
    kw = dict(PRM, obs_radius=2.5)
    a, _ = _gpu(crp, torch, B, w.spacing, kw, P, None)
    b, _ = _gpu(crp, torch, B, w.spacing, kw, P, ((-1e4,) * 3, (1e4,) * 3))
    for k in ("pos", "dir", "length", "status", "n_accepted", "n_rejected", "h_next"):
        assert np.array_equal(a[k], b[k]), k


def test_groups_with_and_without_box(dev, oracle_mod, small):
    torch, crp = dev
    w, B, P = small
    _say("case: two parameter groups, one with a box")
    Q = _in_box(P, BOX)
    f = crp.make_field(B, w.spacing, dtype="f64")
    prms = [crp.make_params(**PRM, box=BOX), crp.make_params(**PRM)]
    pidx = np.arange(len(Q["energy"])) % 2
    st = crp.particles_to_device(Q["pos"], Q["dir"], Q["energy"], Q["charge"], param_index=pidx)
    crp.crp_propagate([f], prms, st)
    torch.cuda.synchronize()
    g = crp.particles_to_host(st)
    for gi, box in ((0, BOX), (1, None)):
        sel = np.nonzero(pidx == gi)[0]
        o = _oracle(oracle_mod, B, w.spacing, PRM, Q, box, sel=sel)
        compare({k: v[sel] for k, v in g.items()}, o, f"group {gi}")
    assert _inside(g["pos"][pidx == 0], BOX)
    assert not _inside(g["pos"][pidx == 1], BOX)


def test_resumed_in_chunks_equals_one_call(dev, small):
    torch, crp = dev
    w, B, P = small
    _say("case: reflective run resumed every 50 accepted steps")
    Q = _in_box(P, BOX)
    sel = slice(0, 300)
    kw = dict(PRM, l_max=5.0)
    whole, _ = _gpu(crp, torch, B, w.spacing, kw, Q, BOX, sel=sel)
    g, state = _gpu(crp, torch, B, w.spacing, kw, Q, BOX, sel=sel, max_steps=50)
    f = crp.make_field(B, w.spacing, dtype="f64")
    prm = crp.make_params(**kw, box=BOX, max_steps=50)
    rounds = 0
    while np.any(g["status"] == 3):
        st = state["status"]
        st[st == 3] = 0
        crp.crp_propagate([f], [prm], state)
        torch.cuda.synchronize()
        g = crp.particles_to_host(state)
        rounds += 1
    assert rounds >= 2
    for k in ("pos", "dir", "length", "h_next", "status", "n_accepted", "n_rejected"):
        assert np.array_equal(whole[k], g[k]), k


def test_modulated_field_in_box(dev, oracle_mod, small):
    torch, crp = dev
    w, B, P = small
    _say("case: modulated field in a reflective box")
    fs, ps, rs = ci.config_seeds(0)
    M = ci.lognormal_modulation(24, 0.25, 1.0, 1.0, rs)
    mod = crp.make_modulation(M, 0.25, origin=(-3.0, -3.0, -3.0), dtype="f64")
    Q = _in_box(P, BOX)
    g, _ = _gpu(crp, torch, B, w.spacing, PRM, Q, BOX, modulation=mod)
    o = _oracle(oracle_mod, B, w.spacing, PRM, Q, BOX, modulation=oracle_mod.Modulation(M, 0.25, (-3.0,) * 3))
    compare(g, o, "modulated box")
    assert _inside(g["pos"], BOX)


def test_reflective_workload_sample(dev, oracle_mod):
    """The reflective workload at full size (256^3 FP32 vector grid, 440^3 FP32
    modulation, 132 Mpc box, 1e6 nuclei) in one launch; a sample against the oracle."""
    torch, crp = dev
    w = ci.get_config("reflective_132box")
    fs, ps, rs = ci.config_seeds(w.index)
    B = ci.kolmogorov_field(w.grid_n, w.spacing, w.l_min, w.l_max, w.b_rms, fs, dtype=np.float32)
    M = ci.lognormal_modulation(w.mod_n, w.mod_spacing, w.mod_l_corr, w.mod_sigma, rs, dtype=np.float32)
    P = ci.isotropic_particles(w.n_particles, w.e_min, w.e_max, w.charges, ps)
    P["pos"] = ci.box_positions(w.n_particles, w.reflect_box[0], w.reflect_box[1], ci.position_seed(w.index))
    o0 = (w.mod_origin,) * 3
    _say(f"case: reflective workload, {w.n_particles} particles, box {w.reflect_box}")
    mod = crp.make_modulation(M, w.mod_spacing, origin=o0)
    kw = dict(tol=w.tol, h_min=w.h_min, h_max=w.h_max, obs_radius=w.obs_radius, l_max=w.max_length)
    g, _ = _gpu(crp, torch, B, w.spacing, kw, P, w.reflect_box, layout="cell8", dtype="f32", modulation=mod)
    assert np.all(g["status"] == 2)
    assert _inside(g["pos"], w.reflect_box)
    rng = np.random.default_rng(9)
    sel = np.sort(rng.choice(w.n_particles, 300, replace=False))
    o = _oracle(oracle_mod, B, w.spacing, kw, P, w.reflect_box, modulation=oracle_mod.Modulation(M, w.mod_spacing, o0),
                sel=sel)
    r = compare({k: v[sel] for k, v in g.items()}, o, "reflective workload sample")
    _say(f"  bitwise fraction {r['bitwise_fraction']}")


@pytest.mark.parametrize("prec", ["mixed_f64acc", "mixed_dfacc"])
def test_mixed_kernel_reflects(dev, small, prec):
    """The mixed-precision kernel (FP16 grid, FP32 stages) in a reflective box:
    the zero-field billiard against its closed form within the FP32 stage
    rounding, and in a field every particle stays in the box with unit
    direction and the exact length stop."""
    torch, crp = dev
    w, B, P = small
    pv = {"mixed_f64acc": crp.CRP_PREC_MIXED_F64ACC, "mixed_dfacc": crp.CRP_PREC_MIXED_DFACC}[prec]
    _say(f"case: mixed kernel ({prec}) in a reflective box")
    rng = np.random.default_rng(15)
    n = 2000
    u0 = rng.standard_normal((n, 3))
    u0 /= np.linalg.norm(u0, axis=1, keepdims=True)
    x0 = rng.uniform(-0.5, 0.5, size=(n, 3))
    lo, hi, L = np.array([-1.0, -0.75, -1.25]), np.array([1.0, 1.25, 0.5]), 7.3
    f0 = crp.make_field(np.zeros((4, 4, 4, 3), np.float32), 1.0, dtype="f16")
    st = crp.particles_to_device(x0, u0, np.full(n, 1e18), np.ones(n, np.int32))
    crp.crp_propagate([f0], [crp.make_params(1e-6, 1e-9, 0.2, l_max=L, box=(lo, hi))], st, precision=pv)
    torch.cuda.synchronize()
    g = crp.particles_to_host(st)
    assert np.all(g["status"] == 2) and np.all(g["length"] == L)
    wdt = hi - lo
    r = np.mod(x0 + L * u0 - lo, 2 * wdt)
    fold = np.where(r <= wdt, lo + r, lo + 2 * wdt - r)
    sign = np.where(np.mod(np.floor((x0 + L * u0 - lo) / wdt), 2) == 0, 1.0, -1.0)
    near_face = np.min(np.minimum(np.abs(fold - lo), np.abs(hi - fold)), axis=1) < 1e-4
    ok = ~near_face  # a fold within 1e-4 of a face may be taken on the other side of it
    assert np.mean(ok) > 0.99
    assert np.max(np.abs(g["pos"][ok] - fold[ok])) < 1e-5
    assert np.max(np.abs(g["dir"][ok] - sign[ok] * u0[ok])) < 1e-5
    Q = _in_box(P, BOX)
    fm = crp.make_field(B.astype(np.float32), w.spacing, dtype="f16")
    st = crp.particles_to_device(Q["pos"], Q["dir"], Q["energy"], Q["charge"])
    crp.crp_propagate([fm], [crp.make_params(**PRM, box=BOX)], st, precision=pv)
    torch.cuda.synchronize()
    h = crp.particles_to_host(st)
    assert np.all(h["status"] == 2) and np.all(h["length"] == PRM["l_max"])
    assert _inside(h["pos"], BOX)
    assert np.max(np.abs(np.linalg.norm(h["dir"], axis=1) - 1.0)) < 1e-6
