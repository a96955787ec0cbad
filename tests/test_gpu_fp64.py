"""GPU parity of the FP64-state propagation path against the FP64 CPU oracle.

Every call goes through the C ABI (libcrp.so).  The design goal is bitwise
equality of every particle's state; the gate is the stated tolerance
(arrival direction <= 1e-6 rad, relative position <= 1e-9).
"""
import math
import sys
from fractions import Fraction

import numpy as np
import pytest

import crp_inputs as ci
from gpu_common import compare, require_gpu, run_gpu, run_oracle, workload

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    return require_gpu()


@pytest.fixture(scope="module")
def c1():
    return workload(0)


@pytest.fixture(scope="module")
def c2_field():
    w, B, P = workload(1, n=20000)
    return w, B, P


# --------------------------------------------------------------- arithmetic

def test_device_arithmetic_matches_host(dev, oracle_mod):
    torch, crp = dev
    _say("case: device arithmetic conformance")
    rng = np.random.default_rng(1)
    x = np.concatenate([10.0 ** rng.uniform(-300, 300, 200000), rng.uniform(0, 4, 200000),
                        2.0 ** np.arange(-60, 60), [1.0, 0.25, 5e-324, 1.7e308]])
    xt = torch.from_numpy(x).cuda()
    out = torch.empty_like(xt)
    for op, ref in [(0, np.sqrt(x)), (1, 1.0 / x), (5, 1.0 / np.sqrt(np.sqrt(x)))]:
        crp.crp_selftest_arith(xt, out, op)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        assert np.array_equal(got, ref), f"op {op}: {np.count_nonzero(got != ref)} mismatches"
    y = np.concatenate([rng.uniform(-1e6, 1e6, 4000), rng.standard_normal(4000) * 1e-3])
    crp.crp_selftest_arith(torch.from_numpy(y).cuda(), out[:len(y)], 3)
    torch.cuda.synchronize()
    assert np.array_equal(out[:len(y)].cpu().numpy(), np.floor(y))
    e = 10.0 ** rng.uniform(-12, 6, 20000)
    et = torch.from_numpy(e).cuda()
    o5 = torch.empty_like(et)
    crp.crp_selftest_arith(et, o5, 4)
    torch.cuda.synchronize()
    ref5 = np.array([oracle_mod.inv_fifth_root(v) for v in e])
    assert np.array_equal(o5.cpu().numpy(), ref5)
    trip = rng.standard_normal((3000, 3)) * np.array([1e3, 1e-3, 1.0])
    tt = torch.from_numpy(trip.reshape(-1).copy()).cuda()
    of = torch.empty(3000, dtype=torch.float64, device="cuda")
    crp.crp_selftest_arith(tt, of, 2)
    torch.cuda.synchronize()
    reff = np.array([float(Fraction(a) * Fraction(b) + Fraction(c)) for a, b, c in trip])
    assert np.array_equal(of.cpu().numpy(), reff)


# --------------------------------------------------------------- parity

def test_small_fp64_workload_full(dev, oracle_mod, c1):
    torch, crp = dev
    w, B, P = c1
    _say("case: 1000 protons, 32^3 FP64 grid, L = 50 Mpc")
    cnt = torch.zeros(crp.NCOUNTERS, dtype=torch.int64, device="cuda")
    g, _, _ = run_gpu(crp, torch, B, w.spacing, w, P, counters=cnt)
    o = run_oracle(oracle_mod, B, w.spacing, w, P)
    r = compare(g, o, "small")
    c = cnt.cpu().numpy()
    assert c[1] == o["counters"]["accepted"] and c[2] == o["counters"]["rejected"]
    assert c[5] == len(P["energy"])
    assert np.array_equal(g["time"], g["length"] * oracle_mod.constants()["MPC_OVER_C"])
    _say("small:", r)


def test_single_group_uses_its_field(dev, oracle_mod, c1):
    """One parameter group naming the second of two fields (no per-particle
    groups): the launch must use that field."""
    torch, crp = dev
    w, B, P = c1
    _say("case: one parameter group on field 1 of 2")
    other = np.ascontiguousarray(B[::-1] * 2.0)
    f0 = crp.make_field(other, w.spacing, dtype="f64")
    f1 = crp.make_field(B, w.spacing, dtype="f64")
    prm = crp.make_params(w.tol, w.h_min, w.h_max, obs_radius=1.5, l_max=20.0, field_index=1)
    st = crp.particles_to_device(P["pos"], P["dir"], P["energy"], P["charge"])
    crp.crp_propagate([f0, f1], [prm], st)
    torch.cuda.synchronize()
    g = crp.particles_to_host(st)
    o = run_oracle(oracle_mod, B, w.spacing, w, P, radius=1.5, l_max=20.0)
    compare(g, o, "field 1 of 2")


@pytest.mark.parametrize("n", [1, 63, 65, 257, 3001])
def test_ragged_sizes(dev, oracle_mod, c1, n):
    torch, crp = dev
    w, B, P = c1
    _say(f"case: ragged n={n}")
    sel = slice(0, n)
    g, _, _ = run_gpu(crp, torch, B, w.spacing, w, P if n <= 1000 else
                      ci.isotropic_particles(n, w.e_min, w.e_max, w.charges, np.random.SeedSequence(9)),
                      sel=sel, radius=1.5, l_max=20.0)
    Q = P if n <= 1000 else ci.isotropic_particles(n, w.e_min, w.e_max, w.charges, np.random.SeedSequence(9))
    o = run_oracle(oracle_mod, B, w.spacing, w, Q, sel=sel, radius=1.5, l_max=20.0)
    compare(g, o, f"ragged {n}")


def test_empty_call(dev, c1):
    torch, crp = dev
    w, B, P = c1
    _say("case: n = 0")
    st = crp.particles_to_device(P["pos"][:0], P["dir"][:0], P["energy"][:0], P["charge"][:0])
    f = crp.make_field(B, w.spacing, dtype="f64")
    crp.crp_propagate([f], [crp.make_params(w.tol, w.h_min, w.h_max, l_max=5.0)], st)
    torch.cuda.synchronize()


def test_production_grid_sample(dev, oracle_mod, c2_field):
    """256^3 FP32 grid, mixed nuclei, sphere r = 20 Mpc or L = 1 Gpc (first 20000 particles)."""
    torch, crp = dev
    w, B, P = c2_field
    _say("case: 256^3 FP32 grid, 20000 mixed nuclei")
    g, _, _ = run_gpu(crp, torch, B, w.spacing, w, P)
    o = run_oracle(oracle_mod, B, w.spacing, w, P)
    r = compare(g, o, "production sample")
    _say("production sample:", r, "arrived", int(np.sum(g["status"] == 1)))


@pytest.mark.parametrize("tuning", [
    dict(block_size=64, blocks_per_cu=1, refill_threshold=1, order_by_rigidity=0),
    dict(block_size=128, blocks_per_cu=0, refill_threshold=1, order_by_rigidity=1),
    dict(block_size=256, blocks_per_cu=2, refill_threshold=16, order_by_rigidity=1),
    dict(block_size=256, blocks_per_cu=8, refill_threshold=64, order_by_rigidity=0),
    dict(block_size=256, blocks_per_cu=4, refill_threshold=1, order_by_rigidity=1, cache_cells=-1),
    dict(block_size=256, blocks_per_cu=4, refill_threshold=32, order_by_rigidity=1, cache_cells=1),
])
def test_results_independent_of_launch_configuration(dev, c2_field, tuning):
    torch, crp = dev
    w, B, P = c2_field
    _say(f"case: tuning {tuning}")
    sel = slice(0, 4000)
    ref, _, _ = run_gpu(crp, torch, B, w.spacing, w, P, sel=sel)
    g, _, _ = run_gpu(crp, torch, B, w.spacing, w, P, sel=sel, tuning=crp.make_tuning(**tuning))
    for k in ("pos", "dir", "length", "h_next", "status", "n_accepted", "n_rejected"):
        assert np.array_equal(ref[k], g[k]), k


def test_automatic_cell_cache_choice(dev):
    """cache_cells = 0 (automatic): on for LINEAR; for CELL8 only above 2048
    particles per compute unit, with one parameter group or several.  Read
    from the launch counters: with the cache fewer than 6 cell loads per
    evaluation, without it exactly 6."""
    torch, crp = dev
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    w, B, P = workload(1, n=2048 * cus + 4096)
    f_lin = crp.make_field(B, w.spacing, dtype="f32", layout="linear")
    f_c8 = crp.make_field(B, w.spacing, dtype="f32", layout="cell8")
    prm = crp.make_params(w.tol, w.h_min, w.h_max, obs_radius=w.obs_radius, l_max=2.0)

    def loads_per_eval(field, n, groups=1):
        s = crp.particles_to_device(P["pos"][:n], P["dir"][:n], P["energy"][:n], P["charge"][:n],
                                    param_index=None if groups == 1 else np.zeros(n, dtype=np.int32))
        c = torch.zeros(crp.NCOUNTERS, dtype=torch.int64, device="cuda")
        crp.crp_propagate([field], [prm] * groups, s, counters=c)
        torch.cuda.synchronize()
        c = c.cpu().numpy()
        return c[6] / (6.0 * c[0])

    small, large = 4096, 2048 * cus + 4096
    _say(f"case: automatic cell cache, {cus} compute units, {small} and {large} particles")
    assert loads_per_eval(f_lin, small) < 0.9
    assert loads_per_eval(f_c8, small) == 1.0
    assert loads_per_eval(f_c8, large) < 0.9
    assert loads_per_eval(f_c8, large, groups=2) < 0.9
    assert loads_per_eval(f_lin, small, groups=2) < 0.9


def test_cell8_layout_bitwise_equal_to_linear(dev, c2_field):
    torch, crp = dev
    w, B, P = c2_field
    _say("case: CELL8 layout")
    sel = slice(0, 4000)
    a, _, _ = run_gpu(crp, torch, B, w.spacing, w, P, sel=sel, layout="linear")
    b, _, _ = run_gpu(crp, torch, B, w.spacing, w, P, sel=sel, layout="cell8")
    for k in ("pos", "dir", "length", "h_next", "status", "n_accepted", "n_rejected"):
        assert np.array_equal(a[k], b[k]), k


def test_resume_after_budget_bitwise(dev, oracle_mod, c1):
    torch, crp = dev
    w, B, P = c1
    _say("case: resume after max_steps")
    sel = slice(0, 300)
    full, _, _ = run_gpu(crp, torch, B, w.spacing, w, P, sel=sel, radius=2.0)
    g, state, f = run_gpu(crp, torch, B, w.spacing, w, P, sel=sel, radius=2.0, max_steps=5)
    prm = crp.make_params(w.tol, w.h_min, w.h_max, obs_radius=2.0, l_max=w.max_length, max_steps=5)
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
        assert np.array_equal(full[k], g[k]), k
    o = run_oracle(oracle_mod, B, w.spacing, w, P, sel=sel, radius=2.0)
    compare(g, o, "resume")


def test_off_centre_sphere_and_backtracking(dev, oracle_mod, c1):
    torch, crp = dev
    w, B, P = c1
    _say("case: off-centre sphere, negative charges")
    Q = dict(P)
    Q["charge"] = np.where(np.arange(len(P["charge"])) % 2 == 0, 1, -1).astype(np.int32)
    c = (0.3, -0.2, 0.1)
    g, _, _ = run_gpu(crp, torch, B, w.spacing, w, Q, radius=3.0, center=c)
    o = run_oracle(oracle_mod, B, w.spacing, w, Q, radius=3.0, center=c)
    compare(g, o, "off-centre")


def test_bad_inputs_and_inactive(dev, oracle_mod, c1):
    torch, crp = dev
    w, B, P = c1
    _say("case: bad inputs and inactive particles")
    n = 8
    pos = np.zeros((n, 3))
    pos[2, 0] = np.nan
    d = P["dir"][:n].copy()
    d[3] = 0.0
    E = P["energy"][:n].copy()
    E[4] = -1.0
    Z = P["charge"][:n].copy()
    Z[5] = 0
    st = crp.particles_to_device(pos, d, E, Z)
    s = st["status"]
    s[6] = 2
    s[7] = 1
    f = crp.make_field(B, w.spacing, dtype="f64")
    crp.crp_propagate([f], [crp.make_params(w.tol, w.h_min, w.h_max, l_max=10.0)], st)
    torch.cuda.synchronize()
    g = crp.particles_to_host(st)
    assert list(g["status"]) == [2, 2, 6, 6, 6, 2, 2, 1]
    o = oracle_mod.propagate(oracle_mod.Grid(B, w.spacing), oracle_mod.params_array(w.tol, w.h_min, w.h_max,
                             l_max=10.0), pos, d, E, Z, status=np.array([0] * 6 + [2, 1], np.int32))
    assert list(o["status"]) == list(g["status"])
    ok = [0, 1, 5]
    for k, ko in (("pos", "pos"), ("dir", "dir"), ("length", "length")):
        assert np.array_equal(g[k][ok], o[ko][ok]), k


def test_nonfinite_cell(dev, oracle_mod, c1):
    torch, crp = dev
    w, B, P = c1
    _say("case: NaN grid cell")
    Bn = B.copy()
    Bn[0, 0, 0, 1] = np.nan
    sel = slice(0, 200)
    g, _, _ = run_gpu(crp, torch, Bn, w.spacing, w, P, sel=sel, l_max=10.0)
    o = run_oracle(oracle_mod, Bn, w.spacing, w, P, sel=sel, l_max=10.0)
    assert np.all(g["status"] == 4)
    compare(g, o, "nan cell")


@pytest.mark.parametrize("bad", ["tol", "hmin", "order", "nolimit", "lmax", "nfield"])
def test_invalid_arguments_rejected_before_launch(dev, c1, bad):
    torch, crp = dev
    w, B, P = c1
    st = crp.particles_to_device(P["pos"][:4], P["dir"][:4], P["energy"][:4], P["charge"][:4])
    f = crp.make_field(B, w.spacing, dtype="f64")
    kw = dict(tol=w.tol, h_min=w.h_min, h_max=w.h_max, l_max=5.0)
    if bad == "tol":
        kw["tol"] = 0.0
    elif bad == "hmin":
        kw["h_min"] = -1.0
    elif bad == "order":
        kw["h_min"] = 2.0
    elif bad == "nolimit":
        kw["l_max"] = math.inf
    elif bad == "lmax":
        kw["l_max"] = float("nan")
    prm = crp.make_params(**kw)
    if bad == "nfield":
        prm.field_index = 3
    before = {k: v.clone() for k, v in st.items() if v is not None}
    with pytest.raises(crp.CRPError) as ei:
        crp.crp_propagate([f], [prm], st)
    assert ei.value.status == crp.CRP_ERR_INVALID
    torch.cuda.synchronize()
    for k, v in before.items():
        assert torch.equal(v, st[k]), k
