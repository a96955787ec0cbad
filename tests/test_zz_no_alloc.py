"""The allocation-free propagation entry point (crp_propagate_noalloc, for
callers that cannot allocate device memory) against crp_propagate, through
the C ABI: identical results bit for bit on two calls in a row, the second
with fewer particles (the shared scratch array keeps the first call's
contents, which must not leak into the second)."""
import sys

import numpy as np
import pytest

from gpu_common import require_gpu, workload

pytestmark = pytest.mark.gpu

KEYS = ("pos", "dir", "length", "h_next", "status", "n_accepted", "n_rejected", "time")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("layout, cache", [("cell8", 1), ("linear", -1)])
def test_noalloc_matches_workspace_entry_point(oracle_mod, layout, cache):
    torch, crp = require_gpu()
    w, B, P = workload(1, n=6000)
    f = crp.make_field(B, w.spacing, dtype="f32", layout=layout)
    prm = crp.make_params(w.tol, w.h_min, w.h_max, obs_radius=w.obs_radius, l_max=w.max_length)
    tun = crp.make_tuning(cache_cells=cache)
    _say(f"case: no-alloc entry point, {layout}, cache {cache}, scratch {crp.crp_noalloc_scratch_bytes()} B")
    for n in (6000, 1500):
        ref = crp.particles_to_device(P["pos"][:n], P["dir"][:n], P["energy"][:n], P["charge"][:n])
        got = crp.particles_to_device(P["pos"][:n], P["dir"][:n], P["energy"][:n], P["charge"][:n])
        cr = torch.zeros(crp.NCOUNTERS, dtype=torch.int64, device="cuda")
        cg = torch.zeros(crp.NCOUNTERS, dtype=torch.int64, device="cuda")
        crp.crp_propagate([f], [prm], ref, tuning=tun, counters=cr)
        crp.crp_propagate_noalloc([f], [prm], got, tuning=tun, counters=cg)
        torch.cuda.synchronize()
        a, b = crp.particles_to_host(ref), crp.particles_to_host(got)
        for k in KEYS:
            assert np.array_equal(a[k], b[k]), (n, k)
        # the counters that do not depend on which lane ran which particle
        # (cell loads and wavefront iterations do)
        assert torch.equal(cr[:6], cg[:6]), (n, cr.tolist(), cg.tolist())
        assert int(cg[5]) == n
        _say(f"  n={n}: bitwise equal, {int(cg[1])} accepted steps")


def test_noalloc_several_groups_and_mixed_precision(oracle_mod):
    torch, crp = require_gpu()
    w, B, P = workload(1, n=3000)
    f = crp.make_field(B, w.spacing, dtype="f32", layout="cell8")
    f16 = crp.make_field(B, w.spacing, dtype="f16", layout="cell8")
    prms = [crp.make_params(w.tol, w.h_min, w.h_max, obs_radius=r, l_max=w.max_length) for r in (5.0, 12.0)]
    pidx = (np.arange(3000) % 2).astype(np.int32)
    _say("case: no-alloc entry point, two parameter groups; mixed precision")
    for n, fields, prec in ((3000, [f], crp.CRP_PREC_FP64), (1000, [f16], crp.CRP_PREC_MIXED_F64ACC)):
        ref = crp.particles_to_device(P["pos"][:n], P["dir"][:n], P["energy"][:n], P["charge"][:n],
                                      param_index=pidx[:n])
        got = crp.particles_to_device(P["pos"][:n], P["dir"][:n], P["energy"][:n], P["charge"][:n],
                                      param_index=pidx[:n])
        crp.crp_propagate(fields, prms, ref, precision=prec)
        crp.crp_propagate_noalloc(fields, prms, got, precision=prec)
        torch.cuda.synchronize()
        a, b = crp.particles_to_host(ref), crp.particles_to_host(got)
        for k in KEYS:
            assert np.array_equal(a[k], b[k]), (n, k)
        _say(f"  n={n} precision {prec}: bitwise equal")
