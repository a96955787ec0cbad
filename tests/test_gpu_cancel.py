"""The caller's cancel word (crp_tuning.cancel): a call stops early when it is
set, the particles it stopped carry status CANCELLED with their state saved,
the ones it never started stay ACTIVE and untouched, and resuming gives the
bit-identical result of an uninterrupted call (section 3.1: propagation ends
when completed or aborted)."""
import sys

import numpy as np
import pytest

from gpu_common import require_gpu, workload

pytestmark = pytest.mark.gpu

KEYS = ("pos", "dir", "length", "h_next", "status", "n_accepted", "n_rejected")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def setup():
    torch, crp = require_gpu()
    w, B, P = workload(1, n=40000)
    f32 = crp.make_field(B, w.spacing, dtype="f32", layout="cell8")
    f16 = crp.make_field(B, w.spacing, dtype="f16", layout="cell8")
    prm = crp.make_params(w.tol, w.h_min, w.h_max, obs_radius=w.obs_radius, l_max=w.max_length)
    return torch, crp, w, P, {0: f32, 1: f16}, prm


def _state(crp, P):
    return crp.particles_to_device(P["pos"], P["dir"], P["energy"], P["charge"])


def _resume_until_done(torch, crp, field, prm, st, precision, tun):
    for _ in range(20):
        s = st["status"]
        if not bool((s == 5).any() | (s == 0).any()):
            return
        s[s == 5] = 0
        crp.crp_propagate([field], [prm], st, precision=precision, tuning=tun)
        torch.cuda.synchronize()
    raise AssertionError("resumed calls did not finish")


@pytest.mark.parametrize("precision", [0, 1])
def test_cancel_before_the_call_starts_nothing(setup, precision):
    torch, crp, w, P, fields, prm = setup
    _say(f"case: cancel word set before the call, precision {precision}")
    flag = torch.ones(1, dtype=torch.int32, device="cuda")
    st = _state(crp, P)
    before = crp.particles_to_host(st)
    crp.crp_propagate([fields[precision]], [prm], st, precision=precision,
                      tuning=crp.make_tuning(blocks_per_cu=2, cancel=flag))
    torch.cuda.synchronize()
    after = crp.particles_to_host(st)
    for k in KEYS:
        assert np.array_equal(before[k], after[k]), k
    assert np.all(after["status"] == 0)


@pytest.mark.parametrize("precision", [0, 1])
def test_cancel_during_the_call_resumes_bitwise(setup, precision):
    """The word is set from a second stream after a spin while the
    propagation runs; how many particles the cancel caught depends on when
    the second stream's kernel runs, but the resumed result never does."""
    torch, crp, w, P, fields, prm = setup
    ref = _state(crp, P)
    crp.crp_propagate([fields[precision]], [prm], ref, precision=precision)
    torch.cuda.synchronize()
    ref = crp.particles_to_host(ref)
    flag = torch.zeros(1, dtype=torch.int32, device="cuda")
    tun = crp.make_tuning(blocks_per_cu=1, cancel=flag)
    st = _state(crp, P)
    side = torch.cuda.Stream()
    torch.cuda.synchronize()
    crp.crp_propagate([fields[precision]], [prm], st, precision=precision, tuning=tun)
    with torch.cuda.stream(side):
        torch.cuda._sleep(20_000_000)  # ~10 ms of spinning on the other stream
        flag.fill_(1)
    torch.cuda.synchronize()
    mid = crp.particles_to_host(st)
    n_cancel, n_untouched = int(np.sum(mid["status"] == 5)), int(np.sum(mid["status"] == 0))
    _say(f"case: cancel during the call, precision {precision}: {n_cancel} cancelled, {n_untouched} not started")
    assert set(np.unique(mid["status"])) <= {0, 1, 2, 5}
    assert np.all(mid["n_accepted"][mid["status"] == 5] > 0)
    flag.zero_()
    _resume_until_done(torch, crp, fields[precision], prm, st, precision, tun)
    out = crp.particles_to_host(st)
    for k in KEYS:
        assert np.array_equal(out[k], ref[k]), k
