#!/usr/bin/env python3
"""Throughput benchmark of the propagation hot path on one MI355X.

Workload (default, production_256cube): 1e6 nuclei (Z uniform in {1, 2, 7,
26}, E log-uniform in 1e18..1e20 eV, isotropic from the origin) in a 256^3
FP32 Kolmogorov grid (spacing 50 kpc, l_min 100 kpc, l_max 5 Mpc, B_rms 1 nG),
tolerance 1e-4, steps 1 kpc .. 1 Mpc, stop at the r = 20 Mpc sphere or at
1 Gpc of path.  A step of the benchmark propagates every particle until it
stops.  Other workloads: --workload small_fp64_32cube | batched_64x64cube |
precision_1024cube | adjoint_128cube | modulated_256cube (the production
vector grid times a 440^3 modulation grid at 300 kpc, section 3.2) |
reflective_132box (that modulated field inside a reflective 132 Mpc box, the
particles starting uniformly in it, 100 Mpc of path; section 4) | lens_nside64
(3,145,728 protons at 10 EeV traced back through the production field to a
20 Mpc sphere, then a HEALPix nside-64 lens built and applied; section 3.3).

Prints one JSON line: particle-steps/s (accepted Cash-Karp steps per second of
the whole job), the lookup roofline of the propagation kernel (algorithmic
bytes of the field lookups per launch / average launch time, against the HBM
peak), the mixed-precision kernel on the same inputs, and the CPU oracle timed
on a bounded sample of the same workload.
"""
import argparse
import dataclasses
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-steps/s + gather GB/s vs roofline; adjoint/forward time; err vs FP64"
HBM_PEAK_GBPS = 8000.0
# MI355X published vector peaks (TFLOP/s, fma counted as two operations)
FP64_VECTOR_PEAK_TFLOPS = 78.6
FP32_VECTOR_PEAK_TFLOPS = 157.3
# Floating-point operations of one Cash-Karp evaluation of the FP64 path
# (fma = 2; add, mul, div, sqrt = 1), from its arithmetic: 6 lookups of 72
# (cell fractions 9, three trilinear components of 7 lerps 63), 6 Lorentz
# terms of 12, the stage states 240, the fifth-order solution 60 and error
# vector 66, two norms 12, the error ratio 2, and the controller, stop and
# bid arithmetic of an accepted step about 74.
FLOPS_PER_EVALUATION = 950
BYTES_PER_VALUE = {"f64": 8, "f32": 4, "f16": 2, "bf16": 2}
# the propagation kernel's device sources (its profiles are tied to their hash)
KERNEL_SOURCES = ["crp_device.h", "lane.h", "propagate_fp64.hip", "crp_internal.h"]
PRECISIONS = {"fp64": 0, "mixed_f64acc": 1, "mixed_dfacc": 2}
PRECISION_LAYOUT = "cell8"  # storage of the precision leg's 1024^3 grids


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1410_5323_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str, layout: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"traffic_propagate_fp64_{workload}_{layout}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("kernel_source_sha") != kernel_source_hash():
        return None
    return t.get("hbm_bytes_per_launch")


def angle(a, b):
    import numpy as np
    return np.arctan2(np.linalg.norm(np.cross(a, b), axis=1), np.sum(a * b, axis=1))


def build_modulation(w):
    """The modulation grid of a modulated workload (numpy FP32), else None."""
    import numpy as np

    import crp_inputs as ci
    if not w.mod_n:
        return None
    _, _, rs = ci.config_seeds(w.index)
    return ci.lognormal_modulation(w.mod_n, w.mod_spacing, w.mod_l_corr, w.mod_sigma, rs, dtype=np.float32)


def build_inputs(w, n_override):
    """Field grids (numpy, FP32 or FP64), per-group stop radii and the particle list."""
    import numpy as np

    import crp_inputs as ci
    fs, ps, rs = ci.config_seeds(w.index)
    gdt = np.float64 if w.grid_dtype == "f64" else np.float32
    if w.n_realisations:
        table = ci.realisation_table(w, rs)
        P = ci.realisation_particles(w, table, ps)
        seeds = fs.spawn(w.n_realisations)
        grids = [ci.kolmogorov_field(w.grid_n, w.spacing, w.l_min, w.l_max, float(table["b_rms"][r]), seeds[r],
                                     dtype=gdt) for r in range(w.n_realisations)]
        radii = [float(r) for r in table["radius"]]
    else:
        n = w.n_particles if n_override is None else n_override
        P = ci.isotropic_particles(n, w.e_min, w.e_max, w.charges, ps, charge_rule=w.charge_rule)
        if w.reflect_box is not None:
            P["pos"] = ci.box_positions(n, w.reflect_box[0], w.reflect_box[1], ci.position_seed(w.index))
        if w.lens_nside:
            # the drawn directions are where the particles are observed to come
            # from; backtracking starts from the reversed velocity
            P["sky"] = P["dir"].copy()
            P["dir"] = -P["dir"]
        grids = [ci.kolmogorov_field(w.grid_n, w.spacing, w.l_min, w.l_max, w.b_rms, fs, dtype=gdt)]
        radii = [w.obs_radius]
    return grids, radii, P


def cpu_baseline(grids, radii, w, P, sample: int, modulation=None):
    """The oracle, as it stands, on the first `sample` particles, all host cores."""
    import numpy as np

    from oracle import oracle as O
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    omp = os.environ.get("OMP_NUM_THREADS")
    threads = min(cores, int(omp)) if omp and omp.isdigit() else cores
    pidx = P.get("param_index")
    groups = np.zeros(sample, np.int64) if pidx is None else pidx[:sample]
    out = {"pos": np.zeros((sample, 3)), "dir": np.zeros((sample, 3)), "length": np.zeros(sample),
           "status": np.zeros(sample, np.int32), "n_acc": np.zeros(sample, np.int64)}
    acc = evals = 0
    t0 = time.perf_counter()
    for gi in np.unique(groups):
        sel = np.nonzero(groups == gi)[0]
        prm = O.params_array(w.tol, w.h_min, w.h_max, radius=radii[gi], l_max=w.max_length, box=w.reflect_box,
                             backtrack=w.lens_nside > 0)
        mod = None if modulation is None else O.Modulation(modulation, w.mod_spacing, (w.mod_origin,) * 3)
        r = O.propagate(O.Grid(grids[gi], w.spacing, modulation=mod), prm, P["pos"][sel], P["dir"][sel], P["energy"][sel],
                        P["charge"][sel], nthreads=threads)
        for k in out:
            out[k][sel] = r[k]
        acc += int(np.sum(r["n_acc"]))
        evals += r["counters"]["evals"]
    dt = time.perf_counter() - t0
    return {"value": acc / dt, "unit": "particle-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"first {sample} particles of the same seeded list ({acc} accepted steps, "
                      f"{evals} evaluations, {dt:.1f} s)"}, out


def lens_leg(crp, torch, w, P, state, reps: int = 20) -> dict:
    """Lens of the workload's rigidity from the backtracking pass just timed:
    observed pixels of the launches, lens construction and lens application
    (one map and 64 maps), each timed with events on the current stream."""
    import numpy as np
    nside = w.lens_nside
    npix = crp.healpix_npix(nside)
    stream = torch.cuda.current_stream()
    sky = [torch.from_numpy(np.ascontiguousarray(P["sky"][:, k])).cuda() for k in range(3)]
    n = int(sky[0].numel())
    ws = torch.empty(crp.crp_lens_workspace_bytes(nside, n), dtype=torch.uint8, device="cuda")

    def ev_ms(fn, count):
        out = []
        for _ in range(count):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            fn()
            b.record(stream)
            b.synchronize()
            out.append(a.elapsed_time(b))
        return out

    rows = crp.crp_healpix_pixels(nside, *sky)
    pix_ms = ev_ms(lambda: crp.crp_healpix_pixels(nside, *sky, pix=rows), 5)
    lens = crp.crp_lens_build(nside, rows, state, workspace=ws)
    outs = (torch.empty_like(lens.row_ptr), torch.empty(n, dtype=torch.int32, device="cuda"),
            torch.empty(n, dtype=torch.float32, device="cuda"))
    build_ms = ev_ms(lambda: crp.crp_lens_build(nside, rows, state, workspace=ws, out=outs), 5)
    out = {"nside": nside, "pixels": npix, "launches": n, "nnz": lens.nnz, "entries_per_row": lens.nnz / npix,
           "escaped_fraction": float((state["status"] == 1).float().mean().item()),
           "matrix_MB": lens.nbytes() / 1e6, "pixels_ms": float(np.median(pix_ms)),
           "build_ms": float(np.median(build_ms))}
    g = torch.Generator(device="cuda")
    g.manual_seed(5)
    for nvec in (1, 64):
        x = torch.rand((npix, nvec) if nvec > 1 else (npix,), generator=g, device="cuda", dtype=torch.float32)
        y = torch.empty_like(x)
        crp.crp_lens_apply(lens, x, y)
        ms = float(np.median(ev_ms(lambda: crp.crp_lens_apply(lens, x, y), reps)))
        alg = 8 * lens.nnz + 8 * (npix + 1) + 2 * 4 * npix * nvec
        out[f"apply_{nvec}"] = {"ms": ms, "algorithmic_bytes": alg, "GB_per_s": alg / (ms * 1e-3) / 1e9,
                                "frac_of_hbm_peak": alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS}
    return out


def lens_cpu_baseline(w, P, ref, m: int) -> dict:
    """The lens oracle on the oracle's own backtracking of the first m launches."""
    import numpy as np

    from oracle import lens as LN
    nside = w.lens_nside
    t0 = time.perf_counter()
    rows = LN.pix_ring(nside, P["sky"][:m, 0], P["sky"][:m, 1], P["sky"][:m, 2])
    row_ptr, col, val = LN.lens_matrix(nside, rows, ref["dir"][:, 0], ref["dir"][:, 1], ref["dir"][:, 2],
                                       ref["status"] == 1)
    t1 = time.perf_counter()
    x = np.random.default_rng(5).random((LN.npix(nside), 64)).astype(np.float32)
    LN.lens_apply(row_ptr, col, val, x)
    t2 = time.perf_counter()
    return {"kind": "oracle", "sample": f"first {m} launches", "build_launches_per_s": m / (t1 - t0),
            "apply_64_ms": (t2 - t1) * 1e3, "nnz": int(len(col))}


def gather_ceiling(field, lanes: int = 262144, per_lane: int = 200, reps: int = 3) -> dict:
    """Achievable lookup rate of the grid: the gather microbenchmark (same
    field, dtype, layout and FP64 trilinear arithmetic as the propagation
    kernel; independent lookups at uniformly random positions, so no cache
    locality), best of `reps` launches timed with HIP events."""
    import torch

    from paper_1410_5323_amd import crp
    sink = torch.empty(lanes, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    crp.crp_bench_gather(field, lanes, per_lane, 0.0, 1, sink)
    best = float("inf")
    for r in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        crp.crp_bench_gather(field, lanes, per_lane, 0.0, 2 + r, sink)
        b.record(stream)
        torch.cuda.synchronize()
        best = min(best, a.elapsed_time(b) / 1e3)
    return {"lookups_per_s": lanes * per_lane / best, "lanes": lanes, "lookups_per_lane": per_lane}


def replay_ceiling(field, w, P, sample: int = 16384, lanes: int = 131072, reps: int = 3) -> dict:
    """Achievable lookup rate on the cell sequences of real trajectories: a
    sample of the workload's particles (spread evenly over its list) is
    propagated on this field with a tape at every accepted step; the recorded
    steps (state and size), particle after particle, are dealt out to `lanes`
    lanes in equal runs, and the replay microbenchmark looks the field up at
    the six stage points of every step with the propagation kernel's lookup
    and per-lane cell cache, all lookups independent.  Best of `reps`."""
    import numpy as np
    import torch

    from paper_1410_5323_amd import crp
    n = len(P["energy"])
    sel = np.linspace(0, n - 1, min(sample, n)).astype(np.int64)
    m = len(sel)
    prm = crp.make_params(w.tol, w.h_min, w.h_max, obs_radius=w.obs_radius, l_max=w.max_length)

    def fresh():
        return crp.particles_to_device(P["pos"][sel], P["dir"][sel], P["energy"][sel], P["charge"][sel])

    st = fresh()
    crp.crp_propagate([field], [prm], st)
    torch.cuda.synchronize()
    total = int(st["n_accepted"].sum().item())
    tape = crp.Tape(m, every_k=1, capacity=total + 2 * m + 1024)
    st = fresh()
    crp.crp_propagate([field], [prm], st, tape=tape)
    torch.cuda.synchronize()
    if tape.overflowed():
        raise RuntimeError("replay ceiling: tape pool too small")
    used = tape.records_needed()
    ck = tape.checkpoints[:8 * used].view(used, 8).cpu().numpy()
    links = tape.links[:used].cpu().numpy()
    fin = tape.finals.view(m, 4).cpu().numpy()
    final_len = st["length"].cpu().numpy()
    del tape
    # per-particle record order: walk each particle's links back from its last record
    owner = np.full(used, -1, np.int64)
    cur = fin[:, 2].astype(np.int64)
    pid = np.arange(m)
    while True:
        live = cur >= 0
        if not live.any():
            break
        owner[cur[live]] = pid[live]
        cur[live] = links[cur[live]]
    keep = owner >= 0
    idx = np.nonzero(keep)[0]
    order = idx[np.lexsort((idx, owner[idx]))]
    own = owner[order]
    L = ck[order, 6]
    # step size: next record's length minus this one's; a particle's last
    # record steps to its final length
    nxt_same = np.concatenate([own[1:] == own[:-1], [False]])
    h = np.where(nxt_same, np.concatenate([L[1:], [0.0]]) - L, final_len[own] - L)
    good = h > 0.0
    rec = np.concatenate([ck[order][:, :6], h[:, None]], axis=1)[good]
    per_lane = len(rec) // lanes
    if per_lane < 1:
        raise RuntimeError("replay ceiling: too few recorded steps for the lanes")
    rec = rec[:per_lane * lanes].reshape(lanes, per_lane, 7).transpose(1, 2, 0).copy()  # [step][7][lane]
    dev_rec = torch.from_numpy(rec).cuda()
    del rec
    sink = torch.empty(lanes, dtype=torch.float64, device="cuda")
    misses = torch.empty(lanes, dtype=torch.int64, device="cuda")
    stream = torch.cuda.current_stream()
    out = {"sampled_particles": int(m), "recorded_steps": int(good.sum()), "lanes": lanes,
           "steps_per_lane": int(per_lane), "lookups_per_lane": 6 * int(per_lane)}
    for cache in (True, False):
        crp.crp_bench_gather_replay(field, dev_rec, lanes, per_lane, cache, sink, misses)
        best = float("inf")
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            crp.crp_bench_gather_replay(field, dev_rec, lanes, per_lane, cache, sink, misses)
            b.record(stream)
            torch.cuda.synchronize()
            best = min(best, a.elapsed_time(b) / 1e3)
        look = 6.0 * per_lane * lanes
        key = "with_cell_cache" if cache else "without_cell_cache"
        out[key] = {"lookups_per_s": look / best, "ms": best * 1e3,
                    "cache_hit_rate": 1.0 - float(misses.sum().item()) / look}
    del dev_rec
    torch.cuda.empty_cache()
    return out


def rotate_directions(u, eps: float):
    """Rotate each unit vector by eps radians about an axis normal to it (a fixed
    recipe, so the perturbed inputs are reproducible)."""
    import numpy as np
    ax = np.cross(u, np.array([0.3, 0.5, 0.81]))
    ax /= np.linalg.norm(ax, axis=1)[:, None]
    return u * np.cos(eps) + np.cross(ax, u) * np.sin(eps)


def error_report(test: dict, ref: dict, probe: dict, rigidity, radius: float) -> dict:
    """Angular and time errors of `test` against the FP64 results `ref`, per
    rigidity decile, next to the FP64 path's own noise floor (`probe`: the FP64
    path with every initial direction rotated by 1e-7 rad)."""
    import numpy as np
    a = angle(test["dir"], ref["dir"])
    fl = angle(probe["dir"], ref["dir"])
    dl = np.abs(test["length"] - ref["length"]) / ref["length"]
    fdl = np.abs(probe["length"] - ref["length"]) / ref["length"]
    delay = np.maximum(ref["length"] - radius, 1e-300)
    dd = np.abs(test["length"] - ref["length"]) / delay
    edges = np.quantile(rigidity, np.linspace(0, 1, 11))
    dec = np.clip(np.searchsorted(edges, rigidity, side="right") - 1, 0, 9)
    rows = []
    for d in range(10):
        k = dec == d
        rows.append({"rigidity_V": [float(edges[d]), float(edges[d + 1])],
                     "angle_p50_rad": float(np.median(a[k])), "noise_floor_angle_p50_rad": float(np.median(fl[k])),
                     "angle_ratio_to_floor": float(np.median(a[k]) / max(np.median(fl[k]), 1e-300)),
                     "time_rel_p50": float(np.median(dl[k])), "noise_floor_time_rel_p50": float(np.median(fdl[k]))})
    return {"angle_rad": {"p50": float(np.median(a)), "p95": float(np.percentile(a, 95)),
                          "frac_below_1e-4": float(np.mean(a <= 1e-4))},
            "noise_floor_angle_rad": {"p50": float(np.median(fl)), "p95": float(np.percentile(fl, 95)),
                                      "frac_below_1e-4": float(np.mean(fl <= 1e-4))},
            "time_rel": {"p50": float(np.median(dl)), "p95": float(np.percentile(dl, 95))},
            "time_delay_rel": {"p50": float(np.median(dd)), "p95": float(np.percentile(dd, 95))},
            "per_rigidity_decile": rows, "particles": int(len(a))}


def classify_and_error(O, grid, prm, P, sub, test_dirs, probe_eps=1e-15, chaos_tol=1e-6, nthreads=0):
    """Lyapunov probe on the subset: the oracle at u0 and at u0 rotated by
    probe_eps; a particle is non-chaotic when its arrival direction moves by
    at most chaos_tol.  Returns (reference results, non-chaotic mask)."""
    import numpy as np
    s = slice(0, sub)
    ref = O.propagate(grid, prm, P["pos"][s], P["dir"][s], P["energy"][s], P["charge"][s], nthreads=nthreads)
    probe = O.propagate(grid, prm, P["pos"][s], rotate_directions(P["dir"][s], probe_eps), P["energy"][s],
                        P["charge"][s], nthreads=nthreads)
    return ref, angle(probe["dir"], ref["dir"]) <= chaos_tol


def angle_stats(a, mask):
    import numpy as np
    b = a[mask]
    if b.size == 0:
        return {"particles": 0}
    return {"particles": int(b.size), "p50": float(np.median(b)), "p95": float(np.percentile(b, 95)),
            "max": float(np.max(b)), "frac_below_1e-4": float(np.mean(b <= 1e-4))}


def precision_leg(tols=(1e-4, 1e-6, 1e-8), subset: int = 10000, bound: float = 1e-4) -> dict:
    """Mixed precision at the stated error on the precision workload (1024^3
    Kolmogorov grid at 10 kpc, 4e6 nuclei, sphere at 10 Mpc).

    For each tolerance, loosest first: the oracle on the FP32 grid runs the
    first `subset` particles, and again with every initial direction rotated
    by 1e-15 rad; a particle whose arrival direction moves by <= 1e-6 rad is
    non-chaotic.  The mixed kernel (FP16 grid, FP32 stages, FP64
    accumulation) runs the same subset; the 95th percentile of its
    arrival-direction error against the oracle over the non-chaotic particles
    decides.  At the loosest tolerance where that is <= 1e-4 rad, the FP64
    path and the mixed kernel (FP16 and BF16 grids, FP64 and double-float
    accumulation) each propagate all 4e6 particles, timed with HIP events,
    for the speed-up; the errors on the subset are taken from those runs,
    against the oracle on the FP32 grid (total) and on the dequantised 16-bit
    grid (arithmetic only)."""
    import numpy as np
    import torch

    import crp_inputs as ci
    from oracle import oracle as O
    from paper_1410_5323_amd import crp
    w = ci.get_config("precision_1024cube")
    t0 = time.perf_counter()
    grids, radii, P = build_inputs(w, None)
    B32 = grids[0]
    n = len(P["energy"])
    log(f"bench: precision leg inputs in {time.perf_counter() - t0:.1f} s ({w.grid_n}^3, n={n})")
    stream = torch.cuda.current_stream()
    pristine = crp.particles_to_device(P["pos"], P["dir"], P["energy"], P["charge"], mass=P["mass"])
    ws = torch.empty(crp.crp_workspace_bytes(n, 1, 1), dtype=torch.uint8, device="cuda")
    # CELL8 grids (FP32 137 GB, FP16/BF16 69 GB each): at tol 1e-8 the FP64 pass took 11.2 s against 12.1 s
    # with LINEAR storage and the FP16 mixed pass 8.8 s against 11.5 s.  They are made when first needed and
    # freed when done, so at most FP32 and one 16-bit grid are resident.
    fields = {}

    def field(dt):
        if dt not in fields:
            src = torch.from_numpy(B32).cuda()
            fields[dt] = crp.make_field(src, w.spacing, dtype=dt, layout=PRECISION_LAYOUT)
            del src
            torch.cuda.synchronize()
            torch.cuda.empty_cache()
        return fields[dt]

    def drop(dt):
        fields.pop(dt, None)
        torch.cuda.synchronize()
        torch.cuda.empty_cache()

    tun64 = crp.make_tuning(256, 2, 32, 1, 0)
    tunmx = crp.make_tuning(256, 4, 32, 1, 0)
    g32 = O.Grid(B32, w.spacing)
    sub = slice(0, subset)

    def run(dt, precision, tol, m=None):
        prm = crp.make_params(tol, w.h_min, w.h_max, obs_radius=w.obs_radius, l_max=w.max_length)
        st = crp.clone_particles(pristine) if m is None else {k: (v[:m].clone() if v is not None else None)
                                                               for k, v in pristine.items()}
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        crp.crp_propagate([field(dt)], [prm], st, precision=precision, tuning=tun64 if precision == 0 else tunmx,
                          workspace=ws)
        b.record(stream)
        torch.cuda.synchronize()
        host = crp.particles_to_host(st)
        del st
        return a.elapsed_time(b), host

    rows = []
    chosen = None
    for tol in tols:
        prm_o = O.params_array(tol, w.h_min, w.h_max, radius=w.obs_radius, l_max=w.max_length)
        t1 = time.perf_counter()
        ref, calm = classify_and_error(O, g32, prm_o, P, subset, None)
        t_or = time.perf_counter() - t1
        _, mx = run("f16", crp.CRP_PREC_MIXED_F64ACC, tol, m=subset)
        a = angle(mx["dir"], ref["dir"])
        row = {"tol": tol, "non_chaotic_fraction": float(np.mean(calm)),
               "angle_vs_oracle_non_chaotic": angle_stats(a, calm),
               "angle_vs_oracle_all": angle_stats(a, np.ones_like(calm)), "oracle_s": t_or}
        log(f"bench: precision leg tol {tol}: {row}")
        rows.append(row)
        if row["angle_vs_oracle_non_chaotic"].get("p95", np.inf) <= bound:
            chosen = (tol, ref, calm, prm_o)
            break
    out = {"workload": w.name, "particles": n, "grid": f"{w.grid_n}^3", "layout": PRECISION_LAYOUT,
           "error_subset": subset,
           "non_chaotic": "oracle arrival direction moves by <= 1e-6 rad when u0 is rotated by 1e-15 rad",
           "bound_rad": bound, "sweep": rows}
    if chosen is None:
        out["result"] = f"no tolerance in {list(tols)} meets p95 <= {bound} rad on the non-chaotic particles"
        return out
    tol, ref, calm, prm_o = chosen
    ms64, h64 = run("f32", 0, tol)
    drop("f32")
    log(f"bench: precision leg fp64 pass {ms64:.1f} ms at tol {tol}")
    runs = {}
    for name, dt, pr in (("f16", "f16", crp.CRP_PREC_MIXED_F64ACC), ("f16_dfacc", "f16", crp.CRP_PREC_MIXED_DFACC),
                         ("bf16", "bf16", crp.CRP_PREC_MIXED_F64ACC)):
        if dt == "bf16":
            drop("f16")
        runs[name] = run(dt, pr, tol)
        log(f"bench: precision leg mixed {name} pass {runs[name][0]:.1f} ms")
    drop("bf16")
    a64 = angle(h64["dir"][sub], ref["dir"])
    res = {"tol": tol, "non_chaotic_fraction": float(np.mean(calm)), "non_chaotic_particles": int(np.sum(calm)),
           "fp64_ms": ms64, "fp64_accepted_steps": int(np.sum(h64["n_accepted"])),
           "fp64_path_vs_oracle_bitwise": float(np.mean(np.all(h64["dir"][sub] == ref["dir"], axis=1))),
           "fp64_path_angle_max": float(np.max(a64))}
    for name, (ms, hx) in runs.items():
        a = angle(hx["dir"][sub], ref["dir"])
        dl = np.abs(hx["length"][sub] - ref["length"]) / ref["length"]
        delay = np.maximum(ref["length"] - w.obs_radius, 1e-300)
        dd = np.abs(hx["length"][sub] - ref["length"]) / delay
        res[name] = {"ms": ms, "speedup_vs_fp64": ms64 / ms,
                     "total_error": {"angle_non_chaotic": angle_stats(a, calm),
                                     "angle_all": angle_stats(a, np.ones_like(calm)),
                                     "length_rel_p95_non_chaotic": float(np.percentile(dl[calm], 95)),
                                     "time_delay_rel_p95_non_chaotic": float(np.percentile(dd[calm], 95))}}
    # arithmetic-only error: the oracle on the values the device stores
    for name, rnd in (("f16", ci.round_to_f16), ("bf16", ci.round_to_bf16)):
        gq = O.Grid(rnd(B32), w.spacing)
        rq = O.propagate(gq, prm_o, P["pos"][sub], P["dir"][sub], P["energy"][sub], P["charge"][sub])
        del gq
        a = angle(runs[name][1]["dir"][sub], rq["dir"])
        res[name]["arithmetic_error"] = {"angle_non_chaotic": angle_stats(a, calm)}
    out["result"] = res
    log(f"bench: precision leg result {res}")
    return out


def adjoint_leg(reps: int = 2):
    """Adjoint/forward cost on the differentiation workload (1e5 protons and
    iron, 128^3 FP32 grid, sphere at 10 Mpc, checkpoints every 64 steps): the
    plain forward, the taped forward and the adjoint (grid-gradient zeroing
    included), each timed with HIP events on the launch stream."""
    import numpy as np
    import torch

    import crp_inputs as ci
    from paper_1410_5323_amd import crp
    w = ci.get_config("adjoint_128cube")
    grids, radii, P = build_inputs(w, None)
    n = len(P["energy"])
    layout = "cell8"
    f = crp.make_field(grids[0], w.spacing, dtype="f32", layout=layout)
    prm = crp.make_params(w.tol, w.h_min, w.h_max, obs_radius=w.obs_radius, l_max=w.max_length)
    init = crp.particles_to_device(P["pos"], P["dir"], P["energy"], P["charge"])
    ws = torch.empty(crp.crp_workspace_bytes(n, 1, 1), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()

    def ev_time(fn):
        out = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            fn()
            b.record(stream)
            torch.cuda.synchronize()
            out.append(a.elapsed_time(b))
        return float(np.mean(out))

    st = crp.clone_particles(init)
    crp.crp_propagate([f], [prm], st, workspace=ws)  # warm-up
    torch.cuda.synchronize()
    tape = crp.Tape(n, every_k=w.checkpoint_every)  # default pool: 64 records per particle
    steps = int(st["n_accepted"].sum())

    # state copies happen outside the timed region: time only the launches
    def timed_fwd(tp):
        times = []
        for _ in range(reps):
            s = crp.clone_particles(init)
            if tp is not None:
                tp.reset()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            crp.crp_propagate([f], [prm], s, workspace=ws, tape=tp)
            b.record(stream)
            torch.cuda.synchronize()
            times.append(a.elapsed_time(b))
        return float(np.mean(times))

    t_fwd = timed_fwd(None)
    t_tape = timed_fwd(tape)
    if tape.overflowed():
        raise RuntimeError(f"adjoint leg: tape pool too small ({tape.records_needed()} records needed)")
    rng = np.random.default_rng(5)
    gd = torch.from_numpy(rng.standard_normal((n, 3))).cuda()
    gt = torch.from_numpy(rng.standard_normal(n) * 1e-14).cuda()
    gu = torch.empty(n, 3, dtype=torch.float64, device="cuda")
    gg = torch.zeros(grids[0].shape, dtype=torch.float64, device="cuda")
    # parallel replay of the particles with at least half the most steps
    replay = tape.replay_steps(0.5)
    aws = crp.adjoint_workspace(n, tape, replay_steps=replay)
    aws0 = crp.adjoint_workspace(n, tape, replay_steps=0)

    def adj(ws):
        gg.zero_()
        crp.crp_propagate_adjoint(f, prm, init, tape, gd, gt, gu, gg, workspace=ws)

    t_adj = ev_time(lambda: adj(aws))
    gu_par = gu.clone()
    t_adj0 = ev_time(lambda: adj(aws0))
    same = bool(torch.equal(gu_par.view(torch.int64), gu.view(torch.int64)))
    fin = torch.isfinite(gu).all(dim=1)
    return {"workload": w.name, "particles": n, "layout": layout, "accepted_steps": steps,
            "forward_ms": t_fwd, "taped_forward_ms": t_tape, "adjoint_ms": t_adj,
            "adjoint_over_forward": t_adj / t_fwd,
            "gradient_over_forward": (t_tape + t_adj) / t_fwd,
            "parallel_replay_steps": replay, "parallel_replay_bytes": aws.numel() - aws0.numel(),
            "adjoint_ms_without_parallel_replay": t_adj0,
            "parallel_replay_same_bits": same,
            "tape_records_used": tape.records_needed(), "tape_bytes_used": tape.records_needed() * 72 + n * 32,
            "finite_gradient_fraction": float(fin.float().mean()),
            "note": "gradient = taped forward + adjoint (the autograd path); the adjoint replays the checkpoint "
                    "segments of the particles with at least half the most steps in parallel before its sweep"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="production_256cube")
    ap.add_argument("--n", type=int, default=None, help="particle count (default: the workload's)")
    ap.add_argument("--layout", default=None, choices=["linear", "cell8"],
                    help="default: cell8 up to 512^3, linear above")
    ap.add_argument("--precision", default="fp64", choices=list(PRECISIONS))
    ap.add_argument("--grid-dtype", default=None, choices=["f64", "f32", "f16", "bf16"])
    ap.add_argument("--mixed-grid-dtype", default="f16", choices=["f32", "f16", "bf16"])
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision comparison")
    ap.add_argument("--block-size", type=int, default=256)
    ap.add_argument("--blocks-per-cu", type=int, default=None,
                    help="persistent blocks per CU (default 2 for the FP64 kernel, whose occupancy is 2 waves/SIMD; "
                         "4 for the mixed kernel)")
    ap.add_argument("--refill-threshold", type=int, default=32)
    ap.add_argument("--cache-cells", type=int, default=0, help="1 on, -1 off, 0 automatic")
    ap.add_argument("--no-order", action="store_true")
    ap.add_argument("--autotune", type=int, default=None, help="1: tune the launch (default on for batches)")
    ap.add_argument("--graph", type=int, default=None, help="1: replay a captured hipGraph (default on for batches)")
    ap.add_argument("--tol", type=float, default=None,
                    help="integrator tolerance in place of the workload's (e.g. to see where the mixed kernel's "
                         "direction error falls below 1e-4 rad)")
    ap.add_argument("--cpu-sample", type=int, default=200000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint/forward cost leg")
    ap.add_argument("--precision-leg", action="store_true",
                    help="only the mixed-precision leg on the 1024^3 precision workload")
    ap.add_argument("--no-replay-ceiling", action="store_true",
                    help="skip the lookup ceiling measured on replayed trajectories")
    ap.add_argument("--no-precision-leg", action="store_true",
                    help="skip the mixed-precision leg (1024^3, run by default with the production workload)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy 1 GiB twice with the streaming kernel (known bytes, to scale HBM counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}): particles are independent, so the "
              "path shards by particles, but no multi-GPU run is measured here.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import crp_inputs as ci
    from paper_1410_5323_amd import crp

    if not torch.cuda.is_available():
        print("bench.py: no GPU available", file=sys.stderr)
        sys.exit(1)
    crp.lib()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_calibration:
        nb = 1 << 30
        src = torch.ones(nb // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(2):
            crp.crp_bench_stream(src, dst, nb, None, 4096)
        torch.cuda.synchronize()
        assert torch.equal(src, dst)
        print(json.dumps({"copy_calibration": {"bytes_read_per_launch": nb, "bytes_written_per_launch": nb,
                                               "launches": 2, "kernel": "k_stream_copy"}}), flush=True)
        return

    if args.precision_leg:
        print(json.dumps({"precision_leg": precision_leg()}), flush=True)
        return

    w = ci.get_config(args.workload)
    if args.tol is not None:
        if not args.tol > 0.0:
            print("bench.py: --tol must be positive", file=sys.stderr)
            sys.exit(2)
        w = dataclasses.replace(w, tol=args.tol)
    batched = w.n_realisations > 0
    use_graph = bool(args.graph if args.graph is not None else batched)
    use_tuner = bool(args.autotune if args.autotune is not None else batched)
    t0 = time.perf_counter()
    grids, radii, P = build_inputs(w, args.n)
    n = len(P["energy"])
    log(f"bench: inputs generated in {time.perf_counter() - t0:.1f} s ({w.name}, n={n}, {len(grids)} field(s))")

    prec = PRECISIONS[args.precision]
    gdt_name = args.grid_dtype or ("f16" if prec != 0 else ("f64" if w.grid_dtype == "f64" else "f32"))
    # CELL8 wherever its grids fit in 60% of the device memory (one 128 B record per cell in FP32): with the
    # register cell cache it is faster at every size measured, 1024^3 included (1.60 s against 2.21 s LINEAR
    # for the FP64 path, 1.03 s against 2.01 s for the mixed kernel)
    cell8_bytes = len(grids) * w.grid_n ** 3 * 32 * BYTES_PER_VALUE[args.grid_dtype or w.grid_dtype]
    layout = args.layout or ("cell8" if cell8_bytes <= 0.6 * torch.cuda.get_device_properties(0).total_memory
                             else "linear")
    params = [crp.make_params(w.tol, w.h_min, w.h_max, obs_radius=radii[r], l_max=w.max_length, field_index=r,
                              box=w.reflect_box, backtrack=w.lens_nside > 0) for r in range(len(grids))]
    pristine = crp.particles_to_device(P["pos"], P["dir"], P["energy"], P["charge"], mass=P["mass"],
                                       param_index=P.get("param_index"))
    state = crp.clone_particles(pristine)
    ws = torch.empty(crp.crp_workspace_bytes(n, len(grids), len(params)), dtype=torch.uint8, device=dev)
    counters = torch.zeros(crp.NCOUNTERS, dtype=torch.int64, device=dev)
    bpc = args.blocks_per_cu if args.blocks_per_cu is not None else (2 if prec == 0 else 4)
    tuning = crp.make_tuning(args.block_size, bpc, args.refill_threshold, 0 if args.no_order else 1,
                             args.cache_cells)
    mixed_tuning = crp.make_tuning(args.block_size, args.blocks_per_cu if args.blocks_per_cu is not None else 4,
                                   args.refill_threshold, 0 if args.no_order else 1, args.cache_cells)

    def timed(fields, precision, tun, steps, warmup, label):
        """Warm-up passes, then `steps` timed passes of the whole hot path."""
        graph = crp.Graph(fields, params, state, precision=precision, tuning=tun, counters=counters,
                          workspace=ws) if use_graph else None
        stream = torch.cuda.current_stream()

        def step(ev=None):
            for k, v in pristine.items():
                if v is not None:
                    state[k].copy_(v, non_blocking=True)
            if ev is not None:
                ev[0].record(stream)
            if graph is not None:
                graph.launch()
            else:
                crp.crp_propagate(fields, params, state, precision=precision, tuning=tun, counters=counters,
                                  workspace=ws)
            if ev is not None:
                ev[1].record(stream)

        for i in range(warmup):
            step()
            torch.cuda.synchronize()
            log(f"bench: {label} warmup {i + 1}/{warmup} done")
        counters.zero_()
        events = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                  for _ in range(steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            step(events[i])
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        launch_ms = [a.elapsed_time(b) for a, b in events]
        log(f"bench: {label}: {steps} timed steps in {elapsed:.3f} s; launch ms {['%.1f' % x for x in launch_ms]}")
        if graph is not None:
            graph.close()
        return {"elapsed": elapsed, "launch_ms": launch_ms, "counters": counters.cpu().numpy().astype(np.int64),
                "host": crp.particles_to_host(state)}

    mod_np = build_modulation(w)
    mod = None if mod_np is None else crp.make_modulation(mod_np, w.mod_spacing, origin=(w.mod_origin,) * 3)
    fields = [crp.make_field(g, w.spacing, dtype=gdt_name, layout=layout, modulation=mod) for g in grids]
    tuned = None
    if use_tuner:
        from paper_1410_5323_amd.autotune import autotune
        tuning = autotune(fields, params, pristine, precision=prec, log=log)
        tuned = {k: getattr(tuning, k) for k in ("block_size", "blocks_per_cu", "refill_threshold",
                                                 "order_by_rigidity", "cache_cells")}
        log(f"bench: autotuned launch {tuned}")
    head = timed(fields, prec, tuning, args.steps, args.warmup, f"{args.precision}/{gdt_name}/{layout}")
    c = head["counters"]
    elapsed = head["elapsed"]
    accepted = int(c[1])
    evals = int(c[0])
    avg_launch_s = float(np.mean(head["launch_ms"])) / 1e3
    bytes_per_eval = 6 * 8 * 3 * BYTES_PER_VALUE[gdt_name]
    if mod is not None:
        bytes_per_eval += 6 * 8 * 4  # the modulation grid's 8 FP32 corners per lookup
    evals_per_launch = evals / args.steps
    steps_per_launch = accepted / args.steps
    # lookup bytes: the survey's unit is one accepted step (6 lookups); every
    # rejected attempt and event iteration adds as much again
    gather_step_GBps = bytes_per_eval * steps_per_launch / avg_launch_s / 1e9
    gather_eval_GBps = bytes_per_eval * evals_per_launch / avg_launch_s / 1e9
    tflops = FLOPS_PER_EVALUATION * evals_per_launch / avg_launch_s / 1e12
    vpeak = FP64_VECTOR_PEAK_TFLOPS if prec == 0 else FP32_VECTOR_PEAK_TFLOPS
    traffic = measured_traffic(w.name, layout) if prec == 0 else None
    host = head["host"]
    gc = gather_ceiling(fields[0])
    lookup_bytes = bytes_per_eval / 6
    gc["algorithmic_GB_per_s"] = gc["lookups_per_s"] * lookup_bytes / 1e9
    gc["kernel_lookups_per_s"] = 6 * evals_per_launch / avg_launch_s
    gc["kernel_fraction"] = gc["kernel_lookups_per_s"] / gc["lookups_per_s"]
    gc = {"uniform_random": gc}
    if not batched and not args.no_replay_ceiling and fields[0].desc.dtype in (crp.CRP_F64, crp.CRP_F32):
        rc = replay_ceiling(fields[0], w, P)
        best = rc["with_cell_cache"]["lookups_per_s"]
        rc["algorithmic_GB_per_s"] = best * lookup_bytes / 1e9
        rc["kernel_fraction"] = gc["uniform_random"]["kernel_lookups_per_s"] / best
        gc["replayed_trajectories"] = rc
    log(f"bench: gather ceiling {gc}")
    statuses = {k: int(np.sum(host["status"] == v)) for k, v in crp.STATUS.items() if np.any(host["status"] == v)}
    del fields
    torch.cuda.empty_cache()

    result = {
        "metric": METRIC,
        "value": accepted / elapsed,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == 0 else "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "particles": n, "fields": len(grids), "grid": f"{w.grid_n}^3 {gdt_name}",
                   "grid_spacing_mpc": w.spacing, "layout": layout, "tol": w.tol,
                   "h_min_mpc": w.h_min, "h_max_mpc": w.h_max,
                   "obs_radius_mpc": [min(radii), max(radii)] if batched else w.obs_radius,
                   "modulation": None if mod is None else f"{w.mod_n}^3 f32, {w.mod_spacing} Mpc, log-normal "
                                                          f"sigma {w.mod_sigma}, correlation {w.mod_l_corr} Mpc",
                   "reflective_box_mpc": w.reflect_box, "l_max_mpc": w.max_length, "precision": args.precision,
                   "hipgraph": use_graph,
                   "tuning": tuned or {"block_size": args.block_size, "blocks_per_cu": bpc,
                                       "refill_threshold": args.refill_threshold,
                                       "order_by_rigidity": not args.no_order, "cache_cells": args.cache_cells}},
        # The pass is set by its longest trajectories' chains of dependent FP64
        # evaluations (arithmetic and lookup latency), not by a bandwidth: the
        # measured HBM traffic is a fifth of the peak.  The roofline reported is
        # the arithmetic one; the lookup bandwidth is in detail.gather.
        "roofline": {"bound": "alu", "achieved": tflops, "peak": vpeak, "unit": "TFLOP/s",
                     "frac": tflops / vpeak, "traffic": traffic},
        "detail": {"accepted_steps_per_launch": accepted / args.steps,
                   "evaluations_per_launch": evals_per_launch,
                   "rejected_per_launch": int(c[2]) / args.steps,
                   "event_evaluations_per_launch": int(c[3]) / args.steps,
                   "floor_hits_per_launch": int(c[4]) / args.steps,
                   "cell_loads_per_launch": int(c[6]) / args.steps,
                   "cell_cache_hit_rate": 1.0 - int(c[6]) / max(1, 6 * evals),
                   "wave_iterations_per_launch": int(c[7]) / args.steps,
                   "lane_utilisation": evals / max(1, 64 * int(c[7])),
                   # the longest trajectory's attempts bound the pass from below: at one
                   # attempt per loop iteration its lane needs that many iterations in a row
                   "max_attempts_one_particle": int(np.max(host["n_accepted"] + host["n_rejected"]))
                   if n else 0,
                   "launch_us_per_attempt_of_longest": avg_launch_s * 1e6
                   / max(1, int(np.max(host["n_accepted"] + host["n_rejected"])) if n else 1),
                   "evaluations_per_s": evals / elapsed,
                   "avg_launch_ms": avg_launch_s * 1e3,
                   "algorithmic_bytes_per_evaluation": bytes_per_eval,
                   "flops_per_evaluation": FLOPS_PER_EVALUATION,
                   "gather": {"algorithmic_bytes_per_accepted_step": bytes_per_eval,
                              "GB_per_s_accepted_steps": gather_step_GBps,
                              "frac_of_hbm_peak_accepted_steps": gather_step_GBps / HBM_PEAK_GBPS,
                              "GB_per_s_all_evaluations": gather_eval_GBps,
                              "measured_hbm_GB_per_s": None if traffic is None else traffic / avg_launch_s / 1e9,
                              "measured_frac_of_hbm_peak": None if traffic is None
                              else traffic / avg_launch_s / 1e9 / HBM_PEAK_GBPS},
                   "limiter": "the longest trajectory: max_attempts_one_particle dependent evaluations at "
                              "launch_us_per_attempt_of_longest each",
                   "statuses": statuses,
                   "gather_ceiling": gc,
                   "kernel_source_sha": kernel_source_hash()},
    }

    mixed_host = None
    if prec == 0 and not args.no_mixed and not batched and not w.lens_nside:
        mdt = args.mixed_grid_dtype
        mfields = [crp.make_field(g, w.spacing, dtype=mdt, layout=layout, modulation=mod) for g in grids]
        mix = timed(mfields, PRECISIONS["mixed_f64acc"], mixed_tuning, args.steps, 1, f"mixed_f64acc/{mdt}/{layout}")
        del mfields
        torch.cuda.empty_cache()
        mixed_host = mix["host"]
        mavg = float(np.mean(mix["launch_ms"]))
        result["mixed_production"] = {"precision": "mixed_f64acc", "grid": f"{w.grid_n}^3 {mdt}", "layout": layout,
                           "avg_launch_ms": mavg, "speedup_vs_fp64": avg_launch_s * 1e3 / mavg,
                           "accepted_steps_per_s": int(mix["counters"][1]) / mix["elapsed"]}
        # noise floor of the FP64 path on the error sample: the same run with each
        # initial direction rotated by 1e-7 rad
        m = min(args.cpu_sample, n)
        pf = [crp.make_field(g, w.spacing, dtype=gdt_name, layout=layout, modulation=mod) for g in grids]
        probe = crp.particles_to_device(P["pos"][:m], rotate_directions(P["dir"][:m], 1e-7), P["energy"][:m],
                                        P["charge"][:m])
        crp.crp_propagate(pf, params[:1], probe, tuning=tuning)
        torch.cuda.synchronize()
        probe_host = crp.particles_to_host(probe)
        del pf, probe
        torch.cuda.empty_cache()
        rig = P["energy"][:m] / P["charge"][:m]
        ref64 = {k: v[:m] for k, v in host.items()}
        result["mixed_production"]["error_vs_fp64"] = error_report({k: v[:m] for k, v in mixed_host.items()}, ref64,
                                                        probe_host, rig, radii[0])
        result["mixed_production"]["error_vs_fp64"]["reference"] = ("FP64 path on the FP32 grid (bitwise equal to the oracle "
                                                         "on this sample)")

    if w.lens_nside:
        result["lens"] = lens_leg(crp, torch, w, P, state)
        log(f"bench: lens leg {result['lens']}")

    if not args.no_adjoint:
        del state, pristine, ws
        torch.cuda.empty_cache()
        log("bench: adjoint/forward leg (adjoint_128cube)")
        result["adjoint"] = adjoint_leg()
        log(f"bench: adjoint leg {result['adjoint']}")
        torch.cuda.empty_cache()

    if not args.no_precision_leg and w.name == "production_256cube" and prec == 0:
        log("bench: mixed-precision leg (precision_1024cube)")
        torch.cuda.empty_cache()
        result["mixed"] = precision_leg()
        torch.cuda.empty_cache()

    if not args.no_cpu_baseline:
        m = min(args.cpu_sample, n)
        log(f"bench: timing the CPU oracle on the first {m} particles")
        cb, ref = cpu_baseline(grids, radii, w, P, m, modulation=mod_np)
        result["cpu_baseline"] = cb
        if prec == 0:
            g = {k: v[:m] for k, v in host.items()}
            bit = (np.all(g["pos"] == ref["pos"], axis=1) & np.all(g["dir"] == ref["dir"], axis=1)
                   & (g["length"] == ref["length"]) & (g["status"] == ref["status"]))
            result["detail"]["parity_sample"] = {"particles": m, "bitwise_fraction": float(np.mean(bit)),
                                                 "max_angle_rad": float(np.max(angle(g["dir"], ref["dir"])))}
        if w.lens_nside:
            result["lens"]["cpu_baseline"] = lens_cpu_baseline(w, P, ref, m)
        if mixed_host is not None:
            a = angle(mixed_host["dir"][:m], ref["dir"])
            result["mixed_production"]["angle_vs_oracle_rad"] = {"p50": float(np.percentile(a, 50)),
                                                      "p95": float(np.percentile(a, 95)),
                                                      "frac_below_1e-4": float(np.mean(a <= 1e-4)),
                                                      "sample": m, "reference": "oracle on the FP32 grid"}
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
