"""Checks of the seeded synthetic inputs (field realisations and particle lists).

The field must be divergence-free in spectral space, have exactly the
requested rms, a shell power spectrum with the Kolmogorov slope and a
coherence length close to the analytic one; particles must be isotropic
with log-uniform energies; everything must be reproducible from the seeds.
"""
import numpy as np
import pytest

import crp_inputs as ci


@pytest.fixture(scope="module")
def field64():
    return ci.kolmogorov_field(64, 1.0, 4.0, 32.0, 1.0, np.random.SeedSequence(7))


def test_rms_exact(field64):
    ms = np.mean(np.sum(field64 * field64, axis=-1))
    assert abs(np.sqrt(ms) - 1.0) < 1e-14


def test_spectrally_divergence_free(field64):
    n = field64.shape[0]
    Bk = [np.fft.rfftn(field64[..., c]) for c in range(3)]
    nx, ny, nz, _ = ci.spectral_mask(n, 1.0, 4.0, 32.0)
    div = nx * Bk[0] + ny * Bk[1] + nz * Bk[2]
    assert np.max(np.abs(div)) <= 1e-12 * np.max(np.abs(np.stack(Bk)))


def test_power_only_inside_band(field64):
    n = field64.shape[0]
    Bk = np.stack([np.fft.rfftn(field64[..., c]) for c in range(3)])
    _, _, _, mask = ci.spectral_mask(n, 1.0, 4.0, 32.0)
    p = np.sum(np.abs(Bk) ** 2, axis=0)
    assert np.max(p[~mask]) <= 1e-20 * np.max(p)


def test_kolmogorov_slope():
    n = 128
    B = ci.kolmogorov_field(n, 1.0, 2.5, 64.0, 1.0, np.random.SeedSequence(8))
    Bk = np.stack([np.fft.rfftn(B[..., c]) for c in range(3)])
    nx, ny, nz, mask = ci.spectral_mask(n, 1.0, 2.5, 64.0)
    k = np.sqrt(nx * nx + ny * ny + nz * nz + 0.0)
    p = np.sum(np.abs(Bk) ** 2, axis=0)
    # mean mode power per shell ~ k^(-11/3)
    edges = np.geomspace(4, 40, 12)
    km, pm = [], []
    for a, b in zip(edges[:-1], edges[1:]):
        sel = mask & (k >= a) & (k < b)
        km.append(np.mean(k[sel]))
        pm.append(np.mean(p[sel]))
    slope = np.polyfit(np.log(km), np.log(pm), 1)[0]
    assert abs(slope + 11.0 / 3.0) < 0.1, slope


def _expected_discrete_lc(n, h, lmin, lmax):
    i = np.fft.fftfreq(n, 1.0 / n)
    nx, ny, nz = np.meshgrid(i, i, i, indexing="ij")
    n2 = nx ** 2 + ny ** 2 + nz ** 2
    m = ((n2 >= (n * h / lmax) ** 2 * (1 - 1e-12)) & (n2 <= (n * h / lmin) ** 2 * (1 + 1e-12))
         & (np.abs(nx) != n // 2) & (np.abs(ny) != n // 2) & (np.abs(nz) != n // 2))
    w = np.where(m, np.maximum(n2, 1) ** (-11.0 / 6.0), 0.0)
    return n * h * w[0].sum() / w.sum()


def test_coherence_length_close_to_formula():
    """Twice the one-sided integral of the normalised correlation along the axes.

    The periodic line integral of <B(0).B(r e_a)>/<B^2> equals the box length
    times the fraction of power in the k_a = 0 plane.  Its expectation over
    realisations is fixed by the mode weights; that expectation is within 10 %
    of the continuum formula of Harari, Mollerach & Roulet for this band."""
    n, h, lmin, lmax = 128, 1.0, 4.0, 32.0
    vals = []
    for s in range(4):
        B = ci.kolmogorov_field(n, h, lmin, lmax, 1.0, np.random.SeedSequence(100 + s))
        Bk = np.stack([np.fft.fftn(B[..., c]) for c in range(3)])
        p = np.sum(np.abs(Bk) ** 2, axis=0)
        tot = p.sum()
        vals += [n * h * p[0, :, :].sum() / tot, n * h * p[:, 0, :].sum() / tot,
                 n * h * p[:, :, 0].sum() / tot]
    lc = np.mean(vals)
    expect = _expected_discrete_lc(n, h, lmin, lmax)
    assert abs(lc / expect - 1.0) < 0.08, (lc, expect)
    assert abs(expect / ci.coherence_length(lmin, lmax) - 1.0) < 0.1


def test_field_reproducible_and_seed_dependent():
    a = ci.kolmogorov_field(16, 0.1, 0.2, 1.6, 1.0, np.random.SeedSequence(1))
    b = ci.kolmogorov_field(16, 0.1, 0.2, 1.6, 1.0, np.random.SeedSequence(1))
    c = ci.kolmogorov_field(16, 0.1, 0.2, 1.6, 1.0, np.random.SeedSequence(2))
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    assert a.dtype == np.float64 and a.shape == (16, 16, 16, 3)
    f32 = ci.kolmogorov_field(16, 0.1, 0.2, 1.6, 1.0, np.random.SeedSequence(1), dtype=np.float32)
    assert np.array_equal(f32, a.astype(np.float32))


def test_particles_isotropic_and_log_uniform():
    p = ci.isotropic_particles(200000, 1e18, 1e20, (1, 2, 7, 26), np.random.SeedSequence(3))
    u = p["dir"]
    assert np.max(np.abs(np.linalg.norm(u, axis=1) - 1)) < 1e-15
    assert np.all(np.abs(u.mean(0)) < 0.01)
    le = np.log10(p["energy"])
    assert le.min() >= 18 and le.max() <= 20 and abs(le.mean() - 19) < 0.01
    assert set(np.unique(p["charge"])) == {1, 2, 7, 26}
    assert np.array_equal(p["mass"], np.where(p["charge"] == 1, 1, 2 * p["charge"]))
    assert np.all(p["pos"] == 0)


def test_config_seeds_are_stable():
    a = ci.config_seeds(1)[1].generate_state(4)
    b = ci.config_seeds(1)[1].generate_state(4)
    c = ci.config_seeds(2)[1].generate_state(4)
    assert np.array_equal(a, b) and not np.array_equal(a, c)


def test_batched_realisation_table():
    w = ci.get_config(2)
    _, ps, rs = ci.config_seeds(2)
    t = ci.realisation_table(w, rs)
    assert len(t["count"]) == 64
    assert np.all((t["b_rms"] >= 0.1) & (t["b_rms"] <= 10))
    assert np.all((t["count"] >= 100) & (t["count"] <= 100000))
    assert np.all((t["radius"] >= 1) & (t["radius"] <= 50))


def test_alternate_charges():
    w = ci.get_config(4)
    p = ci.isotropic_particles(10, w.e_min, w.e_max, w.charges, np.random.SeedSequence(0),
                               charge_rule=w.charge_rule)
    assert list(p["charge"]) == [1, 26] * 5
