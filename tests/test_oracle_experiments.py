"""Pins for the oracle's experiment-side functions: the laser phase at birth
(Sec. 2.2, Figs. 6, 13, 14, using the phase defined under Eq. (2)) and the
hollow-cylinder / annulus ion distribution (Sec. 2.2, Fig. 8).

Independent checks: the phase is tied to the field model -- the order-1 radial
field divided by its envelope is cos(phase), and with the carrier phase moved
by pi/2 it is sin(phase) -- plus the on-axis closed form; the annulus radii are
exact on a cylinder surface, area-uniform in between, and reduce to the
filled-cylinder sampler when r_in = 0.
"""
import numpy as np
import pytest

C = 299792458.0


def _field_phase_parts(orc, L, x, y, z, t):
    """Order-1 Er divided by its amplitude factor (r/w0) A exp(-rho^2/D - s^2)/D."""
    E, _ = orc.field(L, x, y, z, t)
    r = np.hypot(x, y)
    Er = (E[:, 0] * x + E[:, 1] * y) / r
    k = 2 * np.pi / L.lambda_
    zr = 0.5 * k * L.w0 ** 2
    D = 1 + (z / zr) ** 2
    tau0 = L.tau_fwhm / np.sqrt(2 * np.log(2))
    s = (t - z / C) / tau0
    amp = r / L.w0 * L.amp * np.exp(-(r / L.w0) ** 2 / D - s * s) / D
    return Er / amp


def test_birth_phase_matches_order1_field(orc):
    rng = np.random.default_rng(7)
    n = 400
    L = orc.laser_intensity(0.8e-6, 2.5e-6, 30e-15, 1e20, field=orc.RP_O1, phi0=0.3)
    x = rng.uniform(-4e-6, 4e-6, n)
    y = rng.uniform(-4e-6, 4e-6, n)
    z = rng.uniform(-60e-6, 60e-6, n)
    t = z / C + rng.uniform(-40e-15, 40e-15, n)
    ph = orc.birth_phase(L, t, x, y, z, 1)
    assert np.all((ph >= 0) & (ph < 2 * np.pi))
    cos_f = _field_phase_parts(orc, L, x, y, z, t)
    Ls = orc.laser_intensity(0.8e-6, 2.5e-6, 30e-15, 1e20, field=orc.RP_O1, phi0=0.3 + np.pi / 2)
    sin_f = _field_phase_parts(orc, Ls, x, y, z, t)
    # phases of ~1e3 rad: absolute agreement limited by rounding of k z and omega t
    assert np.max(np.abs(cos_f - np.cos(ph))) < 1e-9
    assert np.max(np.abs(sin_f - np.sin(ph))) < 1e-9


def test_birth_phase_on_axis_closed_form(orc):
    L = orc.laser_intensity(1.0e-6, 3e-6, 30e-15, 1e20, phi0=1.1)
    om = 2 * np.pi * C / L.lambda_
    t = np.array([0.0, 1e-15, -2.5e-15, 7e-15])
    ph = orc.birth_phase(L, t, np.zeros(4), np.zeros(4), np.zeros(4), 1)
    want = np.mod(-om * t - 1.1, 2 * np.pi)
    assert np.max(np.abs(ph - want)) < 1e-12


def test_birth_phase_slots_and_unborn(orc):
    L = orc.laser_intensity(0.8e-6, 2.5e-6, 30e-15, 1e20)
    x = np.array([1e-6, -2e-6])
    y = np.array([0.5e-6, 0.0])
    z = np.array([3e-6, -1e-6])
    tb = np.array([1e-15, np.inf, 2e-15, -3e-15, 4e-15, np.inf])
    ph = orc.birth_phase(L, tb, x, y, z, 3)
    assert np.isnan(ph[1]) and np.isnan(ph[5])
    one = orc.birth_phase(L, tb[3:5], x[1:], y[1:], z[1:], 2)
    assert np.array_equal(one, ph[3:5])


def test_annulus_surface_exact(orc):
    x, y, z = orc.sample_atoms_annulus(5, 2, 0, 2000, 2e-6, 2e-6, 10e-6)
    assert np.max(np.abs(np.hypot(x, y) / 2e-6 - 1)) < 4e-16
    assert np.all(np.abs(z) <= 10e-6)


def test_annulus_area_uniform(orc):
    n = 200000
    r_in, r_out = 1e-6, 4e-6
    x, y, z = orc.sample_atoms_annulus(9, 0, 0, n, r_in, r_out, 5e-6)
    r2 = x * x + y * y
    assert r2.min() >= r_in ** 2 * (1 - 1e-15) and r2.max() <= r_out ** 2 * (1 + 1e-15)
    # (r^2 - r_in^2)/(r_out^2 - r_in^2) is U(0,1): compare deciles (KS-style bound)
    u = np.sort((r2 - r_in ** 2) / (r_out ** 2 - r_in ** 2))
    ks = np.max(np.abs(u - (np.arange(n) + 0.5) / n))
    assert ks < 1.63 / np.sqrt(n)   # 1% level
    ang = np.arctan2(y, x)
    assert abs(np.mean(np.cos(ang))) < 5 / np.sqrt(n) and abs(np.mean(np.sin(ang))) < 5 / np.sqrt(n)
    assert abs(np.mean(z)) < 5 * 5e-6 / np.sqrt(3 * n)


def test_annulus_reduces_to_filled_cylinder(orc):
    a = orc.sample_atoms(3, 1, 100, 5000, 3e-6, 7e-6)
    b = orc.sample_atoms_annulus(3, 1, 100, 5000, 0.0, 3e-6, 7e-6)
    for u, v in zip(a, b):   # r_max sqrt(u) vs sqrt(u r_max^2): a rounding apart
        assert np.max(np.abs(u - v)) <= 4 * np.finfo(float).eps * 3e-6


def _brute_hist2d(a, b, uz, na, alo, ahi, nb, blo, bhi):
    """Pure-Python loop over explicit bin edges (small inputs only)."""
    ea = [alo + (ahi - alo) * i / na for i in range(na + 1)]
    eb = [blo + (bhi - blo) * i / nb for i in range(nb + 1)]
    counts = np.zeros((2, na, nb), dtype=np.uint64)
    out = nan = 0
    for ai, bi, ui in zip(a, b, uz):
        if np.isnan(ai) or np.isnan(bi) or np.isnan(ui):
            nan += 1
            continue
        ia = next((i for i in range(na) if ea[i] <= ai < ea[i + 1]), None)
        ib = next((i for i in range(nb) if eb[i] <= bi < eb[i + 1]), None)
        if ia is None or ib is None:
            out += 1
            continue
        counts[0 if ui > 0 else 1, ia, ib] += 1
    return counts, out, nan


def test_histogram2d_brute_force(orc):
    rng = np.random.default_rng(11)
    n = 3000
    a = rng.uniform(-0.5, 2 * np.pi + 0.5, n)
    b = rng.uniform(-1e-7, 4.2e-6, n)
    uz = rng.normal(size=n)
    uz[::97] = 0.0          # exactly zero counts as backward
    a[5::131] = np.nan
    uz[7::173] = np.nan
    # keep values away from bin edges, where the two bin rules may round apart
    wa, wb = 2 * np.pi / 24, 4e-6 / 16
    for v, lo, w in ((a, 0.0, wa), (b, 0.0, wb)):
        f = (v - lo) / w
        near = np.abs(f - np.round(f)) < 1e-9
        v[near] += 0.25 * w
    counts, tallies = orc.histogram2d(a, b, uz, 24, 0.0, 2 * np.pi, 16, 0.0, 4e-6)
    bc, out, nan = _brute_hist2d(a, b, uz, 24, 0.0, 2 * np.pi, 16, 0.0, 4e-6)
    assert np.array_equal(counts, bc)
    assert tallies[0] == out and tallies[1] == nan
    assert counts.sum() + out + nan == n
    assert counts[1].sum() >= np.count_nonzero(uz == 0.0)


def test_histogram2d_matches_numpy(orc):
    rng = np.random.default_rng(12)
    a = rng.uniform(0, 1, 5000)
    b = rng.uniform(0, 1, 5000)
    uz = np.ones(5000)
    c1, t1 = orc.histogram2d(a, b, uz, 8, 0.0, 1.0, 5, 0.0, 1.0)
    ref, _, _ = np.histogram2d(a, b, bins=(8, 5), range=((0, 1), (0, 1)))
    assert np.array_equal(c1[0], ref.astype(np.uint64)) and c1[1].sum() == 0
    c2, t2 = orc.histogram2d(-uz, b, -uz, 1, -2.0, 0.0, 1, 0.0, 1.0)
    assert c2[1, 0, 0] == 5000 and t2.sum() == 0
