"""Pins for the oracle's ionization-time sampling (Sec. 2.1 'Ionization':
charge states ionized one after another, outer shell first; t0 the birth
time).  Reading: inverse-survival sampling, P(t_k > t) = exp(-int w_k dt),
with the integral accumulated from the previous birth.

Independent checks: the closed form in a static uniform field, a brute-force
crossing computed with a different quadrature and a bracketing root finder, a
Kolmogorov-Smirnov test of the survival law, translation invariance of the
arrival window for a plane wave, and panel refinement.
"""
import numpy as np
import pytest
from scipy import optimize, stats

C = 299792458.0


def test_uniform_field_closed_form(orc):
    E0 = 1.2e11
    L = orc.laser_intensity(0.8e-6, 3e-6, 30e-15, 1e21, field=orc.UNIFORM_EB,
                            test_E=(E0, 0, 0), test_B=(0, 0, 0), window=orc.WIN_LAB)
    n = 64
    x, y, z = np.zeros(n), np.zeros(n), np.zeros(n)
    tb = orc.ionize(L, 3, 1, 100, x, y, z, 1, 3).reshape(n, 3)
    ts = -L.t_before
    for i in range(n):
        t = ts
        for s, k in enumerate((1, 2, 3)):
            Ek = -np.log(orc.uniform(3, 1, [100 + i], k + 2)[0])
            w = orc.adk_rate(k, E0)
            t = t + Ek / w
            if t > L.t_after:
                assert np.all(np.isinf(tb[i, s:])) and np.all(tb[i, s:] > 0)
                break
            # tolerance: rounding of a plain sum over up to ~1e5 panels
            assert abs(tb[i, s] - t) <= 1e-11 * max(abs(t), L.lambda_ / C), (i, s)


def _brute_force_times(orc, L, x, y, z, thresholds, k_first, sub=50, ng=20):
    """Sequential crossing times with GL-20 on sub-panels of T/sub and brentq."""
    T = L.lambda_ / C
    ts, te = z / C - L.t_before, z / C + L.t_after
    xg, wg = np.polynomial.legendre.leggauss(ng)

    def rate(k, t):
        t = np.atleast_1d(t)
        E, _ = orc.field(L, x + 0 * t, y + 0 * t, z + 0 * t, t)
        return orc.adk_rate_batch(k, np.linalg.norm(E, axis=1))

    def integral(k, a, b):
        h, m = 0.5 * (b - a), 0.5 * (a + b)
        return h * np.sum(wg * rate(k, m + h * xg))

    out = []
    t_prev = ts
    for s, Ek in enumerate(thresholds):
        k = k_first + s
        I, a = 0.0, t_prev
        found = None
        while a < te:
            b = min(a + T / sub, te)
            seg = integral(k, a, b)
            if I + seg >= Ek:
                I0, a0 = I, a
                found = optimize.brentq(lambda t: I0 + integral(k, a0, t) - Ek, a0, b,
                                        xtol=1e-30, rtol=1e-15)
                break
            I += seg
            a = b
        if found is None:
            out += [np.inf] * (len(thresholds) - s)
            break
        out.append(found)
        t_prev = found
    return np.array(out)


def test_brute_force_crossings(orc):
    L = orc.laser_intensity(0.8e-6, 3e-6, 30e-15, 1e21, field=orc.RP_O5)
    T = L.lambda_ / C
    pts = [(2.1e-6, 0.4e-6, 3e-6), (-0.5e-6, 1.0e-6, -20e-6)]
    for i, (x, y, z) in enumerate(pts):
        tb = orc.ionize(L, 0, 0, i, [x], [y], [z], 1, 4)
        thr = [-np.log(orc.uniform(0, 0, [i], k + 2)[0]) for k in range(1, 5)]
        ref = _brute_force_times(orc, L, x, y, z, thr, 1)
        assert np.all(np.isfinite(tb))
        assert np.max(np.abs(tb - ref)) < 1e-7 * T, (tb - ref) / T


def test_survival_law_ks(orc):
    """t_1 of many independent thresholds at one position follows
    P(t_1 <= t) = 1 - exp(-int_ts^t w_1 dt)."""
    L = orc.laser_intensity(0.8e-6, 3e-6, 30e-15, 4.5e15, field=orc.RP_O1,
                            window=orc.WIN_LAB, t_before=60e-15, t_after=60e-15)
    T = L.lambda_ / C
    x, y, z = 2.0e-6, 0.0, 0.0
    n = 2000
    tb = orc.ionize(L, 11, 0, 0, np.full(n, x), np.full(n, y), np.full(n, z), 1, 1)
    born = tb[np.isfinite(tb)]
    # cumulative integral on a fine grid (GL-20 per T/40 sub-panel)
    ts, te = -L.t_before, L.t_after
    xg, wg = np.polynomial.legendre.leggauss(20)
    edges = np.arange(ts, te + T / 40, T / 40)
    edges[-1] = te
    h = 0.5 * (edges[1:] - edges[:-1])
    m = 0.5 * (edges[1:] + edges[:-1])
    tt = (m[:, None] + h[:, None] * xg[None, :]).ravel()
    E, _ = orc.field(L, x + 0 * tt, y + 0 * tt, z + 0 * tt, tt)
    w = orc.adk_rate_batch(1, np.linalg.norm(E, axis=1)).reshape(-1, xg.size)
    cum = np.concatenate([[0.0], np.cumsum(h * (w @ wg))])
    p_born = 1 - np.exp(-cum[-1])
    assert 0.2 < p_born < 0.95
    # fraction born
    assert abs(born.size / n - p_born) < 4 * np.sqrt(p_born * (1 - p_born) / n)
    cdf = lambda t: (1 - np.exp(-np.interp(t, edges, cum))) / p_born
    assert stats.kstest(born, cdf).pvalue > 1e-3


def test_plane_wave_arrival_invariance(orc):
    """Fields depending on t - z/c only: with the arrival window the birth
    times shift exactly with z/c."""
    L = orc.laser_intensity(0.8e-6, 3e-6, 30e-15, 1e21, field=orc.PLANE_LP)
    T = L.lambda_ / C
    n = 8
    zs = np.linspace(-30e-6, 30e-6, n)
    tb = orc.ionize(L, 1, 0, 0, np.zeros(n), np.zeros(n), zs, 1, 6).reshape(n, 6)
    tb0 = orc.ionize(L, 1, 0, 0, np.zeros(n), np.zeros(n), np.zeros(n), 1, 6).reshape(n, 6)
    fin = np.isfinite(tb0)
    assert fin.sum() > 20
    assert np.array_equal(np.isfinite(tb), fin)
    d = (tb - zs[:, None] / C) - tb0
    assert np.max(np.abs(d[fin])) < 1e-9 * T


def test_panel_refinement(orc):
    L = orc.laser_intensity(0.8e-6, 3e-6, 30e-15, 1e21, field=orc.RP_O5)
    T = L.lambda_ / C
    x, y, z = orc.sample_atoms(0, 0, 0, 6, 2 * L.w0, orc.rayleigh(L))
    tb = orc.ionize(L, 0, 0, 0, x, y, z, 1, 10)
    L.dt = L.dt / 2
    tb2 = orc.ionize(L, 0, 0, 0, x, y, z, 1, 10)
    fin = np.isfinite(tb)
    assert np.array_equal(fin, np.isfinite(tb2))
    assert np.max(np.abs(tb[fin] - tb2[fin])) < 1e-8 * T


def test_weak_field_never_ionizes(orc):
    L = orc.laser_intensity(0.8e-6, 3e-6, 30e-15, 1e12, field=orc.RP_O5)
    tb = orc.ionize(L, 0, 0, 0, [1e-6], [0.0], [0.0], 1, 10)
    assert np.all(np.isposinf(tb))
    # on the axis only Ez acts
    L2 = orc.laser_intensity(0.8e-6, 3e-6, 30e-15, 1e21, field=orc.RP_O5, ez_scale=0.0)
    tb2 = orc.ionize(L2, 0, 0, 0, [0.0], [0.0], [0.0], 1, 10)
    assert np.all(np.isposinf(tb2))
