"""Pins for the oracle's linearly polarized focus (Sec. 2.2 compares the
radially polarized pulse with a linearly polarized one, Fig. 4; the field is
the same Lax-series construction with the vector potential along x).

Independent checks: Maxwell's equations in vacuum by finite differences --
Faraday's law and div B hold to the differencing floor (the fields come from
potentials), Gauss's and Ampere's laws leave residuals that fall with
eps = w0/z_r at the rates the truncation of the series sets; the field at
the focus; the paraxial peak intensity and power of a Gaussian beam; the
symmetries of a beam polarized along x; and the plane-wave limit."""
import numpy as np
import pytest

from test_oracle_fields import C, EPS0, _maxwell


@pytest.mark.parametrize("order,eps_pair,slopes", [
    (21, (0.04, 0.16), (5, 4)), (23, (0.04, 0.16), (7, 6)), (25, (0.08, 0.24), (9, 8))])
def test_lp_maxwell_residuals(orc, order, eps_pair, slopes):
    r1 = _maxwell(orc, order, eps_pair[0])
    r2 = _maxwell(orc, order, eps_pair[1])
    got = np.log(r2[[0, 2]] / r1[[0, 2]]) / np.log(eps_pair[1] / eps_pair[0])
    assert np.all(np.abs(got - np.array(slopes)) < 0.15), got
    # Faraday and div B: at the finite-difference floor for every eps
    assert r1[1] < 5e-11 and r2[1] < 5e-11 and r1[3] < 1e-12 and r2[3] < 1e-12


def test_lp_field_at_focus(orc):
    """At the focus, psi = 1 and psi_s = -1 for the paraxial term, so
    Ex = c By = E0 (1 - eps^2/2) cos(omega t + phi0), Ey = Ez = Bz = 0."""
    lam, w0 = 1e-6, 2.5e-6
    L = orc.laser_intensity(lam, w0, 1.0, 1e20, field=orc.LP_O1, phi0=0.4)
    k = 2 * np.pi / lam
    eps = 2 / (k * w0)
    t = np.linspace(-2e-15, 2e-15, 17)
    E, B = orc.field(L, 0 * t, 0 * t, 0 * t, t)
    want = L.amp * (1 - eps ** 2 / 2) * np.cos(C * k * t + 0.4)
    assert np.allclose(E[:, 0], want, rtol=0, atol=1e-13 * L.amp)
    assert np.allclose(C * B[:, 1], want, rtol=0, atol=1e-13 * L.amp)
    assert np.all(np.abs(E[:, 1:]) < 1e-15 * L.amp) and np.all(np.abs(B[:, [0, 2]]) < 1e-15 * L.amp / C)


def test_lp_intensity_and_power(orc):
    """A paraxial Gaussian beam with peak field E0 has peak intensity
    eps0 c E0^2 / 2 = I (the amplitude from intensity) and power
    pi w0^2 I / 2; the order-1 beam matches both up to O(eps^2)."""
    lam, w0, I = 1e-6, 6e-6, 1e20
    L = orc.laser_intensity(lam, w0, 1.0, I, field=orc.LP_O1)
    k = 2 * np.pi / lam
    eps = 2 / (k * w0)
    T = lam / C
    ts = (np.arange(32) + 0.5) / 32 * T

    def S_z(x, y):
        s = 0.0
        for t in ts:
            E, B = orc.field(L, x, y, 0 * x, t + 0 * x)
            s = s + (E[:, 0] * B[:, 1] - E[:, 1] * B[:, 0]) / (4e-7 * np.pi)
        return s / len(ts)

    peak = S_z(np.zeros(1), np.zeros(1))[0] * 1e-4   # W/cm^2
    assert abs(peak / I - 1) < eps ** 2
    r = np.linspace(0, 4 * w0, 801)
    ph = (np.arange(16) + 0.5) / 16 * 2 * np.pi
    ring = np.array([S_z(ri * np.cos(ph), ri * np.sin(ph)).mean() for ri in r])
    P = np.trapezoid(ring * 2 * np.pi * r, r)
    assert abs(P / (np.pi * w0 ** 2 * I * 1e4 / 2) - 1) < 2 * eps ** 2


def test_lp_symmetries(orc):
    """Polarization along x: Ex, By even in x and y; Ey odd in both; Ez odd in
    x, even in y; Bz even in x, odd in y; Bx = 0."""
    L = orc.laser_intensity(0.8e-6, 1.5e-6, 1.0, 1e20, field=orc.LP_O5)
    rng = np.random.default_rng(4)
    n = 50
    x, y = rng.uniform(-3e-6, 3e-6, (2, n))
    z = rng.uniform(-10e-6, 10e-6, n)
    t = z / C + rng.uniform(-3e-15, 3e-15, n)
    E, B = orc.field(L, x, y, z, t)
    Ex_, Bx_ = orc.field(L, -x, y, z, t)
    Ey_, By_ = orc.field(L, x, -y, z, t)
    tol = 1e-12 * L.amp
    assert np.allclose(Ex_[:, 0], E[:, 0], atol=tol) and np.allclose(Ey_[:, 0], E[:, 0], atol=tol)
    assert np.allclose(Ex_[:, 1], -E[:, 1], atol=tol) and np.allclose(Ey_[:, 1], -E[:, 1], atol=tol)
    assert np.allclose(Ex_[:, 2], -E[:, 2], atol=tol) and np.allclose(Ey_[:, 2], E[:, 2], atol=tol)
    assert np.allclose(Bx_[:, 2], B[:, 2], atol=tol / C) and np.allclose(By_[:, 2], -B[:, 2], atol=tol / C)
    assert np.all(B[:, 0] == 0.0)


def test_lp_plane_wave_limit(orc):
    """For a wide waist (eps -> 0) the field near the axis and the focus is the
    x-polarized plane wave of the same amplitude, envelope and phase."""
    lam = 0.8e-6
    L = orc.laser_intensity(lam, 2e-3, 30e-15, 1e20, field=orc.LP_O5, phi0=0.3)
    P = orc.laser_intensity(lam, 2e-3, 30e-15, 1e20, field=orc.PLANE_LP, phi0=0.3)
    rng = np.random.default_rng(6)
    n = 40
    x, y = rng.uniform(-1e-6, 1e-6, (2, n))
    z = rng.uniform(-5e-6, 5e-6, n)
    t = z / C + rng.uniform(-40e-15, 40e-15, n)
    E, B = orc.field(L, x, y, z, t)
    Ep, Bp = orc.field(P, x, y, z, t)
    assert np.allclose(E, Ep, rtol=0, atol=2e-5 * L.amp)
    assert np.allclose(B, Bp, rtol=0, atol=2e-5 * L.amp / C)
