"""Pins for the oracle's Newton-Lorentz push (Eqs. (7)-(14): dp/dt =
-e(E + v x B), gamma^2 = 1 + p^2/(m c)^2, electrons born at rest).

Independent checks: hyperbolic motion in a uniform E field, gyration radius
and period in a uniform B field, the exact linear invariant and the energy
integral of crossed static fields, the plane-wave canonical-momentum and
light-front invariants (gamma - u_z = 1) with Lawson-Woodward zero net gain,
fourth-order convergence, the x-z-plane reduction (Eqs. (15)-(17)) and
rotational symmetry of the radially polarized focus.
"""
import numpy as np
import pytest
from scipy import integrate, special

C = 299792458.0
QE = 1.602176634e-19
ME = 9.1093837015e-31


def test_uniform_E_hyperbolic(orc):
    E0 = 1e13
    L = orc.laser_intensity(0.8e-6, 3e-6, 30e-15, 1e21, field=orc.UNIFORM_EB,
                            test_E=(E0, 0, 0), test_B=(0, 0, 0))
    t0, t1 = 1.234e-15, 201.234e-15
    x0 = np.array([1e-6, -2e-6, 3e-6])
    xf, uf = orc.push_one(L, t0, t1, L.dt, x0, [0, 0, 0])
    a = QE * E0 / (ME * C)
    tau = t1 - t0
    assert abs(uf[0] - (-a * tau)) < 1e-12 * a * tau
    assert uf[1] == 0 and uf[2] == 0
    dx = -(ME * C * C / (QE * E0)) * (np.sqrt(1 + (a * tau) ** 2) - 1)
    assert abs((xf[0] - x0[0]) - dx) < 1e-10 * abs(dx)
    assert xf[1] == x0[1] and xf[2] == x0[2]


def test_uniform_B_gyration(orc):
    B0 = 1e3
    L = orc.laser_intensity(0.8e-6, 3e-6, 30e-15, 1e21, field=orc.UNIFORM_EB,
                            test_E=(0, 0, 0), test_B=(0, 0, B0))
    uperp = 2.0
    gam = np.sqrt(1 + uperp**2)
    R = uperp * ME * C / (QE * B0)
    Tg = 2 * np.pi * gam * ME / (QE * B0)
    x0 = np.zeros(3)
    xf, uf = orc.push_one(L, 0.0, Tg, L.dt, x0, [uperp, 0, 0])
    assert np.linalg.norm(xf - x0) < 1e-9 * R           # closed orbit after one period
    assert abs(np.linalg.norm(uf) - uperp) < 1e-10 * uperp
    xh, uh = orc.push_one(L, 0.0, Tg / 2, L.dt, x0, [uperp, 0, 0])
    assert abs(np.linalg.norm(xh - x0) - 2 * R) < 1e-9 * R   # diameter after half a turn
    assert np.allclose(uh, [-uperp, 0, 0], rtol=0, atol=1e-9 * uperp)
    # sense of rotation for negative charge: counter-clockwise seen from +z
    xq, _ = orc.push_one(L, 0.0, Tg / 4, L.dt, x0, [uperp, 0, 0])
    assert xq[1] > 0.9 * R


def test_crossed_fields_invariants(orc):
    E0, B0 = 3e11, 2e3
    L = orc.laser_intensity(0.8e-6, 3e-6, 30e-15, 1e21, field=orc.UNIFORM_EB,
                            test_E=(E0, 0, 0), test_B=(0, 0, B0))
    x0 = np.array([0.3e-6, 0.1e-6, -0.2e-6])
    for t1 in (30e-15, 150e-15, 400e-15):
        xf, uf = orc.push_one(L, 0.0, t1, L.dt, x0, [0, 0, 0])
        dx = xf[0] - x0[0]
        # exact linear invariant: u_y - (e B0/(m c)) (x - x0) = 0 (y translation)
        s = QE * B0 / (ME * C)
        assert abs(uf[1] - s * dx) < 1e-12 * max(1.0, abs(uf[1]))
        assert uf[2] == 0.0
        # energy integral: gamma - 1 = -(e E0 / (m c^2)) (x - x0)
        gam = np.sqrt(1 + uf @ uf)
        assert abs((gam - 1) + QE * E0 * dx / (ME * C * C)) < 1e-10 * max(1.0, gam - 1)


def _plane_A(L, s):
    """(e/(m c)) * integral_{-inf}^{s} E_x ds' of the plane-wave test model,
    E_x = A exp(-s^2/tau0^2) cos(omega s + phi0), in closed form through the
    Faddeeva function w(z) = exp(-z^2) erfc(-i z)."""
    om = 2 * np.pi * C / L.lambda_
    tau0 = L.tau_fwhm / np.sqrt(2 * np.log(2))
    z = s / tau0 - 0.5j * om * tau0
    pref = 0.5 * tau0 * np.sqrt(np.pi)
    ph = np.exp(-(s / tau0) ** 2 + 1j * om * s)
    if s <= 0:
        I = pref * ph * special.wofz(-1j * z)
    else:
        I = pref * (2 * np.exp(-0.25 * (om * tau0) ** 2) - ph * special.wofz(1j * z))
    return QE / (ME * C) * L.amp * np.real(np.exp(1j * L.phi0) * I)


def test_plane_A_closed_form_vs_quadrature():
    class _L:
        lambda_, tau_fwhm, amp, phi0 = 0.8e-6, 8e-15, 1e12, 0.4
    om = 2 * np.pi * C / _L.lambda_
    tau0 = _L.tau_fwhm / np.sqrt(2 * np.log(2))
    f = lambda q: _L.amp * np.exp(-(q / tau0) ** 2) * np.cos(om * q + _L.phi0)
    for s in (-7e-15, -1e-15, 0.0, 2e-15, 9e-15):
        val, _ = integrate.quad(f, -8 * tau0, s, limit=500, epsabs=0, epsrel=1e-12,
                                points=np.linspace(-8 * tau0, s, 200)[1:-1])
        assert abs(QE / (ME * C) * val - _plane_A(_L, s)) < 1e-10 * QE / (ME * C) * _L.amp * tau0


def test_plane_wave_invariants(orc):
    L = orc.laser_intensity(0.8e-6, 3e-6, 30e-15, 2e18, field=orc.PLANE_LP, window=orc.WIN_LAB,
                            phi0=0.4)
    a0 = QE * L.amp / (ME * C * 2 * np.pi * C / L.lambda_)
    assert 0.5 < a0 < 2
    for t0 in (-20e-15, -3e-15, 11e-15):
        xf, uf = orc.push_one(L, t0, L.t_after, L.dt, [0, 0, 0], [0, 0, 0])
        sf = L.t_after - xf[2] / C
        # canonical momentum: u_x = -(e/(m c)) int_{s0}^{s} E_x ds
        ux_ref = -(_plane_A(L, sf) - _plane_A(L, t0))
        assert abs(uf[0] - ux_ref) < 1e-7 * a0, (t0, uf[0], ux_ref)
        assert uf[1] == 0.0
        gam = np.sqrt(1 + uf @ uf)
        # light-front invariant and u_z = u_x^2/2 (RK4 truncation ~ (omega dt)^4)
        assert abs(gam - uf[2] - 1) < 1e-6
        assert abs(uf[2] - uf[0] ** 2 / 2) < 1e-6


def test_lawson_woodward(orc):
    """Born at rest before the pulse: no net energy gain once it has passed."""
    L = orc.laser_intensity(0.8e-6, 3e-6, 30e-15, 1e19, field=orc.PLANE_LP, window=orc.WIN_LAB)
    xf, uf = orc.push_one(L, -L.t_before, L.t_after, L.dt, [0, 0, 0], [0, 0, 0])
    sf = L.t_after - xf[2] / C
    assert sf > 4 * L.tau_fwhm                      # the pulse has gone by
    K = np.sqrt(1 + uf @ uf) - 1
    # exact net gain ~ exp(-(t_before/tau0)^2) ~ 1e-15; RK4 truncation ~ 1e-7
    assert np.linalg.norm(uf) < 1e-6 and K < 1e-6
    # during the pulse it was strongly driven
    xm, um = orc.push_one(L, -L.t_before, 0.0, L.dt, [0, 0, 0], [0, 0, 0])
    assert np.linalg.norm(um) > 0.1


def test_rk4_fourth_order(orc):
    """Global error of the position against hyperbolic motion falls as h^4
    (the x equation is a quadrature of a smooth function of time)."""
    E0 = 1e10  # time scale m c/(e E0) = 170 fs
    L = orc.laser_intensity(0.8e-6, 3e-6, 30e-15, 1e21, field=orc.UNIFORM_EB,
                            test_E=(E0, 0, 0), test_B=(0, 0, 0))
    a = QE * E0 / (ME * C)
    t1 = 401e-15
    dx = -(ME * C * C / (QE * E0)) * (np.sqrt(1 + (a * t1) ** 2) - 1)
    errs = []
    for h in (16e-15, 8e-15, 4e-15, 2e-15):
        xf, uf = orc.push_one(L, 0.0, t1, h, [0, 0, 0], [0, 0, 0])
        errs.append(abs(xf[0] - dx) / abs(dx))
    p = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(p - 4) < 0.15), (p, errs)


def test_rk4_step_refinement_rp(orc):
    """In the focus the production step dt = T/200 is converged: halving it
    moves the final momentum by far less than its size."""
    L = orc.laser_intensity(0.8e-6, 3e-6, 30e-15, 1e19, field=orc.RP_O5)
    x0 = np.array([2.0e-6, 0.5e-6, 1.0e-6])
    a_x, a_u = orc.push_one(L, -10e-15, 10e-15, L.dt, x0, [0, 0, 0])
    b_x, b_u = orc.push_one(L, -10e-15, 10e-15, L.dt / 2, x0, [0, 0, 0])
    assert np.linalg.norm(a_u - b_u) < 1e-7 * np.linalg.norm(a_u)


def test_xz_plane_reduction(orc):
    """Eqs. (15)-(17): an electron born in y = 0 keeps p_y = 0 and y = 0."""
    L = orc.laser_intensity(0.8e-6, 3e-6, 30e-15, 1e21, field=orc.RP_O5)
    tb = np.array([-20e-15, -5e-15, 3e-15])
    out = orc.push(L, tb, [1.7e-6], [0.0], [2e-6], 3)
    assert np.all(out[1] == 0.0) and np.all(out[4] == 0.0)
    assert np.all(np.abs(out[0]) > 0)


def test_rotation_symmetry(orc):
    L = orc.laser_intensity(0.8e-6, 3e-6, 30e-15, 1e20, field=orc.RP_O5)
    r, al = 2.2e-6, 0.7
    tb = np.array([-12e-15])
    a = orc.push(L, tb, [r], [0.0], [1e-6], 1)
    b = orc.push(L, tb, [r * np.cos(al)], [r * np.sin(al)], [1e-6], 1)
    ua = np.array([a[0][0], a[1][0], a[2][0]])
    ub = np.array([b[0][0], b[1][0], b[2][0]])
    R = np.array([[np.cos(al), -np.sin(al), 0], [np.sin(al), np.cos(al), 0], [0, 0, 1]])
    assert np.linalg.norm(R @ ua - ub) < 1e-9 * np.linalg.norm(ua)


def test_batch_push_window_and_unborn(orc):
    L = orc.laser_intensity(0.8e-6, 3e-6, 30e-15, 1e21, field=orc.RP_O5)
    x0, y0, z0 = np.array([1e-6, 2e-6]), np.array([0.5e-6, -1e-6]), np.array([-5e-6, 8e-6])
    tb = np.array([-30e-15 - 5e-6 / C, np.inf, np.inf, 10e-15 + 8e-6 / C])
    out = orc.push(L, tb, x0, y0, z0, 2)
    assert np.all(np.isnan([o[1] for o in out])) and np.all(np.isnan([o[2] for o in out]))
    # births before the window: invalid (NaN) beyond one step ahead of the
    # window start, valid within it (reading of the window convention)
    ts0 = z0[0] / C - L.t_before
    early = orc.push(L, np.array([ts0 - 1.5 * L.dt, ts0 - 0.5 * L.dt]), x0[:1], y0[:1], z0[:1], 2)
    assert np.all(np.isnan([o[0] for o in early])) and np.all(np.isfinite([o[1] for o in early]))
    for s, a in ((0, 0), (3, 1)):
        te = z0[a] / C + L.t_after
        xf, uf = orc.push_one(L, tb[s], te, L.dt, [x0[a], y0[a], z0[a]], [0, 0, 0])
        assert np.array_equal([out[0][s], out[1][s], out[2][s]], uf)
        assert np.array_equal([out[3][s], out[4][s], out[5][s]], xf)


def test_double_push_resolves_sensitive_electrons(orc):
    """The RK4 answer is the map in exact arithmetic.  For the most
    rounding-sensitive electrons of the 1024-atom ensemble (0.8 um, w0 3 um,
    30 fs, 1e21 W/cm^2, order 5; found by comparing the double and
    extended-precision builds over all 8192 electrons), plain double
    accumulation of the state missed the extended result by 4e-8..4e-7 for
    these six; with the compensated accumulation the double push stays within
    1e-8 of the extended build's on the same inputs."""
    import ctypes as C
    L = orc.laser_intensity(0.8e-6, 3e-6, 30e-15, 1e21)
    zr = orc.rayleigh(L)
    # (atom, charge state)
    picks = [(997, 1), (580, 5), (708, 2), (105, 3), (278, 6), (840, 5)]
    atoms = np.array([a for a, _ in picks], dtype=np.uint64)
    ch = orc.chain(L, 0, 0, atoms, 2 * L.w0, zr, 1, 8)
    sl = np.array([i * 8 + (k - 1) for i, (_, k) in enumerate(picks)])
    tb = ch["t_birth"][sl]
    assert np.all(np.isfinite(tb))
    x, y, z = ch["x"], ch["y"], ch["z"]
    idx = np.arange(len(picks))
    d = orc.push(L, tb, x[idx], y[idx], z[idx], 1)
    ext = [np.zeros(len(picks)) for _ in range(6)]
    orc.lib_extended().orc_push(C.byref(L), len(picks), np.ascontiguousarray(tb),
                                x[idx].copy(), y[idx].copy(), z[idx].copy(), 1, *ext)
    Kd = orc.epilogue(*d[:3])[0]
    Ke = orc.epilogue(*ext[:3])[0]
    assert np.all(np.abs(Kd - Ke) <= 1e-8 * Ke), np.abs(Kd - Ke) / Ke
