"""Pins for the oracle's radiation reaction (Sec. 2.1, Eq. (3)) and quantum
parameter (Eqs. (4)-(6)).

Independent checks: the power the Eq. (3) term removes is beta^2 times the
Lienard power of the Lorentz motion (computed here from the acceleration,
not from the fields' invariant); the energy of an electron gyrating in a
uniform magnetic field decays as the closed form of that term predicts; chi
is E/E_cr at rest (Eq. (5)) and gamma (1 + beta) E/E_cr head-on against a
plane wave (Eq. (4)); with the term switched off the push is the plain one.
"""
import json
import math
import os

import numpy as np
from scipy.optimize import brentq

C = 299792458.0
QE = 1.602176634e-19
ME = 9.1093837015e-31
EPS0 = 8.8541878128e-12
HBAR = 1.054571817e-34
GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def test_rr_off_is_the_plain_push(orc):
    L = orc.laser_intensity(0.8e-6, 3e-6, 30e-15, 1e21)
    rng = np.random.default_rng(3)
    n = 6
    x, y = rng.uniform(-3e-6, 3e-6, (2, n))
    z = rng.uniform(-20e-6, 20e-6, n)
    tb = np.repeat(z / C, 2) + rng.normal(0, 20e-15, 2 * n)
    a = orc.push(L, tb, x, y, z, 2)
    b = orc.push_rr(L, 0, tb, x, y, z, 2)
    for u, v in zip(a, b[:6]):
        assert np.array_equal(u, v)
    assert np.all(b[6] > 0)


def test_rr_power_is_beta2_lienard(orc):
    L = orc.laser_intensity(0.8e-6, 2.5e-6, 30e-15, 1e22)
    rng = np.random.default_rng(4)
    for _ in range(40):
        pos = rng.uniform(-3e-6, 3e-6, 3)
        t = pos[2] / C + rng.uniform(-30e-15, 30e-15)
        u = rng.normal(size=3) * 10 ** rng.uniform(-1, 3)
        du_rr, chi = orc.rr_terms(L, t, np.concatenate([pos, u]))
        E, B = (a[0] for a in orc.field(L, *[np.array([c]) for c in pos], np.array([t])))
        g = math.sqrt(1 + u @ u)
        v = C * u / g
        # Lorentz motion: du/dt, then the velocity's rate of change
        dudt = -QE / (ME * C) * (E + np.cross(v, B))
        acc = C * (dudt / g - u * (u @ dudt) / g ** 3)
        P_lienard = QE ** 2 * g ** 6 / (6 * math.pi * EPS0 * C ** 3) * (
            acc @ acc - np.cross(v, acc) @ np.cross(v, acc) / C ** 2)
        P_rr = -(ME * C * du_rr) @ v
        beta2 = (v @ v) / C ** 2
        # the Lienard bracket cancels to ~1/gamma^2 of its terms: tolerance ~ eps gamma^2
        assert abs(P_rr - beta2 * P_lienard) <= 1e-13 * (1 + g * g) * beta2 * P_lienard
        # the radiation term is antiparallel to the velocity
        assert np.linalg.norm(np.cross(du_rr, v)) <= 1e-12 * np.linalg.norm(du_rr) * np.linalg.norm(v)


def test_rr_uniform_magnetic_field_decay(orc):
    """v perpendicular to B: d gamma/dt = -K (gamma^2 - 1)^2 / gamma^2 with
    K = e^4 B^2 / (6 pi eps0 m^3 c^3); its antiderivative in gamma is
    G = -gamma / (2 (gamma^2 - 1)) + ln((gamma - 1)/(gamma + 1)) / 4."""
    B0 = 1e5
    L = orc.laser_intensity(0.8e-6, 3e-6, 30e-15, 1e21, field=orc.UNIFORM_EB, test_B=(0, 0, B0))
    g0 = 1000.0
    u0 = np.array([math.sqrt(g0 ** 2 - 1), 0.0, 0.0])
    T = 1e-12
    _, uf, chi_max = orc.push_one_rr(L, 1, 0.0, T, 1e-17, np.zeros(3), u0)
    gf = math.sqrt(1 + uf @ uf)
    K = QE ** 4 * B0 ** 2 / (6 * math.pi * EPS0 * ME ** 3 * C ** 3)
    G = lambda g: -g / (2 * (g * g - 1)) + 0.25 * math.log((g - 1) / (g + 1))
    want = brentq(lambda g: G(g) - G(g0) + K * T, 1.0 + 1e-9, g0, xtol=1e-14, rtol=1e-15)
    assert want < 0.5 * g0                      # a strong effect is being tested
    assert abs(gf / want - 1) < 1e-9, (gf, want)
    assert abs(uf[2]) == 0.0
    # chi is largest at the start: gamma beta B c / E_cr
    assert abs(chi_max / (math.sqrt(g0 ** 2 - 1) * C * B0 / orc.critical_field()) - 1) < 1e-12
    # without the term, gamma is conserved
    _, uf0, _ = orc.push_one_rr(L, 0, 0.0, T, 1e-17, np.zeros(3), u0)
    assert abs(math.sqrt(1 + uf0 @ uf0) / g0 - 1) < 1e-10


def test_chi_at_rest_is_field_over_critical(orc):
    E0 = GOLD["chi_at_5e21"]["E0_V_m"]
    L = orc.laser_intensity(0.8e-6, 3e-6, 30e-15, 1e21, field=orc.UNIFORM_EB, test_E=(E0, 0, 0))
    _, _, chi = orc.push_one_rr(L, 0, 0.0, 1e-18, 1e-18, np.zeros(3), np.zeros(3))
    Ecr = orc.critical_field()
    assert abs(Ecr / (ME ** 2 * C ** 3 / (QE * HBAR)) - 1) < 1e-15
    assert abs(chi / (E0 / Ecr) - 1) < 1e-15
    # the paper quotes E_cr = 1.326e18 V/m and chi = 1.463e-4 (rounded constants)
    g = GOLD["chi_at_5e21"]
    assert abs(Ecr / g["Ecr_V_m"] - 1) < 3e-3
    assert abs(chi / g["chi"] - 1) < 3e-3


def test_chi_head_on_and_co_propagating_plane_wave(orc):
    L = orc.laser_intensity(0.8e-6, 3e-6, 30e-15, 1e21, field=orc.PLANE_LP)
    Ecr = orc.critical_field()
    for u0 in (0.5, 10.0, 300.0):
        g = math.sqrt(1 + u0 * u0)
        _, chi = orc.rr_terms(L, 0.0, np.array([0, 0, 0, 0, 0, -u0]))
        assert abs(chi / ((g + u0) * L.amp / Ecr) - 1) < 1e-14     # gamma (1 + beta) E / E_cr
        _, chi = orc.rr_terms(L, 0.0, np.array([0, 0, 0, 0, 0, u0]))
        assert abs(chi / (L.amp / ((g + u0) * Ecr)) - 1) < 1e-9    # gamma (1 - beta) E / E_cr
