"""The linearly polarized focus as the GPU evaluates it (term tables of
rpdla_lp_coeffs.hpp, written by gen_lp_coeffs.py from a symbolic
derivation) against the oracle's field (derivatives of the same Lax series
taken by hyper-dual arithmetic), on the CPU: the tables are evaluated here
in numpy exactly as the kernel combines them, and must reproduce the oracle
to rounding.  Also: the header is the generator's current output."""
import os
import re
import subprocess
import sys

import numpy as np
import pytest

CSRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                    "paper_2509_01741_amd", "csrc")
C = 299792458.0


def test_header_is_the_generator_output():
    out = subprocess.run([sys.executable, os.path.join(CSRC, "gen_lp_coeffs.py")],
                         capture_output=True, text=True, check=True).stdout
    assert out == open(os.path.join(CSRC, "rpdla_lp_coeffs.hpp")).read()


def _tables():
    txt = open(os.path.join(CSRC, "rpdla_lp_coeffs.hpp")).read()
    tabs = {}
    for name, order, body in re.findall(r"constexpr Term k(\w+?)_O(\d)\[\d+\] = \{(.*?)\};", txt):
        terms = re.findall(r"\{(\d+), (\d+), (\d+), ([-0-9.e+]+), ([-0-9.e+]+)\}", body)
        tabs[(name, int(order))] = [(int(n), int(m), int(j), float(re_), float(im))
                                    for n, m, j, re_, im in terms]
    return tabs


def _gpu_form(tabs, order, L, x, y, z, t):
    """The kernel's combination in SI units: sum_n c_n(s, eps) q^n times
    g e^{i Psi}, with q = (1 + i zeta)/D, Psi = phi0 + omega t - k z -
    s zeta / D, g = A exp(-s/D - (t - z/c)^2/tau0^2)."""
    k = 2 * np.pi / L.lambda_
    w0 = L.w0
    zr = 0.5 * k * w0 * w0
    eps = w0 / zr
    rx, ry = x / w0, y / w0
    s = rx * rx + ry * ry
    zeta = z / zr
    D = 1 + zeta * zeta
    q = (1 + 1j * zeta) / D
    tau0 = L.tau_fwhm / np.sqrt(2 * np.log(2))
    g = L.amp * np.exp(-s / D - ((t - z / C) / tau0) ** 2)
    base = g * np.exp(1j * (L.phi0 + C * k * t - k * z - s * zeta / D))

    def U(name):
        return sum((re_ + 1j * im) * eps ** j * s ** m * q ** n
                   for n, m, j, re_, im in tabs[(name, order)])

    wx0, wxr, wz = base * U("AX0"), base * U("AXR"), base * U("AZ")
    E = np.stack([(wx0 + rx * rx * wxr).real, (rx * ry * wxr).real, (rx * wz).real], -1)
    B = np.stack([0 * s, (base * U("BY")).real / C, eps * ry * (base * U("S")).imag / C], -1)
    return E, B


@pytest.mark.parametrize("order", [1, 3, 5])
def test_gpu_tables_reproduce_oracle_field(orc, order):
    tabs = _tables()
    L = orc.laser_intensity(0.8e-6, 1.2e-6, 25e-15, 1e21, field=20 + order, phi0=0.3)
    rng = np.random.default_rng(order)
    n = 300
    x, y = rng.uniform(-3, 3, (2, n)) * L.w0
    z = rng.uniform(-2, 2, n) * orc.rayleigh(L)
    t = z / C + rng.uniform(-40e-15, 40e-15, n)
    Eo, Bo = orc.field(L, x, y, z, t)
    Eg, Bg = _gpu_form(tabs, order, L, x, y, z, t)
    scale = L.amp
    assert np.max(np.abs(Eg - Eo)) <= 1e-13 * scale
    assert np.max(np.abs(Bg - Bo)) <= 1e-13 * scale / C
