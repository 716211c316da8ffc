"""Pins for the oracle's tunnelling rate (semi-classical tunnelling model the
paper cites in Sec. 1 and Sec. 2.1 'Ionization'; static ADK form).

Independent checks: the textbook static hydrogen rate w = (4/F) exp(-2/(3F))
(atomic units), the hydrogen-like scaling w_Z(F) = Z^2 w_H(F/Z^3) that an exact
tunnelling rate obeys for Ip = Z^2/2, the zero conventions, the Gauss-Legendre
table against numpy, and the neon potentials against their ordering/shell gap.
"""
import numpy as np
import pytest

TAUA = 2.4188843265857e-17
EA = 5.14220674763e11


def test_hydrogen_closed_form(orc):
    for F in np.geomspace(1e-3, 1e3, 61):
        ln_w = orc.adk_lnrate_general(0.5, 1.0, F)
        ref = np.log(4.0 / F) - 2.0 / (3.0 * F) - np.log(TAUA)
        assert abs(ln_w - ref) <= 1e-13 * max(1.0, abs(ref)), F


@pytest.mark.parametrize("Z", [2, 3, 7, 10])
def test_hydrogenlike_scaling(orc, Z):
    for F in np.geomspace(1e-2, 1e4, 25):
        lw = orc.adk_lnrate_general(Z * Z / 2.0, float(Z), F)
        lh = orc.adk_lnrate_general(0.5, 1.0, F / Z**3)
        assert abs(lw - (lh + 2 * np.log(Z))) < 1e-12 * max(1.0, abs(lw))


def test_rate_zero_conventions(orc):
    assert orc.adk_rate(1, 0.0) == 0.0
    assert orc.adk_rate(9, 1e9) == 0.0           # ln w far below -700
    assert orc.adk_lnrate(9, 1e9) < -700
    w = orc.adk_rate(1, 1e11)
    assert w > 0 and abs(np.log(w) - orc.adk_lnrate(1, 1e11)) < 1e-12


def test_rate_increases_below_barrier(orc):
    # below the suppression field every state's rate grows with the field
    ip = orc.ne_ip_ev() / 27.211386245988
    for k in range(1, 11):
        fbsi = ip[k - 1] ** 2 / (4 * k)
        F = np.geomspace(1e-3, 0.5, 50) * fbsi
        lw = [orc.adk_lnrate(k, f * EA) for f in F]
        assert np.all(np.diff(lw) > 0), k


def test_gl4_table(orc):
    x, w = orc.gl4()
    xr, wr = np.polynomial.legendre.leggauss(4)
    assert np.allclose(x, xr, rtol=0, atol=2e-16) and np.allclose(w, wr, rtol=0, atol=2e-16)
    # exact for polynomials up to degree 7
    for d in range(8):
        assert abs(np.sum(w * x**d) - (0 if d % 2 else 2.0 / (d + 1))) < 1e-15


def test_neon_table_shape(orc):
    ip = orc.ne_ip_ev()
    assert np.all(np.diff(ip) > 0)
    assert ip[8] / ip[7] > 4      # K-shell gap between the 8th and 9th electrons (Sec. 2.1)
    assert abs(ip[9] - 13.6057 * 100 * (1 + 0)) / ip[9] < 0.01  # Ne9+ is hydrogen-like: Z^2 Ry
