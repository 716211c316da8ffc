"""Pins for the oracle's outputs: kinetic energy (gamma - 1) m c^2 (text after
Eq. (14)), polar emission angle, azimuth psi = atan2(p_y, p_x) (Fig. 5 text),
forward/backward by the final direction of motion, and the energy-angle
histogram -- checked against direct pure-Python definitions on small inputs.
"""
import math

import numpy as np

MEC2 = 0.51099895000


def test_epilogue_definitions(orc):
    rng = np.random.default_rng(4)
    u = rng.normal(size=(500, 3)) * np.exp(rng.uniform(-8, 7, size=(500, 1)))
    K, th, ps, fwd = orc.epilogue(u[:, 0], u[:, 1], u[:, 2])
    for i in range(500):
        ux, uy, uz = (float(v) for v in u[i])
        g = math.sqrt(1 + ux * ux + uy * uy + uz * uz)
        kref = (g - 1) * MEC2
        # cancellation-free form agrees with (gamma-1) m c^2 where the latter is accurate
        assert abs(K[i] - kref) <= 1e-15 * g * MEC2 + 1e-12 * kref
        assert abs(th[i] - math.atan2(math.hypot(ux, uy), uz)) < 1e-15
        assert ps[i] == math.atan2(uy, ux)
        assert fwd[i] == (1 if uz > 0 else 0)
    # tiny momenta: no cancellation
    K, _, _, _ = orc.epilogue([1e-9], [0.0], [0.0])
    assert abs(K[0] - MEC2 * 0.5e-18) < 1e-12 * MEC2 * 0.5e-18


def _hist_ref(tb, ux, uy, uz, nE, nA, lo, hi, angle):
    counts = np.zeros((2, nE, nA), dtype=np.uint64)
    tal = np.zeros(6, dtype=np.uint64)
    w = (hi - lo) / nE
    for i in range(len(tb)):
        if not tb[i] < math.inf:
            tal[4] += 1
            continue
        if math.isnan(ux[i]) or math.isnan(uy[i]) or math.isnan(uz[i]):
            tal[5] += 1
            continue
        u2 = ux[i] ** 2 + uy[i] ** 2 + uz[i] ** 2
        K = MEC2 * u2 / (math.sqrt(1 + u2) + 1)
        d = 0 if uz[i] > 0 else 1
        tal[d] += 1
        lk = math.log10(K) if K > 0 else -math.inf
        fe = math.floor((lk - lo) / w) if lk > -math.inf else -1
        if fe < 0:
            tal[2] += 1
            continue
        if fe >= nE:
            tal[3] += 1
            continue
        if angle == 0:
            a = math.floor(math.atan2(math.hypot(ux[i], uy[i]), uz[i]) / math.pi * nA)
        else:
            a = math.floor((math.atan2(uy[i], ux[i]) + math.pi) / (2 * math.pi) * nA)
        a = min(max(a, 0), nA - 1)
        counts[d, fe, a] += 1
    return counts, tal


def test_histogram_brute_force(orc):
    rng = np.random.default_rng(9)
    n = 4000
    u = rng.normal(size=(n, 3)) * np.exp(rng.uniform(-6, 9, size=(n, 1)))
    tb = rng.normal(size=n)
    tb[rng.uniform(size=n) < 0.1] = np.inf
    u[rng.uniform(size=n) < 0.02, 1] = np.nan
    u[:5] = [[0, 0, 0], [0, 0, 1e-30], [0, 0, -3], [0, 0, 5], [0, 1e-3, 0]]
    tb[:5] = 0.0
    for angle, nE, nA in ((orc.ANG_POLAR, 64, 36), (orc.ANG_AZIMUTH, 50, 20)):
        c, t = orc.histogram(tb, u[:, 0], u[:, 1], u[:, 2], nE, nA, -3.0, 4.0, angle)
        cr, tr = _hist_ref(tb, u[:, 0], u[:, 1], u[:, 2], nE, nA, -3.0, 4.0, angle)
        assert np.array_equal(c, cr) and np.array_equal(t, tr)
        assert t[0] + t[1] + t[4] + t[5] == n
        assert c.sum() + t[2] + t[3] == t[0] + t[1]
