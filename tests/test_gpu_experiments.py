"""Kernels of the paper's single-particle studies (Sec. 2.2) against the
oracle -- hollow-cylinder sampling (Fig. 8), laser phase and radius at birth
(Figs. 6, 13, 14), the forward/backward two-dimensional histogram (Figs. 13,
14) -- on seeded inputs handed to both sides."""
import math

import numpy as np
import pytest

import seeded_inputs as SI
from gpu_common import C_LIGHT, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env(orc):
    torch = require_gpu()
    from paper_2509_01741_amd import binding as B
    return torch, B, orc


def _t(torch, a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


@pytest.mark.parametrize("r_in,r_out", [(2e-6, 2e-6), (1e-6, 4e-6), (0.0, 3e-6), (0.0, 0.0)])
def test_sample_annulus_parity(env, r_in, r_out):
    torch, B, O = env
    for n, first in ((1, 0), (257, 5), (1000, 987654321)):
        g = B.rpdla_sample_atoms_annulus(4, 6, first, n, r_in, r_out, 20e-6, device="cuda")
        o = O.sample_atoms_annulus(4, 6, first, n, r_in, r_out, 20e-6)
        for a, b in zip(g, o):
            a = a.cpu().numpy()
            assert np.all(np.abs(a - b) <= 8 * np.finfo(float).eps * max(r_out, 20e-6)), \
                np.max(np.abs(a - b))
        if r_in == r_out:
            r = np.hypot(g[0].cpu().numpy(), g[1].cpu().numpy())
            assert np.all(np.abs(r - r_out) <= 4 * np.finfo(float).eps * r_out)


@pytest.mark.parametrize("spa", [1, 3])
def test_birth_phase_parity(env, spa):
    torch, B, O = env
    L = B.rpdla_laser_init_intensity(0.8e-6, 2.5e-6, 53e-15, 5e20, phi0=0.4)
    OL = O.laser_intensity(0.8e-6, 2.5e-6, 53e-15, 5e20, phi0=0.4)
    n = 2000
    xs, ys, zs = SI.cylinder_atoms(50 + spa, n, 4e-6, 60e-6)
    tbs = SI.birth_times(50 + spa, zs, spa, 53e-15, spread=1.5)
    ph, rb = B.rpdla_birth_phase(L, _t(torch, tbs), _t(torch, xs), _t(torch, ys), _t(torch, zs),
                                 spa)
    ph, rb = ph.cpu().numpy(), rb.cpu().numpy()
    oph = O.birth_phase(OL, tbs, xs, ys, zs, spa)
    born = np.isfinite(tbs)
    assert 0 < born.sum() < tbs.size
    assert np.array_equal(np.isnan(ph), ~born) and np.array_equal(np.isnan(rb), ~born)
    d = np.abs(ph[born] - oph[born])
    d = np.minimum(d, 2 * np.pi - d)           # equal phases may sit either side of 0 / 2 pi
    assert d.max() <= 1e-10, d.max()
    assert np.all((ph[born] >= 0) & (ph[born] < 2 * np.pi))
    r = np.repeat(np.hypot(xs, ys), spa)[born]
    assert np.all(np.abs(rb[born] - r) <= 2 * np.finfo(float).eps * r)
    # without the radius output
    ph2, none = B.rpdla_birth_phase(L, _t(torch, tbs), _t(torch, xs), _t(torch, ys),
                                    _t(torch, zs), spa, want_radius=False)
    assert none is None and np.array_equal(ph2.cpu().numpy(), ph, equal_nan=True)


def test_histogram2d_exact(env):
    torch, B, O = env
    n = 50000
    xs, ys, zs = SI.cylinder_atoms(61, n, 4e-6, 10e-6)
    u = SI.momenta(61, n)
    a = np.mod(np.arctan2(ys, xs) + zs * 1e5, 2 * np.pi)     # phase-like values in [0, 2 pi)
    b = np.hypot(xs, ys)
    uz = u[:, 2].copy()
    uz[::101] = 0.0
    a[3::211] = np.nan
    uz[5::307] = np.nan
    b[7::401] = 5e-6                                         # outside the radius range
    for na, nb in ((36, 40), (7, 3), (1, 1)):
        spec = B.rpdla_hist2d_spec(na, nb, 0.0, 2 * math.pi, 0.0, 4e-6)
        c, t = B.rpdla_histogram2d(_t(torch, a), _t(torch, b), _t(torch, uz), spec)
        c2, t2 = B.rpdla_histogram2d(_t(torch, a), _t(torch, b), _t(torch, uz), spec, c, t)
        oc, ot = O.histogram2d(a, b, uz, na, 0.0, 2 * math.pi, nb, 0.0, 4e-6)
        assert np.array_equal(c2.cpu().numpy().astype(np.uint64), 2 * oc)
        assert np.array_equal(t2.cpu().numpy().astype(np.uint64), 2 * ot)
        assert int(oc.sum() + ot.sum()) == n
    e = torch.empty(0, dtype=torch.float64, device="cuda")
    c, t = B.rpdla_histogram2d(e, e, e, B.rpdla_hist2d_spec(2, 2, 0.0, 1.0, 0.0, 1.0))
    assert int(c.sum()) == 0 and int(t.sum()) == 0
