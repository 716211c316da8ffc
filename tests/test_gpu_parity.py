"""GPU parity: every entry point of the C ABI (through the Python binding)
against the CPU oracle on the same seeded inputs, element by element.

Tolerances: birth times |dt| <= 1e-10 max(|t|, T); final energy
|dK| <= 1e-8 K + 1e-12 MeV and forward/backward agreement for >= 99.9% of
electrons; positions of sampled atoms to rounding; histogram counts exact
when the oracle bins the GPU's own momenta.
"""
import numpy as np
import pytest

import seeded_inputs as SI
from gpu_common import (BEAM, C_LIGHT, allowed_failures, check_fp64, energy_parity, gpu_energy,
                        require_gpu)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env(orc):
    torch = require_gpu()
    from paper_2509_01741_amd import binding as B
    return torch, B, orc


def _lasers(B, O, order=5, **kw):
    L = B.rpdla_laser_init_intensity(BEAM["lam"], BEAM["w0"], BEAM["tau"], BEAM["I"])
    OL = O.laser_intensity(BEAM["lam"], BEAM["w0"], BEAM["tau"], BEAM["I"])
    L.field = order
    OL.field = order
    for k, v in kw.items():
        L.set(**{k: v})
        O._set(OL, k, v)
    return L, OL


Z_HALF = 35e-6   # about one Rayleigh length of BEAM


def _atoms(torch, seed, n, r_max=2 * BEAM["w0"], z_half=Z_HALF):
    """Seeded positions as numpy arrays (oracle) and device tensors (GPU)."""
    xs, ys, zs = SI.cylinder_atoms(seed, n, r_max, z_half)
    return (xs, ys, zs), tuple(_t(torch, a) for a in (xs, ys, zs))


def _t(torch, a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


def test_sample_atoms(env):
    torch, B, O = env
    for n, first in ((1, 0), (257, 5), (1000, 123456789)):
        x, y, z = B.rpdla_sample_atoms(7, 3, first, n, 6e-6, 35e-6)
        ox, oy, oz = O.sample_atoms(7, 3, first, n, 6e-6, 35e-6)
        for g, o in ((x, ox), (y, oy), (z, oz)):
            g = g.cpu().numpy()
            assert np.all(np.abs(g - o) <= 4e-16 * 6e-6 * 8), np.max(np.abs(g - o))
    # empty input is a no-op
    e = torch.empty(0, dtype=torch.float64, device="cuda")
    B.rpdla_sample_atoms(0, 0, 0, 0, 1.0, 1.0, e, e, e)


def _check_tb(gtb, otb, T):
    fin = np.isfinite(otb)
    assert np.array_equal(fin, np.isfinite(gtb)), "born / unborn pattern differs"
    assert np.all(np.isposinf(gtb[~fin]))
    err = np.abs(gtb[fin] - otb[fin]) / np.maximum(np.abs(otb[fin]), T)
    assert err.size == 0 or err.max() <= 1e-10, err.max()
    return fin


@pytest.mark.parametrize("order", [1, 3, 5])
def test_ionize_parity_rp(env, order):
    torch, B, O = env
    L, OL = _lasers(B, O, order)
    n = 300
    (xs, ys, zs), (x, y, z) = _atoms(torch, 10 + order, n)
    tb = B.rpdla_ionize(L, 0, 0, 0, x, y, z, 1, 10)
    otb = O.ionize(OL, 0, 0, 0, xs, ys, zs, 1, 10)
    fin = _check_tb(tb.cpu().numpy(), otb, L.lambda_ / C_LIGHT)
    assert fin.sum() > n * 7          # L shell is always stripped at 1e21 W/cm^2
    assert 0 < fin.reshape(n, 10)[:, 8:].sum() < 2 * n  # K shell sometimes


@pytest.mark.parametrize("case", ["uniform", "plane", "lab", "ez0", "er_half", "kwindow"])
def test_ionize_parity_variants(env, case):
    torch, B, O = env
    kw, kf, kl = {}, 1, 8
    if case == "uniform":
        kw = dict(field=11, test_E=(1.2e11, 3e10, 0.0), window=1)
    elif case == "plane":
        kw = dict(field=10)
    elif case == "lab":
        kw = dict(window=1)
    elif case == "ez0":
        kw = dict(ez_scale=0.0)
    elif case == "er_half":
        kw = dict(er_scale=0.5, phi0=0.7)
    elif case == "kwindow":
        kf, kl = 7, 9
    L, OL = _lasers(B, O, 5, **kw)
    n = 130
    (xs, ys, zs), (x, y, z) = _atoms(torch, 20, n)
    tb = B.rpdla_ionize(L, 1, 2, 0, x, y, z, kf, kl)
    otb = O.ionize(OL, 1, 2, 0, xs, ys, zs, kf, kl)
    _check_tb(tb.cpu().numpy(), otb, L.lambda_ / C_LIGHT)


def test_ionize_uniform_closed_form(env):
    """GPU birth times in a static uniform field: t_k - t_{k-1} = E_k / w_k."""
    torch, B, O = env
    E0 = 1.2e11
    L, OL = _lasers(B, O, 5, field=11, test_E=(E0, 0, 0), window=1)
    n = 64
    zero = torch.zeros(n, dtype=torch.float64, device="cuda")
    tb = B.rpdla_ionize(L, 3, 1, 100, zero, zero, zero, 1, 2).cpu().numpy().reshape(n, 2)
    for i in range(n):
        t = -L.t_before
        for s, k in enumerate((1, 2)):
            t += -np.log(O.uniform(3, 1, [100 + i], k + 2)[0]) / O.adk_rate(k, E0)
            if t > L.t_after:
                assert np.all(np.isposinf(tb[i, s:]))
                break
            assert abs(tb[i, s] - t) <= 1e-11 * max(abs(t), L.lambda_ / C_LIGHT)


def _push_case(env, order, n_atoms, prec=0, **kw):
    torch, B, O = env
    L, OL = _lasers(B, O, order, **kw)
    K = 8
    (xs, ys, zs), (x, y, z) = _atoms(torch, 30 + order, n_atoms)
    tbs = SI.birth_times(30 + order, zs, K, BEAM["tau"])
    out = B.rpdla_push(L, prec, _t(torch, tbs), x, y, z, K)
    g = [o.cpu().numpy() for o in out]
    ref = O.push(OL, tbs, xs, ys, zs, K)
    return tbs, g, ref, O, OL, (xs, ys, zs)


@pytest.mark.parametrize("order", [1, 5])
def test_push_parity_fp64(env, order):
    """FP64 push on identical seeded inputs (positions, birth times): the FP64
    energy rule of oracle/parity.py against the double oracle's push and the
    extended-precision build's push of the same inputs, all electrons."""
    torch, B, _ = env
    otb, g, ref, O, OL, (xs, ys, zs) = _push_case(env, order, 150)
    fin = np.isfinite(otb)
    for a in g:
        assert np.all(np.isnan(a[~fin])) and np.all(np.isfinite(a[fin]))
    Kg, fg = gpu_energy(B, torch, *(a[fin] for a in g[:3]))
    assert fin.sum() >= 1000
    check_fp64(O, OL, Kg, fg, otb, xs, ys, zs, 8, extended_push=True,
               label=f" push order {order}")
    assert Kg.max() > 1.0    # MeV-scale acceleration happens
    # final positions
    for a, r in zip(g[3:], ref[3:]):
        d = np.abs(a[fin] - r[fin])
        assert np.quantile(d, 0.999) < 1e-12 + 1e-8 * np.abs(r[fin]).max()


def test_push_closed_forms_gpu(env):
    """Uniform E: u_x = -(eE/mc) t exactly and hyperbolic position;
    crossed E, B: u_y - (e B/(m c)) (x - x0) = 0 exactly (linear invariant)."""
    torch, B, O = env
    QE, ME = 1.602176634e-19, 9.1093837015e-31
    E0 = 1e12
    L = B.rpdla_laser_init_intensity(0.8e-6, 3e-6, 30e-15, 1e21)
    L.set(field=11, test_E=(E0, 0, 0), window=1)
    tb = np.array([-100e-15, 0.0, 123e-15, np.inf])
    x0 = np.array([1e-6]); y0 = np.array([2e-6]); z0 = np.array([-3e-6])
    out = [o.cpu().numpy() for o in B.rpdla_push(L, 0, _t(torch, tb), _t(torch, x0), _t(torch, y0),
                                                 _t(torch, z0), 4)]
    a = QE * E0 / (ME * C_LIGHT)
    tau = L.t_after - tb[:3]
    assert np.all(np.abs(out[0][:3] + a * tau) <= 1e-12 * a * tau)
    dx = -(ME * C_LIGHT**2 / (QE * E0)) * (np.sqrt(1 + (a * tau) ** 2) - 1)
    assert np.all(np.abs(out[3][:3] - x0[0] - dx) <= 1e-9 * np.abs(dx))
    assert np.all(np.isnan([o[3] for o in out]))
    B0 = 2e3
    L.set(test_E=(3e11, 0, 0), test_B=(0, 0, B0))
    out = [o.cpu().numpy() for o in B.rpdla_push(L, 0, _t(torch, tb[:3]), _t(torch, x0),
                                                 _t(torch, y0), _t(torch, z0), 3)]
    s = QE * B0 / (ME * C_LIGHT)
    assert np.all(np.abs(out[1] - s * (out[3] - x0[0])) <= 1e-12 * np.maximum(1, np.abs(out[1])))
    assert np.all(out[2] == 0.0)


def test_push_plane_wave_parity(env):
    torch, B, O = env
    L, OL = _lasers(B, O, 5, field=10, window=1)
    tb = np.linspace(-60e-15, 40e-15, 200)
    z0 = np.zeros(200)
    out = [o.cpu().numpy() for o in B.rpdla_push(L, 0, _t(torch, tb), _t(torch, z0), _t(torch, z0),
                                                 _t(torch, z0), 1)]
    ref = O.push(OL, tb, z0, z0, z0, 1)
    Kg, fg = gpu_energy(B, torch, *out[:3])
    Ko, _, _, fo = O.epilogue(*ref[:3])
    ok, same_dir = energy_parity(Kg, fg, Ko, fo)
    assert ok.all() and same_dir.all()
    g = np.sqrt(1 + out[0] ** 2 + out[1] ** 2 + out[2] ** 2)
    # light-front invariant gamma - u_z = 1 up to the RK4 truncation error,
    # which at a0 ~ 22 and dt = T/200 reaches ~1e-4 gamma (the oracle shares it)
    viol = np.abs(g - out[2] - 1) / g
    assert viol.max() < 3e-4, viol.max()


def test_mixed_vs_fp64(env):
    """Mixed form against the FP64 form on the same slots: per-electron
    |dK|/K <= 1e-3 for the large majority and the ensemble mean within 0.1%.
    The ensemble is ~3.5e4 electrons: on a few thousand, one ill-conditioned
    electron of ~100 MeV off by a few percent moves the mean by 0.1% alone."""
    torch, B, O = env
    L, _ = _lasers(B, O, 5)
    n, K = 4000, 10
    x, y, z = B.rpdla_sample_atoms(0, 9, 0, n, 2 * L.w0, B.rpdla_rayleigh(L))
    tb = B.rpdla_ionize(L, 0, 9, 0, x, y, z, 1, K)
    a = [o.cpu().numpy() for o in B.rpdla_push(L, 0, tb, x, y, z, K)]
    b = [o.cpu().numpy() for o in B.rpdla_push(L, 1, tb, x, y, z, K)]
    fin = np.isfinite(tb.cpu().numpy())
    Ka, fa = gpu_energy(B, torch, *(v[fin] for v in a[:3]))
    Kb, fb = gpu_energy(B, torch, *(v[fin] for v in b[:3]))
    rel = np.abs(Kb - Ka) / Ka
    frac = np.mean(rel <= 1e-3)
    print(f"mixed: frac(|dK|/K <= 1e-3) = {frac:.4f}, mean dK/K = {Kb.mean() / Ka.mean() - 1:.2e}")
    # measured on this beam (1e21 W/cm^2, w0 3 um): 98.6% within 1e-3; the
    # rest are trajectories whose energy amplifies rounding (see DESIGN)
    assert np.median(rel) < 1e-6
    assert frac >= 0.98, frac
    assert abs(Kb.mean() / Ka.mean() - 1) <= 1e-3
    assert np.mean(fa == fb) >= 0.999


def test_mixed_vs_oracle(env):
    """The single-configuration mixed push against the double oracle's push of
    the same seeded inputs, electron by electron: |dK|/K <= 1e-3 for >= 98%
    of the electrons (the target of the mixed form; the rest amplify float
    rounding), median below 1e-6, the ensemble-mean energy within 0.1%, the
    same direction for >= 99.9%."""
    torch, B, O = env
    otb, g, ref, O, OL, _ = _push_case(env, 5, 150, prec=1)
    fin = np.isfinite(otb)
    for a in g:
        assert np.all(np.isnan(a[~fin])) and np.all(np.isfinite(a[fin]))
    Kg, fg = gpu_energy(B, torch, *(a[fin] for a in g[:3]))
    Ko, _, _, fo = O.epilogue(*(r[fin] for r in ref[:3]))
    rel = np.abs(Kg - Ko) / Ko
    mean_err = Kg.mean() / Ko.mean() - 1
    hist = np.histogram(np.log10(np.maximum(rel, 1e-17)), bins=np.arange(-17, 2))[0]
    print(f"mixed vs oracle: {fin.sum()} electrons, within 1e-3 {np.mean(rel <= 1e-3):.4f}, "
          f"median {np.median(rel):.1e}, mean energy {mean_err:.1e}, direction changes "
          f"{(fg != fo).sum()}; electrons per decade of |dK|/K from 1e-17: {hist.tolist()}")
    assert np.mean(rel <= 1e-3) >= 0.98
    assert np.median(rel) < 1e-6
    assert abs(mean_err) <= 1e-3
    assert (fg != fo).sum() <= allowed_failures(fin.sum()) + 1


def test_autotune_and_shape_independence(env):
    """The autotuner reports timings and stores a shape; results do not
    depend on the launch shape (bitwise)."""
    torch, B, O = env
    L, _ = _lasers(B, O, 5)
    rep = B.rpdla_autotune(L, 0, 4096, 1, 10)
    assert rep["field"] == 5 and len(rep["push_ms"]) == 6 and len(rep["ionize_ms"]) == 3
    n, K = 300, 10
    x, y, z = B.rpdla_sample_atoms(0, 4, 0, n, 2 * L.w0, B.rpdla_rayleigh(L))
    outs = []
    for blk, gf in ((64, 1), (256, 2), (128, 1)):
        B.rpdla_set_launch_shape(B.RPDLA_KERNEL_IONIZE, 5, 0, blk, 1)
        B.rpdla_set_launch_shape(B.RPDLA_KERNEL_PUSH, 5, 0, blk, gf)
        tb = B.rpdla_ionize(L, 0, 4, 0, x, y, z, 1, K)
        o = B.rpdla_push(L, 0, tb, x, y, z, K)
        outs.append([tb.cpu().numpy()] + [a.cpu().numpy() for a in o])
    B.rpdla_set_launch_shape(B.RPDLA_KERNEL_IONIZE, 5, 0, 256, 1)
    B.rpdla_set_launch_shape(B.RPDLA_KERNEL_PUSH, 5, 0, 256, 1)
    for other in outs[1:]:
        for a, b in zip(outs[0], other):
            assert np.array_equal(a, b, equal_nan=True)


def test_kernel_occupancy(env):
    """The push and ionize kernels keep every value in registers (no scratch)
    and reach the resident waves their launch bounds ask for."""
    torch, B, O = env
    want = {(B.RPDLA_KERNEL_PUSH, B.RPDLA_FP64): 4, (B.RPDLA_KERNEL_PUSH, B.RPDLA_MIXED): 7,
            (B.RPDLA_KERNEL_IONIZE, B.RPDLA_FP64): 3, (B.RPDLA_KERNEL_BATCHED_PUSH, B.RPDLA_FP64): 4,
            (B.RPDLA_KERNEL_BATCHED_PUSH, B.RPDLA_MIXED): 6}
    for (kind, prec), waves in want.items():
        r = B.rpdla_kernel_occupancy(kind, 5, prec)
        print(f"[occupancy] kind {kind} precision {prec}: {r}")
        assert 0 < r["vgprs"] <= 512 // waves
        assert r["scratch_bytes"] == 0
        assert r["waves_per_simd"] >= waves


def test_epilogue_parity(env):
    torch, B, O = env
    n = 5000
    u = SI.momenta(12, n)
    u[:3] = [[0, 0, 0], [0, 0, -2.0], [1e-9, 0, 0]]
    u[3] = np.nan
    K, th, ps, fw = (o.cpu().numpy() for o in B.rpdla_epilogue(*(_t(torch, u[:, i]) for i in range(3))))
    oK, oth, ops, ofw = O.epilogue(u[4:, 0], u[4:, 1], u[4:, 2])
    assert np.all(np.abs(K[4:] - oK) <= 1e-15 * oK + 1e-300)
    assert np.all(np.abs(th[4:] - oth) <= 1e-15) and np.all(np.abs(ps[4:] - ops) <= 1e-15)
    assert np.array_equal(fw[4:], ofw) and fw[3] == -1 and np.isnan(K[3])


def test_histogram_exact(env):
    torch, B, O = env
    rng = np.random.default_rng(11)
    n = 20000
    u = rng.normal(size=(n, 3)) * np.exp(rng.uniform(-6, 9, size=(n, 1)))
    tb = rng.normal(size=n)
    tb[rng.uniform(size=n) < 0.1] = np.inf
    u[rng.uniform(size=n) < 0.01, 2] = np.nan
    for angle, nE, nA in ((0, 256, 180), (1, 97, 33)):
        spec = B.rpdla_hist_spec(nE, nA, -3.0, 4.0, angle)
        c, t = B.rpdla_histogram(_t(torch, tb), _t(torch, u[:, 0]), _t(torch, u[:, 1]),
                                 _t(torch, u[:, 2]), spec)
        c2, t2 = B.rpdla_histogram(_t(torch, tb), _t(torch, u[:, 0]), _t(torch, u[:, 1]),
                                   _t(torch, u[:, 2]), spec, c, t)  # accumulates
        oc, ot = O.histogram(tb, u[:, 0], u[:, 1], u[:, 2], nE, nA, -3.0, 4.0, angle)
        assert np.array_equal(c2.cpu().numpy().astype(np.uint64), 2 * oc)
        assert np.array_equal(t2.cpu().numpy().astype(np.uint64), 2 * ot)


def test_end_to_end_small(env):
    """sample -> ionize -> push -> histogram on the GPU versus the oracle chain."""
    torch, B, O = env
    L, OL = _lasers(B, O, 5)
    n, K = 60, 10
    x, y, z = B.rpdla_sample_atoms(0, 0, 0, n, 2 * L.w0, B.rpdla_rayleigh(L))
    tb = B.rpdla_ionize(L, 0, 0, 0, x, y, z, 1, K)
    out = B.rpdla_push(L, 0, tb, x, y, z, K)
    spec = B.rpdla_hist_spec(256, 180, -3.0, 4.0, 0)
    c, t = B.rpdla_histogram(tb, *out[:3], spec)
    ox, oy, oz = O.sample_atoms(0, 0, 0, n, 2 * OL.w0, O.rayleigh(OL))
    otb = O.ionize(OL, 0, 0, 0, ox, oy, oz, 1, K)
    ref = O.push(OL, otb, ox, oy, oz, K)
    oc, ot = O.histogram(otb, *ref[:3], 256, 180, -3.0, 4.0, 0)
    _check_tb(tb.cpu().numpy(), otb, L.lambda_ / C_LIGHT)
    t = t.cpu().numpy().astype(np.uint64)
    assert t[4] == ot[4] and t[5] == ot[5] == 0
    # counts: identical up to electrons sitting on a bin edge or flipping direction
    diff = np.abs(c.cpu().numpy().astype(np.int64) - oc.astype(np.int64)).sum()
    assert diff <= 2 * allowed_failures(int(t[0] + t[1])) + 2


def test_edge_cases(env):
    torch, B, O = env
    L, OL = _lasers(B, O, 5)
    e = torch.empty(0, dtype=torch.float64, device="cuda")
    assert B.rpdla_ionize(L, 0, 0, 0, e, e, e, 1, 10).numel() == 0
    assert all(o.numel() == 0 for o in B.rpdla_push(L, 0, e, e, e, e, 10))
    # a weak pulse ionizes nothing: every slot unborn, every output NaN
    Lw = B.rpdla_laser_init_intensity(0.8e-6, 3e-6, 30e-15, 1e10)
    x, y, z = B.rpdla_sample_atoms(0, 0, 0, 33, 6e-6, 35e-6)
    tb = B.rpdla_ionize(Lw, 0, 0, 0, x, y, z, 1, 10)
    assert torch.isinf(tb).all()
    out = B.rpdla_push(Lw, 0, tb, x, y, z, 10)
    assert all(torch.isnan(o).all() for o in out)
    c, t = B.rpdla_histogram(tb, *out[:3], B.rpdla_hist_spec(8, 4, -3.0, 4.0, 0))
    assert t.cpu().tolist() == [0, 0, 0, 0, 330, 0] and int(c.sum()) == 0
    # a single atom, one state
    (x1s, y1s, z1s), (x1, y1, z1) = _atoms(torch, 40, 1)
    tb1 = B.rpdla_ionize(L, 0, 0, 0, x1, y1, z1, 1, 1)
    o1 = O.ionize(OL, 0, 0, 0, x1s, y1s, z1s, 1, 1)
    _check_tb(tb1.cpu().numpy(), o1, L.lambda_ / C_LIGHT)


def test_invalid_arguments(env):
    torch, B, O = env
    L, _ = _lasers(B, O, 5)
    x = torch.zeros(4, dtype=torch.float64, device="cuda")
    with pytest.raises(B.RpdlaError) as ei:
        B.rpdla_ionize(L, 0, 0, 0, x, x, x, 0, 3)
    assert ei.value.status == B.RPDLA_EINVAL
    bad = B.rpdla_laser_init_intensity(0.8e-6, 3e-6, 30e-15, 1e21)
    bad.dt = -1.0
    with pytest.raises(B.RpdlaError):
        B.rpdla_push(bad, 0, x, x, x, x, 1)
    with pytest.raises(B.RpdlaError):
        B.rpdla_push(L, 7, x, x, x, x, 1)
    with pytest.raises(B.RpdlaError):
        B.rpdla_histogram(x, x, x, x, B.rpdla_hist_spec(4, 4, 1.0, 1.0, 0))
    with pytest.raises(TypeError):
        B.rpdla_ionize(L, 0, 0, 0, x.float(), x, x, 1, 2)


@pytest.mark.parametrize("order", [5, 25])
def test_ionize_work_order_bitwise(env, order):
    """From 16,384 atoms on, rpdla_ionize hands the atoms to the lanes in the
    order of their work key (a radix sort), so that a wave holds atoms of
    alike windows.  Each atom's arithmetic is the same either way, so the
    birth times equal, bit for bit, those of calls below that size, which
    take the atoms in index order (the same atoms, addressed by
    first_atom)."""
    torch, B, O = env
    L, _ = _lasers(B, O, order)
    n, parts, seed, cfg = 20000, (0, 7000, 14000, 20000), 21, 4
    x, y, z = B.rpdla_sample_atoms(seed, cfg, 0, n, 2 * BEAM["w0"], B.rpdla_rayleigh(L))
    print(f"ionize in work order: field {order}, {n} atoms, states 1-10", flush=True)
    tb = B.rpdla_ionize(L, seed, cfg, 0, x, y, z, 1, 10).cpu().numpy()
    ref = np.concatenate([
        B.rpdla_ionize(L, seed, cfg, a, x[a:b].contiguous(), y[a:b].contiguous(),
                       z[a:b].contiguous(), 1, 10).cpu().numpy() for a, b in zip(parts, parts[1:])])
    torch.cuda.synchronize()
    born = np.isfinite(tb)
    assert 0 < born.sum() < tb.size
    assert np.array_equal(tb.view(np.uint64), ref.view(np.uint64))


def test_push_queue_parts_small_and_ragged(env):
    """The push draws slots from eight contiguous parts of the slot range (one
    per XCD) and moves on to the other parts when its own runs dry.  For slot
    counts below, at and around multiples of eight (several parts empty), every
    slot is pushed exactly once: outputs prefilled with a marker all change,
    and equal, bit for bit, the same slots of one launch over all of them."""
    torch, B, O = env
    L, _ = _lasers(B, O, 5)
    n_atoms, K = 130, 8
    x, y, z = B.rpdla_sample_atoms(3, 9, 0, n_atoms, 2 * BEAM["w0"], B.rpdla_rayleigh(L))
    tb = B.rpdla_ionize(L, 3, 9, 0, x, y, z, 1, K)
    full = [o.cpu().numpy() for o in B.rpdla_push(L, B.RPDLA_FP64, tb, x, y, z, K)]
    for n in (1, 2, 7, 8, 9, 15, 16, 17, 63, 65, 1000, n_atoms * K):
        print(f"push queue parts: {n} slots", flush=True)
        out = tuple(torch.full((n,), 12345.0, dtype=torch.float64, device="cuda") for _ in range(6))
        B.rpdla_push(L, B.RPDLA_FP64, tb[:n].contiguous(), x, y, z, K, out=out)
        torch.cuda.synchronize()
        for o, f in zip(out, full):
            a = o.cpu().numpy()
            assert not np.any(a == 12345.0), n
            assert np.array_equal(a.view(np.uint64), f[:n].view(np.uint64)), n
