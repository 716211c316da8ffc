"""The workloads besides the benchmark's, at their full sizes where a test can
afford it: the 64-configuration FP64 sweep (65,536 atoms each), the mixed
versus FP64 ensemble (1e6 atoms, 1e7 slots), and the large chunked mixed
sweep at its full chunk size.  Checked through properties that hold at any
size (batched equals the single-configuration path bit for bit, tallies
account for every slot, the mixed form's error statistics) and on sampled
atoms that the oracle recomputes from the seed with its own chain."""
import sys
import time

import numpy as np
import pytest

from gpu_common import C_LIGHT, allowed_failures, check_fp64, gpu_energy, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env(orc):
    torch = require_gpu()
    from paper_2509_01741_amd import binding as B, pipeline, workloads
    return torch, B, pipeline, workloads, orc


def _log(msg):
    print(f"[configs] {msg}", file=sys.stderr, flush=True)


def _single(B, L, seed, cfg_id, n, kf, kl, r_factor, precision, spec):
    x, y, z = B.rpdla_sample_atoms(seed, cfg_id, 0, n, r_factor * L.w0, B.rpdla_rayleigh(L))
    tb = B.rpdla_ionize(L, seed, cfg_id, 0, x, y, z, kf, kl)
    out = B.rpdla_push(L, precision, tb, x, y, z, kl - kf + 1)
    c, t = B.rpdla_histogram(tb, *out[:3], spec)
    return (c, t), (x, y, z, tb, out)


def _oracle_atoms(O, OL, seed, cfg_id, idx, r_factor, kf, kl):
    pos = [O.sample_atoms(seed, cfg_id, int(i), 1, r_factor * OL.w0, O.rayleigh(OL)) for i in idx]
    xs, ys, zs = (np.concatenate([p[j] for p in pos]) for j in range(3))
    otb = np.concatenate([O.ionize(OL, seed, cfg_id, int(i), xs[j:j + 1], ys[j:j + 1],
                                   zs[j:j + 1], kf, kl) for j, i in enumerate(idx)])
    return xs, ys, zs, otb


def _oracle_laser(O, rec):
    if "I" in rec:
        return O.laser_intensity(rec["lam"], rec["w0"], rec["tau"], rec["I"])
    return O.laser_power(rec["lam"], rec["w0"], rec["tau"], rec["P"])


def _batched_vs_single(torch, B, c, arr, tal_b, counts_b, single, n, K, label, exact=False):
    """Element by element: positions and birth times bit-identical (the same
    sampling and ionization arithmetic), final energies within 1e-8 of the
    single-configuration push for >= 99.9% of the electrons and the same
    direction for >= 99.9% (the two push kernels are separate compilations
    of the same arithmetic, so their rounding differs), unborn and NaN tallies
    equal."""
    from oracle import parity
    (sc, st), (x, y, z, tb, out) = single
    st = st.cpu().numpy()
    assert torch.equal(arr["x"][c, :n], x) and torch.equal(arr["z"][c, :n], z)
    assert torch.equal(arr["t_birth"][c, :n].reshape(-1), tb)
    assert st[4] == tal_b[c, 4] and st[5] == tal_b[c, 5] == 0         # unborn, NaN
    fin = torch.isfinite(tb)
    Kb, fb = gpu_energy(B, torch, *(arr[k][c, :n].reshape(-1)[fin] for k in ("ux", "uy", "uz")))
    Ks, fs = gpu_energy(B, torch, *(o[fin] for o in out[:3]))
    ok = parity.within(Kb, Ks)
    same = fb == fs
    nb = int(fin.sum())
    rel = np.abs(Kb - Ks) / Ks
    l1 = int((sc - counts_b[c]).abs().sum())
    _log(f"{label} cfg {c}: {nb} electrons; batched vs single: {(~ok).sum()} beyond 1e-8 "
         f"(median {np.median(rel):.1e}, max {rel.max():.1e}), {(~same).sum()} direction "
         f"changes, histogram L1 {l1}")
    assert (~ok).sum() <= allowed_failures(nb)
    assert (~same).sum() <= allowed_failures(nb)
    if exact:
        # the FP64 batched and single pushes compile to the same arithmetic
        for k, o in zip(("ux", "uy", "uz"), out[:3]):
            assert torch.equal(arr[k][c, :n].reshape(-1)[fin], o[fin]), (label, c, k)
        assert l1 == 0


def _oracle_check_batched(O, OL, torch, B, arr, c, atoms, seed, cfg_id, r_factor, kf, kl, first,
                          label, Kx=None, mixed=False):
    """Sampled atoms of the batched chunk (chunk start `first`) against the
    oracle: positions and birth times from the oracle's own sampling and
    ionization from the seed; FP64 energies by the rule of oracle/parity.py
    (the double oracle's push of the same inputs, and the extended-precision
    chain Kx when given); mixed energies against the double oracle."""
    K = kl - kf + 1
    idx = np.asarray(atoms)
    xs, ys, zs, otb = _oracle_atoms(O, OL, seed, cfg_id, first + idx, r_factor, kf, kl)
    loc = torch.as_tensor(idx, device="cuda")
    gx = [arr[k][c][loc].cpu().numpy() for k in ("x", "y", "z")]
    assert np.max(np.abs(gx[0] - xs)) <= 1e-20
    gtb = arr["t_birth"][c][loc].cpu().numpy().ravel()
    fin = np.isfinite(otb)
    assert np.array_equal(fin, np.isfinite(gtb))
    T = OL.lambda_ / C_LIGHT
    assert np.all(np.abs(gtb[fin] - otb[fin]) <= 1e-10 * np.maximum(np.abs(otb[fin]), T))
    g = [arr[k][c][loc].cpu().numpy().ravel()[fin] for k in ("ux", "uy", "uz")]
    Kg, fg = gpu_energy(B, torch, *g)
    if not mixed:
        return Kg, fg, gtb, gx
    ref = O.push(OL, gtb, *gx, K)
    Ko = O.epilogue(*(r[fin] for r in ref[:3]))[0]
    rel = np.abs(Kg - Ko) / Ko
    _log(f"{label}: {fin.sum()} electrons, mixed vs oracle median {np.median(rel):.1e}, "
         f"within 1e-3 {np.mean(rel <= 1e-3):.4f}, max {rel.max():.1e}")
    assert np.median(rel) < 1e-6 and np.mean(rel <= 1e-3) >= 0.98
    return Kg, fg, gtb, gx


@pytest.mark.timeout(900)
def test_sweep64_full_size(env):
    torch, B, P, W, O = env
    wl = W.SWEEP_FP64
    n, K = wl["atoms"], wl["k_last"] - wl["k_first"] + 1
    n_cfg = len(wl["lasers"])
    spec = P.hist_spec(wl["hist"])
    steps = torch.zeros(n_cfg, dtype=torch.int64, device="cuda")
    ws = torch.empty(B.rpdla_batched_workspace_bytes(n_cfg, n, wl["k_first"], wl["k_last"]),
                     dtype=torch.uint8, device="cuda")
    s = torch.cuda.Stream()
    t0 = time.time()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(s):
        e0.record(s)
        counts, tallies = P.run_sweep(wl, B.RPDLA_FP64, stream=s, workspace=ws,
                                      electron_steps=steps)
        e1.record(s)
    s.synchronize()
    batched_ms = e0.elapsed_time(e1)
    tal = tallies.cpu().numpy()
    _log(f"sweep64 FP64 full size: {time.time() - t0:.1f} s, {int(steps.sum()):.3e} electron-steps")
    assert np.all(tal[:, 0] + tal[:, 1] + tal[:, 4] + tal[:, 5] == n * K)
    assert np.all(tal[:, 5] == 0)
    assert np.all(counts.sum(dim=(1, 2, 3)).cpu().numpy() + tal[:, 2] + tal[:, 3]
                  == tal[:, 0] + tal[:, 1])
    arr = B.batched_chunk_arrays(ws, n_cfg, n, wl["k_first"], wl["k_last"])
    base = wl["cfg_id"] * 1000
    # every configuration through the single-configuration path too: element by
    # element against the batched sweep, and the same work timed both ways
    single_ms = 0.0
    for c in range(n_cfg):
        rec = wl["lasers"][c]
        L = P.laser_of(rec, wl["field_order"])
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        single = _single(B, L, wl["seed"], base + c, n, wl["k_first"], wl["k_last"],
                         wl["r_factor"], B.RPDLA_FP64, spec)
        b.record()
        b.synchronize()
        single_ms += a.elapsed_time(b)
        _batched_vs_single(torch, B, c, arr, tal, counts, single, n, K, "sweep64", exact=True)
        del single
    _log(f"sweep64 FP64, the same work: batched sweep {batched_ms / 1e3:.2f} s, the 64 "
         f"configurations one by one through the single-configuration path {single_ms / 1e3:.2f} s "
         f"(batched / single = {batched_ms / single_ms:.3f})")
    # every configuration: 64 sampled atoms against the oracle, element by
    # element, under the FP64 rule (pooled over the configurations)
    from golden.make_extended_refs import load
    from oracle import parity
    Kx_all, atoms_all, cfg_ids, cfgs = load("rp_ne_sweep64_sampled")
    pool = {k: [] for k in ("Kg", "fg", "Kop", "fop", "Kx")}
    t0 = time.time()
    for j, c in enumerate(cfgs):
        c = int(c)
        assert int(cfg_ids[j]) == base + c
        OL = _oracle_laser(O, wl["lasers"][c])
        OL.field = wl["field_order"]
        Kg, fg, gtb, gx = _oracle_check_batched(O, OL, torch, B, arr, c, atoms_all[j].astype(np.int64),
                                                wl["seed"], base + c, wl["r_factor"], wl["k_first"],
                                                wl["k_last"], 0, f"sweep64 batched cfg {c}")
        fin = np.isfinite(gtb)
        Kx = Kx_all[j].ravel()
        assert np.array_equal(np.isfinite(Kx), fin)
        ref = O.push(OL, gtb, *gx, K)
        Kop, _, _, fop = O.epilogue(*(r[fin] for r in ref[:3]))
        for k, v in (("Kg", Kg), ("fg", fg), ("Kop", Kop), ("fop", fop), ("Kx", Kx[fin])):
            pool[k].append(v)
        mo = int((~parity.within(Kg, Kop)).sum())
        mx = int((~parity.within(Kg, Kx[fin])).sum())
        _log(f"sweep64 cfg {c}: {fin.sum()} electrons of {atoms_all.shape[1]} atoms; beyond 1e-8 "
             f"of the double oracle {mo}, of the extended oracle {mx}, direction changes "
             f"{int((fg != fop).sum())} ({time.time() - t0:.0f} s)")
    from gpu_common import check_fp64_values
    check_fp64_values(*(np.concatenate(pool[k]) for k in ("Kg", "fg", "Kop", "fop")),
                      Kx=np.concatenate(pool["Kx"]),
                      label=f" sweep64 batched, {len(cfgs)} configurations x {atoms_all.shape[1]} atoms")


def test_mixed_vs_fp64_full_size(env):
    torch, B, P, W, O = env
    wl = W.MIXED_AB
    ens = P.Ensemble(wl, precision=B.RPDLA_FP64)
    ens.sample()
    ens.ionize()
    ens.push()
    mixed = B.rpdla_push(ens.L, B.RPDLA_MIXED, ens.tb, ens.x, ens.y, ens.z, ens.K)
    torch.cuda.synchronize()
    fin = torch.isfinite(ens.tb)
    K64, f64 = (torch.as_tensor(a, device="cuda") for a in
                gpu_energy(B, torch, *(o[fin] for o in ens.out[:3])))
    Kmx, fmx = (torch.as_tensor(a, device="cuda") for a in
                gpu_energy(B, torch, *(o[fin] for o in mixed[:3])))
    rel = ((Kmx - K64).abs() / K64).double()
    frac = float((rel <= 1e-3).double().mean())
    mean_err = float(Kmx.double().mean() / K64.double().mean() - 1)
    same = float((f64 == fmx).double().mean())
    hist = np.histogram(np.log10(np.maximum(rel.cpu().numpy(), 1e-17)), bins=np.arange(-17, 2))[0]
    _log(f"mixed vs FP64, {int(fin.sum())} electrons: frac(<=1e-3) {frac:.5f}, median "
         f"{float(rel.median()):.2e}, mean energy {mean_err:.2e}, same direction {same:.6f}; "
         f"electrons per decade of |dK|/K from 1e-17 to 10: {hist.tolist()}")
    assert float(rel.median()) < 1e-6
    assert frac >= 0.999
    assert abs(mean_err) <= 1e-4
    assert same >= 0.9999
    # the FP64 form on sampled atoms, recomputed by the oracle from the seed
    from golden.make_extended_refs import load
    rec = wl["lasers"][0]
    OL = _oracle_laser(O, rec)
    OL.field = wl["field_order"]
    n, K = ens.n, ens.K
    Kx, atoms, _, _ = load("rp_ne_mixed_1m_sampled")
    idx = atoms[0].astype(np.int64)
    xs, ys, zs, otb = _oracle_atoms(O, OL, wl["seed"], wl["cfg_id"], idx, wl["r_factor"],
                                    wl["k_first"], wl["k_last"])
    gtb = ens.tb.reshape(n, K)[torch.as_tensor(idx, device="cuda")].cpu().numpy().ravel()
    ofin = np.isfinite(otb)
    assert np.array_equal(ofin, np.isfinite(gtb))
    T = rec["lam"] / C_LIGHT
    assert np.all(np.abs(gtb[ofin] - otb[ofin]) <= 1e-10 * np.maximum(np.abs(otb[ofin]), T))
    sl = torch.as_tensor((idx[:, None] * K + np.arange(K)[None, :]).ravel(), device="cuda")
    Kg, fg = gpu_energy(B, torch, *(o[sl].cpu().numpy()[ofin] for o in ens.out[:3]))
    gx = [a[torch.as_tensor(idx, device="cuda")].cpu().numpy() for a in (ens.x, ens.y, ens.z)]
    Kx = Kx[0].ravel()
    assert np.array_equal(np.isfinite(Kx), ofin)
    check_fp64(O, OL, Kg, fg, gtb, *gx, K, Kx=Kx[ofin], label=" mixed-ab FP64")


def test_large_chunked_mixed_full_chunk(env):
    """Two of the large sweep's configurations streamed in chunks of the full
    chunk size (1e6 atoms, then a 37-atom chunk replayed from the captured
    graph): every slot accounted for, births and directions as in the
    single-configuration mixed path, and the last chunk's electrons against
    the oracle's own chain."""
    torch, B, P, W, O = env
    wl = dict(W.LARGE_MIXED)
    wl["lasers"] = [wl["lasers"][0], wl["lasers"][-1]]
    apc = wl["chunk"]
    n = apc + 37
    K = wl["k_last"] - wl["k_first"] + 1
    spec = P.hist_spec(wl["hist"])
    ws = torch.empty(B.rpdla_batched_workspace_bytes(2, apc, wl["k_first"], wl["k_last"]),
                     dtype=torch.uint8, device="cuda")
    s = torch.cuda.Stream()
    t0 = time.time()
    with torch.cuda.stream(s):
        counts, tallies = P.run_sweep(wl, B.RPDLA_MIXED, atoms_per_cfg=n, stream=s, workspace=ws)
    s.synchronize()
    _log(f"large mixed, 2 configs x {n} atoms in chunks of {apc}: {time.time() - t0:.1f} s")
    tal = tallies.cpu().numpy()
    assert np.all(tal[:, 0] + tal[:, 1] + tal[:, 4] + tal[:, 5] == n * K)
    arr = B.batched_chunk_arrays(ws, 2, apc, wl["k_first"], wl["k_last"])
    base = wl["cfg_id"] * 1000
    for c, rec in enumerate(wl["lasers"]):
        L = P.laser_of(rec, wl["field_order"])
        (sc, st), (sx, sy, sz, stb, sout) = _single(B, L, wl["seed"], base + c, n, wl["k_first"],
                                                   wl["k_last"], wl["r_factor"], B.RPDLA_MIXED,
                                                   spec)
        st = st.cpu().numpy()
        born = int(st[0] + st[1])
        l1 = int((sc - counts[c]).abs().sum())
        bwd = tal[c, 1] / max(1, tal[c, 0] + tal[c, 1])
        # the last chunk element by element against the single-configuration
        # mixed path (same births; separate compilations of the same float
        # arithmetic, so energies agree to the mixed form's own rounding)
        sl = slice(apc * K, n * K)
        assert torch.equal(arr["t_birth"][c, :37].reshape(-1), stb[sl])
        fin = torch.isfinite(stb[sl])
        Kb, fb = gpu_energy(B, torch, *(arr[k][c, :37].reshape(-1)[fin] for k in ("ux", "uy", "uz")))
        Ks, fs = gpu_energy(B, torch, *(o[sl][fin] for o in sout[:3]))
        rel = np.abs(Kb - Ks) / Ks
        _log(f"large cfg {c} (lambda {rec['lam'] * 1e6:.1f} um, w0 {rec['w0'] * 1e6:.1f} um): "
             f"backward fraction {bwd:.4f}; whole ensemble vs single path: forward "
             f"{int(tal[c, 0])} vs {int(st[0])}, histogram L1 {l1} of {born}; last chunk: "
             f"{int(fin.sum())} electrons, max |dK|/K {rel.max():.1e}, direction changes "
             f"{int((fb != fs).sum())}")
        assert st[4] == tal[c, 4] and st[5] == tal[c, 5] == 0
        # two float compilations differ by the mixed form's rounding (~1e-7),
        # which the ill-conditioned tail amplifies past 1e-3 for about one
        # electron in a hundred (the tail the mixed-vs-FP64 comparison shows)
        assert (rel <= 1e-3).mean() >= 0.98, (rel <= 1e-3).mean()
        assert int((fb != fs).sum()) <= allowed_failures(int(fin.sum())) + 1
        assert abs(int(tal[c, 0]) - int(st[0])) <= allowed_failures(born) + 1
        assert l1 <= 0.01 * born + 4
        OL = _oracle_laser(O, rec)
        OL.field = wl["field_order"]
        _oracle_check_batched(O, OL, torch, B, arr, c, np.arange(37), wl["seed"], base + c,
                              wl["r_factor"], wl["k_first"], wl["k_last"], apc,
                              f"large batched cfg {c} last chunk", mixed=True)
