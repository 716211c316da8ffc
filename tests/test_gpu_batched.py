"""Batched persistent sweep (one push launch over several configurations,
LDS configuration table, per-configuration queues, separate binning pass,
hipGraph chunk replay) against the
single-configuration path and the oracle."""
import sys

import numpy as np
import pytest

from gpu_common import allowed_failures, require_gpu

pytestmark = pytest.mark.gpu

SPEC = (64, 36, -3.0, 4.0, 0)


@pytest.fixture(scope="module")
def env(orc):
    torch = require_gpu()
    from paper_2509_01741_amd import binding as B
    return torch, B, orc


def _lasers(B):
    out = []
    for lam, P in ((0.8e-6, 0.5e15), (1.0e-6, 2e15), (2.0e-6, 1e15)):
        L = B.rpdla_laser_init_power(lam, 2 * lam, 10 * lam / 299792458.0, P)
        out.append(L)
    return out


def _single(B, torch, L, seed, cfg_id, n, K, spec):
    x, y, z = B.rpdla_sample_atoms(seed, cfg_id, 0, n, 2.0 * L.w0, B.rpdla_rayleigh(L))
    tb = B.rpdla_ionize(L, seed, cfg_id, 0, x, y, z, 1, K)
    out = B.rpdla_push(L, 0, tb, x, y, z, K)
    return B.rpdla_histogram(tb, *out[:3], spec), (x, y, z, tb, out)


def test_batched_equals_single_path(env):
    torch, B, O = env
    lasers = _lasers(B)
    spec = B.rpdla_hist_spec(*SPEC)
    n, K, base = 40, 10, 500
    counts, tallies = B.rpdla_run_batched(lasers, 3, base, n, n, 2.0, 1, K, 0, spec)
    for c, L in enumerate(lasers):
        (sc, st), _ = _single(B, torch, L, 3, base + c, n, K, spec)
        assert np.array_equal(st.cpu().numpy(), tallies[c].cpu().numpy()), c
        diff = np.abs(sc.cpu().numpy() - counts[c].cpu().numpy()).sum()
        assert diff == 0, (c, diff)
        assert int(st[4]) + int(st[0]) + int(st[1]) == n * K


def test_batched_graph_chunks(env):
    """Chunks of 15 atoms (graph captured once, replayed 3 times, last chunk
    partial) give exactly the one-chunk result; a second call reuses it."""
    torch, B, O = env
    lasers = _lasers(B)
    spec = B.rpdla_hist_spec(*SPEC)
    n, K = 40, 10
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        c1, t1 = B.rpdla_run_batched(lasers, 4, 7, n, n, 2.0, 1, K, 0, spec, stream=s)
        c3, t3 = B.rpdla_run_batched(lasers, 4, 7, n, 15, 2.0, 1, K, 0, spec, stream=s)
        ws = torch.empty(B.rpdla_batched_workspace_bytes(3, 15, 1, K), dtype=torch.uint8,
                         device="cuda")
        c4 = torch.zeros_like(c3)
        t4 = torch.zeros_like(t3)
        for _ in range(2):   # same arguments: cached graph, results accumulate
            B.rpdla_run_batched(lasers, 4, 7, n, 15, 2.0, 1, K, 0, spec, c4, t4, ws, stream=s)
    s.synchronize()
    assert np.array_equal(c1.cpu().numpy(), c3.cpu().numpy())
    assert np.array_equal(t1.cpu().numpy(), t3.cpu().numpy())
    assert np.array_equal(2 * c1.cpu().numpy(), c4.cpu().numpy())
    assert np.array_equal(2 * t1.cpu().numpy(), t4.cpu().numpy())


def test_batched_vs_oracle(env):
    torch, B, O = env
    lam, P = 1.0e-6, 2e15
    L = B.rpdla_laser_init_power(lam, 2 * lam, 10 * lam / 299792458.0, P)
    OL = O.laser_power(lam, 2 * lam, 10 * lam / 299792458.0, P)
    spec = B.rpdla_hist_spec(*SPEC)
    n, K = 30, 10
    counts, tallies = B.rpdla_run_batched([L], 5, 9, n, n, 2.0, 1, K, 0, spec)
    ox, oy, oz = O.sample_atoms(5, 9, 0, n, 2 * OL.w0, O.rayleigh(OL))
    otb = O.ionize(OL, 5, 9, 0, ox, oy, oz, 1, K)
    ref = O.push(OL, otb, ox, oy, oz, K)
    oc, ot = O.histogram(otb, *ref[:3], *SPEC)
    t = tallies[0].cpu().numpy().astype(np.uint64)
    assert t[4] == ot[4] and t[5] == 0
    nb = int(ot[0] + ot[1])
    assert abs(int(t[0]) - int(ot[0])) <= allowed_failures(nb) + 1
    diff = np.abs(counts[0].cpu().numpy().astype(np.int64) - oc.astype(np.int64)).sum()
    assert diff <= 2 * allowed_failures(nb) + 2


def test_batched_mixed_precision(env):
    torch, B, O = env
    lasers = _lasers(B)
    spec = B.rpdla_hist_spec(*SPEC)
    n, K = 40, 10
    c64, t64 = B.rpdla_run_batched(lasers, 2, 0, n, n, 2.0, 1, K, 0, spec)
    cmx, tmx = B.rpdla_run_batched(lasers, 2, 0, n, n, 2.0, 1, K, 1, spec)
    t64, tmx = t64.cpu().numpy(), tmx.cpu().numpy()
    assert np.array_equal(t64[:, 4], tmx[:, 4])            # same births (FP64 ionization)
    nb = t64[:, 0] + t64[:, 1]
    assert np.all(np.abs(t64[:, 0] - tmx[:, 0]) <= 0.02 * nb + 1)
    # energy spectra agree bin-for-bin up to electrons near bin edges
    d = np.abs(c64.cpu().numpy() - cmx.cpu().numpy()).sum(axis=(1, 2, 3))
    assert np.all(d <= 0.1 * nb + 2), d


def test_single_chunk_graph_replays(env):
    """A one-chunk sweep on a side stream is captured into a graph once and
    replayed: three calls with the same buffers, with the program's own eager
    work and synchronizations between them, each equal to the eager result on
    the null stream."""
    torch, B, O = env
    lasers = _lasers(B)
    spec = B.rpdla_hist_spec(*SPEC)
    n, K = 40, 10
    c0, t0 = B.rpdla_run_batched(lasers, 6, 11, n, n, 2.0, 1, K, 0, spec)   # null stream: eager
    torch.cuda.synchronize()
    g0 = B.rpdla_batched_graphs()
    s = torch.cuda.Stream()
    counts = torch.zeros_like(c0)
    tallies = torch.zeros_like(t0)
    ws = torch.empty(B.rpdla_batched_workspace_bytes(3, n, 1, K), dtype=torch.uint8, device="cuda")
    for rep in range(3):
        with torch.cuda.stream(s):
            counts.zero_()
            tallies.zero_()
            B.rpdla_run_batched(lasers, 6, 11, n, n, 2.0, 1, K, 0, spec, counts, tallies, ws,
                                stream=s)
        s.synchronize()
        assert float(torch.arange(1000, device="cuda", dtype=torch.float64).sum()) == 499500.0
        assert torch.equal(counts, c0) and torch.equal(tallies, t0), rep
        assert B.rpdla_batched_graphs() == g0 + 1


def test_chunk_ranges_add_up_to_the_whole_stream(env):
    """rpdla_run_batched_range: a 3-chunk stream run as chunk 0, then chunks
    1..2 (graph-replayed on a side stream), gives the counts, tallies and
    electron-steps of one whole call, and leaves the last chunk's arrays of the
    whole call."""
    torch, B, O = env
    lasers = _lasers(B)
    spec = B.rpdla_hist_spec(*SPEC)
    n, apc, K = 70, 25, 10                       # chunks of 25, 25 and 20 atoms
    ws_a = torch.empty(B.rpdla_batched_workspace_bytes(3, apc, 1, K), dtype=torch.uint8,
                       device="cuda")
    ws_b = torch.empty_like(ws_a)
    st_a = torch.zeros(3, dtype=torch.int64, device="cuda")
    st_b = torch.zeros(3, dtype=torch.int64, device="cuda")
    c_a, t_a = B.rpdla_run_batched(lasers, 6, 11, n, apc, 2.0, 1, K, 0, spec, workspace=ws_a,
                                   electron_steps=st_a)
    c_b, t_b = B.rpdla_run_batched(lasers, 6, 11, n, apc, 2.0, 1, K, 0, spec, workspace=ws_b,
                                   electron_steps=st_b, chunks=(0, 1))
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        B.rpdla_run_batched(lasers, 6, 11, n, apc, 2.0, 1, K, 0, spec, c_b, t_b, ws_b, stream=s,
                            electron_steps=st_b, chunks=(1, -1))
    s.synchronize()
    print(f"[batched] chunk ranges: {int(st_a.sum())} electron-steps whole, "
          f"{int(st_b.sum())} in parts", file=sys.stderr, flush=True)
    assert torch.equal(c_a, c_b) and torch.equal(t_a, t_b) and torch.equal(st_a, st_b)
    arr_a = B.batched_chunk_arrays(ws_a, 3, apc, 1, K)
    arr_b = B.batched_chunk_arrays(ws_b, 3, apc, 1, K)
    assert torch.equal(arr_a["x"][:, :20], arr_b["x"][:, :20])
    tb = arr_a["t_birth"][:, :20]
    assert torch.equal(tb, arr_b["t_birth"][:, :20])
    born = torch.isfinite(tb)                    # momenta are written for born slots only
    for k in ("ux", "uz"):
        assert torch.equal(arr_a[k][:, :20][born], arr_b[k][:, :20][born]), k
