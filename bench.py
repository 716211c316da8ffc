"""Benchmark: one step = the whole hot path over the full FP64 ensemble
(1e6 neon atoms, charge states 1..10, ~1e7 electron slots, radially polarized
focus 0.8 um / w0 3 um / 30 fs / 1e21 W/cm^2, field order 5, dt = T/200):
sample atoms -> ionization times -> FP64 push -> energy-angle histogram, all
on one MI355X.  Prints ONE JSON line on stdout; progress goes to stderr.

value = electron-steps of the step / wall time of the step (GPU events around
the timed region, inputs resident in HBM).  The same run also times the mixed
FP32/FP64 push on the same birth times and reports its speedup and energy
error against the FP64 push, the FP64 push kernel's roofline fraction
(algorithmic FP64 FLOPs per electron-step x electron-steps / kernel time,
against the MI355X FP64 vector peak) and the CPU oracle's rate on a bounded
sample of the same ensemble.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

C_LIGHT = 299792458.0
# FP64 floating-point operations of one RK4 step of one electron with the
# order-5 radial field, counted from the implemented formulas (mul, add and
# the hardware reciprocal / reciprocal-square-root estimates = 1 FLOP,
# fma = 2; the carrier, exponential, reciprocal and reciprocal square root
# at the operations of their polynomial and Newton sequences).  Per
# right-hand side: field 183 (position terms 8, reciprocal 7, phase and
# envelope arguments 7, exponential 29, half-angle carrier of the two-part
# phase 39, amplitude with cos = 1 - sigma^2 and sin = sigma kappa 7,
# w-recurrence 30, brackets 54, axial and radial scales 2) + Lorentz 27
# (gamma 15, velocity 3, force from the radial parts 9); per step 4 x 210 +
# RK4 115 (stage arguments 48, slope sums 24, increments 15, compensated sums
# of the seven state variables 28) = 955.
ALGO_FLOP_PER_STEP = 955.0
FP64_VECTOR_PEAK_TFLOPS = 78.6
# Published FP32 vector peak (it counts packed FP32 FMAs; the kernels are
# compiled without packed FP32).
FP32_VECTOR_PEAK_TFLOPS = 157.3
PROFILE_COUNTERS_FILE = os.path.join(ROOT, "profiles", "push_ionize_rp_ne_fp64_1m_counters.json")
# two counter passes (one rocprofv3 run each): instruction and FLOP counts,
# then cycles, issue and lane activity
COUNTERS = ["SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_VALU_FLOPS_FP64", "SQ_INSTS_VALU_FLOPS_FP32",
            "SQ_INSTS_VALU_FMA_F64", "SQ_INSTS_VALU_MUL_F64", "SQ_INSTS_VALU_ADD_F64",
            "SQ_INSTS_VALU_TRANS_F32"]
COUNTERS2 = ["GRBM_GUI_ACTIVE", "GRBM_COUNT", "SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_BUSY_CU_CYCLES",
             "SQ_ACTIVE_INST_VALU", "SQ_THREAD_CYCLES_VALU", "SQ_WAIT_INST_ANY", "SQ_WAVE_CYCLES"]
COUNTERS_RUN = ("rocprofv3 --pmc {ctrs} --output-format csv -d $R/gpurun_out/{d} -o run -- python3 "
                "$R/bench.py --steps 1 --warmup 0 --no-cpu-baseline --no-adaptive --no-batched "
                "--no-mixed-workload")
COUNTERS_CMD = COUNTERS_RUN.format(ctrs=" ".join(COUNTERS), d="pmcS")
COUNTERS2_CMD = COUNTERS_RUN.format(ctrs=" ".join(COUNTERS2), d="pmcC")
COUNTER_KERNELS = (("fp64", "push_kernel<5, rpdla::ElecF64>"),
                   ("mixed", "push_kernel<5, rpdla::ElecMixed>"),
                   ("ionize", "ionize_kernel<5>"))
PROFILE_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "push_fp64_rp_ne_fp64_1m_traffic.json")
# sources that define the FP64 push kernel (its traffic figure is tied to them)
KERNEL_SOURCES = ["rpdla_device.hpp", "rpdla_kernels.hpp", "rpdla_fastmath.hpp",
                  "rpdla_fastmath_coeffs.hpp"]


def kernel_source_hash():
    """Hash of the kernel sources: measured traffic is reported only for the
    kernel build it was measured on."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2509_01741_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def electron_steps(tb, z, K, L):
    """Number of RK4 steps the push takes for every born slot (ceil of the
    window remainder over dt), summed -- the unit of the metric."""
    import torch
    fin = torch.isfinite(tb)
    zz = z.repeat_interleave(K)
    tz = zz / C_LIGHT if L.window == 0 else torch.zeros_like(zz)
    n = torch.ceil(((tz + L.t_after) - tb) / L.dt)
    return int(n[fin].clamp(min=0).sum().item()), int(fin.sum().item())


# Atoms of the benchmark ensemble (the first ones, by index) on which the
# oracle runs: its chain is timed for the CPU baseline and its results are
# compared with the GPU's; the extended-precision reference for them is
# stored under tests/golden (rp_ne_fp64_1m_head, 1200 atoms).
ORACLE_SAMPLE_ATOMS = 1000


def cpu_model():
    """The host CPU as /proc/cpuinfo names it, with its family / model /
    stepping numbers (a virtual machine may report only a generic name)."""
    info = {}
    try:
        for line in open("/proc/cpuinfo"):
            if ":" in line:
                k, v = (t.strip() for t in line.split(":", 1))
                if k in ("model name", "cpu family", "model", "stepping") and k not in info:
                    info[k] = v
            if not line.strip() and info:
                break
    except OSError:
        return None
    if "model name" not in info:
        return None
    ids = [f"{k} {info[k]}" for k in ("cpu family", "model", "stepping") if k in info]
    return info["model name"] + (f" ({', '.join(ids)})" if ids else "")


def kinetic_mev(u):
    import numpy as np
    u2 = u[0] ** 2 + u[1] ** 2 + u[2] ** 2
    return 0.51099895 * u2 / (np.sqrt(1.0 + u2) + 1.0)


def cpu_baseline(ens, mixed_out=None):
    """The oracle's whole chain (sampling, ionization, push, kinetic energy)
    over the first ORACLE_SAMPLE_ATOMS atoms of the same ensemble, timed on
    the host's cores; then its results against the GPU's (fp64_vs_oracle)."""
    import numpy as np
    import oracle as O
    wl = ens.wl
    rec = wl["lasers"][0]
    OL = O.laser_intensity(rec["lam"], rec["w0"], rec["tau"], rec["I"])
    OL.field = ens.L.field
    kf, kl = wl["k_first"], wl["k_last"]
    K = kl - kf + 1
    na = min(ORACLE_SAMPLE_ATOMS, ens.n)
    t0 = time.perf_counter()
    ch = O.chain(OL, wl["seed"], wl["cfg_id"], np.arange(na), wl["r_factor"] * OL.w0,
                 O.rayleigh(OL), kf, kl)
    secs = time.perf_counter() - t0
    fin = np.isfinite(ch["t_birth"])
    steps = float(np.ceil((np.repeat(ch["z"], K)[fin] / C_LIGHT + OL.t_after - ch["t_birth"][fin])
                          / OL.dt).sum())
    base = dict(value=steps / secs, unit="electron-steps/s", cores=O.num_threads(),
                nproc=os.cpu_count(), cpu_model=cpu_model(), kind="oracle",
                sample=f"the oracle's whole chain (sampling, ionization, FP64 push) over the first "
                       f"{na} atoms of the same ensemble: {int(fin.sum())} electrons, "
                       f"{int(steps)} electron-steps in {secs:.1f} s")
    try:
        parity = fp64_vs_oracle(ens, OL, K, na, ch, mixed_out)
    except Exception as e:  # a reported statistic only
        log(f"FP64 vs oracle statistics unavailable: {e!r}")
        parity = None
    return base, parity


def fp64_vs_oracle(ens, OL, K, na, ch, mixed_out=None):
    """The GPU's results for the oracle's sample against the oracle, every
    electron classified by the rule of oracle/parity.py: birth times; final
    energies against the double oracle's push of the GPU's own inputs and
    against the extended-precision oracle's chain (stored reference);
    directions; the mixed form against the extended reference."""
    import numpy as np
    import oracle as O
    from oracle import parity
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from golden.make_extended_refs import load
    n = na * K
    tg = ens.tb[:n].cpu().numpy()
    ug = [o[:n].cpu().numpy() for o in ens.out[:3]]
    gx = [a[:na].cpu().numpy() for a in (ens.x, ens.y, ens.z)]
    T = OL.lambda_ / C_LIGHT
    fo, fg = np.isfinite(ch["t_birth"]), np.isfinite(tg)
    both = fo & fg
    dt_rel = np.abs(ch["t_birth"][both] - tg[both]) / np.maximum(np.abs(ch["t_birth"][both]), T)
    Kg, dirg = kinetic_mev([u[fg] for u in ug]), ug[2][fg] > 0
    ref = O.push(OL, tg, *gx, K)
    Kop, dirop = kinetic_mev([u[fg] for u in ref[:3]]), ref[2][fg] > 0
    Kx_all, atoms, _, _ = load("rp_ne_fp64_1m_head")
    Kx = Kx_all[0][:na].ravel()
    assert np.array_equal(np.isfinite(Kx), fo)
    v = parity.fp64_energy_verdict(Kg, dirg, Kop, dirop, Kx=Kx[fg], Koc=ch["K"][fg])
    out = dict(electrons=int(fg.sum()), born_mismatch=int((fo != fg).sum()),
               birth_time_max_rel=float(dt_rel.max()) if dt_rel.size else 0.0,
               energy_rule=v, raw_chain_frac_le_1e8=float(parity.within(Kg, ch["K"][fg]).mean()),
               note="energy_rule: oracle/parity.py -- GPU vs the double oracle's push of the "
                    "same inputs, GPU vs the extended-precision oracle (every electron), "
                    "directions; raw_chain = GPU chain vs the double oracle's own chain")
    if mixed_out is not None:
        um = [o[:n].cpu().numpy() for o in mixed_out[:3]]
        Km = kinetic_mev([u[fg] for u in um])
        rel = np.abs(Km - Kx[fg]) / Kx[fg]
        out["mixed_vs_extended"] = dict(
            frac_rel_err_le_1e3=float(np.mean(rel <= 1e-3)), median_rel_err=float(np.median(rel)),
            mean_energy_rel_err=float(Km.mean() / Kx[fg].mean() - 1),
            hist_decades_from_1e17=np.histogram(np.log10(np.maximum(rel, 1e-17)),
                                                  bins=np.arange(-17, 2))[0].tolist())
    return out


def rel_err_histogram(rel):
    """Electrons per decade of relative error, from 1e-17 to 10 (the first bin
    also holds exact agreement), as a list of 18 counts."""
    import torch
    lg = torch.log10(rel.double().clamp(min=1e-17)).clamp(max=0.999)
    return torch.histc(lg, bins=18, min=-17.0, max=1.0).long().cpu().tolist()


def quantile_sorted(x, q):
    """q-quantile of a 1-D tensor by sorting (any length)."""
    v = x.double().sort().values
    return float(v[min(v.numel() - 1, int(q * v.numel()))].item())


def measure_mixed_workload(wl):
    """FP64 and mixed push of one full single-laser ensemble (the mixed form's
    own workload: 1 PW into w0 = 1.5 um): times, speedup, mixed-vs-FP64
    energy errors."""
    import torch
    from paper_2509_01741_amd import binding as B
    from paper_2509_01741_amd import pipeline
    ens = pipeline.Ensemble(wl, precision=B.RPDLA_FP64)
    ens.sample()
    ens.ionize()
    torch.cuda.synchronize()
    ev = lambda: torch.cuda.Event(enable_timing=True)
    outs = tuple(torch.empty_like(o) for o in ens.out)
    a, b, c = ev(), ev(), ev()
    a.record()
    B.rpdla_push(ens.L, B.RPDLA_FP64, ens.tb, ens.x, ens.y, ens.z, ens.K, ens.out)
    b.record()
    B.rpdla_push(ens.L, B.RPDLA_MIXED, ens.tb, ens.x, ens.y, ens.z, ens.K, outs)
    c.record()
    torch.cuda.synchronize()
    ms64, msmx = a.elapsed_time(b), b.elapsed_time(c)
    steps, born = electron_steps(ens.tb, ens.z, ens.K, ens.L)
    fin = torch.isfinite(ens.tb)

    def kin(o):
        u2 = o[0][fin] ** 2 + o[1][fin] ** 2 + o[2][fin] ** 2
        return 0.51099895 * u2 / (torch.sqrt(1 + u2) + 1), o[2][fin] > 0

    K64, f64 = kin(ens.out)
    Kmx, fmx = kin(outs)
    rel = (Kmx - K64).abs() / K64
    return dict(workload=wl["name"], atoms=ens.n, born_electrons=born, electron_steps=steps,
                fp64_push_ms=round(ms64, 2), mixed_push_ms=round(msmx, 2),
                fp64_electron_steps_per_s=steps / (ms64 * 1e-3),
                mixed_electron_steps_per_s=steps / (msmx * 1e-3), speedup=ms64 / msmx,
                frac_rel_err_le_1e3=float((rel <= 1e-3).double().mean().item()),
                median_rel_err=float(rel.median().item()),
                p99_rel_err=quantile_sorted(rel, 0.99),
                mean_energy_rel_err=float((Kmx.double().mean() / K64.double().mean() - 1).item()),
                same_direction=float((f64 == fmx).double().mean().item()),
                rel_err_hist_decades_from_1e17=rel_err_histogram(rel))


def measure_sweep(wl, precision, atoms_per_cfg, atoms_per_chunk, chunks_total=None):
    """One timed batched sweep on a side stream (its chunk sequence captured
    into a hipGraph at the call and replayed per chunk; the capture is inside
    the timed region); electron-steps counted by the library."""
    import torch
    from paper_2509_01741_amd import binding as B
    from paper_2509_01741_amd import pipeline
    n_cfg = len(wl["lasers"])
    spec = pipeline.hist_spec(wl["hist"])
    dev = torch.device("cuda")
    counts = torch.zeros((n_cfg, 2, spec.nE, spec.nA), dtype=torch.int64, device=dev)
    tallies = torch.zeros((n_cfg, B.RPDLA_NTALLY), dtype=torch.int64, device=dev)
    steps = torch.zeros(n_cfg, dtype=torch.int64, device=dev)
    ws = torch.empty(B.rpdla_batched_workspace_bytes(n_cfg, atoms_per_chunk, wl["k_first"],
                                                     wl["k_last"]), dtype=torch.uint8, device=dev)
    st = torch.cuda.Stream()
    ev = lambda: torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    g0 = B.rpdla_batched_graphs()
    with torch.cuda.stream(st):
        a, b = ev(), ev()
        a.record(st)
        pipeline.run_sweep(wl, precision, atoms_per_cfg, atoms_per_chunk, stream=st, workspace=ws,
                           counts=counts, tallies=tallies, electron_steps=steps)
        b.record(st)
    st.synchronize()
    ms = a.elapsed_time(b)
    n_steps = int(steps.sum().item())
    tal = tallies.sum(0).cpu().tolist()
    bwd = tallies[:, 1].double() / (tallies[:, 0] + tallies[:, 1]).clamp(min=1).double()
    chunks = -(-atoms_per_cfg // atoms_per_chunk)
    return dict(workload=wl["name"], precision="mixed" if precision == B.RPDLA_MIXED else "f64",
                configs=n_cfg, atoms_per_cfg=atoms_per_cfg, atoms_per_chunk=atoms_per_chunk,
                chunks_timed=chunks, chunks_total=chunks_total or chunks,
                graph_captured=B.rpdla_batched_graphs() > g0, ms=round(ms, 2),
                electron_steps=n_steps, electron_steps_per_s=n_steps / (ms * 1e-3),
                born=int(tal[0] + tal[1]), backward_fraction_min_max=[float(bwd.min()), float(bwd.max())],
                occupancy=occupancy(2, int(wl["field_order"]), precision))


def measure_stream(wl, precision):
    """The whole chunked stream of a batched workload (every chunk of every
    configuration), run chunk by chunk with rpdla_run_batched_range on one
    side stream so that each chunk reports as it ends; the chunks are the
    ones one rpdla_run_batched call would run."""
    import torch
    from paper_2509_01741_amd import binding as B
    from paper_2509_01741_amd import pipeline
    n_cfg = len(wl["lasers"])
    spec = pipeline.hist_spec(wl["hist"])
    dev = torch.device("cuda")
    n, apc = int(wl["atoms"]), int(wl["chunk"])
    n_chunks = -(-n // apc)
    lasers = [pipeline.laser_of(r, wl.get("field_order", 5)) for r in wl["lasers"]]
    counts = torch.zeros((n_cfg, 2, spec.nE, spec.nA), dtype=torch.int64, device=dev)
    tallies = torch.zeros((n_cfg, B.RPDLA_NTALLY), dtype=torch.int64, device=dev)
    steps = torch.zeros(n_cfg, dtype=torch.int64, device=dev)
    ws = torch.empty(B.rpdla_batched_workspace_bytes(n_cfg, apc, wl["k_first"], wl["k_last"]),
                     dtype=torch.uint8, device=dev)
    st = torch.cuda.Stream()
    ev = lambda: torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    total_ms = 0.0
    for i in range(n_chunks):
        a, b = ev(), ev()
        with torch.cuda.stream(st):
            a.record(st)
            B.rpdla_run_batched(lasers, wl["seed"], wl["cfg_id"] * 1000, n, apc, wl["r_factor"],
                                wl["k_first"], wl["k_last"], precision, spec, counts, tallies, ws,
                                stream=st, electron_steps=steps, chunks=(i, 1))
            b.record(st)
        b.synchronize()
        total_ms += a.elapsed_time(b)
        log(f"stream {wl['name']}: chunk {i + 1}/{n_chunks} {a.elapsed_time(b) / 1e3:.1f} s")
    n_steps = int(steps.sum().item())
    tal = tallies.sum(0).cpu().tolist()
    bwd = tallies[:, 1].double() / (tallies[:, 0] + tallies[:, 1]).clamp(min=1).double()
    return dict(workload=wl["name"], precision="mixed" if precision == B.RPDLA_MIXED else "f64",
                configs=n_cfg, atoms_per_cfg=n, atoms_per_chunk=apc, chunks=n_chunks,
                ms=round(total_ms, 2), electron_steps=n_steps,
                electron_steps_per_s=n_steps / (total_ms * 1e-3), born=int(tal[0] + tal[1]),
                unborn=int(tal[4]), nan=int(tal[5]),
                backward_fraction_per_config=[round(float(v), 6) for v in bwd.cpu().tolist()])


PUSH_KERNEL_NAME = "push_kernel<5, rpdla::ElecF64>"
TRAFFIC_CMD = ("rocprofv3 --pmc {ctr} --output-format csv -d $R/gpurun_out/{d} -o run -- python3 "
               "$R/bench.py --steps 1 --warmup 0 --no-cpu-baseline --no-mixed --no-adaptive "
               "--no-batched --copy-ref-mib 512")


def _counter_rows(d, counter):
    """(kernel name, summed counter value) per dispatch from a rocprofv3
    --pmc csv output directory."""
    import csv
    import glob
    rows = []
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                if r.get("Counter_Name") == counter:
                    rows.append((r["Kernel_Name"], float(r["Counter_Value"])))
    if not rows:
        raise SystemExit(f"no {counter} rows under {d}")
    return rows


def write_traffic_summary(fetch_dir, write_dir, atoms=1_000_000, copy_mib=512, slots_per_atom=10,
                          out_json=PROFILE_TRAFFIC_FILE):
    """Turn the FETCH_SIZE and WRITE_SIZE runs (TRAFFIC_CMD) into the push
    kernel's HBM bytes per launch, scaled by what the same counters read for
    the plain copy of copy_mib MiB, and write out_json and the .md beside it
    (profiles/*_traffic.{json,md} by default)."""
    out = {}
    for counter, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        rows = _counter_rows(d, counter)
        copy = [v for k, v in rows if "copyBuffer" in k or "copy" in k.lower()]
        push = [v for k, v in rows if PUSH_KERNEL_NAME in k]
        ion = [v for k, v in rows if "ionize_kernel<5>" in k]
        if not copy or len(push) != 1:
            raise SystemExit(f"{counter}: need one copy and one push dispatch, got {len(copy)}, "
                             f"{len(push)}")
        out[counter] = dict(copy_kib=max(copy), push_kib=push[0], ionize_kib=ion[0] if ion else None)
    ref_kib = copy_mib * 1024.0
    f_scale = out["FETCH_SIZE"]["copy_kib"] / ref_kib
    w_scale = out["WRITE_SIZE"]["copy_kib"] / ref_kib
    rd = out["FETCH_SIZE"]["push_kib"] * 1024.0 / f_scale
    wr = out["WRITE_SIZE"]["push_kib"] * 1024.0 / w_scale
    algo = atoms * slots_per_atom * (8 + 48) + atoms * 24
    rec = dict(kernel=PUSH_KERNEL_NAME, workload="rp_ne_fp64_1m", atoms=atoms,
               bytes_per_launch=rd + wr, read_bytes=rd, write_bytes=wr, algorithmic_bytes=algo,
               fetch_scale=f_scale, write_scale=w_scale, kernel_source_hash=kernel_source_hash(),
               command=TRAFFIC_CMD.format(ctr="FETCH_SIZE (then WRITE_SIZE)", d="pmcF|pmcW"),
               summary_command=f"python3 bench.py --traffic-from {fetch_dir} {write_dir}")
    with open(out_json, "w") as fh:
        json.dump(rec, fh, indent=1)
        fh.write("\n")
    md = [
        "# HBM traffic of the FP64 push, 1e6-atom ensemble (states 1-10, order 5)",
        "",
        "Two counter runs on the MI355X box, then the summary (from the repository root, "
        "R=$GRAFT_REPO_ROOT):",
        "",
        "```",
        "cd /tmp && export TMPDIR=/tmp",
        TRAFFIC_CMD.format(ctr="FETCH_SIZE", d="pmcF"),
        TRAFFIC_CMD.format(ctr="WRITE_SIZE", d="pmcW"),
        f"cd $R && python3 bench.py --traffic-from gpurun_out/pmcF gpurun_out/pmcW",
        "```",
        "",
        "| kernel | FETCH_SIZE (KiB) | WRITE_SIZE (KiB) |",
        "|---|---|---|",
        f"| plain device copy ({copy_mib} MiB) | {out['FETCH_SIZE']['copy_kib']:.0f} | "
        f"{out['WRITE_SIZE']['copy_kib']:.0f} |",
        f"| `{PUSH_KERNEL_NAME}` | {out['FETCH_SIZE']['push_kib']:.0f} | "
        f"{out['WRITE_SIZE']['push_kib']:.0f} |",
    ]
    if out["FETCH_SIZE"]["ionize_kib"] is not None:
        md.append(f"| `ionize_kernel<5>` | {out['FETCH_SIZE']['ionize_kib']:.0f} | "
                  f"{out['WRITE_SIZE']['ionize_kib']:.0f} |")
    md += [
        "",
        f"Calibration on the copy of {ref_kib:.0f} KiB: FETCH_SIZE scale {f_scale:.3f}, "
        f"WRITE_SIZE scale {w_scale:.3f}.",
        f"Scaled push traffic per launch: read {rd / 1e6:.1f} MB + write {wr / 1e6:.1f} MB = "
        f"{(rd + wr) / 1e6:.1f} MB (algorithmic: {atoms * slots_per_atom:.0e} slots x (8 B birth "
        f"time + 48 B outputs) + {atoms:.0e} atoms x 24 B = {algo / 1e6:.1f} MB).",
        "Spread over the multi-second launch this is well under 1 GB/s against 8 TB/s: the kernel",
        "is bound by FP64 arithmetic.  The excess over the algorithmic bytes comes from the",
        "scattered 8-byte output stores (each lane finishes its electron at its own time, so the",
        "six stores of one electron land in six partly written sectors).",
        "",
        f"Kernel source hash {kernel_source_hash()} (bench.py reports this traffic only for",
        "that build of the push kernel).",
    ]
    with open(out_json.replace(".json", ".md"), "w") as fh:
        fh.write("\n".join(md) + "\n")
    print(json.dumps(rec))
    return rec


def _per_dispatch(counter_dir):
    """{form: {dispatch id: {counter: value summed over its dimensions}}}."""
    import csv
    import glob
    per = {}
    for f in glob.glob(os.path.join(counter_dir, "**", "*counter_collection.csv"), recursive=True):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                for form, name in COUNTER_KERNELS:
                    if name in r["Kernel_Name"] and "batch" not in r["Kernel_Name"]:
                        d = per.setdefault(form, {}).setdefault(int(r["Dispatch_Id"]), {})
                        d[r["Counter_Name"]] = d.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    return per


def write_counter_summary(counter_dir, bench_json, counter_dir2=None, out_json=PROFILE_COUNTERS_FILE):
    """Turn the counter runs (COUNTERS_CMD, and COUNTERS2_CMD into counter_dir2)
    and the first run's bench line into per-unit FLOPs, issue rates, clock and
    lane activity of the FP64 and mixed pushes and the ionization kernel, and
    write out_json and the .md beside it."""
    # one launch per form: bench.py calls the mixed push twice (untimed, then
    # timed), so take the last dispatch of each kernel, the timed one
    vals = {form: disp[max(disp)] for form, disp in _per_dispatch(counter_dir).items()}
    vals2 = {}
    if counter_dir2:
        vals2 = {form: disp[max(disp)] for form, disp in _per_dispatch(counter_dir2).items()}
    line = [l for l in open(bench_json) if l.startswith("{")][-1]
    b = json.loads(line)
    steps = b["config"]["electron_steps"]
    atoms = b["config"]["atoms"]
    ms = {"fp64": b["roofline"]["push_ms"], "mixed": b["mixed"]["push_ms"], "ionize": b["ionize_ms"]}
    units = {"fp64": ("electron-step", steps), "mixed": ("electron-step", steps),
             "ionize": ("atom", atoms)}
    rec = dict(workload="rp_ne_fp64_1m", electron_steps=steps, atoms=atoms,
               kernel_source_hash=kernel_source_hash(), command=COUNTERS_CMD,
               command2=COUNTERS2_CMD if counter_dir2 else None,
               summary_command=f"python3 bench.py --counters-from {counter_dir} BENCH_STDOUT"
                               + (f" {counter_dir2}" if counter_dir2 else ""))
    forms = [f for f in ("fp64", "mixed", "ionize") if f in vals]
    md = ["# Push and ionization counters, benchmark ensemble (1e6 atoms, states 1-10, order 5)",
          "", "Two counter runs, then the summary (from the repository root, R=$GRAFT_REPO_ROOT):", "",
          "```", "cd /tmp && export TMPDIR=/tmp", COUNTERS_CMD + " > $R/gpurun_out/pmcS.json",
          COUNTERS2_CMD + " > $R/gpurun_out/pmcC.json",
          "cd $R && python3 bench.py --counters-from gpurun_out/pmcS gpurun_out/pmcS.json gpurun_out/pmcC",
          "```", "", f"{steps:.4e} electron-steps per push launch, {atoms} atoms per ionization launch.",
          "", "| counter (summed over the dispatch) | " + " | ".join(forms) + " |",
          "|---" * (len(forms) + 1) + "|"]
    for ctr in COUNTERS:
        md.append(f"| {ctr} | " + " | ".join(f"{vals[f].get(ctr, float('nan')):.4e}" for f in forms) + " |")
    for ctr in COUNTERS2:
        if vals2:
            md.append(f"| {ctr} (second run) | "
                      + " | ".join(f"{vals2.get(f, {}).get(ctr, float('nan')):.4e}" for f in forms) + " |")
    md += ["", "Derived (SQ instruction counts are per wave instruction; a wave is 64 lanes):", ""]
    for form in forms:
        v, v2 = vals[form], vals2.get(form, {})
        unit, n_units = units[form]
        f64 = 64 * v.get("SQ_INSTS_VALU_FLOPS_FP64", 0.0)
        f32 = 64 * v.get("SQ_INSTS_VALU_FLOPS_FP32", 0.0)
        t = ms[form] * 1e-3
        r = dict(ms=ms[form], unit=unit, fp64_flop_per_unit=f64 / n_units,
                 fp32_flop_per_unit=f32 / n_units, fp64_tflops=f64 / t / 1e12,
                 fp32_tflops=f32 / t / 1e12,
                 valu_per_cu_cycle_at_2p4ghz=v["SQ_INSTS_VALU"] / t / (256 * 2.4e9),
                 fp64_arith_frac=(v.get("SQ_INSTS_VALU_FMA_F64", 0) + v.get("SQ_INSTS_VALU_MUL_F64", 0)
                                  + v.get("SQ_INSTS_VALU_ADD_F64", 0)) / v["SQ_INSTS_VALU"])
        if form != "ionize":
            r["fp64_flop_per_step"] = r["fp64_flop_per_unit"]
            r["fp32_flop_per_step"] = r["fp32_flop_per_unit"]
        if v2.get("GRBM_GUI_ACTIVE"):
            # GRBM_GUI_ACTIVE is summed over the 8 XCDs: cycles of the dispatch
            cyc = v2["GRBM_GUI_ACTIVE"] / 8.0
            r["clock_ghz"] = cyc / t / 1e9
            r["valu_per_cu_cycle"] = v2["SQ_INSTS_VALU"] / (256 * cyc)
            r["salu_per_valu"] = v2.get("SQ_INSTS_SALU", 0.0) / v2["SQ_INSTS_VALU"]
            if v2.get("SQ_ACTIVE_INST_VALU"):
                r["active_lanes_per_valu_cycle"] = (v2.get("SQ_THREAD_CYCLES_VALU", 0.0)
                                                    / v2["SQ_ACTIVE_INST_VALU"])
        else:
            r["valu_per_cu_cycle"] = r["valu_per_cu_cycle_at_2p4ghz"]
        rec[form] = r
        line = (f"- {form}: {r['fp64_flop_per_unit']:.0f} FP64 + {r['fp32_flop_per_unit']:.0f} FP32 "
                f"FLOPs per {unit}; {r['fp64_tflops']:.1f} TFLOP/s FP64 + {r['fp32_tflops']:.1f} "
                f"TFLOP/s FP32 in {ms[form]:.1f} ms; FP64 add/mul/fma are "
                f"{100 * r['fp64_arith_frac']:.0f}% of VALU instructions")
        if "clock_ghz" in r:
            line += (f"; clock {r['clock_ghz']:.2f} GHz (GRBM_GUI_ACTIVE / 8 XCDs over the launch), "
                     f"{r['valu_per_cu_cycle']:.2f} VALU wave instructions per CU per measured cycle, "
                     f"{r['salu_per_valu']:.2f} SALU per VALU instruction")
            if "active_lanes_per_valu_cycle" in r:
                line += (f", {r['active_lanes_per_valu_cycle']:.1f} active lanes per wave-cycle of VALU "
                         "work (SQ_THREAD_CYCLES_VALU / SQ_ACTIVE_INST_VALU)")
        md.append(line + ".")
    md += ["", "A wave64 FP64 instruction occupies its SIMD for 4 cycles: the FP64 ceiling is 1.0 wave",
           "instruction per CU per cycle (78.6 TFLOP/s of FMAs at 2.4 GHz).  The mixed push issues",
           "more than that, so its FP32 instructions do not hold their SIMD for 4 cycles each; it is",
           "set against the published peaks (157.3 TFLOP/s FP32, counted with packed FMAs, which the",
           "kernels do not use).  FLOPs per unit count every lane of a wave instruction (SQ counts",
           "are per wave); the active-lane figure gives the share of lanes doing work.  The counters",
           "are taken from one launch per kernel: the timed one, the last of each kernel in the run.",
           "",
           f"Kernel source hash {kernel_source_hash()} (bench.py uses these figures only for",
           "that build of the kernels)."]
    with open(out_json, "w") as fh:
        json.dump(rec, fh, indent=1)
        fh.write("\n")
    with open(out_json.replace(".json", ".md"), "w") as fh:
        fh.write("\n".join(md) + "\n")
    print(json.dumps(rec))
    return rec


def occupancy(kind, field, precision):
    """Registers and resident waves per SIMD of a kernel (None if the query fails)."""
    try:
        from paper_2509_01741_amd import binding as B
        return B.rpdla_kernel_occupancy(kind, field, precision)
    except Exception:
        return None


KSTATS_CMD = ("rocprofv3 --kernel-trace --stats --output-format csv -d $R/gpurun_out/ktrace -o run "
              "-- python3 $R/bench.py --steps 1 --warmup 0 --no-cpu-baseline")
PROFILE_KSTATS_FILE = os.path.join(ROOT, "profiles", "push_fp64_rp_ne_fp64_1m_kernel_stats.md")


def _short_kernel_name(name):
    """Kernel name without its argument list (and shortened if still long)."""
    head = name.split("(", 1)[0]
    return head if len(head) <= 80 else head[:77] + "..."


def write_kernel_stats_summary(trace_dir, bench_json, out_md=PROFILE_KSTATS_FILE):
    """Turn the kernel-trace statistics of one bench run (KSTATS_CMD) into the
    kernel-time table, with the benchmark step's own dispatches set against
    bench.py's HIP-event times of the same run."""
    import csv
    import glob

    def one(pattern):
        files = glob.glob(os.path.join(trace_dir, "**", pattern), recursive=True)
        if not files:
            raise SystemExit(f"no {pattern} under {trace_dir}")
        return list(csv.DictReader(open(files[0])))

    stats, trace = one("*kernel_stats.csv"), one("*kernel_trace.csv")
    line = [l for l in open(bench_json) if l.startswith("{")][-1]
    b = json.loads(line)
    md = ["# Kernel time, FP64 full ensemble (1e6 atoms, states 1-10, order-5 field), the mixed and",
          "# controlled-step pushes of the same slots, and the batched sweeps", "",
          "Command (on the MI355X box, from the repository root, R=$GRAFT_REPO_ROOT), then the summary:",
          "", "```", "cd /tmp && export TMPDIR=/tmp", KSTATS_CMD + " > $R/gpurun_out/ktrace.json",
          "cd $R && python3 bench.py --kernel-stats-from gpurun_out/ktrace gpurun_out/ktrace.json",
          "```", "", "`run_kernel_stats.csv`, kernels above 0.01% of GPU time (durations in ms):", "",
          "| kernel | calls | total ms | average ms | % |", "|---|---|---|---|---|"]
    for r in stats:
        pct = float(r["Percentage"])
        if pct < 0.01:
            continue
        md.append(f"| `{_short_kernel_name(r['Name'])}` | {r['Calls']} | "
                  f"{float(r['TotalDurationNs']) / 1e6:.2f} | {float(r['AverageNs']) / 1e6:.2f} | {pct:.2f} |")
    # the benchmark step is the first ionization and the first FP64 push dispatch
    # (one timed step, no warm-up); later ones belong to the mixed workload
    first = {}
    for r in sorted(trace, key=lambda r: int(r["Dispatch_Id"])):
        for key, pat in (("ionize", "rpdla::ionize_kernel<5>("),
                         ("push", "rpdla::push_kernel<5, rpdla::ElecF64>(")):
            if pat in r["Kernel_Name"] and key not in first:
                first[key] = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6
    md += ["", "The benchmark step's dispatches in `run_kernel_trace.csv` against bench.py's own "
           "HIP-event times of the same profiled run:", "",
           "| kernel | trace ms | bench.py ms |", "|---|---|---|",
           f"| `push_kernel<5, ElecF64>` (1e7 slots) | {first.get('push', float('nan')):.2f} | "
           f"{b['roofline']['push_ms']:.2f} (`push_ms`) |",
           f"| `ionize_kernel<5>` (1e6 atoms) | {first.get('ionize', float('nan')):.2f} | "
           f"{b['ionize_ms']:.2f} (`ionize_ms`) |", "",
           "The second call of each is the FP64 reference of the mixed workload (`rp_ne_mixed_1m`); "
           "the batched kernels belong to the sweeps bench.py also times (64 configurations in FP64 "
           "and mixed precision, 16 large configurations in mixed precision); `push_kernel<5, "
           "ElecDP>` is the controlled-step push of the benchmark slots."]
    with open(out_md, "w") as fh:
        fh.write("\n".join(md) + "\n")
    print("\n".join(md))


def ionize_roofline(atoms, ion_ms):
    """Roofline object of the ionization kernel: its FP64 FLOPs per atom come
    from the counter run (the work is data-dependent: panels are skipped where
    the rate bound vanishes, and the Newton iterations vary), taken on the
    same ensemble at the same size, times this launch's atoms over its time."""
    crec = _counter_record()
    if crec is None or "ionize" not in crec:
        return None
    r = crec["ionize"]
    ach = r["fp64_flop_per_unit"] * atoms / (ion_ms * 1e-3) / 1e12
    return {"bound": "alu", "kernel": "ionize_kernel<5>", "achieved": ach,
            "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": ach / FP64_VECTOR_PEAK_TFLOPS,
            "traffic": None, "flop_per_atom": r["fp64_flop_per_unit"],
            "flop_source": "executed FP64 FLOPs per atom, counter run on this ensemble",
            "valu_per_cu_cycle": r.get("valu_per_cu_cycle"),
            "active_lanes_per_valu_cycle": r.get("active_lanes_per_valu_cycle")}


def _counter_record():
    try:
        rec = json.load(open(PROFILE_COUNTERS_FILE))
        return rec if rec.get("kernel_source_hash") == kernel_source_hash() else None
    except (OSError, ValueError):
        return None


def main():
    if len(sys.argv) == 4 and sys.argv[1] == "--traffic-from":
        write_traffic_summary(sys.argv[2], sys.argv[3])
        return
    if len(sys.argv) == 4 and sys.argv[1] == "--kernel-stats-from":
        write_kernel_stats_summary(sys.argv[2], sys.argv[3])
        return
    if len(sys.argv) in (4, 5) and sys.argv[1] == "--counters-from":
        write_counter_summary(sys.argv[2], sys.argv[3], sys.argv[4] if len(sys.argv) == 5 else None)
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--atoms", type=int, default=None, help="override (testing only)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-adaptive", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--large-stream", action="store_true",
                    help="only run the large mixed workload's whole chunked stream and print it")
    ap.add_argument("--no-mixed-workload", action="store_true",
                    help="skip the mixed form's own workload (counter runs read the last launches)")
    ap.add_argument("--copy-ref-mib", type=int, default=0,
                    help="also run one plain device copy of this many MiB (a known-size "
                         "reference for hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "design (atom chunks per GPU, one all-reduce of the integer histograms) is not "
              "built", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2509_01741_amd import binding as B
    from paper_2509_01741_amd import pipeline, workloads

    torch.cuda.set_device(0)
    if args.large_stream:
        r = measure_stream(workloads.LARGE_MIXED, B.RPDLA_MIXED)
        print(json.dumps({"large_stream": r}), flush=True)
        return
    if args.copy_ref_mib > 0:
        src = torch.ones(args.copy_ref_mib << 17, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy reference: {args.copy_ref_mib} MiB read + written")
        del src, dst
    wl = workloads.FULL_FP64
    ens = pipeline.Ensemble(wl, precision=B.RPDLA_FP64, n_atoms=args.atoms)
    log(f"workload {wl['name']}: {ens.n} atoms x {ens.K} states = {ens.n * ens.K} slots")

    for i in range(args.warmup):
        t0 = time.time()
        ens.step()
        torch.cuda.synchronize()
        log(f"warmup {i + 1}/{args.warmup}: {time.time() - t0:.2f} s")

    ev = lambda: torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_start = ev()
    t_start.record()
    push_ms, ion_ms = [], []
    for i in range(args.steps):
        a, b, c = ev(), ev(), ev()
        ens.sample()
        a.record()
        ens.ionize()
        b.record()
        ens.push()
        c.record()
        ens.histogram()
        push_ms.append((b, c))
        ion_ms.append((a, b))
        c.synchronize()
        log(f"step {i + 1}/{args.steps}: ionize {a.elapsed_time(b):.1f} ms, push {b.elapsed_time(c):.1f} ms")
    t_end = ev()
    t_end.record()
    torch.cuda.synchronize()
    total_ms = t_start.elapsed_time(t_end)
    push_avg = sum(b.elapsed_time(c) for b, c in push_ms) / len(push_ms)
    ion_avg = sum(a.elapsed_time(b) for a, b in ion_ms) / len(ion_ms)
    steps, born = electron_steps(ens.tb, ens.z, ens.K, ens.L)
    ms_per_step = total_ms / args.steps
    value = steps / (ms_per_step * 1e-3)
    push_rate = steps / (push_avg * 1e-3)
    achieved_tflops = ALGO_FLOP_PER_STEP * steps / (push_avg * 1e-3) / 1e12
    tal = ens.tallies.cpu().tolist()
    log(f"{steps:.4e} electron-steps over {born} electrons; step {ms_per_step:.1f} ms; "
        f"push {push_rate:.3e} e-steps/s = {achieved_tflops:.1f} TFLOP/s")

    traffic = None
    if os.path.exists(PROFILE_TRAFFIC_FILE):
        try:
            tr = json.load(open(PROFILE_TRAFFIC_FILE))
            if tr.get("kernel_source_hash") == kernel_source_hash() and tr.get("atoms") == ens.n:
                traffic = tr.get("bytes_per_launch")
        except Exception:
            traffic = None

    mixed = None
    mixed_outs = None
    if not args.no_mixed:
        outs = tuple(torch.empty_like(o) for o in ens.out)
        mixed_outs = outs
        B.rpdla_push(ens.L, B.RPDLA_MIXED, ens.tb, ens.x, ens.y, ens.z, ens.K, outs)
        torch.cuda.synchronize()
        a, b = ev(), ev()
        a.record()
        B.rpdla_push(ens.L, B.RPDLA_MIXED, ens.tb, ens.x, ens.y, ens.z, ens.K, outs)
        b.record()
        torch.cuda.synchronize()
        mix_ms = a.elapsed_time(b)
        fin = torch.isfinite(ens.tb)

        def kin(o):
            u2 = o[0][fin] ** 2 + o[1][fin] ** 2 + o[2][fin] ** 2
            return 0.51099895 * u2 / (torch.sqrt(1 + u2) + 1), o[2][fin] > 0

        K64, f64 = kin(ens.out)
        Kmx, fmx = kin(outs)
        rel = (Kmx - K64).abs() / K64
        mixed = dict(
            push_ms=round(mix_ms, 2),
            electron_steps_per_s=steps / (mix_ms * 1e-3),
            speedup_vs_fp64=push_avg / mix_ms,
            frac_rel_err_le_1e3=float((rel <= 1e-3).double().mean().item()),
            median_rel_err=float(rel.median().item()),
            p99_rel_err=quantile_sorted(rel, 0.99),
            rel_err_hist_decades_from_1e17=rel_err_histogram(rel),
            mean_energy_rel_err=float((Kmx.double().mean() / K64.double().mean() - 1).item()),
            same_direction=float((f64 == fmx).double().mean().item()),
        )
        crec = _counter_record()
        if crec is not None:
            # FLOPs per electron-step of the mixed form from the counter run
            f32 = crec["mixed"]["fp32_flop_per_step"] * steps / (mix_ms * 1e-3) / 1e12
            f64m = crec["mixed"]["fp64_flop_per_step"] * steps / (mix_ms * 1e-3) / 1e12
            mixed["roofline"] = {
                "bound": "alu", "achieved_fp32": f32, "achieved_fp64": f64m,
                "peak_fp32": FP32_VECTOR_PEAK_TFLOPS, "peak_fp64": FP64_VECTOR_PEAK_TFLOPS,
                "unit": "TFLOP/s",
                "frac": f32 / FP32_VECTOR_PEAK_TFLOPS + f64m / FP64_VECTOR_PEAK_TFLOPS,
                "flop_per_electron_step": {"fp32": crec["mixed"]["fp32_flop_per_step"],
                                           "fp64": crec["mixed"]["fp64_flop_per_step"]},
                "valu_per_cu_cycle": crec["mixed"]["valu_per_cu_cycle"],
                "clock_ghz": crec["mixed"].get("clock_ghz"),
                "note": "frac = FP32 share of the published FP32 vector peak (packed FMAs) + "
                        "FP64 share of the FP64 vector peak; FLOPs per electron-step from the "
                        "counter run (executed, every lane of a wave instruction counted)"}
        mixed["occupancy"] = occupancy(0, int(ens.L.field), B.RPDLA_MIXED)
        log(f"mixed: {mixed}")

    if mixed is not None and args.atoms is None and not args.no_mixed_workload:
        # full-size runs only: counter runs at a reduced size read the last
        # push launches, which must stay those of the benchmark ensemble
        mixed["workload_1pw"] = measure_mixed_workload(workloads.MIXED_AB)
        log(f"mixed, 1 PW workload: {mixed['workload_1pw']}")

    adaptive = None
    if not args.no_adaptive:
        # controlled-step push of the same slots (default tolerances, early stop
        # when the energy is constant): time, steps taken, energies against the
        # fixed-step FP64 push
        A = B.adaptive_settings()
        outs = tuple(torch.empty_like(o) for o in ens.out)
        a, b = ev(), ev()
        a.record()
        r = B.rpdla_push_adaptive(ens.L, A, ens.tb, ens.x, ens.y, ens.z, ens.K, outs)
        b.record()
        torch.cuda.synchronize()
        ad_ms = a.elapsed_time(b)
        fin = torch.isfinite(ens.tb)
        u2a = outs[0][fin] ** 2 + outs[1][fin] ** 2 + outs[2][fin] ** 2
        u2f = ens.out[0][fin] ** 2 + ens.out[1][fin] ** 2 + ens.out[2][fin] ** 2
        Ka = u2a / (torch.sqrt(1 + u2a) + 1)
        Kf = u2f / (torch.sqrt(1 + u2f) + 1)
        rel = (Ka - Kf).abs() / Kf
        acc = r[7][fin].double()
        rej = r[8][fin].double()
        adaptive = dict(
            push_ms=round(ad_ms, 2),
            electrons_per_s=int(fin.sum().item()) / (ad_ms * 1e-3),
            speedup_vs_fixed_step=push_avg / ad_ms,
            mean_accepted_steps=float(acc.mean().item()),
            mean_rejected_steps=float(rej.mean().item()),
            field_evaluations_vs_fixed_step=float(6 * (acc + rej).sum().item() / (4 * steps)),
            median_rel_energy_diff_vs_fixed_step=float(rel.median().item()),
            settings=dict(rtol=A.rtol, atol=A.atol, h_max="10 dt", k_tol=A.k_tol),
        )
        log(f"adaptive: {adaptive}")

    batched = None
    if not args.no_batched:
        batched = {}
        sw = workloads.SWEEP_FP64
        r = measure_sweep(sw, B.RPDLA_FP64, sw["atoms"], sw["atoms"])
        log(f"batched sweep FP64: {r}")
        batched["sweep64_fp64"] = r
        r = measure_sweep(sw, B.RPDLA_MIXED, sw["atoms"], sw["atoms"])
        log(f"batched sweep mixed: {r}")
        batched["sweep64_mixed"] = r
        lg = workloads.LARGE_MIXED
        r = measure_sweep(lg, B.RPDLA_MIXED, lg["chunk"], lg["chunk"],
                          chunks_total=-(-lg["atoms"] // lg["chunk"]))
        log(f"large mixed sweep: {r}")
        batched["large16_mixed"] = r

    base = None
    parity = None
    if not args.no_cpu_baseline:
        try:
            base, parity = cpu_baseline(ens, mixed_outs)
            log(f"cpu baseline: {base['value']:.3e} e-steps/s on {base['cores']} threads")
            log(f"FP64 vs oracle: {parity}")
        except Exception as e:  # the oracle is a reported baseline only
            log(f"cpu baseline unavailable: {e!r}")

    rec = wl["lasers"][0]
    out = {
        "metric": "electron-steps/s (FP64 full Monte Carlo step: sample, ionize, push, histogram)",
        "value": value,
        "unit": "electron-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": wl["name"], "atoms": ens.n, "charge_states": [wl["k_first"], wl["k_last"]],
            "slots": ens.n * ens.K, "born_electrons": born, "electron_steps": steps,
            "lambda_um": rec["lam"] * 1e6, "w0_um": rec["w0"] * 1e6, "tau_fwhm_fs": rec["tau"] * 1e15,
            "I_W_cm2": rec["I"], "field_order": int(ens.L.field), "dt": "T/200",
            "window": "[z/c - 5 tau, z/c + 10 tau]",
        },
        "roofline": {
            "bound": "alu", "kernel": "push_kernel<5, ElecF64>",
            "achieved": achieved_tflops, "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved_tflops / FP64_VECTOR_PEAK_TFLOPS, "traffic": traffic,
            "flop_per_electron_step": ALGO_FLOP_PER_STEP, "push_ms": round(push_avg, 2),
            "flop_per_electron_step_counters": (None if _counter_record() is None else
                                                _counter_record()["fp64"]["fp64_flop_per_step"]),
            # issue rate from the counter run (ceiling 1.0 for FP64 code), the
            # kernel's registers and resident waves, HBM rate from the traffic
            "valu_per_cu_cycle": (None if _counter_record() is None else
                                  _counter_record()["fp64"]["valu_per_cu_cycle"]),
            # the clock the counter run measured under this load, and the
            # fraction of the FP64 peak at that clock (the published peak
            # assumes 2.4 GHz)
            "clock_ghz_counters": (None if _counter_record() is None else
                                   _counter_record()["fp64"].get("clock_ghz")),
            "frac_at_measured_clock": (
                None if _counter_record() is None or not _counter_record()["fp64"].get("clock_ghz")
                else achieved_tflops / (FP64_VECTOR_PEAK_TFLOPS
                                        * _counter_record()["fp64"]["clock_ghz"] / 2.4)),
            "occupancy": occupancy(0, int(ens.L.field), B.RPDLA_FP64),
            "hbm_gb_s": None if traffic is None else traffic / (push_avg * 1e-3) / 1e9,
        },
        "push_electron_steps_per_s": push_rate,
        "ionize_ms": round(ion_avg, 2),
        "ionize": ionize_roofline(ens.n, ion_avg),
        "tallies": dict(zip(["fwd", "bwd", "below", "above", "unborn", "nan"], tal)),
        "mixed": mixed,
        "adaptive": adaptive,
        "batched": batched,
        "cpu_baseline": base,
        "fp64_vs_oracle": parity,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
