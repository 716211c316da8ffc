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
# order-5 field (mul, add = 1 FLOP, fma = 2; the sine/cosine, exponential,
# reciprocal and reciprocal square root counted at the operations of their
# polynomial implementations): 4 x (223 field + 27 Lorentz) + 85 RK4 = 1085.
ALGO_FLOP_PER_STEP = 1085.0
FP64_VECTOR_PEAK_TFLOPS = 78.6
# Published FP32 vector peak.  It counts packed FP32 FMAs (two per lane per
# instruction); the kernels are compiled without packed FP32, so an FP32
# instruction, like an FP64 one, occupies its SIMD for 4 cycles per wave64 and
# the ceiling for their unpacked FP32 FMAs is the FP64 figure, 78.6 TFLOP/s.
FP32_VECTOR_PEAK_TFLOPS = 157.3
PROFILE_COUNTERS_FILE = os.path.join(ROOT, "profiles", "push_rp_ne_fp64_100k_counters.json")
COUNTERS = ["SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_VALU_FLOPS_FP64", "SQ_INSTS_VALU_FLOPS_FP32",
            "SQ_INSTS_VALU_FMA_F64", "SQ_INSTS_VALU_MUL_F64", "SQ_INSTS_VALU_ADD_F64",
            "SQ_INSTS_VALU_TRANS_F32"]
COUNTERS_CMD = ("rocprofv3 --pmc " + " ".join(COUNTERS) + " --output-format csv -d "
                "$R/gpurun_out/pmcS -o run -- python3 $R/bench.py --steps 1 --warmup 0 --atoms 100000 "
                "--no-cpu-baseline --no-adaptive --no-batched")
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


def cpu_baseline(ens, budget_s=15.0):
    """Oracle push rate on a bounded sample of the same workload: the oracle
    samples the first atoms and ionizes them itself (same seed and laser), and
    its push over their slots is timed, scaled to ~budget_s."""
    import numpy as np
    import oracle as O
    wl = ens.wl
    rec = wl["lasers"][0]
    OL = O.laser_intensity(rec["lam"], rec["w0"], rec["tau"], rec["I"])
    OL.field = ens.L.field
    kf, kl = wl["k_first"], wl["k_last"]
    K = kl - kf + 1

    def run(na):
        x, y, z = O.sample_atoms(wl["seed"], wl["cfg_id"], 0, na, wl["r_factor"] * OL.w0,
                                 O.rayleigh(OL))
        t = O.ionize(OL, wl["seed"], wl["cfg_id"], 0, x, y, z, kf, kl)
        fin = np.isfinite(t)
        steps = np.ceil((np.repeat(z, K)[fin] / C_LIGHT + OL.t_after - t[fin]) / OL.dt).sum()
        t0 = time.perf_counter()
        out = O.push(OL, t, x, y, z, K)
        return float(steps), time.perf_counter() - t0, (x, y, z, t, out)

    s1, t1, _ = run(4)
    na = int(max(4, min(ens.n, 4 * budget_s / max(t1, 1e-3))))
    s2, t2, sample = run(na)
    base = dict(value=s2 / t2, unit="electron-steps/s", cores=O.num_threads(), kind="oracle",
                sample=f"FP64 push of the slots of the first {na} atoms ({int(s2)} electron-steps, "
                       f"{t2:.1f} s), atoms and birth times from the oracle's own sampling and "
                       f"ionization; order-5 field, same laser")
    try:
        parity = fp64_vs_oracle(ens, OL, K, sample)
    except Exception as e:  # a reported statistic only
        log(f"FP64 vs oracle statistics unavailable: {e!r}")
        parity = None
    return base, parity


def fp64_vs_oracle(ens, OL, K, sample):
    """The GPU's FP64 results for the oracle's sample (the first atoms of the
    same ensemble) against the oracle's: birth times, energies, directions.
    Electrons outside 1e-8 are re-pushed by the oracle with birth times moved
    by 1e-15 relative; those whose own energy then moves by more than 1e-10
    are ill-conditioned (a rounding-level change of the input moves them)."""
    import numpy as np
    import oracle as O
    x, y, z, t, out = sample
    n = t.size
    tg = ens.tb[:n].cpu().numpy()
    ug = [o[:n].cpu().numpy() for o in ens.out[:3]]
    T = OL.lambda_ / C_LIGHT
    fo, fg = np.isfinite(t), np.isfinite(tg)
    both = fo & fg
    dt_rel = np.abs(t[both] - tg[both]) / np.maximum(np.abs(t[both]), T)

    def kin(u):
        u2 = u[0][both] ** 2 + u[1][both] ** 2 + u[2][both] ** 2
        return 0.51099895 * u2 / (np.sqrt(1.0 + u2) + 1.0), u[2][both] > 0

    Ko, dir_o = kin(out)
    Kg, dir_g = kin(ug)
    rel = np.abs(Kg - Ko) / Ko
    ok = np.abs(Kg - Ko) <= 1e-8 * Ko + 1e-12
    bad = np.nonzero(both)[0][~ok]
    ill = 0
    if bad.size:
        tp = t[bad] + 1e-15 * np.maximum(np.abs(t[bad]), T)
        xs, ys, zs = (np.repeat(a, K)[bad] for a in (x, y, z))
        pert = O.push(OL, tp, xs, ys, zs, 1)
        u2 = pert[0] ** 2 + pert[1] ** 2 + pert[2] ** 2
        Kp = 0.51099895 * u2 / (np.sqrt(1.0 + u2) + 1.0)
        ill = int((np.abs(Kp - Ko[~ok]) / Ko[~ok] > 1e-10).sum())
    well = int(both.sum()) - ill
    return dict(electrons=int(both.sum()), born_mismatch=int((fo != fg).sum()),
                birth_time_max_rel=float(dt_rel.max()) if dt_rel.size else 0.0,
                energy_frac_le_1e8=float(ok.mean()), energy_median_rel=float(np.median(rel)),
                ill_conditioned=ill,
                energy_frac_le_1e8_well_conditioned=float((ok.sum()) / max(well, 1)) if ill
                else float(ok.mean()),
                same_direction=float((dir_o == dir_g).mean()),
                note="sample of the CPU baseline; ill-conditioned = the oracle's own energy "
                     "moves by more than 1e-10 when the birth time moves by 1e-15 relative")


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
                mean_energy_rel_err=float((Kmx.double().mean() / K64.double().mean() - 1).item()),
                same_direction=float((f64 == fmx).double().mean().item()))


def measure_sweep(wl, precision, atoms_per_cfg, atoms_per_chunk):
    """One timed batched sweep (after an untimed one that captures the graph)
    on a side stream; electron-steps counted by the library."""
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
    with torch.cuda.stream(st):
        pipeline.run_sweep(wl, precision, atoms_per_cfg, atoms_per_chunk, stream=st, workspace=ws,
                           counts=counts, tallies=tallies, electron_steps=steps)
        counts.zero_(); tallies.zero_(); steps.zero_()
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
    return dict(workload=wl["name"], precision="mixed" if precision == B.RPDLA_MIXED else "f64",
                configs=n_cfg, atoms_per_cfg=atoms_per_cfg, atoms_per_chunk=atoms_per_chunk,
                chunks=-(-atoms_per_cfg // atoms_per_chunk), ms=round(ms, 2),
                electron_steps=n_steps, electron_steps_per_s=n_steps / (ms * 1e-3),
                born=int(tal[0] + tal[1]), backward_fraction_min_max=[float(bwd.min()), float(bwd.max())],
                occupancy=occupancy(2, int(wl["field_order"]), precision))


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


def write_counter_summary(counter_dir, bench_json, out_json=PROFILE_COUNTERS_FILE):
    """Turn the counter run (COUNTERS_CMD) and that run's bench line into
    per-electron-step FLOPs and issue rates of the FP64 and mixed pushes, and
    write out_json and the .md beside it."""
    import csv
    import glob
    per_dispatch = {}
    for f in glob.glob(os.path.join(counter_dir, "**", "*counter_collection.csv"), recursive=True):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                for form, name in (("fp64", "push_kernel<5, rpdla::ElecF64>"),
                                   ("mixed", "push_kernel<5, rpdla::ElecMixed>")):
                    if name in r["Kernel_Name"] and "batch" not in r["Kernel_Name"]:
                        d = per_dispatch.setdefault(form, {}).setdefault(int(r["Dispatch_Id"]), {})
                        d[r["Counter_Name"]] = d.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    # one launch per form: bench.py calls the mixed push twice (untimed, then
    # timed), so take the last dispatch of each kernel, the timed one
    vals = {form: disp[max(disp)] for form, disp in per_dispatch.items()}
    line = [l for l in open(bench_json) if l.startswith("{")][-1]
    b = json.loads(line)
    steps = b["config"]["electron_steps"]
    ms = {"fp64": b["roofline"]["push_ms"], "mixed": b["mixed"]["push_ms"]}
    rec = dict(workload="rp_ne_fp64_1m at 1e5 atoms", electron_steps=steps,
               kernel_source_hash=kernel_source_hash(), command=COUNTERS_CMD,
               summary_command=f"python3 bench.py --counters-from {counter_dir} BENCH_STDOUT")
    md = ["# FP64 and mixed push counters, 1e5 atoms of the benchmark ensemble (states 1-10, order 5)",
          "", "One counter run, then the summary (from the repository root, R=$GRAFT_REPO_ROOT):", "",
          "```", "cd /tmp && export TMPDIR=/tmp", COUNTERS_CMD + " > $R/gpurun_out/pmcS.json",
          "cd $R && python3 bench.py --counters-from gpurun_out/pmcS gpurun_out/pmcS.json", "```",
          "", f"{steps:.4e} electron-steps per push launch.", "",
          "| counter (summed over the dispatch) | FP64 push | mixed push |", "|---|---|---|"]
    for ctr in COUNTERS:
        md.append(f"| {ctr} | {vals['fp64'].get(ctr, float('nan')):.4e} | "
                  f"{vals['mixed'].get(ctr, float('nan')):.4e} |")
    md += ["", "Derived (SQ counts are per wave instruction; a wave is 64 lanes):", ""]
    for form in ("fp64", "mixed"):
        v = vals[form]
        f64 = 64 * v.get("SQ_INSTS_VALU_FLOPS_FP64", 0.0)
        f32 = 64 * v.get("SQ_INSTS_VALU_FLOPS_FP32", 0.0)
        t = ms[form] * 1e-3
        issue = v["SQ_INSTS_VALU"] / t / (256 * 2.4e9)
        rec[form] = dict(push_ms=ms[form], fp64_flop_per_step=f64 / steps,
                         fp32_flop_per_step=f32 / steps, valu_per_cu_cycle=issue,
                         fp64_tflops=f64 / t / 1e12, fp32_tflops=f32 / t / 1e12,
                         fp64_arith_frac=(v.get("SQ_INSTS_VALU_FMA_F64", 0) + v.get(
                             "SQ_INSTS_VALU_MUL_F64", 0) + v.get("SQ_INSTS_VALU_ADD_F64", 0))
                         / v["SQ_INSTS_VALU"])
        r = rec[form]
        md.append(f"- {form}: {r['fp64_flop_per_step']:.0f} FP64 + {r['fp32_flop_per_step']:.0f} "
                  f"FP32 FLOPs per electron-step; {r['fp64_tflops']:.1f} TFLOP/s FP64 + "
                  f"{r['fp32_tflops']:.1f} TFLOP/s FP32 in {ms[form]:.1f} ms; "
                  f"{issue:.2f} VALU wave instructions per CU per cycle (256 CU x 2.4 GHz); "
                  f"FP64 add/mul/fma are {100 * r['fp64_arith_frac']:.0f}% of VALU instructions.")
    md += ["", "A wave64 FP64 instruction occupies its SIMD for 4 cycles, and so does an unpacked FP32",
           "one (the kernels are compiled without packed FP32), so the ceiling is 1.0 wave",
           "instruction per CU per cycle for both forms: 78.6 TFLOP/s of FMAs in either precision.",
           "The published 157.3 TFLOP/s FP32 peak counts packed FP32 FMAs.  The counters are taken",
           "from one launch per form: the timed one, the last of each kernel in the run.", "",
           f"Kernel source hash {kernel_source_hash()} (bench.py uses these figures only for",
           "that build of the push kernels)."]
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
    if len(sys.argv) == 4 and sys.argv[1] == "--counters-from":
        write_counter_summary(sys.argv[2], sys.argv[3])
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
    if not args.no_mixed:
        outs = tuple(torch.empty_like(o) for o in ens.out)
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
            p99_rel_err=float(torch.quantile(rel[:1_000_000].double(), 0.99).item()),
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
                "frac_unpacked_ceiling": (f32 + f64m) / FP64_VECTOR_PEAK_TFLOPS,
                "flop_per_electron_step": {"fp32": crec["mixed"]["fp32_flop_per_step"],
                                           "fp64": crec["mixed"]["fp64_flop_per_step"]},
                "valu_per_cu_cycle": crec["mixed"]["valu_per_cu_cycle"],
                "note": "frac = FP32 share of the published FP32 vector peak (packed FMAs) + "
                        "FP64 share of the FP64 vector peak; frac_unpacked_ceiling = both "
                        "against 78.6 TFLOP/s, the ceiling of unpacked FP32 and FP64 FMAs, "
                        "which share the SIMDs at 4 cycles per wave64 instruction"}
        mixed["occupancy"] = occupancy(0, int(ens.L.field), B.RPDLA_MIXED)
        log(f"mixed: {mixed}")

    if mixed is not None and args.atoms is None:
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
        r = measure_sweep(workloads.SWEEP_FP64, B.RPDLA_FP64, 16384, 16384)
        log(f"batched sweep FP64: {r}")
        batched["sweep64_fp64"] = r
        r = measure_sweep(workloads.SWEEP_FP64, B.RPDLA_MIXED, 16384, 16384)
        log(f"batched sweep mixed: {r}")
        batched["sweep64_mixed"] = r
        r = measure_sweep(workloads.LARGE_MIXED, B.RPDLA_MIXED, 100_000, 50_000)
        log(f"large mixed sweep: {r}")
        batched["large16_mixed"] = r

    base = None
    parity = None
    if not args.no_cpu_baseline:
        try:
            base, parity = cpu_baseline(ens)
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
            "occupancy": occupancy(0, int(ens.L.field), B.RPDLA_FP64),
            "hbm_gb_s": None if traffic is None else traffic / (push_avg * 1e-3) / 1e9,
        },
        "push_electron_steps_per_s": push_rate,
        "ionize_ms": round(ion_avg, 2),
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
