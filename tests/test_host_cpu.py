"""Host-side pieces that need no GPU: the binding refuses to load without the
built library (no CPU fallback), bench.py's contract for several GPUs and its
counter-summary arithmetic, and the experiment driver's reductions."""
import json
import math
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_binding_fails_loudly_without_library(tmp_path):
    pkg = tmp_path / "pkgcopy"
    pkg.mkdir()
    (pkg / "__init__.py").write_text("")
    shutil.copy(os.path.join(ROOT, "paper_2509_01741_amd", "binding.py"), pkg / "binding.py")
    r = subprocess.run([sys.executable, "-c", "import pkgcopy.binding"], cwd=tmp_path,
                       capture_output=True, text=True)
    assert r.returncode != 0
    assert "ImportError" in r.stderr and "not built" in r.stderr


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def _write_counters(d, counter, rows):
    d.mkdir(parents=True)
    with open(d / "run_counter_collection.csv", "w") as f:
        f.write("Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value\n")
        for i, (k, v) in enumerate(rows):
            f.write(f'{i},"{k}",{counter},{v}\n')


def test_traffic_summary_arithmetic(tmp_path):
    sys.path.insert(0, ROOT)
    import bench
    push = "void rpdla::push_kernel<5, rpdla::ElecF64>(rpdla::DevCfg, rpdla::PushIO)"
    copy = "__amd_rocclr_copyBuffer"
    _write_counters(tmp_path / "F", "FETCH_SIZE", [(copy, 262144.0), (push, 1000.0),
                                                   ("void rpdla::ionize_kernel<5>(x)", 7.0)])
    _write_counters(tmp_path / "W", "WRITE_SIZE", [(copy, 524288.0), (push, 3000.0),
                                                   ("void rpdla::ionize_kernel<5>(x)", 9.0)])
    out = tmp_path / "t.json"
    rec = bench.write_traffic_summary(str(tmp_path / "F"), str(tmp_path / "W"), out_json=str(out))
    assert rec["fetch_scale"] == 0.5 and rec["write_scale"] == 1.0
    assert rec["read_bytes"] == 1000.0 * 1024 / 0.5 and rec["write_bytes"] == 3000.0 * 1024
    assert rec["algorithmic_bytes"] == 1e6 * 10 * 56 + 1e6 * 24
    assert json.load(open(out))["bytes_per_launch"] == rec["read_bytes"] + rec["write_bytes"]
    assert "ionize_kernel<5>" in open(str(out).replace(".json", ".md")).read()


def test_experiment_reductions():
    torch = pytest.importorskip("torch")
    sys.path.insert(0, ROOT)
    # loads the built library (no GPU call is made): the reductions are plain
    # torch on CPU counts
    from paper_2509_01741_amd import experiments as ex
    assert abs(ex.f_number_waist(0.8e-6) / 2.546479089470325e-06 - 1) < 1e-15
    # phase x radius counts: 8 phase bins x 4 radius bins, direction 1 only
    pr = torch.zeros((2, 8, 4), dtype=torch.int64)
    pr[1, 0, 0] = 30          # phase bin [0, pi/4): within pi/4 of 0
    pr[1, 7, 1] = 10          # [7pi/4, 2pi): within pi/4 of 2 pi
    pr[1, 4, 3] = 60          # around pi
    assert abs(ex.phase_near_zero_fraction(pr, 1, math.pi / 4) - 0.4) < 1e-12
    assert math.isnan(ex.phase_near_zero_fraction(pr, 0, math.pi / 4))
    assert ex.radius_quantile(pr, 1, 4e-6, 0.9) == 4e-6   # 60% in the last radius bin
    assert ex.radius_quantile(pr, 1, 4e-6, 0.3) == 1e-6


def test_counter_summary_arithmetic(tmp_path):
    """bench.py's counter summary on a synthetic pair of counter runs: FLOPs
    per unit, the last dispatch of each kernel, the clock from GRBM_GUI_ACTIVE
    (summed over 8 XCDs) and the issue rate per measured cycle."""
    sys.path.insert(0, ROOT)
    import bench
    f64 = "void rpdla::push_kernel<5, rpdla::ElecF64>(rpdla::DevCfg, rpdla::PushIO)"
    mix = "void rpdla::push_kernel<5, rpdla::ElecMixed>(rpdla::DevCfg, rpdla::PushIO)"
    ion = "void rpdla::ionize_kernel<5>(rpdla::DevCfg, unsigned long, unsigned int, ...)"
    d, d2 = tmp_path / "S", tmp_path / "C"
    d.mkdir()
    d2.mkdir()
    with open(d / "run_counter_collection.csv", "w") as f:
        f.write("Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value\n")
        for k, vals in ((f64, dict(SQ_INSTS_VALU=600.0, SQ_INSTS_VALU_FLOPS_FP64=1000.0,
                                    SQ_INSTS_VALU_FMA_F64=300.0, SQ_INSTS_VALU_MUL_F64=100.0,
                                    SQ_INSTS_VALU_ADD_F64=50.0)),
                        (mix, dict(SQ_INSTS_VALU=400.0, SQ_INSTS_VALU_FLOPS_FP64=100.0,
                                   SQ_INSTS_VALU_FLOPS_FP32=500.0)),
                        (ion, dict(SQ_INSTS_VALU=50.0, SQ_INSTS_VALU_FLOPS_FP64=20.0))):
            # the mixed push is dispatched twice (untimed, then timed): one counts
            for disp in ((0,) if k != mix else (1, 2)):
                for ctr, v in vals.items():
                    f.write(f'{disp},"{k}",{ctr},{v}\n')
    with open(d2 / "run_counter_collection.csv", "w") as f:
        f.write("Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value\n")
        # per-XCD rows, summed by the summary: 8 x 1.2e9 cycles over 1 s = 1.2 GHz
        for x in range(8):
            f.write(f'5,"{f64}",GRBM_GUI_ACTIVE,1.2e9\n')
        f.write(f'5,"{f64}",SQ_INSTS_VALU,600.0\n')
        f.write(f'5,"{f64}",SQ_INSTS_SALU,150.0\n')
        f.write(f'5,"{f64}",SQ_ACTIVE_INST_VALU,1000.0\n')
        f.write(f'5,"{f64}",SQ_THREAD_CYCLES_VALU,32000.0\n')
    bj = tmp_path / "b.json"
    bj.write_text("noise\n" + json.dumps({"config": {"electron_steps": 64.0, "atoms": 4},
                                         "roofline": {"push_ms": 1000.0},
                                         "mixed": {"push_ms": 500.0}, "ionize_ms": 10.0}) + "\n")
    rec = bench.write_counter_summary(str(d), str(bj), str(d2), out_json=str(tmp_path / "c.json"))
    assert rec["fp64"]["fp64_flop_per_step"] == 1000.0          # 64 lanes x 1000 / 64 steps
    assert rec["mixed"]["fp32_flop_per_step"] == 500.0
    assert rec["mixed"]["fp64_flop_per_step"] == 100.0
    assert rec["ionize"]["fp64_flop_per_unit"] == 64 * 20.0 / 4  # per atom
    assert abs(rec["fp64"]["fp64_arith_frac"] - 450.0 / 600.0) < 1e-15
    assert abs(rec["fp64"]["clock_ghz"] - 1.2) < 1e-12
    assert abs(rec["fp64"]["valu_per_cu_cycle"] - 600.0 / (256 * 1.2e9)) < 1e-24
    assert abs(rec["fp64"]["salu_per_valu"] - 0.25) < 1e-15
    assert abs(rec["fp64"]["active_lanes_per_valu_cycle"] - 32.0) < 1e-12
    assert abs(rec["mixed"]["valu_per_cu_cycle"] - 400.0 / 0.5 / (256 * 2.4e9)) < 1e-24


def test_fp64_vs_oracle_statistics():
    """bench.py's FP64-vs-oracle statistic: the oracle's own chain handed in as
    the GPU's results agrees with itself; a planted 1e-6 energy error in one
    electron is counted against both references."""
    import types

    import numpy as np
    import torch

    sys.path.insert(0, ROOT)
    import bench
    import oracle as O
    from paper_2509_01741_amd import workloads

    wl = workloads.FULL_FP64
    rec = wl["lasers"][0]
    OL = O.laser_intensity(rec["lam"], rec["w0"], rec["tau"], rec["I"])
    K = wl["k_last"] - wl["k_first"] + 1
    na = 3
    ch = O.chain(OL, wl["seed"], wl["cfg_id"], np.arange(na), wl["r_factor"] * OL.w0,
                 O.rayleigh(OL), wl["k_first"], wl["k_last"])
    t = ch["t_birth"]
    out = (ch["ux"], ch["uy"], ch["uz"])
    ens = types.SimpleNamespace(tb=torch.from_numpy(t.copy()),
                                out=tuple(torch.from_numpy(o.copy()) for o in out),
                                x=torch.from_numpy(ch["x"]), y=torch.from_numpy(ch["y"]),
                                z=torch.from_numpy(ch["z"]))
    r = bench.fp64_vs_oracle(ens, OL, K, na, ch)
    born = int(np.isfinite(t).sum())
    v = r["energy_rule"]
    assert r["electrons"] == born and r["born_mismatch"] == 0
    assert r["birth_time_max_rel"] == 0.0 and r["raw_chain_frac_le_1e8"] == 1.0
    assert v["misses_vs_oracle"] == 0 and v["same_direction"] == 1.0
    assert v["misses_vs_extended"] == v["oracle_misses_vs_extended"]
    j = int(np.nonzero(np.isfinite(t))[0][0])
    bad = [o.copy() for o in out]
    bad[0][j] *= 1.0 + 1e-6
    ens.out = tuple(torch.from_numpy(o) for o in bad)
    r = bench.fp64_vs_oracle(ens, OL, K, na, ch)
    assert r["energy_rule"]["misses_vs_oracle"] == 1
    assert r["energy_rule"]["misses_vs_extended"] >= 1


def test_parity_rule_counts():
    """oracle/parity.py: misses against each reference are counted over every
    electron, the allowance is floor(0.001 n), and each rule can fail alone."""
    import numpy as np

    sys.path.insert(0, ROOT)
    from oracle import parity
    n = 3000
    K = np.linspace(0.1, 10.0, n)
    f = np.ones(n, dtype=bool)
    assert parity.allowed_misses(n) == 3 and parity.allowed_misses(999) == 0
    v = parity.fp64_energy_verdict(K, f, K, f, Kx=K, Koc=K)
    assert v["passed"] and v["misses_vs_oracle"] == 0 and v["oracle_misses_vs_extended"] == 0
    Kg = K.copy()
    Kg[:3] *= 1 + 2e-8
    assert parity.fp64_energy_verdict(Kg, f, K, f, Kx=K)["passed"]          # 3 of 3000
    Kg[3] *= 1 + 2e-8
    v = parity.fp64_energy_verdict(Kg, f, K, f, Kx=K)
    assert not v["passed"] and v["misses_vs_oracle"] == 4 and v["misses_vs_extended"] == 4
    Kx = K.copy()
    Kx[:4] *= 1 + 2e-8                                                      # only the exact answer differs
    v = parity.fp64_energy_verdict(K, f, K, f, Kx=Kx)
    assert not v["passed"] and v["misses_vs_oracle"] == 0 and v["misses_vs_extended"] == 4
    g = f.copy()
    g[:4] = False                                                           # directions alone
    assert not parity.fp64_energy_verdict(K, g, K, f, Kx=K)["passed"]
    # the absolute floor: 1e-12 MeV
    assert parity.within(np.array([1e-13]), np.array([5e-13])).all()
