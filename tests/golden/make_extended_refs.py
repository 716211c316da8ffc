"""Writes the extended-precision oracle references under tests/golden/.

Every stored value comes from the oracle alone (oracle.chain with
extended=True: the same source as the double oracle, every step in x87
extended precision): for each reference below, the final kinetic energy
[MeV] of every slot (NaN where the state is not born) of the listed atoms,
each computed by the oracle's own chain from the seed -- sampling,
ionization, push.  The double oracle misses these energies by more than 1e-8
for a few electrons in ten thousand; the extended build resolves all of them,
which is why the FP64 parity rule (oracle/parity.py) is stated against it.

Usage:  python tests/golden/make_extended_refs.py [NAME ...]   (all by default)
It takes minutes to tens of minutes per reference on a few cores.
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_2509_01741_amd import workloads as W  # noqa: E402  (parameters only)


def oracle_laser(rec, order=5):
    if "I" in rec:
        L = O.laser_intensity(rec["lam"], rec["w0"], rec["tau"], rec["I"])
    else:
        L = O.laser_power(rec["lam"], rec["w0"], rec["tau"], rec["P"])
    L.field = order
    return L


def sampled_atoms(n_atoms, count, offset):
    """`count` atom indices spread over [0, n_atoms): offset, offset + step, ..."""
    step = max(1, n_atoms // count)
    return np.arange(offset, n_atoms, step, dtype=np.uint64)[:count]


def references():
    """name -> (workload, [(configuration index, cfg_id, atom indices)])."""
    refs = {}
    wl = W.SMALL_FP64
    refs["rp_ne_fp64_1k"] = (wl, [(0, wl["cfg_id"], np.arange(wl["atoms"], dtype=np.uint64))])
    wl = W.FULL_FP64
    refs["rp_ne_fp64_1m_head"] = (wl, [(0, wl["cfg_id"], np.arange(1200, dtype=np.uint64))])
    refs["rp_ne_fp64_1m_sampled"] = (wl, [(0, wl["cfg_id"], sampled_atoms(wl["atoms"], 150, 7))])
    wl = W.MIXED_AB
    refs["rp_ne_mixed_1m_sampled"] = (wl, [(0, wl["cfg_id"], sampled_atoms(wl["atoms"], 40, 11))])
    wl = W.SWEEP_FP64
    refs["rp_ne_sweep64_sampled"] = (
        wl, [(c, wl["cfg_id"] * 1000 + c, sampled_atoms(wl["atoms"], 64, 5))
             for c in range(len(wl["lasers"]))])
    return refs


def oracle_source_sha():
    with open(os.path.join(ROOT, "oracle", "rpdla_oracle.c"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def compute(name, extended=True):
    """Energies of the reference's slots: array [configs, atoms, states]."""
    wl, parts = references()[name]
    K = wl["k_last"] - wl["k_first"] + 1
    out = []
    for c, cfg_id, atoms in parts:
        L = oracle_laser(wl["lasers"][c], wl.get("field_order", 5))
        r = O.chain(L, wl["seed"], cfg_id, atoms, wl["r_factor"] * L.w0, O.rayleigh(L),
                    wl["k_first"], wl["k_last"], extended=extended)
        out.append(r["K"].reshape(atoms.size, K))
    return np.stack(out)


def path_of(name):
    return os.path.join(HERE, f"extended_{name}.npz")


def load(name):
    """(energies [configs, atoms, states], atom indices [configs, atoms],
    cfg_ids [configs], configuration indices [configs])."""
    with np.load(path_of(name), allow_pickle=False) as f:
        return f["K_MeV"], f["atoms"], f["cfg_ids"], f["configs"]


def write(name):
    wl, parts = references()[name]
    t0 = time.time()
    K = compute(name, extended=True)
    np.savez_compressed(path_of(name), K_MeV=K,
                        atoms=np.stack([p[2] for p in parts]).astype(np.uint64),
                        cfg_ids=np.array([p[1] for p in parts], dtype=np.uint64),
                        configs=np.array([p[0] for p in parts], dtype=np.int64))
    meta_path = os.path.join(HERE, "extended_refs.json")
    meta = json.load(open(meta_path)) if os.path.exists(meta_path) else {}
    meta[name] = dict(workload=wl["name"], k_first=wl["k_first"], k_last=wl["k_last"],
                      configs=len(parts), atoms_per_config=int(parts[0][2].size),
                      oracle_source_sha256_16=oracle_source_sha(),
                      seconds=round(time.time() - t0, 1))
    with open(meta_path, "w") as f:
        json.dump(meta, f, indent=1, sort_keys=True)
    print(f"{name}: {K.size} slots, {np.isfinite(K).sum()} born, {time.time() - t0:.0f} s",
          flush=True)


if __name__ == "__main__":
    O.build(force=False)
    for name in (sys.argv[1:] or list(references())):
        write(name)
