"""The hot path for one workload, entirely in the gfx950 kernels: sample
atoms -> ionization times -> push -> histogram (one laser) or the batched
persistent sweep (several lasers).  Python only sequences the C ABI calls.
"""
from __future__ import annotations

import torch

from . import binding as B


def laser_of(rec: dict, order: int = 5) -> B.rpdla_laser:
    """rpdla_laser for a workload laser record (keys lam, w0, tau, I or P)."""
    if "I" in rec:
        L = B.rpdla_laser_init_intensity(rec["lam"], rec["w0"], rec["tau"], rec["I"])
    else:
        L = B.rpdla_laser_init_power(rec["lam"], rec["w0"], rec["tau"], rec["P"])
    L.field = order
    return L


def hist_spec(h: dict, angle: int = B.RPDLA_ANG_POLAR) -> B.rpdla_hist_spec:
    return B.rpdla_hist_spec(h["nE"], h["nA"], h["logE_min"], h["logE_max"], angle)


class Ensemble:
    """Device buffers for one single-laser ensemble, reused across steps."""

    def __init__(self, wl: dict, precision: int = B.RPDLA_FP64, n_atoms: int | None = None,
                 device="cuda"):
        self.wl = wl
        self.L = laser_of(wl["lasers"][0], wl.get("field_order", 5))
        self.precision = precision
        self.n = int(n_atoms if n_atoms is not None else wl["atoms"])
        self.K = wl["k_last"] - wl["k_first"] + 1
        self.spec = hist_spec(wl["hist"])
        dev = torch.device(device)
        f64 = dict(dtype=torch.float64, device=dev)
        self.x, self.y, self.z = (torch.empty(self.n, **f64) for _ in range(3))
        self.tb = torch.empty(self.n * self.K, **f64)
        self.out = tuple(torch.empty(self.n * self.K, **f64) for _ in range(6))
        self.counts = torch.zeros((2, self.spec.nE, self.spec.nA), dtype=torch.int64, device=dev)
        self.tallies = torch.zeros(B.RPDLA_NTALLY, dtype=torch.int64, device=dev)

    def sample(self, stream=None):
        wl, L = self.wl, self.L
        B.rpdla_sample_atoms(wl["seed"], wl["cfg_id"], 0, self.n, wl["r_factor"] * L.w0,
                             B.rpdla_rayleigh(L), self.x, self.y, self.z, stream=stream)

    def ionize(self, stream=None):
        wl = self.wl
        B.rpdla_ionize(self.L, wl["seed"], wl["cfg_id"], 0, self.x, self.y, self.z, wl["k_first"],
                       wl["k_last"], self.tb, stream=stream)

    def push(self, stream=None):
        B.rpdla_push(self.L, self.precision, self.tb, self.x, self.y, self.z, self.K, self.out,
                     stream=stream)

    def histogram(self, stream=None):
        self.counts.zero_()
        self.tallies.zero_()
        ux, uy, uz = self.out[:3]
        B.rpdla_histogram(self.tb, ux, uy, uz, self.spec, self.counts, self.tallies, stream=stream)

    def step(self, stream=None):
        self.sample(stream)
        self.ionize(stream)
        self.push(stream)
        self.histogram(stream)


def run_sweep(wl: dict, precision: int, atoms_per_cfg: int | None = None,
              atoms_per_chunk: int | None = None, stream=None, workspace=None, counts=None,
              tallies=None, electron_steps=None):
    """Batched persistent sweep over every laser of a workload."""
    lasers = [laser_of(r, wl.get("field_order", 5)) for r in wl["lasers"]]
    n = int(atoms_per_cfg if atoms_per_cfg is not None else wl["atoms"])
    apc = int(atoms_per_chunk if atoms_per_chunk is not None else wl.get("chunk", n))
    apc = max(1, min(apc, n)) if n > 0 else 1
    return B.rpdla_run_batched(lasers, wl["seed"], wl["cfg_id"] * 1000, n, apc, wl["r_factor"],
                               wl["k_first"], wl["k_last"], precision, hist_spec(wl["hist"]),
                               counts=counts, tallies=tallies, workspace=workspace, stream=stream,
                               electron_steps=electron_steps)
