"""The paper's single-particle studies (Sec. 2.2) run on the same kernels as
the hot path: ion sampling (filled or hollow cylinder), ionization times,
the push, per-electron outputs, birth phase and radius, and histograms.
Python only sequences the C ABI calls and reduces the kernels' outputs to
the handful of numbers each study reports.

Studies (the paper's figure each one mirrors, with synthetic seeded ions):
  * ``birth_maps``      -- Figs. 6, 13, 14: birth phase and birth radius of
                           forward and backward electrons, and against energy;
  * ``target_radius``   -- Fig. 7: forward/backward yields for filled targets
                           of radius 1 and 4 um (four intensities, read as
                           5e19 .. 5e22 W/cm^2: the paper does not list them);
  * ``hollow_scan``     -- Fig. 8: yields for ions on a cylinder surface of
                           radius 0..4 um, 5e19 W/cm^2;
  * ``field_scale``     -- Fig. 9: yields with Ez or Er multiplied by s in
                           [0, 1], 5e19 W/cm^2;
  * ``wavelength_scan`` -- Fig. 5: energies for 0.8, 1 and 2 um at equal
                           intensity and f-number;
  * ``polarization``    -- Fig. 4: the radially polarized focus against the
                           linearly polarized one at the same intensity,
                           wavelength and f-number (backward electrons).

Paper set-up (Sec. 2.2): 800 nm unless stated, f/5, 53 fs pulses, Ne7+ ions
at rest freeing their eighth electron (charge state 8 only), targets of
radius lambda and length z_r about the focus.  The waist of an f/5 focus is
read as w0 = 2 lambda F / pi (Gaussian-beam optics; the paper gives only F).

Run:  python -m paper_2509_01741_amd.experiments STUDY [--atoms N] [--out FILE]
"""
from __future__ import annotations

import argparse
import json
import math
import sys

import torch

from . import binding as B

UM = 1e-6
FS = 1e-15

# Sec. 2.2: 800 nm, f/5, 53 fs; intensities 5e19, 5e20, 5e21 W/cm^2.
PAPER_LAMBDA = 0.8 * UM
PAPER_FNUM = 5.0
PAPER_TAU = 53 * FS
PAPER_INTENSITIES = (5e19, 5e20, 5e21)
NE7_STATE = 8          # Ne7+ -> Ne8+, the electron the paper follows


def f_number_waist(lam: float, fnum: float = PAPER_FNUM) -> float:
    """Gaussian-beam waist of an f/F focus, w0 = 2 lambda F / pi."""
    return 2.0 * lam * fnum / math.pi


def paper_laser(I_W_cm2: float, lam: float = PAPER_LAMBDA, fnum: float = PAPER_FNUM,
                tau: float = PAPER_TAU, order: int = B.RPDLA_RP_O5, **kw) -> B.rpdla_laser:
    L = B.rpdla_laser_init_intensity(lam, f_number_waist(lam, fnum), tau, I_W_cm2, **kw)
    L.field = order
    return L


def run(L: B.rpdla_laser, n_atoms: int, r_out: float, *, r_in: float = 0.0,
        z_half: float | None = None, k_first: int = NE7_STATE, k_last: int = NE7_STATE,
        seed: int = 0, cfg_id: int = 0, precision: int = B.RPDLA_FP64, stream=None) -> dict:
    """One ensemble through every kernel; device tensors per electron slot:
    t_birth, ux, uy, uz, xf, yf, zf, K, theta, psi, fwd, phase, r_birth."""
    zh = B.rpdla_rayleigh(L) if z_half is None else z_half
    x, y, z = B.rpdla_sample_atoms_annulus(seed, cfg_id, 0, n_atoms, r_in, r_out, zh,
                                           stream=stream, device="cuda")
    tb = B.rpdla_ionize(L, seed, cfg_id, 0, x, y, z, k_first, k_last, stream=stream)
    spa = k_last - k_first + 1
    ux, uy, uz, xf, yf, zf = B.rpdla_push(L, precision, tb, x, y, z, spa, stream=stream)
    K, theta, psi, fwd = B.rpdla_epilogue(ux, uy, uz, stream=stream)
    phase = rb = None
    if L.field not in (B.RPDLA_LP_O1, B.RPDLA_LP_O3, B.RPDLA_LP_O5):
        # the birth phase is the radial focus's carrier phase
        phase, rb = B.rpdla_birth_phase(L, tb, x, y, z, spa, stream=stream)
    return dict(x=x, y=y, z=z, t_birth=tb, ux=ux, uy=uy, uz=uz, xf=xf, yf=yf, zf=zf, K=K,
                theta=theta, psi=psi, fwd=fwd, phase=phase, r_birth=rb, slots_per_atom=spa)


def yields(res: dict) -> dict:
    """Forward/backward counts (kernel tallies) and energy summaries."""
    spec = B.rpdla_hist_spec(1, 1, -30.0, 30.0, B.RPDLA_ANG_POLAR)
    _, t = B.rpdla_histogram(res["t_birth"], res["ux"], res["uy"], res["uz"], spec)
    t = t.cpu().tolist()
    K, fwd = res["K"], res["fwd"]
    out = dict(n_slots=int(res["t_birth"].numel()), forward=t[0], backward=t[1], unborn=t[4],
               nan=t[5])
    for name, flag in (("forward", 1), ("backward", 0)):
        sel = K[fwd == flag]
        out[f"K_max_{name}_MeV"] = float(sel.max()) if sel.numel() else 0.0
        out[f"K_mean_{name}_MeV"] = float(sel.mean()) if sel.numel() else 0.0
    return out


def birth_maps(res: dict, n_phase: int = 36, n_r: int = 40, r_max: float | None = None,
               n_e: int = 40, logE=(-3.0, 3.0)) -> dict:
    """Figs. 13, 14: phase x radius counts of forward and backward electrons;
    Fig. 6: birth phase and radius against log10 of the final energy."""
    rb, ph, uz = res["r_birth"], res["phase"], res["uz"]
    if r_max is None:
        finite = rb[~torch.isnan(rb)]
        r_max = float(finite.max()) * (1 + 1e-12) if finite.numel() else 1.0
    pr, t_pr = B.rpdla_histogram2d(ph, rb, uz, B.rpdla_hist2d_spec(n_phase, n_r, 0.0, 2 * math.pi,
                                                                   0.0, r_max))
    lk = torch.log10(res["K"])
    pe, _ = B.rpdla_histogram2d(ph, lk, uz, B.rpdla_hist2d_spec(n_phase, n_e, 0.0, 2 * math.pi,
                                                                logE[0], logE[1]))
    re_, _ = B.rpdla_histogram2d(rb, lk, uz, B.rpdla_hist2d_spec(n_r, n_e, 0.0, r_max,
                                                                 logE[0], logE[1]))
    return dict(phase_radius=pr, phase_radius_tallies=t_pr, phase_energy=pe, radius_energy=re_,
                r_max=r_max, logE=logE)


def phase_near_zero_fraction(pr_counts: torch.Tensor, direction: int, width: float) -> float:
    """Fraction of direction's electrons whose birth phase lies within
    `width` of 0 (mod 2 pi), from a phase x radius histogram."""
    c = pr_counts[direction].sum(dim=1).double()
    n = c.numel()
    centres = (torch.arange(n, dtype=torch.float64) + 0.5) * (2 * math.pi / n)
    d = torch.minimum(centres, 2 * math.pi - centres)
    tot = float(c.sum())
    return float(c.cpu()[d <= width].sum()) / tot if tot else float("nan")


def radius_quantile(pr_counts: torch.Tensor, direction: int, r_max: float, q: float) -> float:
    """Radius below which a fraction q of direction's electrons were born."""
    c = pr_counts[direction].sum(dim=0).double().cpu()
    cs = torch.cumsum(c, 0)
    if cs[-1] == 0:
        return float("nan")
    i = int(torch.searchsorted(cs, q * cs[-1]))
    return (i + 1) * r_max / c.numel()


# ----------------------------------------------------------------------------- studies

def study_birth_maps(n_atoms: int, intensities=PAPER_INTENSITIES, r_target: float = 4 * UM,
                     seed: int = 0) -> list:
    """Target radius 4 um (the larger target of Fig. 7), wide enough to show
    where forward and backward electrons are born."""
    out = []
    for i, I in enumerate(intensities):
        L = paper_laser(I)
        res = run(L, n_atoms, r_target, seed=seed, cfg_id=100 + i)
        m = birth_maps(res)
        pr = m["phase_radius"]
        out.append(dict(I_W_cm2=I, **yields(res),
                        backward_phase_within_pi4_of_0=phase_near_zero_fraction(pr, 1, math.pi / 4),
                        forward_phase_within_pi4_of_0=phase_near_zero_fraction(pr, 0, math.pi / 4),
                        backward_r90_m=radius_quantile(pr, 1, m["r_max"], 0.9),
                        forward_r90_m=radius_quantile(pr, 0, m["r_max"], 0.9),
                        phase_radius_counts=pr.cpu().tolist(), r_max=m["r_max"]))
    return out


def study_target_radius(n_atoms: int, radii=(1 * UM, 4 * UM), intensities=(5e19, 5e20, 5e21, 5e22),
                        seed: int = 0) -> list:
    out = []
    for i, I in enumerate(intensities):
        L = paper_laser(I)
        for j, R in enumerate(radii):
            res = run(L, n_atoms, R, seed=seed, cfg_id=200 + 10 * i + j)
            out.append(dict(I_W_cm2=I, R_m=R, **yields(res)))
    return out


def study_hollow_scan(n_atoms: int, radii=tuple(0.25 * UM * k for k in range(17)), I: float = 5e19,
                      seed: int = 0) -> list:
    L = paper_laser(I)
    out = []
    for j, R in enumerate(radii):
        res = run(L, n_atoms, R, r_in=R, seed=seed, cfg_id=300 + j)
        out.append(dict(I_W_cm2=I, R_m=R, **yields(res)))
    return out


def study_field_scale(n_atoms: int, scales=(0.0, 0.25, 0.5, 0.75, 1.0), I: float = 5e19,
                      seed: int = 0) -> list:
    out = []
    for which in ("ez_scale", "er_scale"):
        for s in scales:
            L = paper_laser(I, **{which: s})
            res = run(L, n_atoms, PAPER_LAMBDA, seed=seed, cfg_id=400)
            out.append(dict(I_W_cm2=I, knob=which, scale=s, **yields(res)))
    return out


def study_wavelength_scan(n_atoms: int, lams=(0.8 * UM, 1.0 * UM, 2.0 * UM),
                          intensities=PAPER_INTENSITIES, seed: int = 0) -> list:
    out = []
    for i, I in enumerate(intensities):
        for j, lam in enumerate(lams):
            L = paper_laser(I, lam=lam)
            res = run(L, n_atoms, lam, seed=seed, cfg_id=500 + 10 * i + j)
            out.append(dict(I_W_cm2=I, lam_m=lam, **yields(res)))
    return out


def study_polarization(n_atoms: int, intensities=(5e19, 5e20, 5e21), r_target: float = 1 * UM,
                       seed: int = 0) -> list:
    """Fig. 4: radially against linearly polarized focus, same intensity,
    wavelength, f-number and pulse, the same seeded ions."""
    out = []
    for i, I in enumerate(intensities):
        for name, order in (("radial", B.RPDLA_RP_O5), ("linear", B.RPDLA_LP_O5)):
            res = run(paper_laser(I, order=order), n_atoms, r_target, seed=seed,
                      cfg_id=600 + i)
            out.append(dict(I_W_cm2=I, polarization=name, **yields(res)))
    return out


STUDIES = dict(birth_maps=study_birth_maps, target_radius=study_target_radius,
               hollow_scan=study_hollow_scan, field_scale=study_field_scale,
               wavelength_scan=study_wavelength_scan, polarization=study_polarization)


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("study", choices=sorted(STUDIES) + ["all"])
    ap.add_argument("--atoms", type=int, default=100_000)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default=None, help="write the results as JSON here")
    a = ap.parse_args(argv)
    if not torch.cuda.is_available():
        print("experiments need the GPU", file=sys.stderr)
        return 2
    names = sorted(STUDIES) if a.study == "all" else [a.study]
    results = {}
    for n in names:
        results[n] = STUDIES[n](a.atoms, seed=a.seed)
        torch.cuda.synchronize()
        short = [{k: v for k, v in r.items() if k != "phase_radius_counts"} for r in results[n]]
        print(json.dumps({n: short}), flush=True)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(results, f)
    return 0


if __name__ == "__main__":
    sys.exit(main())
