"""Seeded synthetic workloads (parameters only, no physics).

Each workload is the parameter set of one Monte Carlo ensemble shaped like the
paper's runs (Sec. 2.1: ions at rest uniform in a cylinder about the axis;
Sec. 2.2: wavelength scan and intensity scan of a radially polarized focus),
scaled up.  The same records feed the HIP library and the CPU oracle; each
side derives everything else (Rayleigh length, amplitude, step) itself.

Fields of a laser record: ``lam`` wavelength [m], ``w0`` waist [m], ``tau``
intensity FWHM [s], and either ``I`` peak Gaussian-equivalent intensity
[W/cm^2] or ``P`` power [W].  Sampling cylinder: radius ``r_factor * w0``,
half-length one Rayleigh length.
"""
from __future__ import annotations

UM = 1e-6
FS = 1e-15
PW = 1e15
C_LIGHT = 299792458.0


def _cyc(lam):
    """Optical period of wavelength ``lam`` [s]."""
    return lam / C_LIGHT


# Plain FP64 ensemble, small enough for the oracle in full.
SMALL_FP64 = dict(
    name="rp_ne_fp64_1k",
    lasers=[dict(lam=0.8 * UM, w0=3.0 * UM, tau=30 * FS, I=1e21)],
    atoms=1024, k_first=1, k_last=8, seed=0, cfg_id=0, r_factor=2.0,
    field_order=5, hist=dict(nE=256, nA=180, logE_min=-3.0, logE_max=4.0),
)

# Plain FP64 full ensemble, same beam, ten charge states.
FULL_FP64 = dict(
    name="rp_ne_fp64_1m",
    lasers=[dict(lam=0.8 * UM, w0=3.0 * UM, tau=30 * FS, I=1e21)],
    atoms=1_000_000, k_first=1, k_last=10, seed=0, cfg_id=1, r_factor=2.0,
    field_order=5, hist=dict(nE=256, nA=180, logE_min=-3.0, logE_max=4.0),
)


def _sweep_lasers():
    out = []
    for lam_um in (0.8, 1.0, 1.5, 2.0, 3.0, 4.0, 5.0, 10.0):
        for p in (0.5, 1, 2, 5, 10, 20, 50, 100):
            lam = lam_um * UM
            out.append(dict(lam=lam, w0=2.0 * lam, tau=10.0 * _cyc(lam), P=p * PW))
    return out


# Batched sweep: 8 wavelengths x 8 powers in one persistent launch.
SWEEP_FP64 = dict(
    name="rp_ne_sweep64",
    lasers=_sweep_lasers(),
    atoms=65_536, k_first=1, k_last=10, seed=0, cfg_id=2, r_factor=2.0,
    field_order=5, hist=dict(nE=256, nA=180, logE_min=-3.0, logE_max=4.0),
)

# Mixed precision versus FP64.
MIXED_AB = dict(
    name="rp_ne_mixed_1m",
    lasers=[dict(lam=0.8 * UM, w0=1.5 * UM, tau=25 * FS, P=1 * PW)],
    atoms=1_000_000, k_first=1, k_last=10, seed=0, cfg_id=3, r_factor=2.0,
    field_order=5, hist=dict(nE=256, nA=180, logE_min=-3.0, logE_max=4.0),
)


def _large_lasers():
    out = []
    for lam_um in (0.8, 2.0, 5.0, 10.0):
        for wf in (1, 2, 3, 5):
            lam = lam_um * UM
            out.append(dict(lam=lam, w0=wf * lam, tau=10.0 * _cyc(lam), P=20 * PW))
    return out


# Large mixed + batched, streamed in chunks of atoms.
LARGE_MIXED = dict(
    name="rp_ne_large16",
    lasers=_large_lasers(),
    atoms=10_000_000, k_first=1, k_last=10, seed=0, cfg_id=4, r_factor=2.0,
    field_order=5, chunk=1_000_000,
    hist=dict(nE=512, nA=360, logE_min=-3.0, logE_max=4.0),
)

ALL = [SMALL_FP64, FULL_FP64, SWEEP_FP64, MIXED_AB, LARGE_MIXED]
