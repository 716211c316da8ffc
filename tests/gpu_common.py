"""Shared helpers for the GPU tests (inputs and tolerances; no physics)."""
import numpy as np
import pytest

C_LIGHT = 299792458.0

# Plain FP64 ensemble beam: 0.8 um, w0 = 3 um, 30 fs FWHM, 1e21 W/cm^2.
BEAM = dict(lam=0.8e-6, w0=3e-6, tau=30e-15, I=1e21)


def require_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def energy_parity(ux_a, uy_a, uz_a, ux_b, uy_b, uz_b, orc):
    """Fraction of electrons whose kinetic energies agree to 1e-8 relative
    (+1e-12 MeV) and whose forward/backward flags agree."""
    Ka, _, _, fa = orc.epilogue(ux_a, uy_a, uz_a)
    Kb, _, _, fb = orc.epilogue(ux_b, uy_b, uz_b)
    ok = np.abs(Ka - Kb) <= 1e-8 * np.abs(Kb) + 1e-12
    return ok, fa == fb, Ka, Kb


def allowed_failures(n, frac=0.999):
    return int(np.floor((1 - frac) * n))
