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


def gpu_energy(B, torch, ux, uy, uz):
    """Kinetic energy [MeV] and forward flag from the library's own epilogue
    kernel, for GPU momenta (tensors or arrays)."""
    t = [a.contiguous().to(device="cuda", dtype=torch.float64) if isinstance(a, torch.Tensor)
         else torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")
         for a in (ux, uy, uz)]
    K, _, _, fwd = B.rpdla_epilogue(*t)
    return K.cpu().numpy(), fwd.cpu().numpy()


def energy_parity(Kg, fg, Ko, fo):
    """Per electron: energies agree to 1e-8 relative (+1e-12 MeV); directions
    agree."""
    from oracle import parity
    return parity.within(Kg, Ko), np.asarray(fg) == np.asarray(fo)


def allowed_failures(n, frac=0.999):
    from oracle import parity
    return parity.allowed_misses(n, frac)


def check_fp64_values(Kg, fg, Kop, fop, Kx=None, Koc=None, label=""):
    """The FP64 energy rule (oracle/parity.py) on energies the caller computed
    for the same born electrons; asserts and returns the verdict."""
    import sys

    from oracle import parity
    v = parity.fp64_energy_verdict(Kg, fg, Kop, fop, Kx=Kx, Koc=Koc)
    print(parity.summary(v, label), file=sys.stderr, flush=True)
    assert v["passed"], v
    return v


def check_fp64(O, OL, Kg, fg, tb_gpu, xs, ys, zs, K, Kx=None, Koc=None, label="",
               extended_push=False):
    """The FP64 energy rule (oracle/parity.py) for the born slots of
    per-slot arrays: the GPU's energies Kg and flags fg (born slots only),
    tb_gpu the GPU's birth times of all slots, xs, ys, zs the atoms (slot s
    belongs to atom s // K).  The double oracle pushes the same electrons from
    the GPU's births; the extended reference is Kx (born slots), or, with
    extended_push, the extended build's push of the same inputs.  Asserts
    and returns the verdict."""
    fin = np.isfinite(tb_gpu)
    ref = O.push(OL, tb_gpu, xs, ys, zs, K)
    Kop, _, _, fop = O.epilogue(*(r[fin] for r in ref[:3]))
    if extended_push:
        ext = O.push(OL, tb_gpu, xs, ys, zs, K, extended=True)
        Kx = O.epilogue(*(r[fin] for r in ext[:3]))[0]
    return check_fp64_values(Kg, fg, Kop, fop, Kx=Kx, Koc=Koc, label=label)
