"""Python binding of the C ABI in ``include/rpdla.h`` (argument marshalling
only).  Every function has the C name; arrays are torch CUDA tensors (device
memory), the stream is torch's current stream unless one is given.  All the
arithmetic happens in the gfx950 kernels of ``librpdla.so``: if the library
is missing the import fails loudly -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "librpdla.so")

RPDLA_OK, RPDLA_EINVAL, RPDLA_ERANGE, RPDLA_EHIP, RPDLA_ENOMEM, RPDLA_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
RPDLA_RP_O1, RPDLA_RP_O3, RPDLA_RP_O5, RPDLA_PLANE_LP, RPDLA_UNIFORM_EB = 1, 3, 5, 10, 11
RPDLA_LP_O1, RPDLA_LP_O3, RPDLA_LP_O5 = 21, 23, 25
RPDLA_FP64, RPDLA_MIXED = 0, 1
RPDLA_WIN_ARRIVAL, RPDLA_WIN_LAB = 0, 1
RPDLA_ANG_POLAR, RPDLA_ANG_AZIMUTH = 0, 1
RPDLA_NTALLY = 6


class RpdlaError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: status {status}: {detail}")
        self.status = status


class rpdla_laser(C.Structure):
    _fields_ = [
        ("lambda_", C.c_double), ("w0", C.c_double), ("tau_fwhm", C.c_double),
        ("amp", C.c_double), ("phi0", C.c_double),
        ("field", C.c_int32), ("window", C.c_int32),
        ("t_before", C.c_double), ("t_after", C.c_double), ("dt", C.c_double),
        ("ez_scale", C.c_double), ("er_scale", C.c_double),
        ("test_E", C.c_double * 3), ("test_B", C.c_double * 3),
    ]

    def set(self, **kw):
        for k, v in kw.items():
            if k in ("test_E", "test_B"):
                getattr(self, k)[:] = [float(a) for a in v]
            elif k in ("lam", "lambda"):
                self.lambda_ = float(v)
            else:
                setattr(self, k, v)
        return self


class rpdla_hist_spec(C.Structure):
    _fields_ = [("nE", C.c_int32), ("nA", C.c_int32), ("logE_min_MeV", C.c_double),
                ("logE_max_MeV", C.c_double), ("angle", C.c_int32)]


class rpdla_adaptive(C.Structure):
    _fields_ = [("rtol", C.c_double), ("atol", C.c_double), ("h_max", C.c_double),
                ("k_tol", C.c_double), ("max_steps", C.c_int64)]


def adaptive_settings(rtol=1e-9, atol=1e-9, h_max=0.0, k_tol=1e-10, max_steps=10_000_000):
    """rpdla_adaptive with the library's defaults (h_max <= 0: ten steps dt)."""
    return rpdla_adaptive(rtol, atol, h_max, k_tol, max_steps)


class rpdla_hist2d_spec(C.Structure):
    _fields_ = [("na", C.c_int32), ("nb", C.c_int32), ("a_lo", C.c_double), ("a_hi", C.c_double),
                ("b_lo", C.c_double), ("b_hi", C.c_double)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is not built: run `python -m paper_2509_01741_amd.build` "
            "(hipcc, gfx950); the library has no CPU fallback")
    # torch is imported above, so the library's HIP calls bind to the HIP
    # runtime torch already loaded (one runtime per process, one view of the
    # device); a process that loads librpdla.so before torch gets two
    lib = C.CDLL(LIB_PATH)
    vp, i32, i64, u32, u64, d = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32, C.c_uint64, C.c_double
    LP = C.POINTER(rpdla_laser)
    HP = C.POINTER(rpdla_hist_spec)
    sig = {
        "rpdla_laser_init_intensity": (i32, [LP, d, d, d, d]),
        "rpdla_laser_init_power": (i32, [LP, d, d, d, d]),
        "rpdla_rayleigh": (d, [LP]),
        "rpdla_sample_atoms": (i32, [u64, u32, u64, i64, d, d, vp, vp, vp, vp]),
        "rpdla_ionize": (i32, [LP, u64, u32, u64, i64, vp, vp, vp, i32, i32, vp, vp]),
        "rpdla_sample_atoms_annulus": (i32, [u64, u32, u64, i64, d, d, d, vp, vp, vp, vp]),
        "rpdla_birth_phase": (i32, [LP, i64, vp, vp, vp, vp, i32, vp, vp, vp]),
        "rpdla_push_rr": (i32, [LP, i32, i64, vp, vp, vp, vp, i32, vp, vp, vp, vp, vp, vp, vp,
                                vp]),
        "rpdla_push_adaptive": (i32, [LP, C.POINTER(rpdla_adaptive), i64, vp, vp, vp, vp, i32,
                                      vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]),
        "rpdla_batched_workspace_layout": (i32, [i32, i64, i32, i32, C.POINTER(C.c_size_t)]),
        "rpdla_histogram2d": (i32, [i64, vp, vp, vp, C.POINTER(rpdla_hist2d_spec), vp, vp, vp]),
        "rpdla_push": (i32, [LP, i32, i64, vp, vp, vp, vp, i32, vp, vp, vp, vp, vp, vp, vp]),
        "rpdla_push_noalloc": (i32, [LP, i32, i64, vp, vp, vp, vp, i32, vp, vp, vp, vp, vp, vp,
                                     vp]),
        "rpdla_histogram": (i32, [i64, vp, vp, vp, vp, HP, vp, vp, vp]),
        "rpdla_epilogue": (i32, [i64, vp, vp, vp, vp, vp, vp, vp, vp]),
        "rpdla_batched_workspace_bytes": (C.c_size_t, [i32, i64, i32, i32]),
        "rpdla_batched_graphs": (i32, []),
        "rpdla_run_batched": (i32, [LP, i32, u64, u32, i64, i64, d, i32, i32, i32, HP, vp, vp,
                                    vp, vp, C.c_size_t, vp]),
        "rpdla_run_batched_range": (i32, [LP, i32, u64, u32, i64, i64, i64, i64, d, i32, i32, i32,
                                          HP, vp, vp, vp, vp, C.c_size_t, vp]),
        "rpdla_autotune": (i32, [LP, i32, i64, i32, i32, C.c_char_p, C.c_size_t, vp]),
        "rpdla_set_launch_shape": (i32, [i32, i32, i32, i32, i32]),
        "rpdla_get_launch_shape": (i32, [i32, i32, i32, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
        "rpdla_kernel_occupancy": (i32, [i32, i32, i32, C.POINTER(C.c_int32),
                                         C.POINTER(C.c_int32), C.POINTER(C.c_double)]),
        "rpdla_status_string": (C.c_char_p, [i32]),
        "rpdla_last_error": (C.c_char_p, []),
        "rpdla_version": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


def _check(status: int, where: str):
    if status != RPDLA_OK:
        raise RpdlaError(status, where, lib.rpdla_last_error().decode())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _dev(t: torch.Tensor, name: str, n: int, dtype=torch.float64):
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() < n:
        raise ValueError(f"{name} has {t.numel()} elements, need {n}")
    return C.c_void_p(t.data_ptr() if t.numel() else 0)


def _empty(n, like=None, dtype=torch.float64, device=None):
    dev = device if device is not None else (like.device if like is not None else "cuda")
    return torch.empty(n, dtype=dtype, device=dev)


def rpdla_version() -> str:
    return lib.rpdla_version().decode()


def rpdla_laser_init_intensity(lam, w0, tau_fwhm, I_W_cm2, **kw) -> rpdla_laser:
    L = rpdla_laser()
    _check(lib.rpdla_laser_init_intensity(C.byref(L), lam, w0, tau_fwhm, I_W_cm2),
           "rpdla_laser_init_intensity")
    return L.set(**kw)


def rpdla_laser_init_power(lam, w0, tau_fwhm, P_W, **kw) -> rpdla_laser:
    L = rpdla_laser()
    _check(lib.rpdla_laser_init_power(C.byref(L), lam, w0, tau_fwhm, P_W), "rpdla_laser_init_power")
    return L.set(**kw)


def rpdla_rayleigh(L: rpdla_laser) -> float:
    return lib.rpdla_rayleigh(C.byref(L))


def rpdla_sample_atoms(seed, cfg_id, first_atom, n_atoms, r_max, z_half, x=None, y=None, z=None,
                       stream=None, device=None):
    x = _empty(n_atoms, device=device) if x is None else x
    y = _empty(n_atoms, like=x) if y is None else y
    z = _empty(n_atoms, like=x) if z is None else z
    _check(lib.rpdla_sample_atoms(seed, cfg_id, first_atom, n_atoms, r_max, z_half,
                                  _dev(x, "x", n_atoms), _dev(y, "y", n_atoms),
                                  _dev(z, "z", n_atoms), _stream(stream)), "rpdla_sample_atoms")
    return x, y, z


def rpdla_sample_atoms_annulus(seed, cfg_id, first_atom, n_atoms, r_in, r_out, z_half, x=None,
                               y=None, z=None, stream=None, device=None):
    x = _empty(n_atoms, device=device) if x is None else x
    y = _empty(n_atoms, like=x) if y is None else y
    z = _empty(n_atoms, like=x) if z is None else z
    _check(lib.rpdla_sample_atoms_annulus(seed, cfg_id, first_atom, n_atoms, r_in, r_out, z_half,
                                          _dev(x, "x", n_atoms), _dev(y, "y", n_atoms),
                                          _dev(z, "z", n_atoms), _stream(stream)),
           "rpdla_sample_atoms_annulus")
    return x, y, z


def rpdla_birth_phase(L, t_birth, x, y, z, slots_per_atom, phase=None, r_birth=None,
                      want_radius=True, stream=None):
    """Returns (phase, r_birth); r_birth is None when want_radius is False."""
    n = t_birth.numel()
    na = (n + slots_per_atom - 1) // slots_per_atom
    phase = _empty(n, like=t_birth) if phase is None else phase
    if want_radius and r_birth is None:
        r_birth = _empty(n, like=t_birth)
    rp = _dev(r_birth, "r_birth", n) if r_birth is not None else None
    _check(lib.rpdla_birth_phase(C.byref(L), n, _dev(t_birth, "t_birth", n), _dev(x, "x", na),
                                 _dev(y, "y", na), _dev(z, "z", na), slots_per_atom,
                                 _dev(phase, "phase", n), rp, _stream(stream)),
           "rpdla_birth_phase")
    return phase, r_birth


def rpdla_histogram2d(a, b, uz, spec, counts=None, tallies=None, stream=None):
    """counts: int64 tensor [2, na, nb] and tallies: int64 tensor [2] (the
    library adds unsigned 64-bit counts into them)."""
    n = a.numel()
    nbins = 2 * spec.na * spec.nb
    if counts is None:
        counts = torch.zeros((2, spec.na, spec.nb), dtype=torch.int64, device=a.device)
    if tallies is None:
        tallies = torch.zeros(2, dtype=torch.int64, device=a.device)
    _check(lib.rpdla_histogram2d(n, _dev(a, "a", n), _dev(b, "b", n), _dev(uz, "uz", n),
                                 C.byref(spec), _dev(counts, "counts", nbins, torch.int64),
                                 _dev(tallies, "tallies", 2, torch.int64), _stream(stream)),
           "rpdla_histogram2d")
    return counts, tallies


def rpdla_ionize(L, seed, cfg_id, first_atom, x, y, z, k_first, k_last, t_birth=None, stream=None):
    n = x.numel()
    K = k_last - k_first + 1
    t_birth = _empty(n * K, like=x) if t_birth is None else t_birth
    _check(lib.rpdla_ionize(C.byref(L), seed, cfg_id, first_atom, n, _dev(x, "x", n),
                            _dev(y, "y", n), _dev(z, "z", n), k_first, k_last,
                            _dev(t_birth, "t_birth", n * K), _stream(stream)), "rpdla_ionize")
    return t_birth


def rpdla_push(L, precision, t_birth, x0, y0, z0, slots_per_atom, out=None, stream=None):
    n = t_birth.numel()
    na = (n + slots_per_atom - 1) // slots_per_atom
    if out is None:
        out = tuple(_empty(n, like=t_birth) for _ in range(6))
    ux, uy, uz, xf, yf, zf = out
    _check(lib.rpdla_push(C.byref(L), precision, n, _dev(t_birth, "t_birth", n),
                          _dev(x0, "x0", na), _dev(y0, "y0", na), _dev(z0, "z0", na),
                          slots_per_atom, _dev(ux, "ux", n), _dev(uy, "uy", n), _dev(uz, "uz", n),
                          _dev(xf, "xf", n), _dev(yf, "yf", n), _dev(zf, "zf", n),
                          _stream(stream)), "rpdla_push")
    return out


def rpdla_push_noalloc(L, precision, t_birth, x0, y0, z0, slots_per_atom, out, stream=None):
    """rpdla_push without device allocation: the caller passes the six output
    tensors ``out`` = (ux, uy, uz, xf, yf, zf); the library's own 256-byte
    device array holds the work counter (overlapping calls on one GPU race)."""
    n = t_birth.numel()
    na = (n + slots_per_atom - 1) // slots_per_atom
    ux, uy, uz, xf, yf, zf = out
    _check(lib.rpdla_push_noalloc(C.byref(L), precision, n, _dev(t_birth, "t_birth", n),
                                  _dev(x0, "x0", na), _dev(y0, "y0", na), _dev(z0, "z0", na),
                                  slots_per_atom, _dev(ux, "ux", n), _dev(uy, "uy", n),
                                  _dev(uz, "uz", n), _dev(xf, "xf", n), _dev(yf, "yf", n),
                                  _dev(zf, "zf", n), _stream(stream)), "rpdla_push_noalloc")
    return out


def rpdla_push_rr(L, radiation_reaction, t_birth, x0, y0, z0, slots_per_atom, out=None,
                  chi_max=None, want_chi=True, stream=None):
    """FP64 push with Eq. (3)'s radiation term on (1) or off (0); returns
    (ux, uy, uz, xf, yf, zf, chi_max), chi_max None when want_chi is False."""
    n = t_birth.numel()
    na = (n + slots_per_atom - 1) // slots_per_atom
    if out is None:
        out = tuple(_empty(n, like=t_birth) for _ in range(6))
    if want_chi and chi_max is None:
        chi_max = _empty(n, like=t_birth)
    ux, uy, uz, xf, yf, zf = out
    cp = _dev(chi_max, "chi_max", n) if chi_max is not None else None
    _check(lib.rpdla_push_rr(C.byref(L), int(radiation_reaction), n, _dev(t_birth, "t_birth", n),
                             _dev(x0, "x0", na), _dev(y0, "y0", na), _dev(z0, "z0", na),
                             slots_per_atom, _dev(ux, "ux", n), _dev(uy, "uy", n),
                             _dev(uz, "uz", n), _dev(xf, "xf", n), _dev(yf, "yf", n),
                             _dev(zf, "zf", n), cp, _stream(stream)), "rpdla_push_rr")
    return tuple(out) + (chi_max,)


def rpdla_push_adaptive(L, A, t_birth, x0, y0, z0, slots_per_atom, out=None, want_extra=True,
                        stream=None):
    """Controlled-step FP64 push; returns (ux, uy, uz, xf, yf, zf, t_stop,
    steps_accepted, steps_rejected), the last three None when want_extra is
    False."""
    n = t_birth.numel()
    na = (n + slots_per_atom - 1) // slots_per_atom
    if out is None:
        out = tuple(_empty(n, like=t_birth) for _ in range(6))
    ux, uy, uz, xf, yf, zf = out
    ts = acc = rej = None
    if want_extra:
        ts = _empty(n, like=t_birth)
        acc = torch.empty(n, dtype=torch.int64, device=t_birth.device)
        rej = torch.empty(n, dtype=torch.int64, device=t_birth.device)
    _check(lib.rpdla_push_adaptive(
        C.byref(L), C.byref(A), n, _dev(t_birth, "t_birth", n), _dev(x0, "x0", na),
        _dev(y0, "y0", na), _dev(z0, "z0", na), slots_per_atom, _dev(ux, "ux", n),
        _dev(uy, "uy", n), _dev(uz, "uz", n), _dev(xf, "xf", n), _dev(yf, "yf", n),
        _dev(zf, "zf", n), _dev(ts, "t_stop", n) if ts is not None else None,
        _dev(acc, "steps_accepted", n, torch.int64) if acc is not None else None,
        _dev(rej, "steps_rejected", n, torch.int64) if rej is not None else None,
        _stream(stream)), "rpdla_push_adaptive")
    return tuple(out) + (ts, acc, rej)


def rpdla_epilogue(ux, uy, uz, out=None, stream=None):
    """Returns (K_MeV, theta, psi, fwd) tensors for momenta ux, uy, uz."""
    n = ux.numel()
    if out is None:
        out = (_empty(n, like=ux), _empty(n, like=ux), _empty(n, like=ux),
               torch.empty(n, dtype=torch.int32, device=ux.device))
    K, th, ps, fw = out
    _check(lib.rpdla_epilogue(n, _dev(ux, "ux", n), _dev(uy, "uy", n), _dev(uz, "uz", n),
                              _dev(K, "K", n), _dev(th, "theta", n), _dev(ps, "psi", n),
                              _dev(fw, "fwd", n, torch.int32), _stream(stream)), "rpdla_epilogue")
    return out


def rpdla_histogram(t_birth, ux, uy, uz, spec: rpdla_hist_spec, counts=None, tallies=None,
                    stream=None):
    """counts: int64 tensor [2, nE, nA] and tallies: int64 tensor [6] (the
    library adds unsigned 64-bit counts into them)."""
    n = t_birth.numel()
    nb = 2 * spec.nE * spec.nA
    if counts is None:
        counts = torch.zeros((2, spec.nE, spec.nA), dtype=torch.int64, device=t_birth.device)
    if tallies is None:
        tallies = torch.zeros(RPDLA_NTALLY, dtype=torch.int64, device=t_birth.device)
    _check(lib.rpdla_histogram(n, _dev(t_birth, "t_birth", n), _dev(ux, "ux", n),
                               _dev(uy, "uy", n), _dev(uz, "uz", n), C.byref(spec),
                               _dev(counts, "counts", nb, torch.int64),
                               _dev(tallies, "tallies", RPDLA_NTALLY, torch.int64),
                               _stream(stream)), "rpdla_histogram")
    return counts, tallies


RPDLA_KERNEL_PUSH, RPDLA_KERNEL_IONIZE, RPDLA_KERNEL_BATCHED_PUSH = 0, 1, 2


def rpdla_autotune(L, precision, n_atoms=65536, k_first=1, k_last=10, stream=None) -> dict:
    """Tune launch shapes for L's field model and `precision`; returns the report."""
    import json
    buf = C.create_string_buffer(8192)
    _check(lib.rpdla_autotune(C.byref(L), precision, n_atoms, k_first, k_last, buf, len(buf),
                              _stream(stream)), "rpdla_autotune")
    return json.loads(buf.value.decode())


def rpdla_set_launch_shape(kernel, field, precision, block, grid_factor=1):
    _check(lib.rpdla_set_launch_shape(kernel, field, precision, block, grid_factor),
           "rpdla_set_launch_shape")


def rpdla_get_launch_shape(kernel, field, precision):
    b, g = C.c_int32(), C.c_int32()
    _check(lib.rpdla_get_launch_shape(kernel, field, precision, C.byref(b), C.byref(g)),
           "rpdla_get_launch_shape")
    return b.value, g.value


def rpdla_kernel_occupancy(kernel, field, precision) -> dict:
    """Vector registers, scratch bytes per lane and resident waves per SIMD of
    one kernel at its current launch shape (device query)."""
    v, s, w = C.c_int32(), C.c_int32(), C.c_double()
    _check(lib.rpdla_kernel_occupancy(kernel, field, precision, C.byref(v), C.byref(s), C.byref(w)),
           "rpdla_kernel_occupancy")
    return {"vgprs": v.value, "scratch_bytes": s.value, "waves_per_simd": w.value}


def rpdla_batched_workspace_bytes(n_cfg, atoms_per_chunk, k_first, k_last) -> int:
    return int(lib.rpdla_batched_workspace_bytes(n_cfg, atoms_per_chunk, k_first, k_last))


def rpdla_batched_graphs() -> int:
    """Chunk graphs held by the library (rpdla_run_batched on a side stream
    captures one per argument set)."""
    return int(lib.rpdla_batched_graphs())


RPDLA_WS_NARRAYS = 7
WS_ARRAYS = ("x", "y", "z", "t_birth", "ux", "uy", "uz")


def rpdla_batched_workspace_layout(n_cfg, atoms_per_chunk, k_first, k_last) -> dict:
    """Byte offsets of the last chunk's arrays in the batched workspace."""
    off = (C.c_size_t * RPDLA_WS_NARRAYS)()
    _check(lib.rpdla_batched_workspace_layout(n_cfg, atoms_per_chunk, k_first, k_last, off),
           "rpdla_batched_workspace_layout")
    return dict(zip(WS_ARRAYS, (int(v) for v in off)))


def batched_chunk_arrays(workspace, n_cfg, atoms_per_chunk, k_first, k_last) -> dict:
    """Views (float64 tensors) of the last chunk's arrays inside a workspace:
    x, y, z [n_cfg, apc] and t_birth, ux, uy, uz [n_cfg, apc, K]."""
    lay = rpdla_batched_workspace_layout(n_cfg, atoms_per_chunk, k_first, k_last)
    K = k_last - k_first + 1
    out = {}
    for name, o in lay.items():
        shape = (n_cfg, atoms_per_chunk) if name in ("x", "y", "z") else (n_cfg, atoms_per_chunk, K)
        cnt = int(np.prod(shape))
        out[name] = workspace[o:o + 8 * cnt].view(torch.float64).view(*shape)
    return out


def rpdla_run_batched(lasers, seed, cfg_base, atoms_per_cfg, atoms_per_chunk, r_factor, k_first,
                      k_last, precision, spec: rpdla_hist_spec, counts=None, tallies=None,
                      workspace=None, stream=None, device=None, electron_steps=None,
                      chunks=None):
    """Returns (counts [n_cfg, 2, nE, nA], tallies [n_cfg, 6]); electron_steps,
    if given, is an int64 tensor [n_cfg] that accumulates the RK4 steps.
    chunks=(first, count) runs only those chunks of the stream
    (rpdla_run_batched_range)."""
    n_cfg = len(lasers)
    arr = (rpdla_laser * n_cfg)(*lasers)
    nb = 2 * spec.nE * spec.nA
    dev = device if device is not None else "cuda"
    if counts is None:
        counts = torch.zeros((n_cfg, 2, spec.nE, spec.nA), dtype=torch.int64, device=dev)
    if tallies is None:
        tallies = torch.zeros((n_cfg, RPDLA_NTALLY), dtype=torch.int64, device=dev)
    need = rpdla_batched_workspace_bytes(n_cfg, atoms_per_chunk, k_first, k_last)
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=counts.device)
    first, count = (0, -1) if chunks is None else chunks
    _check(lib.rpdla_run_batched_range(arr, n_cfg, seed, cfg_base, atoms_per_cfg, atoms_per_chunk,
                                       first, count, r_factor, k_first, k_last, precision,
                                       C.byref(spec),
                                       _dev(counts, "counts", n_cfg * nb, torch.int64),
                                       _dev(tallies, "tallies", n_cfg * RPDLA_NTALLY, torch.int64),
                                       (C.c_void_p(0) if electron_steps is None else
                                        _dev(electron_steps, "electron_steps", n_cfg,
                                             torch.int64)),
                                       _dev(workspace, "workspace", need, torch.uint8),
                                       C.c_size_t(workspace.numel()), _stream(stream)),
           "rpdla_run_batched_range" if chunks is not None else "rpdla_run_batched")
    return counts, tallies
