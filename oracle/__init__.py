"""Plain FP64 CPU oracle for the ionization-seeded electron-acceleration Monte
Carlo of arXiv 2509.01741 -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the HIP library:
the C source ``rpdla_oracle.c`` carries its own constants, tables, random
number generator and formulas, and is built with plain ``gcc -O2`` (no fast
math) into ``liborc.so`` next to it.

Every function here is a thin numpy <-> ctypes marshalling wrapper over the C
source; each C function cites the section or equation of the paper it
follows.  All quantities are SI.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rpdla_oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")
_LIB_EXT = os.path.join(_HERE, "liborc_ext.so")

RP_O1, RP_O3, RP_O5, PLANE_LP, UNIFORM_EB = 1, 3, 5, 10, 11
LP_O1, LP_O3, LP_O5 = 21, 23, 25
WIN_ARRIVAL, WIN_LAB = 0, 1
ANG_POLAR, ANG_AZIMUTH = 0, 1


def build(force: bool = True) -> str:
    """Compile ``rpdla_oracle.c`` into ``liborc.so`` (gcc -O2, OpenMP) and,
    with -DORC_EXTENDED, into ``liborc_ext.so`` (the same steps in x87
    extended precision)."""
    for path, extra in ((_LIB, []), (_LIB_EXT, ["-DORC_EXTENDED"])):
        if force or not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
            tmp = path + ".tmp%d" % os.getpid()
            cmd = ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared", "-Wall"] + extra + \
                  ["-o", tmp, _SRC, "-lm"]
            subprocess.run(cmd, check=True)
            os.replace(tmp, path)
    return _LIB


class Laser(C.Structure):
    """Mirror of the oracle's own laser record (SI units)."""
    _fields_ = [
        ("lambda_", C.c_double), ("w0", C.c_double), ("tau_fwhm", C.c_double),
        ("amp", C.c_double), ("phi0", C.c_double),
        ("field", C.c_int), ("window", C.c_int),
        ("t_before", C.c_double), ("t_after", C.c_double), ("dt", C.c_double),
        ("ez_scale", C.c_double), ("er_scale", C.c_double),
        ("test_E", C.c_double * 3), ("test_B", C.c_double * 3),
    ]


class HistSpec(C.Structure):
    _fields_ = [("nE", C.c_int), ("nA", C.c_int), ("logE_min_MeV", C.c_double),
                ("logE_max_MeV", C.c_double), ("angle", C.c_int)]


_lib = None
_D = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_U64 = np.ctypeslib.ndpointer(dtype=np.uint64, flags="C_CONTIGUOUS")
_I32 = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_I64 = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")


def lib():
    """The oracle library (plain double), or the one RPDLA_ORACLE_LIB names:
    the mutation check (tests/test_pins_mutations.py) points it at a copy with
    one planted mistake, and the pins are also run against liborc_ext.so."""
    global _lib
    if _lib is None:
        path = os.environ.get("RPDLA_ORACLE_LIB")
        if path is None:
            path = _LIB
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
        _lib = _bind(C.CDLL(path))
    return _lib


_lib_ext = None


def lib_extended():
    """The same oracle built to compute in x87 extended precision."""
    global _lib_ext
    if _lib_ext is None:
        if not os.path.exists(_LIB_EXT) or os.path.getmtime(_LIB_EXT) < os.path.getmtime(_SRC):
            build(force=True)
        _lib_ext = _bind(C.CDLL(_LIB_EXT))
    return _lib_ext


def _bind(L):
    LP = C.POINTER(Laser)
    sig = {
        "orc_constants": (None, [_D]),
        "orc_laser_init_intensity": (None, [LP, C.c_double, C.c_double, C.c_double, C.c_double]),
        "orc_laser_init_power": (None, [LP, C.c_double, C.c_double, C.c_double, C.c_double]),
        "orc_rayleigh": (C.c_double, [LP]),
        "orc_philox4x64_10": (None, [_U64, _U64, _U64]),
        "orc_uniform": (C.c_double, [C.c_uint64, C.c_uint32, C.c_uint64, C.c_int]),
        "orc_uniform_batch": (None, [C.c_uint64, C.c_uint32, C.c_int64, _U64, _I32, _D]),
        "orc_sample_atoms": (None, [C.c_uint64, C.c_uint32, C.c_uint64, C.c_int64,
                                    C.c_double, C.c_double, _D, _D, _D]),
        "orc_field_batch": (None, [LP, C.c_int64, _D, _D, _D, _D, _D, _D]),
        "orc_adk_lnrate_general": (C.c_double, [C.c_double, C.c_double, C.c_double]),
        "orc_adk_lnrate": (C.c_double, [C.c_int, C.c_double]),
        "orc_adk_rate": (C.c_double, [C.c_int, C.c_double]),
        "orc_adk_rate_batch": (None, [C.c_int, C.c_int64, _D, _D]),
        "orc_gl4_table": (None, [_D, _D]),
        "orc_ionize": (None, [LP, C.c_uint64, C.c_uint32, C.c_uint64, C.c_int64,
                              _D, _D, _D, C.c_int, C.c_int, _D]),
        "orc_push_one": (None, [LP, C.c_double, C.c_double, C.c_double, _D, _D, _D, _D]),
        "orc_push": (None, [LP, C.c_int64, _D, _D, _D, _D, C.c_int, _D, _D, _D, _D, _D, _D]),
        "orc_epilogue": (None, [C.c_int64, _D, _D, _D, _D, _D, _D, _I32]),
        "orc_histogram": (None, [C.c_int64, _D, _D, _D, _D, C.POINTER(HistSpec), _U64, _U64]),
        "orc_num_threads": (C.c_int, []),
        "orc_birth_phase": (None, [LP, C.c_int64, _D, _D, _D, _D, C.c_int, _D]),
        "orc_sample_atoms_annulus": (None, [C.c_uint64, C.c_uint32, C.c_uint64, C.c_int64,
                                            C.c_double, C.c_double, C.c_double, _D, _D, _D]),
        "orc_histogram2d": (None, [C.c_int64, _D, _D, _D, C.c_int32, C.c_double, C.c_double,
                                   C.c_int32, C.c_double, C.c_double, _U64, _U64]),
        "orc_critical_field": (C.c_double, []),
        "orc_rr_terms": (None, [LP, C.c_double, _D, _D, _D]),
        "orc_push_one_rr": (None, [LP, C.c_int, C.c_double, C.c_double, C.c_double, _D, _D, _D,
                                   _D, _D]),
        "orc_push_rr": (None, [LP, C.c_int, C.c_int64, _D, _D, _D, _D, C.c_int, _D, _D, _D, _D,
                               _D, _D, _D]),
        "orc_push_one_adaptive": (C.c_int, [LP, C.POINTER(Adaptive), C.c_double, C.c_double,
                                            _D, _D, _D, _D, _D, _I64, _I64]),
        "orc_push_adaptive": (None, [LP, C.POINTER(Adaptive), C.c_int64, _D, _D, _D, _D, C.c_int,
                                     _D, _D, _D, _D, _D, _D, _D, _I64, _I64]),
        "orc_dp_tableau": (None, [_D, _D, _D, _D]),
        "orc_ne_ip_table": (None, [_D]),
        "orc_is_extended": (C.c_int, []),
        "orc_chain": (None, [LP, C.c_uint64, C.c_uint32, _U64, C.c_int64, C.c_double,
                             C.c_double, C.c_int, C.c_int, _D, _D, _D, _D, _D, _D, _D, _D]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    return L


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def constants() -> dict:
    out = np.zeros(8)
    lib().orc_constants(out)
    keys = ["c", "qe", "me", "eps0", "mec2_MeV", "Ea", "tau_a", "Eh_eV"]
    return dict(zip(keys, out.tolist()))


def ne_ip_ev() -> np.ndarray:
    out = np.zeros(10)
    lib().orc_ne_ip_table(out)
    return out


def laser_intensity(lam, w0, tau_fwhm, I_W_cm2, **kw) -> Laser:
    L = Laser()
    lib().orc_laser_init_intensity(C.byref(L), lam, w0, tau_fwhm, I_W_cm2)
    for k, v in kw.items():
        _set(L, k, v)
    return L


def laser_power(lam, w0, tau_fwhm, P_W, **kw) -> Laser:
    L = Laser()
    lib().orc_laser_init_power(C.byref(L), lam, w0, tau_fwhm, P_W)
    for k, v in kw.items():
        _set(L, k, v)
    return L


def _set(L, k, v):
    if k in ("test_E", "test_B"):
        getattr(L, k)[:] = list(v)
    elif k == "lam":
        L.lambda_ = v
    else:
        setattr(L, k, v)


def rayleigh(L: Laser) -> float:
    return lib().orc_rayleigh(C.byref(L))


def philox(ctr, key) -> np.ndarray:
    out = np.zeros(4, dtype=np.uint64)
    lib().orc_philox4x64_10(np.ascontiguousarray(ctr, dtype=np.uint64),
                            np.ascontiguousarray(key, dtype=np.uint64), out)
    return out


def uniform(seed, cfg, atoms, js) -> np.ndarray:
    atoms = np.ascontiguousarray(atoms, dtype=np.uint64)
    js = np.ascontiguousarray(np.broadcast_to(js, atoms.shape), dtype=np.int32)
    u = np.zeros(atoms.shape, dtype=np.float64)
    lib().orc_uniform_batch(seed, cfg, atoms.size, atoms, js, u)
    return u


def sample_atoms(seed, cfg, first_atom, n, r_max, z_half):
    x, y, z = np.zeros(n), np.zeros(n), np.zeros(n)
    lib().orc_sample_atoms(seed, cfg, first_atom, n, r_max, z_half, x, y, z)
    return x, y, z


def field(L: Laser, x, y, z, t):
    x, y, z, t = np.broadcast_arrays(_d(x), _d(y), _d(z), _d(t))
    shp = x.shape
    x, y, z, t = (_d(a.ravel()) for a in (x, y, z, t))
    E = np.zeros((x.size, 3)); B = np.zeros((x.size, 3))
    lib().orc_field_batch(C.byref(L), x.size, x, y, z, t, E, B)
    return E.reshape(shp + (3,)), B.reshape(shp + (3,))


def adk_lnrate(k: int, Emag: float) -> float:
    return lib().orc_adk_lnrate(k, Emag)


def adk_rate(k: int, Emag: float) -> float:
    return lib().orc_adk_rate(k, Emag)


def adk_rate_batch(k: int, Emag) -> np.ndarray:
    Emag = _d(Emag).ravel()
    w = np.zeros(Emag.size)
    lib().orc_adk_rate_batch(k, Emag.size, Emag, w)
    return w


def adk_lnrate_general(Ip_au: float, Z: float, F_au: float) -> float:
    return lib().orc_adk_lnrate_general(Ip_au, Z, F_au)


def gl4():
    x = np.zeros(4); w = np.zeros(4)
    lib().orc_gl4_table(x, w)
    return x, w


def ionize(L: Laser, seed, cfg, first_atom, x, y, z, k_first, k_last):
    x, y, z = _d(x), _d(y), _d(z)
    K = k_last - k_first + 1
    tb = np.zeros(x.size * K)
    lib().orc_ionize(C.byref(L), seed, cfg, first_atom, x.size, x, y, z, k_first, k_last, tb)
    return tb


def push_one(L: Laser, t0, t_end, h, x0, u0):
    xf = np.zeros(3); uf = np.zeros(3)
    lib().orc_push_one(C.byref(L), t0, t_end, h, _d(x0), _d(u0), xf, uf)
    return xf, uf


def push(L: Laser, t_birth, x0, y0, z0, slots_per_atom, extended=False):
    """FP64 push of every slot (extended=True: the extended-precision build,
    same double inputs and outputs)."""
    t_birth = _d(t_birth)
    n = t_birth.size
    out = [np.zeros(n) for _ in range(6)]
    (lib_extended() if extended else lib()).orc_push(C.byref(L), n, t_birth, _d(x0), _d(y0),
                                                     _d(z0), slots_per_atom, *out)
    return tuple(out)  # ux, uy, uz, xf, yf, zf


def epilogue(ux, uy, uz):
    ux, uy, uz = _d(ux), _d(uy), _d(uz)
    n = ux.size
    K, th, ps = np.zeros(n), np.zeros(n), np.zeros(n)
    fwd = np.zeros(n, dtype=np.int32)
    lib().orc_epilogue(n, ux, uy, uz, K, th, ps, fwd)
    return K, th, ps, fwd


def histogram(t_birth, ux, uy, uz, nE, nA, logE_min, logE_max, angle=ANG_POLAR):
    sp = HistSpec(nE, nA, logE_min, logE_max, angle)
    counts = np.zeros(2 * nE * nA, dtype=np.uint64)
    tallies = np.zeros(6, dtype=np.uint64)
    t_birth = _d(t_birth)
    lib().orc_histogram(t_birth.size, t_birth, _d(ux), _d(uy), _d(uz), C.byref(sp),
                        counts, tallies)
    return counts.reshape(2, nE, nA), tallies


def birth_phase(L: Laser, t_birth, x, y, z, slots_per_atom):
    t_birth = _d(t_birth)
    ph = np.zeros(t_birth.size)
    lib().orc_birth_phase(C.byref(L), t_birth.size, t_birth, _d(x), _d(y), _d(z), slots_per_atom, ph)
    return ph


def sample_atoms_annulus(seed, cfg, first_atom, n, r_in, r_out, z_half):
    x, y, z = np.zeros(n), np.zeros(n), np.zeros(n)
    lib().orc_sample_atoms_annulus(seed, cfg, first_atom, n, r_in, r_out, z_half, x, y, z)
    return x, y, z


def histogram2d(a, b, uz, na, a_lo, a_hi, nb, b_lo, b_hi):
    """counts uint64 [2, na, nb] (0 forward: uz > 0) and tallies [2]
    (0 outside the ranges, 1 NaN)."""
    a, b, uz = _d(a), _d(b), _d(uz)
    counts = np.zeros((2, na, nb), dtype=np.uint64)
    tallies = np.zeros(2, dtype=np.uint64)
    lib().orc_histogram2d(a.size, a, b, uz, na, a_lo, a_hi, nb, b_lo, b_hi, counts, tallies)
    return counts, tallies


def critical_field() -> float:
    """E_cr = m^2 c^3 / (e hbar) [V/m]."""
    return lib().orc_critical_field()


def rr_terms(L: Laser, t, Y):
    """Radiation-reaction du/dt (u = p/mc) of Eq. (3) and chi, for state
    Y = (x, y, z, ux, uy, uz) at time t."""
    du = np.zeros(3)
    chi = np.zeros(1)
    lib().orc_rr_terms(C.byref(L), float(t), _d(Y), du, chi)
    return du, float(chi[0])


def push_one_rr(L: Laser, rr, t0, t_end, h, x0, u0):
    """One electron with initial momentum u0: (xf, uf, chi_max)."""
    xf, uf, cm = np.zeros(3), np.zeros(3), np.zeros(1)
    lib().orc_push_one_rr(C.byref(L), int(rr), t0, t_end, h, _d(x0), _d(u0), xf, uf, cm)
    return xf, uf, float(cm[0])


def push_rr(L: Laser, rr, t_birth, x0, y0, z0, slots_per_atom, extended=False):
    """Like push() with Eq. (3)'s radiation term on (rr=1) or off, plus the
    per-electron maximum of chi: (ux, uy, uz, xf, yf, zf, chi_max)."""
    t_birth = _d(t_birth)
    n = t_birth.size
    out = [np.zeros(n) for _ in range(7)]
    (lib_extended() if extended else lib()).orc_push_rr(
        C.byref(L), int(rr), n, t_birth, _d(x0), _d(y0), _d(z0), slots_per_atom, *out)
    return tuple(out)


class Adaptive(C.Structure):
    """Controlled-step push settings (see orc_push_one_adaptive)."""
    _fields_ = [("rtol", C.c_double), ("atol", C.c_double), ("h_max", C.c_double),
                ("k_tol", C.c_double), ("max_steps", C.c_int64)]


def adaptive(rtol=1e-9, atol=1e-9, h_max=None, k_tol=1e-10, max_steps=10_000_000, L=None):
    """Settings; h_max defaults to ten of L's steps dt."""
    if h_max is None:
        h_max = 10.0 * L.dt
    return Adaptive(rtol, atol, h_max, k_tol, max_steps)


def dp_tableau():
    """(c, A, b5, b4) of the oracle's embedded pair."""
    c, a, b5, b4 = np.zeros(7), np.zeros(49), np.zeros(7), np.zeros(7)
    lib().orc_dp_tableau(c, a, b5, b4)
    return c, a.reshape(7, 7), b5, b4


def push_one_adaptive(L: Laser, A: Adaptive, t0, t_end, x0, u0):
    """(xf, uf, t_stop, accepted, rejected, status)."""
    xf, uf, ts = np.zeros(3), np.zeros(3), np.zeros(1)
    na, nr = np.zeros(1, dtype=np.int64), np.zeros(1, dtype=np.int64)
    st = lib().orc_push_one_adaptive(C.byref(L), C.byref(A), t0, t_end, _d(x0), _d(u0), xf, uf,
                                     ts, na, nr)
    return xf, uf, float(ts[0]), int(na[0]), int(nr[0]), st


def push_adaptive(L: Laser, A: Adaptive, t_birth, x0, y0, z0, slots_per_atom):
    """(ux, uy, uz, xf, yf, zf, t_stop, accepted, rejected) per slot."""
    t_birth = _d(t_birth)
    n = t_birth.size
    out = [np.zeros(n) for _ in range(7)]
    na, nr = np.zeros(n, dtype=np.int64), np.zeros(n, dtype=np.int64)
    lib().orc_push_adaptive(C.byref(L), C.byref(A), n, t_birth, _d(x0), _d(y0), _d(z0),
                            slots_per_atom, *out, na, nr)
    return tuple(out) + (na, nr)


def num_threads() -> int:
    return lib().orc_num_threads()


def is_extended(extended=False) -> bool:
    return bool((lib_extended() if extended else lib()).orc_is_extended())


def chain(L: Laser, seed, cfg, atoms, r_max, z_half, k_first, k_last, extended=False):
    """Sampling, ionization, push and kinetic energy of the atoms with the
    given indices in one pass, nothing rounded to double between the steps;
    extended=True runs it in x87 extended precision.  Returns dict x, y, z [n]
    and t_birth, ux, uy, uz, K [n K] (slot j K + s: atom atoms[j], state
    k_first + s)."""
    atoms = np.ascontiguousarray(atoms, dtype=np.uint64).ravel()
    n = atoms.size
    K = k_last - k_first + 1
    out = {k: np.zeros(n) for k in ("x", "y", "z")}
    out.update({k: np.zeros(n * K) for k in ("t_birth", "ux", "uy", "uz", "K")})
    (lib_extended() if extended else lib()).orc_chain(
        C.byref(L), seed, cfg, atoms, n, r_max, z_half, k_first, k_last, out["x"], out["y"],
        out["z"], out["t_birth"], out["ux"], out["uy"], out["uz"], out["K"])
    return out
