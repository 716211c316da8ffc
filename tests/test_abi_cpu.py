"""The C-ABI library without a GPU: it loads, exports every symbol the
header declares, and its host-only entry points (laser set-up, argument
validation) behave as documented.  No compute call is made here."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rpdla.h")
LIB = os.path.join(ROOT, "paper_2509_01741_amd", "librpdla.so")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(rpdla_[a-z_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    # loaded through the binding, which imports torch first: a library loaded
    # before torch binds to a second HIP runtime, and the GPU tests that may
    # follow in the same process would then see two
    if not os.path.exists(LIB):
        from paper_2509_01741_amd.build import build_library
        build_library(force=False)
    from paper_2509_01741_amd import binding as B
    return B.lib


def test_header_symbols_exported(lib):
    names = _declared()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
    nm = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    for n in names:
        assert re.search(r"\bT " + n + r"\b", nm), n


def test_laser_init_matches_oracle(orc):
    from paper_2509_01741_amd import binding as B
    for I in (5e19, 1e21, 5e21):
        L = B.rpdla_laser_init_intensity(0.8e-6, 3e-6, 30e-15, I)
        OL = orc.laser_intensity(0.8e-6, 3e-6, 30e-15, I)
        assert abs(L.amp / OL.amp - 1) < 1e-15
    L = B.rpdla_laser_init_power(1.0e-6, 2e-6, 33e-15, 1e15)
    OL = orc.laser_power(1.0e-6, 2e-6, 33e-15, 1e15)
    assert abs(L.amp / OL.amp - 1) < 1e-15
    assert L.field == 5 and L.window == 0 and L.ez_scale == 1 and L.er_scale == 1
    assert L.t_before == 5 * 33e-15 and L.t_after == 10 * 33e-15
    assert abs(L.dt - 1e-6 / 299792458.0 / 200) < 1e-30
    assert abs(B.rpdla_rayleigh(L) / orc.rayleigh(OL) - 1) < 1e-15


def test_validation_without_gpu():
    from paper_2509_01741_amd import binding as B
    lib = B.lib
    L = B.rpdla_laser_init_intensity(0.8e-6, 3e-6, 30e-15, 1e21)
    p = C.c_void_p(0)
    # k range
    assert lib.rpdla_ionize(C.byref(L), 0, 0, 0, 4, p, p, p, 0, 3, p, p) == B.RPDLA_EINVAL
    assert lib.rpdla_ionize(C.byref(L), 0, 0, 0, 4, p, p, p, 3, 11, p, p) == B.RPDLA_EINVAL
    # null pointers with n > 0
    assert lib.rpdla_ionize(C.byref(L), 0, 0, 0, 4, p, p, p, 1, 3, p, p) == B.RPDLA_EINVAL
    assert b"null" in lib.rpdla_last_error()
    # bad laser
    bad = B.rpdla_laser_init_intensity(0.8e-6, 3e-6, 30e-15, 1e21)
    bad.w0 = 0.0
    assert lib.rpdla_push(C.byref(bad), 0, 4, p, p, p, p, 1, p, p, p, p, p, p, p) == B.RPDLA_EINVAL
    bad = B.rpdla_laser_init_intensity(0.8e-6, 3e-6, 30e-15, 1e21)
    bad.field = 2
    assert lib.rpdla_push(C.byref(bad), 0, 4, p, p, p, p, 1, p, p, p, p, p, p, p) == B.RPDLA_EINVAL
    bad = B.rpdla_laser_init_intensity(0.8e-6, 3e-6, 30e-15, 1e21)
    bad.t_after = 0.0
    assert lib.rpdla_push(C.byref(bad), 0, 4, p, p, p, p, 1, p, p, p, p, p, p, p) == B.RPDLA_EINVAL
    bad = B.rpdla_laser_init_intensity(0.8e-6, 3e-6, 30e-15, 1e21)
    bad.dt = 1e-30
    assert lib.rpdla_push(C.byref(bad), 0, 4, p, p, p, p, 1, p, p, p, p, p, p, p) == B.RPDLA_ERANGE
    # precision, slots_per_atom
    assert lib.rpdla_push(C.byref(L), 3, 4, p, p, p, p, 1, p, p, p, p, p, p, p) == B.RPDLA_EINVAL
    assert lib.rpdla_push(C.byref(L), 0, 4, p, p, p, p, 0, p, p, p, p, p, p, p) == B.RPDLA_EINVAL
    # histogram spec
    sp = B.rpdla_hist_spec(0, 4, -3.0, 4.0, 0)
    assert lib.rpdla_histogram(4, p, p, p, p, C.byref(sp), p, p, p) == B.RPDLA_EINVAL
    sp = B.rpdla_hist_spec(4, 4, 4.0, -3.0, 0)
    assert lib.rpdla_histogram(4, p, p, p, p, C.byref(sp), p, p, p) == B.RPDLA_EINVAL
    # epilogue
    assert lib.rpdla_epilogue(-1, p, p, p, p, p, p, p, p) == B.RPDLA_EINVAL
    assert lib.rpdla_epilogue(3, p, p, p, p, p, p, p, p) == B.RPDLA_EINVAL
    assert lib.rpdla_epilogue(0, p, p, p, p, p, p, p, p) == B.RPDLA_OK
    # sampling
    assert lib.rpdla_sample_atoms(0, 0, 0, -1, 1.0, 1.0, p, p, p, p) == B.RPDLA_EINVAL
    assert lib.rpdla_sample_atoms(0, 0, 0, 5, -1.0, 1.0, p, p, p, p) == B.RPDLA_EINVAL
    # empty calls succeed without touching the device
    assert lib.rpdla_sample_atoms(0, 0, 0, 0, 1.0, 1.0, p, p, p, p) == B.RPDLA_OK
    assert lib.rpdla_push(C.byref(L), 0, 0, p, p, p, p, 1, p, p, p, p, p, p, p) == B.RPDLA_OK
    # batched: workspace size and checks
    assert lib.rpdla_batched_workspace_bytes(0, 10, 1, 10) == 0
    ws = lib.rpdla_batched_workspace_bytes(64, 65536, 1, 10)
    assert ws >= 64 * 65536 * (3 + 10) * 8
    arr = (B.rpdla_laser * 2)(L, L)
    sp = B.rpdla_hist_spec(4, 4, -3.0, 4.0, 0)
    assert lib.rpdla_run_batched(arr, 65, 0, 0, 10, 10, 2.0, 1, 10, 0, C.byref(sp), p, p, p, p,
                                 0, p) == B.RPDLA_EUNSUPPORTED
    assert lib.rpdla_run_batched(arr, 2, 0, 0, 10, 10, 2.0, 1, 10, 0, C.byref(sp), C.c_void_p(256),
                                 C.c_void_p(512), p, C.c_void_p(1024), 16, p) == B.RPDLA_ENOMEM
    # chunk ranges outside a 2-chunk stream (20 atoms, 10 per chunk), checked before any launch
    for first, cnt in ((-1, 1), (0, 3), (3, -1), (1, 2)):
        assert lib.rpdla_run_batched_range(arr, 2, 0, 0, 20, 10, first, cnt, 2.0, 1, 10, 0,
                                           C.byref(sp), C.c_void_p(256), C.c_void_p(512), p,
                                           C.c_void_p(1024), 1 << 40, p) == B.RPDLA_EINVAL
    arr[1].field = 1
    assert lib.rpdla_run_batched(arr, 2, 0, 0, 10, 10, 2.0, 1, 10, 0, C.byref(sp), p, p, p, p, 0,
                                 p) == B.RPDLA_EINVAL
    assert lib.rpdla_status_string(B.RPDLA_ENOMEM) == b"out of memory / workspace too small"
    # launch-shape table (host only)
    assert lib.rpdla_set_launch_shape(0, 5, 0, 100, 1) == B.RPDLA_EINVAL
    assert lib.rpdla_set_launch_shape(3, 5, 0, 128, 1) == B.RPDLA_EINVAL
    assert lib.rpdla_set_launch_shape(0, 5, 0, 128, 9) == B.RPDLA_EINVAL
    assert B.rpdla_get_launch_shape(0, 3, 1) == (256, 1)
    B.rpdla_set_launch_shape(0, 3, 1, 128, 2)
    assert B.rpdla_get_launch_shape(0, 3, 1) == (128, 2)
    B.rpdla_set_launch_shape(0, 3, 1, 256, 1)
    assert lib.rpdla_autotune(C.byref(L), 0, 10, 1, 10, None, 0, p) == B.RPDLA_ERANGE


def test_kernel_occupancy_validation():
    from paper_2509_01741_amd import binding as B
    lib = B.lib
    v, sc, w = C.c_int32(), C.c_int32(), C.c_double()
    ok = (C.byref(v), C.byref(sc), C.byref(w))
    assert lib.rpdla_kernel_occupancy(0, 5, 0, None, C.byref(sc), C.byref(w)) == B.RPDLA_EINVAL
    assert lib.rpdla_kernel_occupancy(3, 5, 0, *ok) == B.RPDLA_EINVAL
    assert lib.rpdla_kernel_occupancy(0, 2, 0, *ok) == B.RPDLA_EINVAL
    assert lib.rpdla_kernel_occupancy(0, 5, 2, *ok) == B.RPDLA_EINVAL


def test_ne_table_matches_oracle(orc):
    """Both sides carry their own copy of the neon potentials; they must agree."""
    src = open(os.path.join(ROOT, "paper_2509_01741_amd", "csrc", "rpdla_api.hip")).read()
    m = re.search(r"kNeIpEv\[10\] = \{([^}]*)\}", src)
    vals = np.array([float(v) for v in m.group(1).replace("\n", " ").split(",")])
    assert np.array_equal(vals, orc.ne_ip_ev())


def test_experiment_entry_points_validation():
    from paper_2509_01741_amd import binding as B
    lib = B.lib
    L = B.rpdla_laser_init_intensity(0.8e-6, 2.5e-6, 30e-15, 5e19)
    p = C.c_void_p(0)
    # annulus sampler: radii order, negative n, empty call
    assert lib.rpdla_sample_atoms_annulus(0, 0, 0, 5, 2.0, 1.0, 1.0, p, p, p, p) == B.RPDLA_EINVAL
    assert lib.rpdla_sample_atoms_annulus(0, 0, 0, 5, -1.0, 1.0, 1.0, p, p, p, p) == B.RPDLA_EINVAL
    assert lib.rpdla_sample_atoms_annulus(0, 0, 0, -1, 0.0, 1.0, 1.0, p, p, p, p) == B.RPDLA_EINVAL
    assert lib.rpdla_sample_atoms_annulus(0, 0, 0, 5, 0.0, 1.0, 1.0, p, p, p, p) == B.RPDLA_EINVAL
    assert lib.rpdla_sample_atoms_annulus(0, 0, 0, 0, 1.0, 1.0, 1.0, p, p, p, p) == B.RPDLA_OK
    # birth phase: slots_per_atom, null pointers, empty call (r_birth may be NULL)
    assert lib.rpdla_birth_phase(C.byref(L), 4, p, p, p, p, 0, p, p, p) == B.RPDLA_EINVAL
    assert lib.rpdla_birth_phase(C.byref(L), 4, p, p, p, p, 1, p, p, p) == B.RPDLA_EINVAL
    assert lib.rpdla_birth_phase(C.byref(L), 0, p, p, p, p, 1, p, p, p) == B.RPDLA_OK
    # 2-d histogram spec
    sp = B.rpdla_hist2d_spec(0, 4, 0.0, 1.0, 0.0, 1.0)
    assert lib.rpdla_histogram2d(4, p, p, p, C.byref(sp), p, p, p) == B.RPDLA_EINVAL
    sp = B.rpdla_hist2d_spec(4, 4, 1.0, 1.0, 0.0, 1.0)
    assert lib.rpdla_histogram2d(4, p, p, p, C.byref(sp), p, p, p) == B.RPDLA_EINVAL
    sp = B.rpdla_hist2d_spec(4, 4, 0.0, 1.0, 0.0, float("nan"))
    assert lib.rpdla_histogram2d(4, p, p, p, C.byref(sp), p, p, p) == B.RPDLA_EINVAL
    sp = B.rpdla_hist2d_spec(1 << 15, 1 << 14, 0.0, 1.0, 0.0, 1.0)
    assert lib.rpdla_histogram2d(4, p, p, p, C.byref(sp), p, p, p) == B.RPDLA_ERANGE
    sp = B.rpdla_hist2d_spec(4, 4, 0.0, 1.0, 0.0, 1.0)
    assert lib.rpdla_histogram2d(4, p, p, p, C.byref(sp), p, p, p) == B.RPDLA_EINVAL
    assert lib.rpdla_histogram2d(0, p, p, p, C.byref(sp), C.c_void_p(256), C.c_void_p(256),
                                 p) == B.RPDLA_OK


def test_hist2d_spec_layout():
    # the ctypes mirror must match the C struct: int32 na, nb then four doubles
    from paper_2509_01741_amd import binding as B
    assert C.sizeof(B.rpdla_hist2d_spec) == 40
    assert B.rpdla_hist2d_spec.a_lo.offset == 8 and B.rpdla_hist2d_spec.b_hi.offset == 32


def test_push_rr_validation():
    from paper_2509_01741_amd import binding as B
    lib = B.lib
    L = B.rpdla_laser_init_intensity(0.8e-6, 2.5e-6, 30e-15, 5e22)
    p = C.c_void_p(0)
    args = lambda rr, n, spa: (C.byref(L), rr, n, p, p, p, p, spa, p, p, p, p, p, p, p, p)
    assert lib.rpdla_push_rr(*args(2, 4, 1)) == B.RPDLA_EINVAL
    assert lib.rpdla_push_rr(*args(-1, 4, 1)) == B.RPDLA_EINVAL
    assert lib.rpdla_push_rr(*args(1, -1, 1)) == B.RPDLA_EINVAL
    assert lib.rpdla_push_rr(*args(1, 4, 0)) == B.RPDLA_EINVAL
    assert lib.rpdla_push_rr(*args(1, 4, 1)) == B.RPDLA_EINVAL      # null pointers
    assert lib.rpdla_push_rr(*args(1, 0, 1)) == B.RPDLA_OK
    bad = B.rpdla_laser_init_intensity(0.8e-6, 2.5e-6, 30e-15, 5e22)
    bad.tau_fwhm = -1.0
    assert lib.rpdla_push_rr(C.byref(bad), 1, 0, p, p, p, p, 1, p, p, p, p, p, p, p,
                             p) == B.RPDLA_EINVAL


def test_push_adaptive_validation():
    from paper_2509_01741_amd import binding as B
    lib = B.lib
    L = B.rpdla_laser_init_intensity(0.8e-6, 3e-6, 30e-15, 1e21)
    p = C.c_void_p(0)

    def call(A, n=4, spa=1):
        return lib.rpdla_push_adaptive(C.byref(L), C.byref(A) if A is not None else None, n, p, p,
                                       p, p, spa, p, p, p, p, p, p, p, p, p, p)
    ok = B.adaptive_settings()
    assert call(None) == B.RPDLA_EINVAL
    assert call(B.adaptive_settings(rtol=-1.0)) == B.RPDLA_EINVAL
    assert call(B.adaptive_settings(rtol=0.0, atol=0.0)) == B.RPDLA_EINVAL
    assert call(B.adaptive_settings(h_max=float("inf"))) == B.RPDLA_EINVAL
    assert call(B.adaptive_settings(max_steps=0)) == B.RPDLA_EINVAL
    assert call(ok, n=-1) == B.RPDLA_EINVAL
    assert call(ok, spa=0) == B.RPDLA_EINVAL
    assert call(ok) == B.RPDLA_EINVAL                # null pointers
    assert call(ok, n=0) == B.RPDLA_OK
    assert C.sizeof(B.rpdla_adaptive) == 40
