"""The double-precision sine/cosine, exponential and reciprocal used by the
GPU kernels (csrc/rpdla_fastmath.hpp), compiled for the host with g++ from
the same header, against libm and mpmath, and the generated coefficient
table against a fresh run of its generator."""
import ctypes as C
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2509_01741_amd", "csrc")

HARNESS = r'''
#include "rpdla_fastmath.hpp"
extern "C" void fm_sincos(long n, const double* x, double* s, double* c) {
    for (long i = 0; i < n; ++i) rpdla::fm::sincos_f64(x[i], s + i, c + i);
}
extern "C" void fm_sincos2(long n, const double* xh, const double* xl, double* s, double* c) {
    for (long i = 0; i < n; ++i) rpdla::fm::sincos2_f64(xh[i], xl[i], s + i, c + i);
}
extern "C" void fm_cis_half2(long n, const double* xh, const double* xl, double* s, double* c) {
    for (long i = 0; i < n; ++i) {
        double sg, kp;
        const unsigned m = rpdla::fm::cis_half2_f64(xh[i], xl[i], &sg, &kp);
        s[i] = rpdla::fm::flip_sign(sg * kp, m);
        c[i] = rpdla::fm::flip_sign(1.0 - sg * sg, m);
    }
}
extern "C" void fm_exp(long n, const double* x, double* y) {
    for (long i = 0; i < n; ++i) y[i] = rpdla::fm::exp_f64(x[i]);
}
extern "C" void fm_exp_fin(long n, const double* x, double* y) {
    for (long i = 0; i < n; ++i) y[i] = rpdla::fm::exp_fin_f64(x[i]);
}
extern "C" void fm_rsqrt_mid(long n, const double* x, double* y) {
    for (long i = 0; i < n; ++i) y[i] = rpdla::fm::rsqrt_mid_f64(x[i]);
}
extern "C" void fm_log(long n, const double* x, double* y) {
    for (long i = 0; i < n; ++i) y[i] = rpdla::fm::log_pos_f64(x[i]);
}
extern "C" void fm_rcp(long n, const double* x, double* y) {
    for (long i = 0; i < n; ++i) y[i] = rpdla::fm::rcp_f64(x[i]);
}
extern "C" void fm_rsqrt(long n, const double* x, double* y) {
    for (long i = 0; i < n; ++i) y[i] = rpdla::fm::rsqrt_ge1_f64(x[i]);
}
'''


@pytest.fixture(scope="module")
def fm(tmp_path_factory):
    d = tmp_path_factory.mktemp("fm")
    src = d / "h.cpp"
    src.write_text(HARNESS)
    so = d / "libfm.so"
    subprocess.run(["g++", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-I" + CSRC,
                    "-o", str(so), str(src)], check=True)
    lib = C.CDLL(str(so))
    P = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
    lib.fm_sincos.argtypes = [C.c_long, P, P, P]
    lib.fm_exp.argtypes = [C.c_long, P, P]
    lib.fm_sincos2.argtypes = [C.c_long, P, P, P, P]
    lib.fm_exp_fin.argtypes = [C.c_long, P, P]
    lib.fm_cis_half2.argtypes = [C.c_long, P, P, P, P]
    lib.fm_rcp.argtypes = [C.c_long, P, P]
    lib.fm_log.argtypes = [C.c_long, P, P]
    lib.fm_rsqrt_mid.argtypes = [C.c_long, P, P]
    lib.fm_rsqrt.argtypes = [C.c_long, P, P]
    return lib


def test_sincos_against_libm(fm):
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.uniform(-1e4, 1e4, 400000), rng.uniform(-4, 4, 100000),
                        np.arange(-64, 65) * np.pi / 4, [0.0, -0.0, 1e-300, 2.0**-30]])
    s = np.zeros_like(x); c = np.zeros_like(x)
    fm.fm_sincos(x.size, x, s, c)
    # absolute error in units of 2^-53 (the functions are bounded by 1)
    es = np.abs(s - np.sin(x)) / 2.0**-53
    ec = np.abs(c - np.cos(x)) / 2.0**-53
    assert es.max() <= 4 and ec.max() <= 4, (es.max(), ec.max())
    assert np.all(s[-4:] == np.sin(x[-4:])) or np.max(np.abs(s[-4:] - x[-4:])) < 1e-300


def test_sincos_against_mpmath(fm):
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 40
    rng = np.random.default_rng(2)
    x = np.concatenate([rng.uniform(-3000, 3000, 300), rng.uniform(-1, 1, 100)])
    s = np.zeros_like(x); c = np.zeros_like(x)
    fm.fm_sincos(x.size, x, s, c)
    for xi, si, ci in zip(x, s, c):
        xs = mp.mpf(xi)
        assert abs(si - mp.sin(xs)) <= 2 * 2.0**-53
        assert abs(ci - mp.cos(xs)) <= 2 * 2.0**-53


def test_sincos_of_unevaluated_sum(fm):
    """sin and cos of x_hi + x_lo taken exactly (mpmath) for phases up to 1e3
    with a low part of a few units: a few 2^-53 absolute, well below
    ulp(x_hi) -- the precision a rounded sum x_hi + x_lo would have lost."""
    mp = pytest.importorskip("mpmath")
    mp.mp.prec = 120
    rng = np.random.default_rng(7)
    xh = rng.uniform(-1e3, 1e3, 3000)
    xl = rng.uniform(-4, 4, 3000)
    s = np.zeros_like(xh); c = np.zeros_like(xh)
    fm.fm_sincos2(xh.size, xh, xl, s, c)
    ref_s = np.array([float(mp.sin(mp.mpf(a) + mp.mpf(b))) for a, b in zip(xh, xl)])
    ref_c = np.array([float(mp.cos(mp.mpf(a) + mp.mpf(b))) for a, b in zip(xh, xl)])
    es = np.abs(s - ref_s) / 2.0**-53
    ec = np.abs(c - ref_c) / 2.0**-53
    assert es.max() <= 8 and ec.max() <= 8, (es.max(), ec.max())
    # the rounded sum loses up to ulp(1e3)/2 = 2^-44 of argument
    s1 = np.zeros_like(xh); c1 = np.zeros_like(xh)
    fm.fm_sincos(xh.size, xh + xl, s1, c1)
    assert np.abs(s1 - ref_s).max() / 2.0**-53 > 4 * es.max()


def test_half_angle_cis_of_unevaluated_sum(fm):
    """The half-angle form of e^{ix} (x = n pi + r, sigma = sqrt2 sin(r/2),
    kappa = sqrt2 cos(r/2), cos x = (-1)^n (1 - sigma^2), sin x = (-1)^n
    sigma kappa) against mpmath for phases up to 1e3 with a low part of a few
    units, the multiples of pi/2 and pi/4 (where the reduction switches n or
    the identities cancel most), and tiny arguments."""
    mp = pytest.importorskip("mpmath")
    mp.mp.prec = 120
    rng = np.random.default_rng(8)
    k = np.arange(-4000, 4001)
    xh = np.concatenate([rng.uniform(-1e3, 1e3, 3000), k * np.pi / 2, k * np.pi / 4,
                         rng.uniform(-1e-3, 1e-3, 200), [0.0, 1e-300, -1e-300]])
    xl = np.concatenate([rng.uniform(-4, 4, 3000), np.zeros(xh.size - 3000)])
    s = np.zeros_like(xh); c = np.zeros_like(xh)
    fm.fm_cis_half2(xh.size, xh, xl, s, c)
    ref_s = np.array([float(mp.sin(mp.mpf(a) + mp.mpf(b))) for a, b in zip(xh, xl)])
    ref_c = np.array([float(mp.cos(mp.mpf(a) + mp.mpf(b))) for a, b in zip(xh, xl)])
    es = np.abs(s - ref_s) / 2.0**-53
    ec = np.abs(c - ref_c) / 2.0**-53
    # absolute errors: a few units of 2^-53 (1 - sigma^2 cancels near cos x = 0)
    assert es.max() <= 8 and ec.max() <= 8, (es.max(), ec.max())
    # sine relative to its size near zero: sigma kappa keeps it
    small = np.abs(ref_s) < 1e-3
    rel = np.abs(s[small] - ref_s[small]) / np.maximum(np.abs(ref_s[small]), 1e-300)
    assert rel.max() <= 8 * 2.0**-53, rel.max()


def test_exp_against_libm(fm):
    rng = np.random.default_rng(3)
    x = np.concatenate([rng.uniform(-745, 5, 400000), rng.uniform(-1, 1, 100000),
                        [0.0, -1e-300, -708.0, -745.0, -746.0, -1e6]])
    y = np.zeros_like(x)
    fm.fm_exp(x.size, x, y)
    ref = np.exp(x)
    norm = ref > 2.2250738585072014e-308
    rel = np.abs(y[norm] - ref[norm]) / ref[norm]
    assert rel.max() <= 3 * 2.0**-53, rel.max()
    assert np.all(np.abs(y[~norm] - ref[~norm]) <= 4.9e-324 * 4)
    assert fm and y[-6] == 1.0 and y[-1] == 0.0 and y[-2] == 0.0


def test_exp_without_guards_equals_exp(fm):
    """The guard-free exponential of the field evaluations returns what the
    guarded one does wherever the guards do not act, and flushes to zero (or
    the smallest denormal, correctly rounded) far below the normal range."""
    rng = np.random.default_rng(4)
    x = np.concatenate([rng.uniform(-745, 5, 400000), rng.uniform(-1, 1, 100000),
                        rng.uniform(-1e5, -745.2, 10000), [0.0, -708.0, -745.0, -1e5]])
    y = np.zeros_like(x); yf = np.zeros_like(x)
    fm.fm_exp(x.size, x, y)
    fm.fm_exp_fin(x.size, x, yf)
    guarded = x < -745.2
    assert np.array_equal(y[~guarded], yf[~guarded])
    assert np.all(yf[guarded] == 0.0)
    ref = np.exp(x[~guarded])
    assert np.all(np.abs(yf[~guarded] - ref) <= np.maximum(3 * 2.0**-53 * ref, 4 * 4.9e-324))


def test_rcp(fm):
    rng = np.random.default_rng(4)
    x = 1.0 + rng.uniform(0, 50, 100000) ** 2
    y = np.zeros_like(x)
    fm.fm_rcp(x.size, x, y)
    rel = np.abs(y - 1.0 / x) * x
    assert rel.max() <= 2 * 2.0**-53


def test_rsqrt(fm):
    rng = np.random.default_rng(5)
    x = np.concatenate([1.0 + rng.uniform(0, 10, 100000) ** 2, np.exp(rng.uniform(0, 40, 100000)),
                        [1.0, 2.0, 4.0, 1e30]])
    y = np.zeros_like(x)
    fm.fm_rsqrt(x.size, x, y)
    rel = np.abs(y - 1.0 / np.sqrt(x)) * np.sqrt(x)
    assert rel.max() <= 3 * 2.0**-53, rel.max()  # reference 1/sqrt rounds twice


def test_coefficients_are_the_generator_output():
    pytest.importorskip("mpmath")
    out = subprocess.run([sys.executable, os.path.join(CSRC, "gen_fastmath.py")],
                         capture_output=True, text=True, check=True).stdout
    assert out.strip() == open(os.path.join(CSRC, "rpdla_fastmath_coeffs.hpp")).read().strip()


def test_log_against_libm_and_mpmath(fm):
    """The logarithm of the tunnelling rate's field argument: within 2 units
    in the last place of libm over the whole positive range (subnormals
    included, the reduction boundaries sqrt(1/2) and sqrt(2) densely), and
    within 2 ulp of a 120-bit mpmath reference on a sample."""
    import mpmath as mp
    rng = np.random.default_rng(5)
    x = np.concatenate([np.exp(rng.uniform(-744, 709, 300000)), rng.uniform(0.5, 2.0, 200000),
                        np.sqrt(2.0) * (1 + rng.uniform(-1e-6, 1e-6, 20000)),
                        np.sqrt(0.5) * (1 + rng.uniform(-1e-6, 1e-6, 20000)),
                        [5e-324, 1e-310, 2.2250738585072014e-308, 1.0, 2.0, 0.5, 1.7976931348623157e308]])
    y = np.zeros_like(x)
    fm.fm_log(x.size, x, y)
    ref = np.log(x)
    ulp = np.abs(y - ref) / np.spacing(np.abs(ref))
    assert ulp[ref != 0].max() <= 2.0, ulp[ref != 0].max()
    assert y[x == 1.0][0] == 0.0
    mp.mp.prec = 120
    idx = rng.choice(x.size, 2000, replace=False)
    err = max(abs((mp.mpf(float(y[i])) - mp.log(mp.mpf(float(x[i])))) / mp.mpf(float(np.spacing(abs(ref[i])))))
              for i in idx if ref[i] != 0)
    assert float(err) <= 2.0, float(err)


def test_rsqrt_mid_range(fm):
    """The reciprocal square root of the rate's |a|^2 over its stated range
    [2^-960, 2^960]: one third-order step from the estimate (the host build
    starts from a float estimate) gives full precision."""
    rng = np.random.default_rng(6)
    x = np.concatenate([2.0 ** rng.uniform(-960, 960, 300000), rng.uniform(0.25, 4.0, 100000),
                        [2.0 ** -960, 2.0 ** 960, 1.0, 4.0]])
    y = np.zeros_like(x)
    fm.fm_rsqrt_mid(x.size, x, y)
    ref = 1.0 / np.sqrt(x)
    rel = np.abs(y - ref) / ref
    assert rel.max() <= 3 * 2.0 ** -53, rel.max()
