"""Mutation check of the oracle's pins: plant one plausible mistake at a time
in a copy of oracle/rpdla_oracle.c (a flipped sign, a dropped or wrong
coefficient, a swapped index or operand, a wrong weight, a missing factor),
build it, and run the oracle's CPU pin tests against it.  Every mutant must
make at least one pin fail; a mutant that passes them all names a part of
the oracle that its pins do not fix.  The mistakes are planted in the
oracle, on the CPU; the HIP library is not involved."""
import concurrent.futures as cf
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "rpdla_oracle.c")
PIN_FILES = sorted(os.path.join("tests", f) for f in os.listdir(os.path.join(ROOT, "tests"))
                   if f.startswith("test_oracle_") and f.endswith(".py"))

# (label, text in the oracle, replacement, which occurrence (0-based))
MUTANTS = [
    # laser set-up
    ("amplitude from intensity", "sqrt(2.0 * I / (ORC_EPS0 * ORC_C))",
     "sqrt(I / (ORC_EPS0 * ORC_C))", 0),
    ("amplitude from power", "sqrt(8.0 * P_W /", "sqrt(4.0 * P_W /", 0),
    ("Rayleigh length", "return 0.5 * k * L->w0 * L->w0;", "return k * L->w0 * L->w0;", 0),
    # random numbers and sampling
    ("Philox multiplier", "M0 = 0xD2E7470EE14C6C93ULL", "M0 = 0xD2E7470EE14C6C95ULL", 0),
    ("Philox Weyl constant", "W1 = 0xBB67AE8584CAA73BULL", "W1 = 0xBB67AE8584CAA73DULL", 0),
    ("uniform offset", "((double)m + 1.0)", "((double)m)", 0),
    ("uniform word", "out[j & 3]", "out[(j + 1) & 3]", 0),
    ("sampler radius law", "orc_real r = r_max * sqrt((orc_real)u0);", "orc_real r = r_max * u0;", 0),
    ("sampler axial range", "*z = z_half * (2.0 * u2 - 1.0);", "*z = z_half * u2;", 0),
    # fields
    ("envelope sign", "exp(-rho2 / D - s * s)", "exp(-rho2 / D + 0.5 * s * s)", 0),
    ("wavefront curvature sign", "- rho2 * zeta / D;", "+ rho2 * zeta / D;", 0),
    ("Gouy phase sign", "cos(Psi + n * gouy)", "cos(Psi - n * gouy)", 0),
    ("amplitude power of D", "pow(D, -0.5 * n)", "pow(D, -0.5 * (n - 1))", 0),
    ("order-3 Er coefficient", "PE += e2 * (-C[3] / 2.0", "PE += e2 * (C[3] / 2.0", 0),
    ("order-3 Bt coefficient", "r2 * C[4] / 2.0 - r4 * C[5] / 4.0);",
     "r2 * C[4] / 2.0 - r4 * C[5] / 2.0);", 0),
    ("order-3 Ez coefficient", "5.0 * r4 * S[5] / 4.0", "3.0 * r4 * S[5] / 4.0", 0),
    ("order-5 Er coefficient", "17.0 * r4 * C[6] / 16.0", "15.0 * r4 * C[6] / 16.0", 0),
    ("order-5 Bt coefficient", "- r6 * C[7] / 4.0 + r8 * C[8] / 32.0);",
     "- r6 * C[7] / 8.0 + r8 * C[8] / 32.0);", 0),
    ("order-1 Ez sign", "orc_real Ez = eps * (S[2] - r2 * S[3]);",
     "orc_real Ez = eps * (S[2] + r2 * S[3]);", 0),
    ("B_x sign", "B[0] = -PB * y / (w0 * ORC_C);", "B[0] = PB * y / (w0 * ORC_C);", 0),
    ("Ez scale", "E[2] = L->ez_scale * Ez;", "E[2] = L->er_scale * Ez;", 0),
    ("plane-wave B sign", "B[1] = ex / ORC_C;", "B[1] = -ex / ORC_C;", 0),
    ("tau0 from FWHM", "L->tau_fwhm / sqrt(2.0 * log((orc_real)2.0))",
     "L->tau_fwhm / sqrt(log((orc_real)2.0))", 0),
    # linearly polarized focus
    ("LP Ez sign", "- iu * eps * rx * psi_s) * ph);", "+ iu * eps * rx * psi_s) * ph);", 0),
    ("LP Ex gauge term", "(psi + 0.5 * e2 * psi_s + e2 * rx * rx * psi_ss)", "(psi + e2 * rx * rx * psi_ss)", 0),
    ("LP By correction", "(psi + iu * 0.5 * e2 * psi_z)", "(psi - iu * 0.5 * e2 * psi_z)", 0),
    ("LP Bz component", "creal(-iu * eps * ry * psi_s * ph)", "creal(-iu * eps * rx * psi_s * ph)", 0),
    ("LP series coefficient", "hd_scale(hd_pow(f, 3), 3.0 / 8.0)", "hd_scale(hd_pow(f, 3), 3.0 / 16.0)", 0),
    ("hyper-dual exp", "e * (x.d + x.b * x.c)", "e * x.d", 0),
    ("hyper-dual inverse", "-q * q * x.c,", "q * q * x.c,", 0),
    ("hyper-dual product", "x.a * y.d + x.b * y.c + x.c * y.b + x.d * y.a", "x.a * y.d + x.b * y.c + x.d * y.a", 0),
    # tunnelling rate
    ("ADK Gamma argument", "lgamma(2.0 * nstar)", "lgamma(nstar)", 0),
    ("ADK field exponent", "(2.0 * nstar - 1.0) * log(2.0 * F0 / F_au)",
     "(2.0 * nstar) * log(2.0 * F0 / F_au)", 0),
    ("ADK exponential", "- 2.0 * F0 / (3.0 * F_au);", "- F0 / (3.0 * F_au);", 0),
    ("ADK charge of state k", "orc_adk_lnrate_r(Ip, (orc_real)k, Emag / ORC_EA)",
     "orc_adk_lnrate_r(Ip, (orc_real)k - 0.5, Emag / ORC_EA)", 0),
    ("ADK potential of state k", "orc_ne_ip_ev[k - 1] / ORC_EH_EV",
     "orc_ne_ip_ev[k < 10 ? k : 9] / ORC_EH_EV", 0),
    # quadrature and ionization
    ("GL-4 weight", "orc_real wa = (18.0 + sqrt(thirty)) / 36.0;",
     "orc_real wa = (18.0 + sqrt(thirty)) / 35.0;", 0),
    ("GL-4 half width", "orc_real h = 0.5 * (b - a), m = 0.5 * (a + b);",
     "orc_real h = (b - a), m = 0.5 * (a + b);", 0),
    ("first threshold stream", "orc_uniform(seed, cfg, atom, k_first + 2)",
     "orc_uniform(seed, cfg, atom, k_first + 3)", 0),
    ("next threshold stream", "orc_uniform(seed, cfg, atom, k_first + s + 2)",
     "orc_uniform(seed, cfg, atom, k_first + s + 1)", 0),
    ("integral not reset at a birth", "I = 0.0;\n                tstart = t;",
     "tstart = t;", 0),
    ("next state starts at window start", "I = 0.0;\n                tstart = t;",
     "I = 0.0;\n                tstart = ts;", 0),
    ("bracket update", "if (gdiff > 0.0) th = t; else tl = t;",
     "if (gdiff > 0.0) tl = t; else th = t;", 0),
    ("window start", "*ts = tz - L->t_before;", "*ts = tz - 0.5 * L->t_before;", 0),
    ("arrival window", "(L->window == ORC_WIN_ARRIVAL) ? z / ORC_C : 0.0",
     "(L->window == ORC_WIN_ARRIVAL) ? 0.0 : 0.0", 0),
    # push
    ("RK4 weights", "(k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i])",
     "(k1[i] + 2.0 * k2[i] + k3[i] + 2.0 * k4[i])", 0),
    ("RK4 stage state", "for (int i = 0; i < 7; ++i) Yt[i] = Y[i] + 0.5 * hn * k2[i];",
     "for (int i = 0; i < 7; ++i) Yt[i] = Y[i] + 0.5 * hn * k1[i];", 0),
    ("retarded-time slope", "dY[6] = 1.0 - Y[5] / gam;", "dY[6] = 1.0;", 0),
    ("retarded-time start", "t0 - x0[2] / ORC_C};", "t0};", 0),
    ("RK4 last step", "orc_real hn = (n == N - 1) ? t_end - ta : h;", "orc_real hn = h;", 0),
    ("magnetic force sign", "dY[5] = q * (E[2] + (vx * B[1] - vy * B[0]));",
     "dY[5] = q * (E[2] - (vx * B[1] - vy * B[0]));", 0),
    ("missing 1/gamma", "orc_real vx = ORC_C * Y[3] / gam,", "orc_real vx = ORC_C * Y[3],", 0),
    ("state accumulation not compensated", "*comp = (t - *sum) - y;", "*comp = 0.0;", 0),
    ("before-window births accepted", "if (!(t0 >= ts - L->dt)) {",
     "if (!(t0 >= ts - 1e3 * L->dt)) {", 0),
    # outputs
    ("kinetic energy", "K_MeV[i] = ORC_MEC2_MEV * u2 / (gam + 1.0);",
     "K_MeV[i] = ORC_MEC2_MEV * u2 / gam;", 0),
    ("polar angle operands", "theta[i] = atan2(sqrt(ux[i] * ux[i] + uy[i] * uy[i]), uz[i]);",
     "theta[i] = atan2(uz[i], sqrt(ux[i] * ux[i] + uy[i] * uy[i]));", 0),
    ("forward flag", "fwd[i] = (uz[i] > 0.0) ? 1 : 0;", "fwd[i] = (uz[i] < 0.0) ? 1 : 0;", 0),
    ("histogram bin width", "/ (double)sp->nE;", "/ (double)(sp->nE - 1);", 0),
    ("histogram direction", "int dir = (uz[i] > 0.0) ? 0 : 1;", "int dir = (uz[i] > 0.0) ? 1 : 0;", 0),
    ("azimuth bins", "floor((ang + ORC_PI) / (2.0 * ORC_PI)", "floor((ang) / (2.0 * ORC_PI)", 0),
    # studies
    ("birth phase Gouy term", "- 2.0 * atan(z / zr)", "- atan(z / zr)", 0),
    ("annulus radius law", "sqrt(r_in * r_in + u0 * (r_out * r_out - r_in * r_in))",
     "(r_in + u0 * (r_out - r_in))", 0),
    ("2-D histogram direction", "const int dir = (uz[i] > 0.0) ? 0 : 1;",
     "const int dir = (uz[i] > 0.0) ? 1 : 0;", 0),
    # radiation reaction and chi
    ("radiation coefficient", "(6.0 * ORC_PI * ORC_EPS0", "(4.0 * ORC_PI * ORC_EPS0", 0),
    ("radiation bracket sign", "- vE * vE;", "+ vE * vE;", 0),
    ("radiation gamma power", "e2 * e2 * gam * gam /", "e2 * e2 * gam /", 0),
    ("chi maximum", "if (chi > cm) cm = chi;", "cm = chi;", 0),
    # controlled-step push
    ("tableau entry", "44.0 / 45.0", "44.0 / 46.0", 0),
    ("embedded weight", "393.0 / 640.0", "393.0 / 641.0", 0),
    ("controller exponent", "0.9 * pow(err, (orc_real)-0.2)", "0.9 * pow(err, (orc_real)-0.25)", 0),
    ("accept threshold", "if (err <= 1.0) {", "if (err <= 2.0) {", 0),
    ("error scaling", "const orc_real scale[6] = {k, k, k, 1.0, 1.0, 1.0};",
     "const orc_real scale[6] = {1.0, 1.0, 1.0, 1.0, 1.0, 1.0};", 0),
    ("stop rule", "if (fabs(g - g_ref) <= A->k_tol * g) break;",
     "if (fabs(g - g_ref) <= 1e3 * A->k_tol * g) break;", 0),
    ("check interval", "if (t - t_ref >= 0.999 * T) {", "if (t - t_ref >= 0.5 * T) {", 0),
]


def _mutate(src, old, new, nth):
    pos = -1
    for _ in range(nth + 1):
        pos = src.find(old, pos + 1)
        if pos < 0:
            raise KeyError(old)
    return src[:pos] + new + src[pos + len(old):]


def _run_pins(lib_path, timeout=600, threads=2):
    env = dict(os.environ, RPDLA_ORACLE_LIB=lib_path, OMP_NUM_THREADS=str(threads))
    cmd = [sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider"] + PIN_FILES
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=timeout)
    return r.returncode, r.stdout[-400:]


def _build(src_text, out_dir, name):
    c_path = os.path.join(out_dir, name + ".c")
    so_path = os.path.join(out_dir, name + ".so")
    with open(c_path, "w") as f:
        f.write(src_text)
    subprocess.run(["gcc", "-O1", "-std=gnu11", "-fopenmp", "-fPIC", "-shared", "-w", "-o",
                    so_path, c_path, "-lm"], check=True)
    return so_path


def test_every_mutant_is_caught():
    src = open(SRC).read()
    with tempfile.TemporaryDirectory() as d:
        # the harness itself: the unchanged oracle passes every pin
        rc, out = _run_pins(_build(src, d, "control"))
        assert rc == 0, out

        def one(i):
            label, old, new, nth = MUTANTS[i]
            so = _build(_mutate(src, old, new, nth), d, "m%02d" % i)
            rc, out = _run_pins(so)
            return label, rc, out

        with cf.ThreadPoolExecutor(max_workers=4) as ex:
            results = list(ex.map(one, range(len(MUTANTS))))
    missed = [(label, rc) for label, rc, _ in results if rc != 1]
    print(f"{len(MUTANTS)} mutants, {len(MUTANTS) - len(missed)} caught")
    assert not missed, missed


@pytest.mark.parametrize("label,old,new,nth", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutation_site_exists(label, old, new, nth):
    """Each planted mistake changes the current oracle source (a stale site
    would make a mutant identical to the oracle)."""
    src = open(SRC).read()
    assert _mutate(src, old, new, nth) != src


def test_pins_hold_for_extended_build():
    """The extended-precision build of the oracle (the same source, every
    step in x87 extended precision) is the reference that decides which
    double results are determined to a tolerance at all, so it must pass the
    same pins as the plain build."""
    import oracle
    oracle.build(force=False)
    rc, out = _run_pins(os.path.join(ROOT, "oracle", "liborc_ext.so"), timeout=900,
                        threads=os.cpu_count() or 2)
    assert rc == 0, out
