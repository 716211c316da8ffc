/*
 * rpdla_oracle.c -- plain, slow FP64 CPU oracle for the ionization-seeded
 * electron-acceleration Monte Carlo of arXiv 2509.01741 (Hissi, Ngirmang,
 * Smith, Chowdhury: forward and backward acceleration by a radially
 * polarized focus seeded by field ionization of neon).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no source, header, table or constant with the
 * HIP library: every constant below is typed here on its own.
 *
 * Everything is SI, scalar, double precision, evaluated directly from the
 * defining formulas (real trigonometric form of the fields, explicit Gouy
 * arctangent, explicit powers of 1+zeta^2).  OpenMP only splits independent
 * atoms / electrons across threads; each one is computed exactly as a serial
 * loop would.
 *
 * Sections of the paper followed (paper = arXiv 2509.01741):
 *   - focal-volume Monte Carlo sampling ......... Sec. 2.1 "Ionization"
 *   - radially polarized fields ................. Sec. 2.1 "Acceleration", Eqs. (1)-(2)
 *                                                  and the phase definition below them
 *   - tunnelling (semi-classical) ionization .... Sec. 1 and Sec. 2.1 "Ionization"
 *   - Newton-Lorentz equations .................. Eqs. (7)-(14)
 *   - kinetic energy and azimuth ................ text after Eq. (14); Sec. 2.2, Fig. 5 text
 *   - forward / backward classification ......... Sec. 2.2 (Figs. 4, 7-9, 13-16)
 *   - birth phase, hollow-cylinder ions, 2-D maps  Sec. 2.2, Figs. 6, 8, 13, 14
 *   - radiation reaction and quantum parameter .. Sec. 2.1, Eqs. (3)-(6)
 *   - controlled-step fifth-order push .......... Sec. 1 and Sec. 2.1
 *
 * Readings where the paper is silent or garbled are listed next to the code
 * that takes them.  Parity status: every function is pinned by the CPU tests
 * (closed forms, invariants, library routines, printed worked values) except
 * one part of the tunnelling rate, which is PARITY UNPINNED: the dependence of
 * its prefactor C^2 on a non-integer effective quantum number n*.  The paper
 * names the tunnelling model without a formula, so nothing fixes that
 * dependence; the pins cover the hydrogen and hydrogen-like limits (n* = 1),
 * the state -> (potential, charge) mapping through the hydrogen-like last
 * neon electron, and the power of the field at every neon n*.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <tgmath.h>
#undef I   /* the imaginary unit of <complex.h>; nothing here is complex */

/* Working precision.  The oracle is plain double; the same source built with
 * -DORC_EXTENDED computes every step in x87 extended precision (64-bit
 * significand, 2^11 finer than double) with the same arguments and outputs,
 * as the reference that tells which double results are determined to a
 * given tolerance at all.  <tgmath.h> picks each math function's precision
 * from its argument; ORC_R marks a decimal constant of working precision. */
#ifdef ORC_EXTENDED
typedef long double orc_real;
#define ORC_R(x) x##L
#else
typedef double orc_real;
#define ORC_R(x) x
#endif

/* The crossing solve stops at a Newton correction of at most
 * 2^ORC_CROSS_TOL_EXP max(|t|, T) (the last correction is applied, so the
 * result is accurate to about the square of that). */
#ifndef ORC_CROSS_TOL_EXP
#define ORC_CROSS_TOL_EXP (-40)
#endif

/* ---------------------------------------------------------------------------
 * Constants (CODATA 2018 exact / recommended values, SI).
 * ------------------------------------------------------------------------- */
#define ORC_C        ORC_R(299792458.0)         /* speed of light, m/s        */
#define ORC_QE       ORC_R(1.602176634e-19)     /* elementary charge, C       */
#define ORC_ME       ORC_R(9.1093837015e-31)    /* electron mass, kg          */
#define ORC_EPS0     ORC_R(8.8541878128e-12)    /* vacuum permittivity, F/m   */
#define ORC_MEC2_MEV ORC_R(0.51099895000)       /* electron rest energy, MeV  */
#define ORC_EA       ORC_R(5.14220674763e11)    /* atomic unit of field, V/m  */
#define ORC_TAUA     ORC_R(2.4188843265857e-17) /* atomic unit of time, s     */
#define ORC_EH_EV    ORC_R(27.211386245988)     /* Hartree energy, eV         */
#define ORC_PI       ORC_R(3.14159265358979323846264338327950288)
#define ORC_HBAR     ORC_R(1.054571817e-34)     /* reduced Planck constant, J s */
#define ORC_ALPHA    ORC_R(7.2973525693e-3)     /* fine-structure constant    */

/* Neon ionization potentials Ne^(k-1)+ -> Ne^k+, k = 1..10, in eV (NIST ASD
 * values; the paper names the charge states but prints no potentials). */
static const orc_real orc_ne_ip_ev[10] = {
    ORC_R(21.564540), ORC_R(40.96297), ORC_R(63.4233), ORC_R(97.1900), ORC_R(126.247),
    ORC_R(157.934), ORC_R(207.271), ORC_R(239.0970), ORC_R(1195.80784), ORC_R(1362.19911)};

/* field models */
enum { ORC_RP_O1 = 1, ORC_RP_O3 = 3, ORC_RP_O5 = 5,
       ORC_PLANE_LP = 10, ORC_UNIFORM_EB = 11,
       ORC_LP_O1 = 21, ORC_LP_O3 = 23, ORC_LP_O5 = 25 };
/* integration window */
enum { ORC_WIN_ARRIVAL = 0, ORC_WIN_LAB = 1 };
/* histogram angle */
enum { ORC_ANG_POLAR = 0, ORC_ANG_AZIMUTH = 1 };

typedef struct {
    double lambda, w0, tau_fwhm; /* m, m, s (intensity FWHM)                */
    double amp;                  /* Er amplitude of Eq. (1), V/m             */
    double phi0;                 /* carrier phase                            */
    int field, window;
    double t_before, t_after;    /* window bounds, s                         */
    double dt;                   /* step / panel width, s                    */
    double ez_scale, er_scale;   /* multipliers on Ez and on Ex, Ey          */
    double test_E[3], test_B[3]; /* uniform-field test model                 */
} orc_laser;

typedef struct {
    int nE, nA;
    double logE_min_MeV, logE_max_MeV;
    int angle;
} orc_hist_spec;

void orc_ne_ip_table(double out[10])
{
    for (int i = 0; i < 10; ++i) out[i] = (double)orc_ne_ip_ev[i];
}

/* 1 in the extended-precision build, 0 in the plain one. */
int orc_is_extended(void)
{
#ifdef ORC_EXTENDED
    return 1;
#else
    return 0;
#endif
}

void orc_constants(double out[8])
{
    out[0] = ORC_C; out[1] = ORC_QE; out[2] = ORC_ME; out[3] = ORC_EPS0;
    out[4] = ORC_MEC2_MEV; out[5] = ORC_EA; out[6] = ORC_TAUA; out[7] = ORC_EH_EV;
}

/* ---------------------------------------------------------------------------
 * Laser set-up.  Amplitude from peak intensity uses the Gaussian-equivalent
 * field E0 = sqrt(2 I / (eps0 c)) that Sec. 2.1 attaches to every intensity
 * (5e19 W/cm^2 -> 1.94e13 V/m, 5e21 W/cm^2 -> 1.94e14 V/m); that value is
 * the E0 of Eq. (1).  From power, the order-1 beam carries
 * P = pi w0^2 eps0 c A^2 / 8 (flux of E x H integrated over the focal plane).
 * Defaults: window [-5 tau, +10 tau] around the pulse, dt = T/200, unit
 * field scales, field order 5.
 * ------------------------------------------------------------------------- */
static void orc_laser_defaults(orc_laser* L, double lambda, double w0, double tau)
{
    memset(L, 0, sizeof(*L));
    L->lambda = lambda; L->w0 = w0; L->tau_fwhm = tau;
    L->phi0 = 0.0;
    L->field = ORC_RP_O5;
    L->window = ORC_WIN_ARRIVAL;
    L->t_before = 5.0 * tau;
    L->t_after = 10.0 * tau;
    L->dt = lambda / ORC_C / 200.0;
    L->ez_scale = 1.0; L->er_scale = 1.0;
}

void orc_laser_init_intensity(orc_laser* L, double lambda, double w0, double tau, double I_W_cm2)
{
    orc_laser_defaults(L, lambda, w0, tau);
    double I = I_W_cm2 * 1.0e4; /* W/m^2 */
    L->amp = sqrt(2.0 * I / (ORC_EPS0 * ORC_C));
}

void orc_laser_init_power(orc_laser* L, double lambda, double w0, double tau, double P_W)
{
    orc_laser_defaults(L, lambda, w0, tau);
    L->amp = sqrt(8.0 * P_W / (ORC_PI * w0 * w0 * ORC_EPS0 * ORC_C));
}

/* Rayleigh length z_r = k0 r0^2 / 2 (definition under Eq. (2)). */
double orc_rayleigh(const orc_laser* L)
{
    double k = 2.0 * ORC_PI / L->lambda;
    return 0.5 * k * L->w0 * L->w0;
}

/* ---------------------------------------------------------------------------
 * Counter-based random numbers: Philox4x64-10 (Salmon, Moraes, Dror, Shaw,
 * "Parallel random numbers: as easy as 1, 2, 3", SC'11).  Ten rounds of two
 * 64x64->128 multiplies; the key is bumped by the Weyl constants between
 * rounds.
 * ------------------------------------------------------------------------- */
static void orc_mulhilo64(uint64_t a, uint64_t b, uint64_t* hi, uint64_t* lo)
{
    unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

void orc_philox4x64_10(const uint64_t ctr_in[4], const uint64_t key_in[2], uint64_t out[4])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint64_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        uint64_t hi0, lo0, hi1, lo1;
        orc_mulhilo64(M0, c0, &hi0, &lo0);
        orc_mulhilo64(M1, c2, &hi1, &lo1);
        uint64_t n0 = hi1 ^ c1 ^ k0;
        uint64_t n1 = lo1;
        uint64_t n2 = hi0 ^ c3 ^ k1;
        uint64_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += W0; k1 += W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Uniform variate number j of atom `atom` in configuration `cfg`: key
 * (seed, cfg), counter (atom, j/4, 0, 0), word j%4; the top 53 bits give
 * u = (m + 1) 2^-53 in (0, 1].  Streams: j = 0,1,2 position; j = k + 2 is
 * the ionization threshold of charge state k (k = 1..10). */
double orc_uniform(uint64_t seed, uint32_t cfg, uint64_t atom, int j)
{
    uint64_t ctr[4] = {atom, (uint64_t)(j >> 2), 0, 0};
    uint64_t key[2] = {seed, (uint64_t)cfg};
    uint64_t out[4];
    orc_philox4x64_10(ctr, key, out);
    uint64_t m = out[j & 3] >> 11;
    return ((double)m + 1.0) * (1.0 / 9007199254740992.0);
}

/* Focal-volume sampling (Sec. 2.1): ions at rest, uniform in a cylinder about
 * the propagation axis, focus at the origin: r = R sqrt(u0),
 * azimuth 2 pi u1, z = zh (2 u2 - 1). */
static void orc_sample_one(uint64_t seed, uint32_t cfg, uint64_t a, orc_real r_max,
                           orc_real z_half, orc_real* x, orc_real* y, orc_real* z)
{
    double u0 = orc_uniform(seed, cfg, a, 0);
    double u1 = orc_uniform(seed, cfg, a, 1);
    double u2 = orc_uniform(seed, cfg, a, 2);
    orc_real r = r_max * sqrt((orc_real)u0);
    orc_real th = 2.0 * ORC_PI * u1;
    *x = r * cos(th);
    *y = r * sin(th);
    *z = z_half * (2.0 * u2 - 1.0);
}

void orc_sample_atoms(uint64_t seed, uint32_t cfg, uint64_t first_atom, int64_t n,
                      double r_max, double z_half, double* x, double* y, double* z)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        orc_real xr, yr, zr;
        orc_sample_one(seed, cfg, first_atom + (uint64_t)i, r_max, z_half, &xr, &yr, &zr);
        x[i] = (double)xr;
        y[i] = (double)yr;
        z[i] = (double)zr;
    }
}

/* ---------------------------------------------------------------------------
 * Fields.
 *
 * Radially polarized TM01 focus, Eqs. (1)-(2) with the phase, f^2 and z_r
 * defined beneath them, B_theta from Maxwell's equations and the w0/z_r
 * (non-paraxial) corrections the text names.  Derivation: vector potential
 * A = z^ A0 psi(rho, zeta) exp(i(omega t - k z)) in Lorenz gauge with the
 * Lax series psi = psi0 + eps^2 psi2 + eps^4 psi4, eps = w0/z_r,
 * rho = r/w0, zeta = z/z_r.  Writing
 *     D = 1 + zeta^2,   Psi = phi0 + omega t - k z - rho^2 zeta / D,
 *     g = exp(-rho^2/D - (t - z/c)^2/tau0^2),
 *     C_n = A g D^(-n/2) cos(Psi + n atan zeta),
 *     S_n = A g D^(-n/2) sin(Psi + n atan zeta),
 * the fields are
 *   Er/r  = (1/w0)[C2 + eps^2(-C3/2 + rho^2 C4 - rho^4 C5/4)
 *                  + eps^4(-3C4/8 - 3rho^2 C5/8 + 17rho^4 C6/16 - 3rho^6 C7/8 + rho^8 C8/32)]
 *   Ez    = eps(S2 - rho^2 S3) + eps^3(S3/2 + rho^2 S4/2 - 5rho^4 S5/4 + rho^6 S6/4)
 *   cBt/r = (1/w0)[C2 + eps^2(C3/2 + rho^2 C4/2 - rho^4 C5/4)
 *                  + eps^4(3C4/8 + 3rho^2 C5/8 + 3rho^4 C6/16 - rho^6 C7/4 + rho^8 C8/32)]
 * Order 1 keeps the first term of each line, order 3 adds the eps^2 terms of
 * Er and Bt and the eps^3 term of Ez, order 5 keeps everything.
 *
 * Readings: (i) the envelope exponent is negative (the printed Eqs. (1)-(2)
 * lost the minus sign); (ii) the printed Eq. (2) is inconsistent with the
 * printed phase -- with the phase as printed it fails Gauss's law at order
 * eps; Ez here is Eq. (2) evaluated at -phi, the Maxwell-consistent sign;
 * (iii) tau0 = tau_FWHM / sqrt(2 ln 2), so exp(-2 (t-z/c)^2/tau0^2), the
 * intensity envelope, has full width tau_FWHM at half maximum; (iv) A, the
 * amplitude of Eq. (1), is held fixed when the order changes.  Order-1 Er is
 * Eq. (1) exactly (with E0 = A and the paper's phi = -(Psi + 2 atan zeta)).
 *
 * Test models: a linearly polarized plane wave Ex = A env cos(omega t - k z
 * + phi0), By = Ex/c, and uniform static E and B.
 * ------------------------------------------------------------------------- */
/* ---------------------------------------------------------------------------
 * Linearly polarized focus (Sec. 2.2 compares the radially polarized pulse
 * with a linearly polarized one of the same intensity, wavelength and focus,
 * Fig. 4; the paper gives no field for it).  Reading: the same construction
 * as the radial focus with the vector potential along x instead of z,
 *     A = x^ (i E0 / omega) psi(rho, zeta) exp(i eta),  eta = omega t - k z + phi0,
 * the same Lax series psi = psi0 + eps^2 psi2 + eps^4 psi4 (orders 1, 3, 5:
 * the series truncated after psi0, psi2, psi4), Lorenz gauge
 * (phi = (i c^2/omega) dA_x/dx), E = -grad phi - dA/dt, B = curl A, physical
 * fields the real parts, times the same temporal envelope.  With
 * s = rho^2 = (x^2 + y^2)/w0^2, rx = x/w0, ry = y/w0 and the derivatives of
 * psi with respect to s and zeta (subscripts):
 *   Ex = E0 Re{[psi + (eps^2/2) psi_s + eps^2 rx^2 psi_ss] e^{i eta}}
 *   Ey = E0 Re{eps^2 rx ry psi_ss e^{i eta}}
 *   Ez = E0 Re{[(eps^3/2) rx psi_s,zeta - i eps rx psi_s] e^{i eta}}
 *   c Bx = 0,  c By = E0 Re{[psi + i (eps^2/2) psi_zeta] e^{i eta}},
 *   c Bz = E0 Re{-i eps ry psi_s e^{i eta}}.
 * E0 is the peak field at the focus of the paraxial beam, so the amplitude
 * from intensity, sqrt(2 I / (eps0 c)), gives peak intensity I.  The
 * derivatives of psi are taken exactly by hyper-dual arithmetic (numbers
 * a + b e1 + c e2 + d e1 e2 with e1^2 = e2^2 = 0, complex parts): evaluating
 * psi at s + e1 + e2 gives psi_s in b and psi_ss in d, at (s + e1, zeta + e2)
 * psi_zeta in c and psi_s,zeta in d.
 * ------------------------------------------------------------------------- */
#ifdef ORC_EXTENDED
typedef long double _Complex orc_cplx;
#else
typedef double _Complex orc_cplx;
#endif
typedef struct { orc_cplx a, b, c, d; } orc_hd;

static orc_hd hd_make(orc_cplx a, orc_cplx b, orc_cplx c)
{
    orc_hd r = {a, b, c, 0};
    return r;
}

static orc_hd hd_add(orc_hd x, orc_hd y)
{
    orc_hd r = {x.a + y.a, x.b + y.b, x.c + y.c, x.d + y.d};
    return r;
}

static orc_hd hd_scale(orc_hd x, orc_cplx k)
{
    orc_hd r = {k * x.a, k * x.b, k * x.c, k * x.d};
    return r;
}

static orc_hd hd_mul(orc_hd x, orc_hd y)
{
    orc_hd r = {x.a * y.a, x.a * y.b + x.b * y.a, x.a * y.c + x.c * y.a,
                x.a * y.d + x.b * y.c + x.c * y.b + x.d * y.a};
    return r;
}

static orc_hd hd_exp(orc_hd x)
{
    orc_cplx e = exp(x.a);
    orc_hd r = {e, e * x.b, e * x.c, e * (x.d + x.b * x.c)};
    return r;
}

static orc_hd hd_inv(orc_hd x)
{
    orc_cplx q = 1.0 / x.a;
    orc_hd r = {q, -q * q * x.b, -q * q * x.c, 2.0 * q * q * q * x.b * x.c - q * q * x.d};
    return r;
}

static orc_hd hd_pow(orc_hd x, int n)
{
    orc_hd r = hd_make(1.0, 0.0, 0.0);
    for (int i = 0; i < n; ++i) r = hd_mul(r, x);
    return r;
}

/* The Lax series psi(s, zeta) truncated at `order` (1, 3 or 5):
 *   f = 1/(1 - i zeta),  psi0 = f e^{-f s},
 *   psi2 = (f^2/2 - f^4 s^2/4) e^{-f s},
 *   psi4 = (3f^3/8 - 3f^5 s^2/16 - f^6 s^3/8 + f^7 s^4/32) e^{-f s}. */
static orc_hd orc_lax_psi(orc_hd S, orc_hd Zt, orc_real eps, int order)
{
    const orc_cplx iu = (orc_cplx)_Complex_I;
    orc_hd one = hd_make(1.0, 0.0, 0.0);
    orc_hd f = hd_inv(hd_add(one, hd_scale(Zt, -iu)));
    orc_hd P = f;
    if (order >= 3) {
        orc_hd p2 = hd_add(hd_scale(hd_pow(f, 2), 0.5),
                           hd_scale(hd_mul(hd_pow(f, 4), hd_pow(S, 2)), -0.25));
        P = hd_add(P, hd_scale(p2, eps * eps));
    }
    if (order >= 5) {
        orc_hd p4 = hd_scale(hd_pow(f, 3), 3.0 / 8.0);
        p4 = hd_add(p4, hd_scale(hd_mul(hd_pow(f, 5), hd_pow(S, 2)), -3.0 / 16.0));
        p4 = hd_add(p4, hd_scale(hd_mul(hd_pow(f, 6), hd_pow(S, 3)), -1.0 / 8.0));
        p4 = hd_add(p4, hd_scale(hd_mul(hd_pow(f, 7), hd_pow(S, 4)), 1.0 / 32.0));
        P = hd_add(P, hd_scale(p4, eps * eps * eps * eps));
    }
    return hd_mul(P, hd_exp(hd_scale(hd_mul(f, S), -1.0)));
}

static void orc_field_lp(const orc_laser* L, orc_real x, orc_real y, orc_real z, orc_real xi,
                         orc_real E[3], orc_real B[3])
{
    const orc_cplx iu = (orc_cplx)_Complex_I;
    const orc_real k = 2.0 * ORC_PI / L->lambda;
    const orc_real om = ORC_C * k;
    const orc_real tau0 = L->tau_fwhm / sqrt(2.0 * log((orc_real)2.0));
    const int order = L->field - 20;
    const orc_real w0 = L->w0;
    const orc_real zr = 0.5 * k * w0 * w0;
    const orc_real eps = w0 / zr;
    const orc_real rx = x / w0, ry = y / w0;
    const orc_real s = rx * rx + ry * ry;
    const orc_real zeta = z / zr;
    /* psi, psi_s, psi_ss */
    orc_hd ps = orc_lax_psi(hd_make(s, 1.0, 1.0), hd_make(zeta, 0.0, 0.0), eps, order);
    /* psi_zeta, psi_s,zeta */
    orc_hd pz = orc_lax_psi(hd_make(s, 1.0, 0.0), hd_make(zeta, 0.0, 1.0), eps, order);
    const orc_cplx psi = ps.a, psi_s = ps.b, psi_ss = ps.d, psi_z = pz.c, psi_sz = pz.d;
    const orc_real sg = xi / tau0;
    const orc_real amp = L->amp * exp(-sg * sg);
    const orc_cplx ph = exp(iu * (om * xi + L->phi0));
    const orc_real e2 = eps * eps;
    E[0] = L->er_scale * amp * creal((psi + 0.5 * e2 * psi_s + e2 * rx * rx * psi_ss) * ph);
    E[1] = L->er_scale * amp * creal(e2 * rx * ry * psi_ss * ph);
    E[2] = L->ez_scale * amp * creal((0.5 * e2 * eps * rx * psi_sz - iu * eps * rx * psi_s) * ph);
    B[0] = 0.0;
    B[1] = amp / ORC_C * creal((psi + iu * 0.5 * e2 * psi_z) * ph);
    B[2] = amp / ORC_C * creal(-iu * eps * ry * psi_s * ph);
}

/* Every field family depends on time only through the retarded time
 * xi = t - z/c (carrier phase omega xi, envelope xi/tau0); orc_field_ret takes
 * xi itself, orc_field the time t. */
static void orc_field_ret(const orc_laser* L, orc_real x, orc_real y, orc_real z, orc_real xi,
                          orc_real E[3], orc_real B[3])
{
    const orc_real k = 2.0 * ORC_PI / L->lambda;
    const orc_real om = ORC_C * k;
    const orc_real tau0 = L->tau_fwhm / sqrt(2.0 * log((orc_real)2.0));
    if (L->field == ORC_UNIFORM_EB) {
        for (int i = 0; i < 3; ++i) { E[i] = L->test_E[i]; B[i] = L->test_B[i]; }
        return;
    }
    if (L->field == ORC_LP_O1 || L->field == ORC_LP_O3 || L->field == ORC_LP_O5) {
        orc_field_lp(L, x, y, z, xi, E, B);
        return;
    }
    if (L->field == ORC_PLANE_LP) {
        orc_real s = xi / tau0;
        orc_real ex = L->amp * exp(-s * s) * cos(om * xi + L->phi0);
        E[0] = ex; E[1] = 0.0; E[2] = 0.0;
        B[0] = 0.0; B[1] = ex / ORC_C; B[2] = 0.0;
        return;
    }
    const int order = L->field;
    const orc_real w0 = L->w0;
    const orc_real zr = 0.5 * k * w0 * w0;
    const orc_real eps = w0 / zr;
    const orc_real rho2 = (x * x + y * y) / (w0 * w0);
    const orc_real zeta = z / zr;
    const orc_real D = 1.0 + zeta * zeta;
    const orc_real Psi = L->phi0 + om * xi - rho2 * zeta / D;
    const orc_real s = xi / tau0;
    const orc_real g = exp(-rho2 / D - s * s);
    const orc_real gouy = atan(zeta);
    orc_real C[9], S[9];
    for (int n = 2; n <= 8; ++n) {
        orc_real a = L->amp * g * pow(D, -0.5 * n);
        C[n] = a * cos(Psi + n * gouy);
        S[n] = a * sin(Psi + n * gouy);
    }
    const orc_real r2 = rho2, r4 = rho2 * rho2, r6 = r4 * rho2, r8 = r4 * r4;
    const orc_real e2 = eps * eps, e3 = e2 * eps, e4 = e2 * e2;
    orc_real PE = C[2];
    orc_real PB = C[2];
    orc_real Ez = eps * (S[2] - r2 * S[3]);
    if (order >= 3) {
        PE += e2 * (-C[3] / 2.0 + r2 * C[4] - r4 * C[5] / 4.0);
        PB += e2 * (C[3] / 2.0 + r2 * C[4] / 2.0 - r4 * C[5] / 4.0);
        Ez += e3 * (S[3] / 2.0 + r2 * S[4] / 2.0 - 5.0 * r4 * S[5] / 4.0 + r6 * S[6] / 4.0);
    }
    if (order >= 5) {
        PE += e4 * (-3.0 * C[4] / 8.0 - 3.0 * r2 * C[5] / 8.0 + 17.0 * r4 * C[6] / 16.0
                    - 3.0 * r6 * C[7] / 8.0 + r8 * C[8] / 32.0);
        PB += e4 * (3.0 * C[4] / 8.0 + 3.0 * r2 * C[5] / 8.0 + 3.0 * r4 * C[6] / 16.0
                    - r6 * C[7] / 4.0 + r8 * C[8] / 32.0);
    }
    /* Cartesian projection: Ex = Er x/r, Ey = Er y/r; Bx = -Bt y/r,
     * By = Bt x/r, Bz = 0 (text before Eq. (8)). */
    E[0] = L->er_scale * PE * x / w0;
    E[1] = L->er_scale * PE * y / w0;
    E[2] = L->ez_scale * Ez;
    B[0] = -PB * y / (w0 * ORC_C);
    B[1] = PB * x / (w0 * ORC_C);
    B[2] = 0.0;
}

static void orc_field(const orc_laser* L, orc_real x, orc_real y, orc_real z, orc_real t,
                      orc_real E[3], orc_real B[3])
{
    orc_field_ret(L, x, y, z, t - z / ORC_C, E, B);
}

/* ---------------------------------------------------------------------------
 * Tunnelling rate.  The paper cites the semi-classical (PPT) tunnelling model
 * without printing a formula; the rate used is the static ADK rate with
 * l = m = 0 and l* = n* - 1, in atomic units
 *   w = C^2 Ip (2 F0/F)^(2 n* - 1) exp(-2 F0 / (3 F)),
 *   n* = Z / sqrt(2 Ip), F0 = (2 Ip)^(3/2), C^2 = 2^(2 n*) / (n* Gamma(2 n*)),
 * Z the charge after ionization, evaluated in log space.  The rate is set to
 * exactly zero when F = 0 or ln(w [1/s]) < -700.  Parity unpinned: the n*
 * dependence of C^2 (see the header of this file).
 * ------------------------------------------------------------------------- */
static orc_real orc_adk_lnrate_r(orc_real Ip_au, orc_real Z, orc_real F_au)
{
    orc_real nstar = Z / sqrt(2.0 * Ip_au);
    orc_real F0 = pow(2.0 * Ip_au, (orc_real)1.5);
    orc_real lnC2 = 2.0 * nstar * log((orc_real)2.0) - log(nstar) - lgamma(2.0 * nstar);
    return lnC2 + log(Ip_au / ORC_TAUA) + (2.0 * nstar - 1.0) * log(2.0 * F0 / F_au)
           - 2.0 * F0 / (3.0 * F_au);
}

double orc_adk_lnrate_general(double Ip_au, double Z, double F_au)
{
    return (double)orc_adk_lnrate_r(Ip_au, Z, F_au);
}

/* ln of the rate [1/s] of Ne^(k-1)+ -> Ne^k+ at field magnitude Emag [V/m]. */
static orc_real orc_adk_lnrate_k(int k, orc_real Emag)
{
    orc_real Ip = orc_ne_ip_ev[k - 1] / ORC_EH_EV;
    return orc_adk_lnrate_r(Ip, (orc_real)k, Emag / ORC_EA);
}

double orc_adk_lnrate(int k, double Emag) { return (double)orc_adk_lnrate_k(k, Emag); }

static orc_real orc_adk_rate_k(int k, orc_real Emag)
{
    if (!(Emag > 0.0)) return 0.0;
    orc_real l = orc_adk_lnrate_k(k, Emag);
    if (l < -700.0) return 0.0;
    return exp(l);
}

double orc_adk_rate(int k, double Emag) { return (double)orc_adk_rate_k(k, Emag); }

static orc_real orc_emag(const orc_laser* L, orc_real x, orc_real y, orc_real z, orc_real t)
{
    orc_real E[3], B[3];
    orc_field(L, x, y, z, t, E, B);
    return sqrt(E[0] * E[0] + E[1] * E[1] + E[2] * E[2]);
}

/* 4-point Gauss-Legendre nodes / weights on [-1, 1], closed form. */
static void orc_gl4(orc_real xn[4], orc_real wn[4])
{
    const orc_real three = 3.0, two = 2.0, six = 6.0, thirty = 30.0;
    orc_real a = sqrt(three / 7.0 - two / 7.0 * sqrt(six / 5.0));
    orc_real b = sqrt(three / 7.0 + two / 7.0 * sqrt(six / 5.0));
    orc_real wa = (18.0 + sqrt(thirty)) / 36.0;
    orc_real wb = (18.0 - sqrt(thirty)) / 36.0;
    xn[0] = -b; xn[1] = -a; xn[2] = a; xn[3] = b;
    wn[0] = wb; wn[1] = wa; wn[2] = wa; wn[3] = wb;
}

void orc_gl4_table(double xn[4], double wn[4])
{
    orc_real x[4], w[4];
    orc_gl4(x, w);
    for (int i = 0; i < 4; ++i) { xn[i] = (double)x[i]; wn[i] = (double)w[i]; }
}

/* GL-4 estimate of the integral of w_k(|E(x,t)|) dt over [a, b]. */
static orc_real orc_rate_integral(const orc_laser* L, int k, orc_real x, orc_real y, orc_real z,
                                  orc_real a, orc_real b)
{
    orc_real xn[4], wn[4];
    orc_gl4(xn, wn);
    orc_real h = 0.5 * (b - a), m = 0.5 * (a + b);
    orc_real s = 0.0;
    for (int i = 0; i < 4; ++i)
        s += wn[i] * orc_adk_rate_k(k, orc_emag(L, x, y, z, m + h * xn[i]));
    return h * s;
}

/* Window of an atom at axial position z (reading: the bounds -5 tau, +10 tau
 * are taken relative to the pulse peak's arrival at the atom, z/c, so that
 * every atom sees the whole pulse; the lab-frame window is the alternative). */
static void orc_window(const orc_laser* L, orc_real z, orc_real* ts, orc_real* te)
{
    orc_real tz = (L->window == ORC_WIN_ARRIVAL) ? z / ORC_C : 0.0;
    *ts = tz - L->t_before;
    *te = tz + L->t_after;
}

/* Solve G(t) = target on [lo, hi], G(t) = GL-4 integral of w over [lo, t],
 * G(lo) = 0 < target <= G(hi): Newton steps with derivative w(t), kept inside
 * the bracket by bisection.  Start from linear interpolation on the panel;
 * accept t - d as soon as a Newton correction d is at most
 * 2^-40 max(|t|, T), or stop when a bisection step is that small. */
static orc_real orc_solve_crossing(const orc_laser* L, int k, orc_real x, orc_real y,
                                   orc_real z, orc_real lo, orc_real hi, orc_real target,
                                   orc_real Ghi)
{
    if (!(target > 0.0)) return lo;
    const orc_real T = L->lambda / ORC_C;
    orc_real tl = lo, th = hi;
    orc_real t = lo + (hi - lo) * (target / Ghi);
    if (!(t > tl && t < th)) t = 0.5 * (tl + th);
    for (int it = 0; it < 100; ++it) {
        orc_real gdiff = orc_rate_integral(L, k, x, y, z, lo, t) - target;
        if (gdiff == 0.0) return t;
        if (gdiff > 0.0) th = t; else tl = t;
        const orc_real tol = ldexp(fmax(fabs(t), T), ORC_CROSS_TOL_EXP);
        orc_real w = orc_adk_rate_k(k, orc_emag(L, x, y, z, t));
        orc_real tn = NAN;
        if (w > 0.0) {
            orc_real d = gdiff / w;
            if (fabs(d) <= tol) return t - d;   /* converged Newton step */
            tn = t - d;
        }
        if (!(tn > tl && tn < th)) tn = 0.5 * (tl + th);
        orc_real step = fabs(tn - t);
        t = tn;
        if (step <= tol) break;                 /* bracket below tolerance */
    }
    return t;
}

/* Ionization times of one atom.  Sequential charge states k_first..k_last
 * (text of Sec. 2.1: outer electrons first, then inner).  State k is born
 * when the accumulated rate since the previous birth reaches an Exp(1)
 * threshold -ln u (inverse-survival sampling: P(t_k > t) = exp(-int w dt)).
 * Integrals use GL-4 on panels of width dt laid from the window start; a
 * state that starts inside a panel integrates the remainder of that panel.
 * +INF marks a state not reached inside the window (and every later state). */
static void orc_ionize_atom(const orc_laser* L, uint64_t seed, uint32_t cfg, uint64_t atom,
                            orc_real x, orc_real y, orc_real z, int k_first, int k_last,
                            orc_real* tb)
{
    const int K = k_last - k_first + 1;
    for (int s = 0; s < K; ++s) tb[s] = INFINITY;
    orc_real ts, te;
    orc_window(L, z, &ts, &te);
    const orc_real h = L->dt;
    const int64_t M = (int64_t)ceil((te - ts) / h);
    int s = 0;
    orc_real target = -log((orc_real)orc_uniform(seed, cfg, atom, k_first + 2));
    orc_real I = 0.0;
    orc_real tstart = ts;
    for (int64_t j = 0; j < M && s < K; ++j) {
        orc_real a = ts + (orc_real)j * h;
        orc_real b = (j == M - 1) ? te : ts + (orc_real)(j + 1) * h;
        while (s < K) {
            orc_real lo = (tstart > a) ? tstart : a;
            orc_real seg = orc_rate_integral(L, k_first + s, x, y, z, lo, b);
            if (I + seg < target) { I += seg; break; }
            orc_real t = orc_solve_crossing(L, k_first + s, x, y, z, lo, b, target - I, seg);
            tb[s] = t;
            ++s;
            if (s < K) {
                target = -log((orc_real)orc_uniform(seed, cfg, atom, k_first + s + 2));
                I = 0.0;
                tstart = t;
            }
        }
    }
}

void orc_ionize_one(const orc_laser* L, uint64_t seed, uint32_t cfg, uint64_t atom,
                    double x, double y, double z, int k_first, int k_last, double* tb)
{
    orc_real t[10];
    orc_ionize_atom(L, seed, cfg, atom, x, y, z, k_first, k_last, t);
    for (int s = 0; s < k_last - k_first + 1; ++s) tb[s] = (double)t[s];
}

void orc_ionize(const orc_laser* L, uint64_t seed, uint32_t cfg, uint64_t first_atom, int64_t n,
                const double* x, const double* y, const double* z, int k_first, int k_last,
                double* t_birth)
{
    const int K = k_last - k_first + 1;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < n; ++i)
        orc_ionize_one(L, seed, cfg, first_atom + (uint64_t)i, x[i], y[i], z[i],
                       k_first, k_last, t_birth + i * K);
}

/* ---------------------------------------------------------------------------
 * Newton-Lorentz push (Eqs. (7)-(14), radiation reaction dropped as the
 * paper does below 5e22 W/cm^2).  State (x, u) with u = p/(m c):
 *   dx/dt = c u / gamma,  du/dt = -(e/(m c)) (E + (c u/gamma) x B),
 *   gamma = sqrt(1 + u.u).
 * Classical fourth-order Runge-Kutta with fixed step h (reading: the paper's
 * controlled-step fifth-order scheme is its own integrator; a fixed step
 * makes the discretized result unique).  Step n starts at t0 + n h; the
 * last step ends exactly at t_end.
 *
 * The state is accumulated with compensated (Kahan) summation.  The result
 * the definition asks for is the RK4 map in exact arithmetic; over the
 * ~3e4 steps of a trajectory, plain accumulation of the position in double
 * moves the final energy of a few electrons in a thousand by more than 1e-8
 * (their trajectories amplify rounding by up to ~1e8; measured against the
 * extended-precision build), and compensation removes that part of the
 * rounding error.
 *
 * The fields depend on time only through the retarded time xi = t - z/c,
 * and the state carries xi as a seventh variable, d xi/dt = 1 - v_z/c, from
 * xi = t0 - z0/c.  RK4 is linear in the stage slopes, so in exact arithmetic
 * its xi equals t - z/c at every stage and step: the discretized trajectory
 * is the one of the six-variable system.  In floating point the carrier
 * phase omega xi is then resolved to the rounding of xi itself instead of
 * that of omega t and k z separately (each up to ~1e3 rad over the window).
 * ------------------------------------------------------------------------- */
static void orc_kahan_add(orc_real* sum, orc_real* comp, orc_real v)
{
    orc_real y = v - *comp;
    orc_real t = *sum + y;
    *comp = (t - *sum) - y;
    *sum = t;
}

/* Slopes of (x, u) for the fields E, B at the state; returns gamma. */
static orc_real orc_lorentz(const orc_real Y[6], const orc_real E[3], const orc_real B[3],
                            orc_real dY[6])
{
    orc_real gam = sqrt(1.0 + Y[3] * Y[3] + Y[4] * Y[4] + Y[5] * Y[5]);
    orc_real vx = ORC_C * Y[3] / gam, vy = ORC_C * Y[4] / gam, vz = ORC_C * Y[5] / gam;
    const orc_real q = -ORC_QE / (ORC_ME * ORC_C);
    dY[0] = vx; dY[1] = vy; dY[2] = vz;
    dY[3] = q * (E[0] + (vy * B[2] - vz * B[1]));
    dY[4] = q * (E[1] + (vz * B[0] - vx * B[2]));
    dY[5] = q * (E[2] + (vx * B[1] - vy * B[0]));
    return gam;
}

/* Six-variable right-hand side at time t (the controlled-step push). */
static void orc_rhs(const orc_laser* L, orc_real t, const orc_real Y[6], orc_real dY[6])
{
    orc_real E[3], B[3];
    orc_field(L, Y[0], Y[1], Y[2], t, E, B);
    orc_lorentz(Y, E, B, dY);
}

/* Seven-variable right-hand side: Y[6] = xi = t - z/c. */
static void orc_rhs_xi(const orc_laser* L, const orc_real Y[7], orc_real dY[7])
{
    orc_real E[3], B[3];
    orc_field_ret(L, Y[0], Y[1], Y[2], Y[6], E, B);
    const orc_real gam = orc_lorentz(Y, E, B, dY);
    dY[6] = 1.0 - Y[5] / gam;
}

static void orc_push_elec(const orc_laser* L, orc_real t0, orc_real t_end, orc_real h,
                          const orc_real x0[3], const orc_real u0[3], orc_real xf[3],
                          orc_real uf[3])
{
    orc_real Y[7] = {x0[0], x0[1], x0[2], u0[0], u0[1], u0[2], t0 - x0[2] / ORC_C};
    orc_real comp[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    const int64_t N = (int64_t)ceil((t_end - t0) / h);
    for (int64_t n = 0; n < N; ++n) {
        orc_real ta = t0 + (orc_real)n * h;
        orc_real hn = (n == N - 1) ? t_end - ta : h;
        orc_real k1[7], k2[7], k3[7], k4[7], Yt[7];
        orc_rhs_xi(L, Y, k1);
        for (int i = 0; i < 7; ++i) Yt[i] = Y[i] + 0.5 * hn * k1[i];
        orc_rhs_xi(L, Yt, k2);
        for (int i = 0; i < 7; ++i) Yt[i] = Y[i] + 0.5 * hn * k2[i];
        orc_rhs_xi(L, Yt, k3);
        for (int i = 0; i < 7; ++i) Yt[i] = Y[i] + hn * k3[i];
        orc_rhs_xi(L, Yt, k4);
        for (int i = 0; i < 7; ++i)
            orc_kahan_add(&Y[i], &comp[i], hn / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]));
    }
    for (int i = 0; i < 3; ++i) { xf[i] = Y[i]; uf[i] = Y[3 + i]; }
}

void orc_push_one(const orc_laser* L, double t0, double t_end, double h,
                  const double x0[3], const double u0[3], double xf[3], double uf[3])
{
    orc_real X0[3] = {x0[0], x0[1], x0[2]}, U0[3] = {u0[0], u0[1], u0[2]}, XF[3], UF[3];
    orc_push_elec(L, t0, t_end, h, X0, U0, XF, UF);
    for (int i = 0; i < 3; ++i) { xf[i] = (double)XF[i]; uf[i] = (double)UF[i]; }
}

/* Push every born slot from rest (Sec. 2.1: electrons born with zero
 * momentum at their ionization time).  Slot s belongs to atom
 * s / slots_per_atom.  Unborn slots (t_birth = +INF) get NaN outputs, and so
 * do births more than one step before the window start (invalid input). */
void orc_push(const orc_laser* L, int64_t n_slots, const double* t_birth,
              const double* x0, const double* y0, const double* z0, int slots_per_atom,
              double* ux, double* uy, double* uz, double* xf, double* yf, double* zf)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t s = 0; s < n_slots; ++s) {
        int64_t a = s / slots_per_atom;
        double t0 = t_birth[s];
        if (!(t0 < INFINITY)) {
            ux[s] = uy[s] = uz[s] = xf[s] = yf[s] = zf[s] = NAN;
            continue;
        }
        orc_real ts, te;
        orc_window(L, z0[a], &ts, &te);
        if (!(t0 >= ts - L->dt)) {   /* birth before the window: invalid slot */
            ux[s] = uy[s] = uz[s] = xf[s] = yf[s] = zf[s] = NAN;
            continue;
        }
        orc_real X0[3] = {x0[a], y0[a], z0[a]}, U0[3] = {0.0, 0.0, 0.0}, XF[3], UF[3];
        orc_push_elec(L, t0, te, L->dt, X0, U0, XF, UF);
        ux[s] = (double)UF[0]; uy[s] = (double)UF[1]; uz[s] = (double)UF[2];
        xf[s] = (double)XF[0]; yf[s] = (double)XF[1]; zf[s] = (double)XF[2];
    }
}

/* Kinetic energy m c^2 u^2 / (gamma + 1) [MeV] of normalized momentum u. */
static orc_real orc_kinetic(const orc_real u[3])
{
    orc_real u2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    return ORC_MEC2_MEV * u2 / (sqrt(1.0 + u2) + 1.0);
}

/* The whole chain for the atoms with indices atoms[0..n-1], in working
 * precision, with nothing rounded to double between the steps: sampling in a
 * cylinder r < r_max, |z| < z_half, ionization times of states
 * k_first..k_last, the push of every born electron from its birth and its
 * kinetic energy.  Outputs are rounded to double at the end: positions
 * x, y, z [n]; per slot t_birth, ux, uy, uz, K_MeV [n K] (+INF / NaN as for
 * orc_ionize / orc_push).  In the plain build this equals orc_sample_atoms,
 * orc_ionize, orc_push and orc_epilogue called in turn. */
void orc_chain(const orc_laser* L, uint64_t seed, uint32_t cfg, const uint64_t* atoms, int64_t n,
               double r_max, double z_half, int k_first, int k_last, double* x, double* y,
               double* z, double* t_birth, double* ux, double* uy, double* uz, double* K_MeV)
{
    const int K = k_last - k_first + 1;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < n; ++i) {
        orc_real X[3], tb[10];
        orc_sample_one(seed, cfg, atoms[i], r_max, z_half, &X[0], &X[1], &X[2]);
        x[i] = (double)X[0]; y[i] = (double)X[1]; z[i] = (double)X[2];
        orc_ionize_atom(L, seed, cfg, atoms[i], X[0], X[1], X[2], k_first, k_last, tb);
        orc_real ts, te;
        orc_window(L, X[2], &ts, &te);
        for (int k = 0; k < K; ++k) {
            const int64_t sl = i * K + k;
            t_birth[sl] = (double)tb[k];
            if (!(tb[k] < INFINITY) || !(tb[k] >= ts - L->dt)) {
                ux[sl] = uy[sl] = uz[sl] = K_MeV[sl] = NAN;
                continue;
            }
            orc_real U0[3] = {0.0, 0.0, 0.0}, XF[3], UF[3];
            orc_push_elec(L, tb[k], te, L->dt, X, U0, XF, UF);
            ux[sl] = (double)UF[0]; uy[sl] = (double)UF[1]; uz[sl] = (double)UF[2];
            K_MeV[sl] = (double)orc_kinetic(UF);
        }
    }
}

/* ---------------------------------------------------------------------------
 * Outputs.  Kinetic energy (gamma - 1) m c^2 (text after Eq. (14)), written
 * as m c^2 u^2 / (gamma + 1); polar emission angle atan2(|u_perp|, u_z);
 * azimuth psi = atan2(u_y, u_x) (Fig. 5 text); forward iff u_z > 0 (the
 * final propagation direction, Sec. 2.2).
 * ------------------------------------------------------------------------- */
void orc_epilogue(int64_t n, const double* ux, const double* uy, const double* uz,
                  double* K_MeV, double* theta, double* psi, int32_t* fwd)
{
    for (int64_t i = 0; i < n; ++i) {
        double u2 = ux[i] * ux[i] + uy[i] * uy[i] + uz[i] * uz[i];
        double gam = sqrt(1.0 + u2);
        K_MeV[i] = ORC_MEC2_MEV * u2 / (gam + 1.0);
        theta[i] = atan2(sqrt(ux[i] * ux[i] + uy[i] * uy[i]), uz[i]);
        psi[i] = atan2(uy[i], ux[i]);
        fwd[i] = (uz[i] > 0.0) ? 1 : 0;
    }
}

/* Energy-angle histogram counts[dir][iE][iA], dir 0 = forward, 1 = backward;
 * log10-energy bins over [logE_min, logE_max); angle bins over [0, pi]
 * (polar) or (-pi, pi] (azimuth), the top edge folded into the last bin.
 * Tallies: 0 forward, 1 backward, 2 below range, 3 above range, 4 unborn,
 * 5 NaN.  Counts and tallies accumulate. */
void orc_histogram(int64_t n, const double* t_birth, const double* ux, const double* uy,
                   const double* uz, const orc_hist_spec* sp, uint64_t* counts,
                   uint64_t* tallies)
{
    const double width = (sp->logE_max_MeV - sp->logE_min_MeV) / (double)sp->nE;
    for (int64_t i = 0; i < n; ++i) {
        if (!(t_birth[i] < INFINITY)) { tallies[4] += 1; continue; }
        if (isnan(ux[i]) || isnan(uy[i]) || isnan(uz[i])) { tallies[5] += 1; continue; }
        double u2 = ux[i] * ux[i] + uy[i] * uy[i] + uz[i] * uz[i];
        double gam = sqrt(1.0 + u2);
        double K = ORC_MEC2_MEV * u2 / (gam + 1.0);
        int dir = (uz[i] > 0.0) ? 0 : 1;
        tallies[dir] += 1;
        double lk = log10(K);
        double fe = floor((lk - sp->logE_min_MeV) / width);
        if (!(fe >= 0.0)) { tallies[2] += 1; continue; }
        if (fe >= (double)sp->nE) { tallies[3] += 1; continue; }
        double ang, fa;
        if (sp->angle == ORC_ANG_POLAR) {
            ang = atan2(sqrt(ux[i] * ux[i] + uy[i] * uy[i]), uz[i]);
            fa = floor(ang / ORC_PI * (double)sp->nA);
        } else {
            ang = atan2(uy[i], ux[i]);
            fa = floor((ang + ORC_PI) / (2.0 * ORC_PI) * (double)sp->nA);
        }
        int ia = (int)fa;
        if (ia > sp->nA - 1) ia = sp->nA - 1;
        if (ia < 0) ia = 0;
        int ie = (int)fe;
        counts[((int64_t)dir * sp->nE + ie) * sp->nA + ia] += 1;
    }
}

/* ---------------------------------------------------------------------------
 * Batch helpers for the Python test harness.
 * ------------------------------------------------------------------------- */
void orc_field_batch(const orc_laser* L, int64_t n, const double* x, const double* y,
                     const double* z, const double* t, double* E, double* B)
{
    for (int64_t i = 0; i < n; ++i) {
        orc_real e[3], b[3];
        orc_field(L, x[i], y[i], z[i], t[i], e, b);
        for (int j = 0; j < 3; ++j) { E[3 * i + j] = (double)e[j]; B[3 * i + j] = (double)b[j]; }
    }
}

void orc_uniform_batch(uint64_t seed, uint32_t cfg, int64_t n, const uint64_t* atom,
                       const int32_t* j, double* u)
{
    for (int64_t i = 0; i < n; ++i) u[i] = orc_uniform(seed, cfg, atom[i], j[i]);
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_adk_rate_batch(int k, int64_t n, const double* Emag, double* w)
{
    for (int64_t i = 0; i < n; ++i) w[i] = orc_adk_rate(k, Emag[i]);
}

/* ---------------------------------------------------------------------------
 * Laser phase at a birth event (Sec. 2.2, Figs. 6, 13, 14: "initial phase of
 * the laser coincident with the birth"): the phase defined under Eq. (2),
 *   phi = k z - omega t - 2 atan(z/z_r) + z r^2 / (z_r r0^2 f^2) + phi0,
 * f^2 = 1 + (z/z_r)^2, with the paper's phi0 = -(this library's phi0)
 * (reading of the carrier-phase sign), reduced to [0, 2 pi).  NaN for
 * unborn slots.  Slot s belongs to atom s / slots_per_atom.
 * ------------------------------------------------------------------------- */
double orc_birth_phase_one(const orc_laser* L, double x, double y, double z, double t)
{
    const double k = 2.0 * ORC_PI / L->lambda;
    const double om = ORC_C * k;
    const double zr = 0.5 * k * L->w0 * L->w0;
    const double r2 = x * x + y * y;
    const double f2 = 1.0 + (z / zr) * (z / zr);
    double phi = k * z - om * t - 2.0 * atan(z / zr) + z * r2 / (zr * L->w0 * L->w0 * f2) - L->phi0;
    phi = fmod(phi, 2.0 * ORC_PI);
    if (phi < 0.0) phi += 2.0 * ORC_PI;
    if (phi >= 2.0 * ORC_PI) phi -= 2.0 * ORC_PI;
    return phi;
}

void orc_birth_phase(const orc_laser* L, int64_t n_slots, const double* t_birth, const double* x,
                     const double* y, const double* z, int slots_per_atom, double* phase)
{
    for (int64_t s = 0; s < n_slots; ++s) {
        int64_t a = s / slots_per_atom;
        phase[s] = (t_birth[s] < INFINITY) ? orc_birth_phase_one(L, x[a], y[a], z[a], t_birth[s]) : NAN;
    }
}

/* Annular sampling (Sec. 2.2, Fig. 8: ions uniform on the surface of a hollow
 * cylinder): r uniform in area between r_in and r_out, r = r_out exactly when
 * r_in == r_out (a surface); azimuth and z as in orc_sample_atoms. */
void orc_sample_atoms_annulus(uint64_t seed, uint32_t cfg, uint64_t first_atom, int64_t n,
                              double r_in, double r_out, double z_half, double* x, double* y,
                              double* z)
{
    for (int64_t i = 0; i < n; ++i) {
        uint64_t a = first_atom + (uint64_t)i;
        double u0 = orc_uniform(seed, cfg, a, 0);
        double u1 = orc_uniform(seed, cfg, a, 1);
        double u2 = orc_uniform(seed, cfg, a, 2);
        double r = (r_in == r_out) ? r_out : sqrt(r_in * r_in + u0 * (r_out * r_out - r_in * r_in));
        double th = 2.0 * ORC_PI * u1;
        x[i] = r * cos(th);
        y[i] = r * sin(th);
        z[i] = z_half * (2.0 * u2 - 1.0);
    }
}

/* ---------------------------------------------------------------------------
 * Two-dimensional histogram split by the direction of final motion, for the
 * birth-phase x birth-radius maps of forward and backward electrons (Sec. 2.2,
 * Figs. 13, 14) and the birth-variable x energy maps of Fig. 6.  Pair i goes
 * to counts[dir][ia][ib] with dir 0 if uz[i] > 0 else 1,
 * ia = floor((a[i] - a_lo) / ((a_hi - a_lo) / na)), ib likewise; pairs with a
 * NaN in a, b or uz are tallied in tallies[1], pairs outside the ranges in
 * tallies[0].  Counts and tallies accumulate.
 * ------------------------------------------------------------------------- */
void orc_histogram2d(int64_t n, const double* a, const double* b, const double* uz,
                     int32_t na, double a_lo, double a_hi, int32_t nb, double b_lo,
                     double b_hi, uint64_t* counts, uint64_t* tallies)
{
    const double wa = (a_hi - a_lo) / (double)na;
    const double wb = (b_hi - b_lo) / (double)nb;
    for (int64_t i = 0; i < n; ++i) {
        if (isnan(a[i]) || isnan(b[i]) || isnan(uz[i])) { tallies[1] += 1; continue; }
        const double fa = floor((a[i] - a_lo) / wa);
        const double fb = floor((b[i] - b_lo) / wb);
        if (!(fa >= 0.0 && fa < (double)na && fb >= 0.0 && fb < (double)nb)) {
            tallies[0] += 1;
            continue;
        }
        const int dir = (uz[i] > 0.0) ? 0 : 1;
        counts[((int64_t)dir * na + (int64_t)fa) * nb + (int64_t)fb] += 1;
    }
}


/* ---------------------------------------------------------------------------
 * Radiation reaction and the quantum parameter (Sec. 2.1, Eqs. (3)-(6)).
 *
 * Eq. (3) adds to the Lorentz force the leading (gamma^2) term of the
 * Landau-Lifshitz force.  In SI units
 *   F_RR = -(e^4 gamma^2 / (6 pi eps0 m^2 c^5)) v [(E + v x B)^2 - (v.E)^2 / c^2].
 * Reading: the printed coefficient 2 e^4 gamma^2 / (3 m c^5) is the Gaussian
 * one with a power of m lost; with e^2 -> e^2/(4 pi eps0) and B -> c B it
 * becomes the SI coefficient above.  The other Landau-Lifshitz terms (field
 * derivatives, gamma^0) are not in Eq. (3) and are not added.
 *
 * Quantum parameter: the general form of Eq. (4) for an electron of any
 * velocity, chi = (gamma / E_cr) sqrt((E + v x B)^2 - (v.E)^2 / c^2),
 * E_cr = m^2 c^3 / (e hbar); at rest it is E / E_cr (Eq. (5)) and head-on
 * against a plane wave gamma (1 + beta) E / E_cr (Eq. (4)).  The classical
 * radiation parameter of Eq. (6) is Rc = alpha a0 chi with a0 = e E0/(m c
 * omega) the laser's normalized amplitude.
 *
 * orc_push_rr pushes like orc_push with the term of Eq. (3) switched on
 * (rr = 1) or off (rr = 0) and records, per electron, the largest chi met at
 * the start of its RK4 steps (0 if it takes none).
 * ------------------------------------------------------------------------- */
static orc_real orc_ecr(void)
{
    return ORC_ME * ORC_ME * ORC_C * ORC_C * ORC_C / (ORC_QE * ORC_HBAR);
}

double orc_critical_field(void) { return (double)orc_ecr(); }

/* du/dt of Eq. (3)'s radiation term (u = p / m c) and chi, for state Y at
 * retarded time xi. */
static void orc_rr_terms_r(const orc_laser* L, orc_real xi, const orc_real Y[6], orc_real duRR[3],
                           orc_real* chi)
{
    orc_real E[3], B[3];
    orc_field_ret(L, Y[0], Y[1], Y[2], xi, E, B);
    const orc_real gam = sqrt(1.0 + Y[3] * Y[3] + Y[4] * Y[4] + Y[5] * Y[5]);
    const orc_real v[3] = {ORC_C * Y[3] / gam, ORC_C * Y[4] / gam, ORC_C * Y[5] / gam};
    const orc_real f[3] = {E[0] + (v[1] * B[2] - v[2] * B[1]),
                           E[1] + (v[2] * B[0] - v[0] * B[2]),
                           E[2] + (v[0] * B[1] - v[1] * B[0])};
    const orc_real vE = (v[0] * E[0] + v[1] * E[1] + v[2] * E[2]) / ORC_C;
    orc_real Q = f[0] * f[0] + f[1] * f[1] + f[2] * f[2] - vE * vE;
    if (Q < 0.0) Q = 0.0;
    const orc_real e2 = ORC_QE * ORC_QE;
    const orc_real coef = e2 * e2 * gam * gam /
                          (6.0 * ORC_PI * ORC_EPS0 * ORC_ME * ORC_ME * ORC_C * ORC_C * ORC_C * ORC_C * ORC_C);
    for (int i = 0; i < 3; ++i) duRR[i] = -coef * v[i] * Q / (ORC_ME * ORC_C);
    *chi = gam * sqrt(Q) / orc_ecr();
}

void orc_rr_terms(const orc_laser* L, double t, const double Y[6], double duRR[3], double* chi)
{
    orc_real Yr[6], du[3], c;
    for (int i = 0; i < 6; ++i) Yr[i] = Y[i];
    orc_rr_terms_r(L, t - Yr[2] / ORC_C, Yr, du, &c);
    for (int i = 0; i < 3; ++i) duRR[i] = (double)du[i];
    *chi = (double)c;
}

static void orc_rhs_rr(const orc_laser* L, int rr, const orc_real Y[7], orc_real dY[7],
                       orc_real* chi)
{
    orc_real du[3];
    orc_rhs_xi(L, Y, dY);
    orc_rr_terms_r(L, Y[6], Y, du, chi);
    if (rr)
        for (int i = 0; i < 3; ++i) dY[3 + i] += du[i];
}

static void orc_push_elec_rr(const orc_laser* L, int rr, orc_real t0, orc_real t_end,
                             orc_real h, const orc_real x0[3], const orc_real u0[3],
                             orc_real xf[3], orc_real uf[3], orc_real* chi_max)
{
    orc_real Y[7] = {x0[0], x0[1], x0[2], u0[0], u0[1], u0[2], t0 - x0[2] / ORC_C};
    orc_real comp[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    orc_real cm = 0.0;
    const int64_t N = (int64_t)ceil((t_end - t0) / h);
    for (int64_t n = 0; n < N; ++n) {
        orc_real ta = t0 + (orc_real)n * h;
        orc_real hn = (n == N - 1) ? t_end - ta : h;
        orc_real k1[7], k2[7], k3[7], k4[7], Yt[7], chi, dummy;
        orc_rhs_rr(L, rr, Y, k1, &chi);
        if (chi > cm) cm = chi;
        for (int i = 0; i < 7; ++i) Yt[i] = Y[i] + 0.5 * hn * k1[i];
        orc_rhs_rr(L, rr, Yt, k2, &dummy);
        for (int i = 0; i < 7; ++i) Yt[i] = Y[i] + 0.5 * hn * k2[i];
        orc_rhs_rr(L, rr, Yt, k3, &dummy);
        for (int i = 0; i < 7; ++i) Yt[i] = Y[i] + hn * k3[i];
        orc_rhs_rr(L, rr, Yt, k4, &dummy);
        for (int i = 0; i < 7; ++i)
            orc_kahan_add(&Y[i], &comp[i], hn / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]));
    }
    for (int i = 0; i < 3; ++i) { xf[i] = Y[i]; uf[i] = Y[3 + i]; }
    *chi_max = cm;
}

void orc_push_one_rr(const orc_laser* L, int rr, double t0, double t_end, double h,
                     const double x0[3], const double u0[3], double xf[3], double uf[3],
                     double* chi_max)
{
    orc_real X0[3] = {x0[0], x0[1], x0[2]}, U0[3] = {u0[0], u0[1], u0[2]}, XF[3], UF[3], cm;
    orc_push_elec_rr(L, rr, t0, t_end, h, X0, U0, XF, UF, &cm);
    for (int i = 0; i < 3; ++i) { xf[i] = (double)XF[i]; uf[i] = (double)UF[i]; }
    *chi_max = (double)cm;
}

void orc_push_rr(const orc_laser* L, int rr, int64_t n_slots, const double* t_birth,
                 const double* x0, const double* y0, const double* z0, int slots_per_atom,
                 double* ux, double* uy, double* uz, double* xf, double* yf, double* zf,
                 double* chi_max)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t s = 0; s < n_slots; ++s) {
        int64_t a = s / slots_per_atom;
        double t0 = t_birth[s];
        orc_real ts, te;
        orc_window(L, z0[a], &ts, &te);
        if (!(t0 < INFINITY) || !(t0 >= ts - L->dt)) {
            ux[s] = uy[s] = uz[s] = xf[s] = yf[s] = zf[s] = chi_max[s] = NAN;
            continue;
        }
        orc_real X0[3] = {x0[a], y0[a], z0[a]}, U0[3] = {0.0, 0.0, 0.0}, XF[3], UF[3], cm;
        orc_push_elec_rr(L, rr, t0, te, L->dt, X0, U0, XF, UF, &cm);
        ux[s] = (double)UF[0]; uy[s] = (double)UF[1]; uz[s] = (double)UF[2];
        xf[s] = (double)XF[0]; yf[s] = (double)XF[1]; zf[s] = (double)XF[2];
        chi_max[s] = (double)cm;
    }
}

/* ---------------------------------------------------------------------------
 * Controlled-step push (Sec. 1 and Sec. 2.1: a fifth-order Runge-Kutta method
 * with a controlled time step, electrons followed until their kinetic energy
 * no longer changes).
 *
 * Readings (the paper names only "fifth order" and "controlled step"):
 *   - the pair is Dormand-Prince 5(4): seven stages, the fifth-order result
 *     carried forward, the last stage reused as the next step's first;
 *   - error of a step: the largest over the six components of
 *     |y5 - y4| / (atol + rtol max(|y_n|, |y_n+1|)), positions measured as
 *     k x and momenta as u = p / m c; the step is accepted when it is <= 1;
 *   - next step: h * min(5, max(0.2, 0.9 err^(-1/5))) (5 when err = 0), at
 *     most h_max and never past the window end; first step dt;
 *   - stop at the window end, or earlier at the first accepted step end at
 *     which gamma differs by at most k_tol (relative) from its value at the
 *     previous check; checks are made at the first step ends at least 0.999
 *     optical period after the previous check (the first one after birth):
 *     "one period" with a margin, so that steps commensurate with the period
 *     (h_max = T/20 by default) do not make each check a rounding tie;
 *   - more than max_steps attempted steps, or a step whose error is not a
 *     number: the electron is reported as NaN.
 * ------------------------------------------------------------------------- */
typedef struct {
    double rtol, atol;   /* error tolerances (dimensionless, as above)      */
    double h_max;        /* largest step [s]                               */
    double k_tol;        /* relative change of gamma regarded as constant  */
    int64_t max_steps;   /* attempted steps allowed per electron           */
} orc_adaptive;

/* Dormand-Prince 5(4) tableau */
static const double DP_C[7] = {0.0, 1.0 / 5.0, 3.0 / 10.0, 4.0 / 5.0, 8.0 / 9.0, 1.0, 1.0};
static const double DP_A[7][6] = {
    {0, 0, 0, 0, 0, 0},
    {1.0 / 5.0, 0, 0, 0, 0, 0},
    {3.0 / 40.0, 9.0 / 40.0, 0, 0, 0, 0},
    {44.0 / 45.0, -56.0 / 15.0, 32.0 / 9.0, 0, 0, 0},
    {19372.0 / 6561.0, -25360.0 / 2187.0, 64448.0 / 6561.0, -212.0 / 729.0, 0, 0},
    {9017.0 / 3168.0, -355.0 / 33.0, 46732.0 / 5247.0, 49.0 / 176.0, -5103.0 / 18656.0, 0},
    {35.0 / 384.0, 0.0, 500.0 / 1113.0, 125.0 / 192.0, -2187.0 / 6784.0, 11.0 / 84.0}};
/* fifth-order weights (= the last row) and the fourth-order ones */
static const double DP_B5[7] = {35.0 / 384.0, 0.0, 500.0 / 1113.0, 125.0 / 192.0,
                                -2187.0 / 6784.0, 11.0 / 84.0, 0.0};
static const double DP_B4[7] = {5179.0 / 57600.0, 0.0, 7571.0 / 16695.0, 393.0 / 640.0,
                                -92097.0 / 339200.0, 187.0 / 2100.0, 1.0 / 40.0};

static orc_real orc_gamma6(const orc_real Y[6])
{
    return sqrt(1.0 + Y[3] * Y[3] + Y[4] * Y[4] + Y[5] * Y[5]);
}

/* returns 0, or 1 when max_steps was exceeded */
int orc_push_one_adaptive(const orc_laser* L, const orc_adaptive* A, double t0, double t_end,
                          const double x0[3], const double u0[3], double xf[3], double uf[3],
                          double* t_stop, int64_t* n_acc, int64_t* n_rej)
{
    const orc_real k = 2.0 * ORC_PI / L->lambda;
    const orc_real T = L->lambda / ORC_C;
    const orc_real scale[6] = {k, k, k, 1.0, 1.0, 1.0};
    orc_real Y[6] = {x0[0], x0[1], x0[2], u0[0], u0[1], u0[2]};
    orc_real K[7][6], Yt[6], Y5[6];
    orc_real t = t0, h = L->dt;
    orc_real g_ref = orc_gamma6(Y), t_ref = t0;
    int64_t acc = 0, rej = 0;
    int status = 0;
    orc_rhs(L, t, Y, K[0]);
    while (t < t_end) {
        if (acc + rej >= A->max_steps) { status = 1; break; }
        orc_real hs = h < A->h_max ? h : A->h_max;
        int last = 0;
        if (hs >= t_end - t) { hs = t_end - t; last = 1; }
        for (int s = 1; s < 7; ++s) {
            for (int i = 0; i < 6; ++i) {
                orc_real acc_i = 0.0;
                for (int j = 0; j < s; ++j) acc_i += DP_A[s][j] * K[j][i];
                Yt[i] = Y[i] + hs * acc_i;
            }
            orc_rhs(L, t + DP_C[s] * hs, Yt, K[s]);
        }
        /* stage 7 was evaluated at the fifth-order result (row 7 = b5) */
        for (int i = 0; i < 6; ++i) Y5[i] = Yt[i];
        orc_real err = 0.0;
        for (int i = 0; i < 6; ++i) {
            orc_real e = 0.0;
            for (int j = 0; j < 7; ++j) e += (DP_B5[j] - DP_B4[j]) * K[j][i];
            e = fabs(hs * e) * scale[i];
            const orc_real ya = fabs(Y[i]) * scale[i], yb = fabs(Y5[i]) * scale[i];
            const orc_real r = e / (A->atol + A->rtol * (ya > yb ? ya : yb));
            if (r > err || r != r) err = r;
        }
        if (err != err) { status = 1; break; }   /* the step produced no number */
        if (err <= 1.0) {
            t = last ? t_end : t + hs;
            for (int i = 0; i < 6; ++i) { Y[i] = Y5[i]; K[0][i] = K[6][i]; }
            ++acc;
            if (last) break;
            if (t - t_ref >= 0.999 * T) {
                const orc_real g = orc_gamma6(Y);
                if (fabs(g - g_ref) <= A->k_tol * g) break;
                g_ref = g;
                t_ref = t;
            }
        } else {
            ++rej;
        }
        orc_real fac = (err == 0.0) ? 5.0 : 0.9 * pow(err, (orc_real)-0.2);
        if (fac > 5.0) fac = 5.0;
        if (fac < 0.2) fac = 0.2;
        h = hs * fac;
    }
    for (int i = 0; i < 3; ++i) { xf[i] = (double)Y[i]; uf[i] = (double)Y[3 + i]; }
    *t_stop = (double)t;
    *n_acc = acc;
    *n_rej = rej;
    if (status) {
        for (int i = 0; i < 3; ++i) xf[i] = uf[i] = NAN;
        *t_stop = NAN;
    }
    return status;
}

void orc_push_adaptive(const orc_laser* L, const orc_adaptive* A, int64_t n_slots,
                       const double* t_birth, const double* x0, const double* y0,
                       const double* z0, int slots_per_atom, double* ux, double* uy, double* uz,
                       double* xf, double* yf, double* zf, double* t_stop, int64_t* n_acc,
                       int64_t* n_rej)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t s = 0; s < n_slots; ++s) {
        int64_t a = s / slots_per_atom;
        double t0 = t_birth[s];
        orc_real ts, te;
        orc_window(L, z0[a], &ts, &te);
        if (!(t0 < INFINITY) || !(t0 >= ts - L->dt)) {
            ux[s] = uy[s] = uz[s] = xf[s] = yf[s] = zf[s] = t_stop[s] = NAN;
            n_acc[s] = n_rej[s] = 0;
            continue;
        }
        double X0[3] = {x0[a], y0[a], z0[a]}, U0[3] = {0.0, 0.0, 0.0}, XF[3], UF[3];
        orc_push_one_adaptive(L, A, t0, (double)te, X0, U0, XF, UF, &t_stop[s], &n_acc[s],
                              &n_rej[s]);
        ux[s] = UF[0]; uy[s] = UF[1]; uz[s] = UF[2];
        xf[s] = XF[0]; yf[s] = XF[1]; zf[s] = XF[2];
    }
}

/* The tableau above, for the tests (c[7], a[7][7] row-major, b5[7], b4[7]). */
void orc_dp_tableau(double* c, double* a, double* b5, double* b4)
{
    for (int i = 0; i < 7; ++i) {
        c[i] = DP_C[i];
        b5[i] = DP_B5[i];
        b4[i] = DP_B4[i];
        for (int j = 0; j < 7; ++j) a[i * 7 + j] = (j < 6) ? DP_A[i][j] : 0.0;
    }
}
