// rpdla_device.hpp -- device-side building blocks for gfx950: per-configuration
// constants in normalized units, the counter-based generator, the radially
// polarized focus and the tunnelling rate.
//
// Normalized units (one set per laser configuration): time tau = omega t,
// length X = k x, momentum u = p/(m c), fields a = e E/(m c omega) and
// b = e B/(m omega).  In them the Newton-Lorentz equations (Eqs. (7)-(14) of
// the paper) read dX/dtau = u/gamma, du/dtau = -(a + (u/gamma) x b).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rpdla_fastmath.hpp"
#include "rpdla_lp_coeffs.hpp"

namespace rpdla {

constexpr int kMaxStates = 10;

// Per-configuration constants, built on the host (rpdla_api.hip) and passed
// by value to kernels, staged in LDS by the batched ionization kernel and read
// with scalar loads by the batched push.
struct DevCfg {
    double omega, inv_omega;     // carrier angular frequency [rad/s]
    double k, inv_k;             // wavenumber [1/m]
    double a0;                   // normalized amplitude e A/(m c omega)
    double inv_w0n2;             // 1/(k w0)^2
    double inv_w0n;              // 1/(k w0)
    double inv_zrn;              // 1/(k z_r)
    double eps, e2, e3, e4;      // eps = w0/z_r and its powers
    double inv_T0n;              // 1/(omega tau0)
    double phi0;                 // carrier phase
    double hn;                   // omega dt
    double tb_n, ta_n;           // omega t_before, omega t_after
    double er_scale, ez_scale;
    double er_w, ez_e;           // er_scale/(k w0) and ez_scale eps (folded products)
    double a0_w, ez_2;           // a0/(k w0) and 2 ez_scale: the FP64 radial field
                                 // carries 1/(k w0) in its amplitude (ez_scale eps k w0 = 2 ez_scale)
    double tE[3], tB[3];         // normalized uniform test fields
    int32_t field, window;
    // tunnelling rate per normalized time for state k (index k-1):
    //   ln w = c0 - c1h ln|a|^2 - c2 / |a|,   w = 0 where ln w < lnw_zero
    double adk_c0[kMaxStates], adk_c1h[kMaxStates], adk_c2[kMaxStates];
    double adk_a2thr[kMaxStates];  // |a|^2 below which ln w < -80 (panels skipped there)
    double lnw_zero;
    double gl_x[4], gl_w[4];       // Gauss-Legendre 4-point nodes / weights on [-1, 1]
    double rr_kappa;               // (2/3) k r_e: Landau-Lifshitz gamma^2 term, normalized
    double chi_eta;                // hbar omega / (m c^2): chi = eta gamma sqrt(Q)
    // controlled-step push: tolerances, largest step (normalized), constant-energy
    // tolerance and attempted-step budget per electron
    double ad_rtol, ad_atol, ad_hmax, ad_ktol;
    int64_t ad_max_steps;
};

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 64x64->128 multiplies, key bumped by the Weyl constants between rounds.
// ---------------------------------------------------------------------------
struct U64x4 { uint64_t v[4]; };

__device__ inline U64x4 philox4x64(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                   uint64_t k0, uint64_t k1)
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
        const uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
        const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += W0; k1 += W1;
    }
    U64x4 o; o.v[0] = c0; o.v[1] = c1; o.v[2] = c2; o.v[3] = c3;
    return o;
}

// (m + 1) 2^-53 with m the top 53 bits: uniform on (0, 1].
__device__ inline double u01(uint64_t w) { return (double)((w >> 11) + 1ull) * 0x1.0p-53; }

// Variate j of atom `atom`: counter (atom, j/4, 0, 0), key (seed, cfg), word j%4.
__device__ inline double uniform_j(uint64_t seed, uint32_t cfg, uint64_t atom, int j)
{
    const U64x4 r = philox4x64(atom, (uint64_t)(j >> 2), 0, 0, seed, (uint64_t)cfg);
    const int w = j & 3;  // word select without a dynamically indexed array
    const uint64_t v = (w == 0) ? r.v[0] : (w == 1) ? r.v[1] : (w == 2) ? r.v[2] : r.v[3];
    return u01(v);
}

// ---------------------------------------------------------------------------
// Radially polarized TM01 focus, series in eps = w0/z_r (Sec. 2.1, Eqs. (1)-(2),
// B_theta from Maxwell's equations, non-paraxial corrections).  With
// rho = r/w0, zeta = z/z_r, D = 1 + zeta^2, q = (1 + i zeta)/D,
// Psi = phi0 + tau - Z - rho^2 zeta/D and g = a0 exp(-rho^2/D - s^2),
// s = (tau - Z)/(omega tau0), the complex amplitudes Q_n = g e^{i Psi} q^n
// (C_n = Re Q_n, S_n = Im Q_n) carry the Gouy phase in the powers of q, so an
// evaluation needs one sine/cosine and one exponential (below the powers are
// formed by repeated multiplication by w = D q).  Then
//   Er/r  = [C2 + e2(-C3/2 + rho^2 C4 - rho^4 C5/4)
//            + e4(-3C4/8 - 3rho^2 C5/8 + 17rho^4 C6/16 - 3rho^6 C7/8 + rho^8 C8/32)] / w0
//   Ez    = eps(S2 - rho^2 S3) + e3(S3/2 + rho^2 S4/2 - 5rho^4 S5/4 + rho^6 S6/4)
//   cBt/r = [C2 + e2(C3/2 + rho^2 C4/2 - rho^4 C5/4)
//            + e4(3C4/8 + 3rho^2 C5/8 + 3rho^4 C6/16 - rho^6 C7/4 + rho^8 C8/32)] / w0
// Order 1 keeps the first term of each bracket, order 3 adds the eps^2 terms
// of Er, Bt and the eps^3 term of Ez, order 5 keeps all.  Ex = Er x/r,
// Ey = Er y/r, Bx = -Bt y/r, By = Bt x/r, Bz = 0.
// ---------------------------------------------------------------------------
template <typename T>
struct Cx { T re, im; };

template <typename T>
__device__ inline Cx<T> cmul(Cx<T> a, Cx<T> b)
{
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}

// The same series arranged for fewer operations (double and float).  With
// w = 1 + i zeta (so q = iD w), write Q_n = iD^(n-2) R_n, R_n = G w^n,
// G = g iD^2 e^{i Psi}: one multiplication by w is two fused multiply-adds.
// The powers of iD then pair with those of rho^2 into rD = rho^2 iD and with
// e2 into E = e2 iD, so each bracket is a polynomial in rD (Horner) and
//   PE = Re{R2 + E (-R3/2 + rD R4 - rD^2 R5/4)
//          + E^2 (-3R4/8 - 3rD R5/8 + 17rD^2 R6/16 - 3rD^3 R7/8 + rD^4 R8/32)}
//   PB = Re{R2 + E (R3/2 + rD R4/2 - rD^2 R5/4)
//          + E^2 (3R4/8 + 3rD R5/8 + 3rD^2 R6/16 - rD^3 R7/4 + rD^4 R8/32)}
//   EZ = eps Im{R2 - rD R3 + E (R3/2 + rD R4/2 - 5rD^2 R5/4 + rD^3 R6/4)}
// (E^2 = e4 iD^2 and eps E = e3 iD: the terms of the series above, term by
// term).
template <int ORDER, typename T>
__device__ inline void rp_brackets(T G_re, T G_im, T zeta, T rD, T E, T& PE, T& PB, T& EZe)
{
    constexpr int NMAX = ORDER >= 5 ? 8 : ORDER >= 3 ? 6 : 3;
    T Rr[NMAX + 1], Ri[NMAX + 1];
    Rr[0] = G_re;
    Ri[0] = G_im;
#pragma unroll
    for (int n = 1; n <= NMAX; ++n) {
        Rr[n] = fma(-zeta, Ri[n - 1], Rr[n - 1]);
        Ri[n] = fma(zeta, Rr[n - 1], Ri[n - 1]);
    }
    PE = Rr[2];
    PB = Rr[2];
    EZe = fma(-rD, Ri[3], Ri[2]);
    if constexpr (ORDER >= 3) {
        // first-order brackets in v = rD/2 (fewer constant factors):
        //   pe2 = 2 R4 v - R5 v^2 - R3/2,  pb2 = R4 v - R5 v^2 + R3/2,
        //   ez3 = 2 I6 v^3 - 5 I5 v^2 + I4 v + I3/2
        const T v = T(0.5) * rD;
        const T h3 = T(0.5) * Rr[3];
        const T a = fma(-Rr[5], v, Rr[4]);
        const T pb2 = fma(a, v, h3);
        const T pe2 = fma(a + Rr[4], v, -h3);
        const T ez3 = fma(fma(fma(Ri[6] + Ri[6], v, T(-5.0) * Ri[5]), v, Ri[4]), v,
                          T(0.5) * Ri[3]);
        EZe = fma(E, ez3, EZe);
        if constexpr (ORDER >= 5) {
            const T t8 = T(0.03125) * Rr[8], t5 = T(0.375) * Rr[5], t4 = T(0.375) * Rr[4];
            const T pe4 = fma(fma(fma(fma(t8, rD, T(-0.375) * Rr[7]), rD, T(1.0625) * Rr[6]), rD, -t5),
                              rD, -t4);
            const T pb4 = fma(fma(fma(fma(t8, rD, T(-0.25) * Rr[7]), rD, T(0.1875) * Rr[6]), rD, t5),
                              rD, t4);
            PE = fma(E, fma(E, pe4, pe2), PE);
            PB = fma(E, fma(E, pb4, pb2), PB);
        } else {
            PE = fma(E, pe2, PE);
            PB = fma(E, pb2, PB);
        }
    }
}

// Double-precision radial field at normalized position (X, Y, Z) and retarded
// time d = tau - Z (every field model depends on time only through d), in
// the parts the force needs: a = (pe X, pe Y, az), b = (-pb Y, pb X, 0).
// With LO the retarded time is the unevaluated sum d + dl (dl small): the
// carrier phase goes to the sine/cosine as the pair (d, phi0 + dl - rD zeta),
// so it is not rounded to a multiple of ulp(d).
template <int ORDER, bool LO, class CFG>
__device__ inline void rp_field_parts_f64(const CFG& c, double X, double Y, double Z, double d,
                                          double dl, double& pe, double& pb, double& az)
{
    const double r2 = (X * X + Y * Y) * c.inv_w0n2;
    const double zeta = Z * c.inv_zrn;
    const double iD = fm::rcp_f64(1.0 + zeta * zeta);
    const double rD = r2 * iD;
    const double psi_lo = fma(-rD, zeta, LO ? c.phi0 + dl : c.phi0);
    const double s = (LO ? d + dl : d) * c.inv_T0n;
    const double g = c.a0_w * fm::exp_fin_f64(-rD - s * s);
    // g e^{i Psi} / D from the half-angle form: the sign (-1)^n goes on the
    // amplitude, cos Psi = 1 - sigma^2 and sin Psi = sigma kappa
    double sg, kp;
    const unsigned sgn = fm::cis_half2_f64(d, psi_lo, &sg, &kp);
    const double gi = fm::flip_sign(g * (iD * iD), sgn);
    const double gs = gi * sg;
    double PE, PB, EZe;
    rp_brackets<ORDER, double>(fma(-gs, sg, gi), gs * kp, zeta, rD, c.e2 * iD, PE, PB, EZe);
    pe = c.er_scale * PE;
    pb = PB;
    az = c.ez_2 * EZe;
}

// The radial field in Cartesian components.  WANT_B = false skips the
// magnetic field (ionization needs |E| only).
template <int ORDER, bool WANT_B, bool LO, class CFG>
__device__ inline void rp_field_f64(const CFG& c, double X, double Y, double Z, double d, double dl,
                                    double& ax, double& ay, double& az, double& bx, double& by)
{
    double pe, pb;
    rp_field_parts_f64<ORDER, LO>(c, X, Y, Z, d, dl, pe, pb, az);
    ax = pe * X;
    ay = pe * Y;
    if constexpr (WANT_B) {
        bx = -pb * Y;
        by = pb * X;
    }
}

// Spatial bound M with |a(X, tau)|^2 <= M^2 exp(-2 s^2): every C_n, S_n is
// bounded by a0 exp(-rho^2/D) D^(-n/2); sum the coefficient magnitudes.
template <int ORDER, class CFG>
__device__ inline double rp_bound2(const CFG& c, double X, double Y, double Z)
{
    const double r2 = (X * X + Y * Y) * c.inv_w0n2;
    const double zeta = Z * c.inv_zrn;
    const double iD = 1.0 / (1.0 + zeta * zeta);
    const double m = sqrt(iD);              // |q|
    const double base = c.a0 * exp(-r2 * iD);
    double p[9];
    p[2] = base * iD;
    for (int n = 3; n <= 8; ++n) p[n] = p[n - 1] * m;
    const double r4 = r2 * r2, r6 = r4 * r2, r8 = r4 * r4;
    double PE = p[2], EZ = c.eps * (p[2] + r2 * p[3]);
    if (ORDER >= 3) {
        PE += c.e2 * (0.5 * p[3] + r2 * p[4] + 0.25 * r4 * p[5]);
        EZ += c.e3 * (0.5 * p[3] + 0.5 * r2 * p[4] + 1.25 * r4 * p[5] + 0.25 * r6 * p[6]);
    }
    if (ORDER >= 5)
        PE += c.e4 * (0.375 * p[4] + 0.375 * r2 * p[5] + 1.0625 * r4 * p[6] + 0.375 * r6 * p[7]
                      + 0.03125 * r8 * p[8]);
    const double et = fabs(c.er_scale) * PE, ez = fabs(c.ez_scale) * EZ;
    return et * et * r2 + ez * ez;
}

// ---------------------------------------------------------------------------
// Linearly polarized focus (Sec. 2.2 compares the radial focus with a linearly
// polarized one, Fig. 4): the same Lax series with the vector potential along
// x (the derivation and the term tables are in gen_lp_coeffs.py).  With
// rx = x/w0, ry = y/w0, s = rx^2 + ry^2 and Q_n = g e^{i Psi} q^n as for the
// radial focus:
//   a_x = Re[sum_n (AX0_n + rx^2 AXR_n) Q_n],  a_y = rx ry Re[sum_n AXR_n Q_n],
//   a_z = rx Re[sum_n AZ_n Q_n],  b_x = 0,  b_y = Re[sum_n BY_n Q_n],
//   b_z = eps ry Im[sum_n S_n Q_n],
// each coefficient a polynomial in s and eps.  The sums are Horner in q.
// ---------------------------------------------------------------------------
template <int N>
__device__ inline Cx<double> lp_coef(const lp::Term (&T)[N], int n, const double* sp,
                                     const double* ep)
{
    double cr = 0.0, ci = 0.0;
#pragma unroll
    for (int t = 0; t < N; ++t) {
        if (T[t].n == n) {
            const double w = ep[T[t].j] * sp[T[t].m];
            if (T[t].re != 0.0) cr += T[t].re * w;
            if (T[t].im != 0.0) ci += T[t].im * w;
        }
    }
    return {cr, ci};
}

// sum_n c_n q^n over n = NMIN..NMAX (Horner, then the factor q^NMIN).
template <int N, int NMIN, int NMAX>
__device__ inline Cx<double> lp_sum(const lp::Term (&T)[N], const double* sp, const double* ep,
                                    Cx<double> q)
{
    Cx<double> u = lp_coef(T, NMAX, sp, ep);
#pragma unroll
    for (int n = NMAX - 1; n >= NMIN; --n) {
        const Cx<double> c = lp_coef(T, n, sp, ep);
        u = cmul(u, q);
        u.re += c.re;
        u.im += c.im;
    }
#pragma unroll
    for (int n = 0; n < NMIN; ++n) u = cmul(u, q);
    return u;
}

// Upper bound of |sum_n c_n Q_n| / (g): sum of the coefficient magnitudes
// times |q|^n.
template <int N>
__device__ inline double lp_bound_sum(const lp::Term (&T)[N], const double* sp, const double* ep,
                                      double qabs)
{
    double b = 0.0;
#pragma unroll
    for (int t = 0; t < N; ++t) {
        double qn = 1.0;
        for (int i = 0; i < T[t].n; ++i) qn *= qabs;
        b += (fabs(T[t].re) + fabs(T[t].im)) * ep[T[t].j] * sp[T[t].m] * qn;
    }
    return b;
}

#define RPDLA_LP_SUM(ORD, NAME, sp, ep, q)                                                   \
    lp_sum<lp::k##NAME##_O##ORD##_N, lp::k##NAME##_O##ORD##_NMIN,                            \
           lp::k##NAME##_O##ORD##_NMAX>(lp::k##NAME##_O##ORD, sp, ep, q)

template <int ORDER>
__device__ inline void lp_sums(const double* sp, const double* ep, Cx<double> q, Cx<double>& ux0,
                               Cx<double>& uxr, Cx<double>& uz, Cx<double>& uby, Cx<double>& us)
{
    if constexpr (ORDER == 1) {
        ux0 = RPDLA_LP_SUM(1, AX0, sp, ep, q); uxr = RPDLA_LP_SUM(1, AXR, sp, ep, q);
        uz = RPDLA_LP_SUM(1, AZ, sp, ep, q); uby = RPDLA_LP_SUM(1, BY, sp, ep, q);
        us = RPDLA_LP_SUM(1, S, sp, ep, q);
    } else if constexpr (ORDER == 3) {
        ux0 = RPDLA_LP_SUM(3, AX0, sp, ep, q); uxr = RPDLA_LP_SUM(3, AXR, sp, ep, q);
        uz = RPDLA_LP_SUM(3, AZ, sp, ep, q); uby = RPDLA_LP_SUM(3, BY, sp, ep, q);
        us = RPDLA_LP_SUM(3, S, sp, ep, q);
    } else {
        ux0 = RPDLA_LP_SUM(5, AX0, sp, ep, q); uxr = RPDLA_LP_SUM(5, AXR, sp, ep, q);
        uz = RPDLA_LP_SUM(5, AZ, sp, ep, q); uby = RPDLA_LP_SUM(5, BY, sp, ep, q);
        us = RPDLA_LP_SUM(5, S, sp, ep, q);
    }
}

template <class CFG>
__device__ inline void lp_powers(const CFG& c, double s, double* sp, double* ep)
{
    sp[0] = 1.0; sp[1] = s; sp[2] = s * s; sp[3] = sp[2] * s; sp[4] = sp[2] * sp[2];
    sp[5] = sp[4] * s;
    ep[0] = 1.0; ep[1] = c.eps; ep[2] = c.e2; ep[3] = c.e3; ep[4] = c.e4; ep[5] = c.e4 * c.eps;
    ep[6] = c.e3 * c.e3; ep[7] = ep[6] * c.eps;
}

template <int ORDER, bool WANT_B, class CFG>
__device__ inline void lp_field_f64(const CFG& c, double X, double Y, double Z, double d,
                                    double& ax, double& ay, double& az, double& bx, double& by,
                                    double& bz)
{
    const double rx = X * c.inv_w0n, ry = Y * c.inv_w0n;
    const double s = rx * rx + ry * ry;
    const double zeta = Z * c.inv_zrn;
    const double iD = fm::rcp_f64(1.0 + zeta * zeta);
    const double Psi = c.phi0 + d - s * zeta * iD;
    const double sg = d * c.inv_T0n;
    const double g = c.a0 * fm::exp_fin_f64(-s * iD - sg * sg);
    double sn, cs;
    fm::sincos_f64(Psi, &sn, &cs);
    const Cx<double> base{g * cs, g * sn};
    double sp[6], ep[8];
    lp_powers(c, s, sp, ep);
    Cx<double> ux0, uxr, uz, uby, us;
    lp_sums<ORDER>(sp, ep, Cx<double>{iD, zeta * iD}, ux0, uxr, uz, uby, us);
    const Cx<double> wx0 = cmul(base, ux0), wxr = cmul(base, uxr), wz = cmul(base, uz);
    ax = c.er_scale * (wx0.re + rx * rx * wxr.re);
    ay = c.er_scale * rx * ry * wxr.re;
    az = c.ez_scale * rx * wz.re;
    bx = 0.0;
    if constexpr (WANT_B) {
        by = cmul(base, uby).re;
        bz = c.eps * ry * cmul(base, us).im;
    } else {
        by = 0.0;
        bz = 0.0;
    }
}

// Spatial bound M with |a(X, tau)|^2 <= M^2 exp(-2 s^2) for the linear focus.
template <int ORDER, class CFG>
__device__ inline double lp_bound2(const CFG& c, double X, double Y, double Z)
{
    const double rx = fabs(X * c.inv_w0n), ry = fabs(Y * c.inv_w0n);
    const double s = rx * rx + ry * ry;
    const double zeta = Z * c.inv_zrn;
    const double iD = 1.0 / (1.0 + zeta * zeta);
    const double qabs = sqrt(iD);
    const double gs = c.a0 * exp(-s * iD);
    double sp[6], ep[8];
    lp_powers(c, s, sp, ep);
    double bx0, bxr, bz;
    if constexpr (ORDER == 1) {
        bx0 = lp_bound_sum(lp::kAX0_O1, sp, ep, qabs); bxr = lp_bound_sum(lp::kAXR_O1, sp, ep, qabs);
        bz = lp_bound_sum(lp::kAZ_O1, sp, ep, qabs);
    } else if constexpr (ORDER == 3) {
        bx0 = lp_bound_sum(lp::kAX0_O3, sp, ep, qabs); bxr = lp_bound_sum(lp::kAXR_O3, sp, ep, qabs);
        bz = lp_bound_sum(lp::kAZ_O3, sp, ep, qabs);
    } else {
        bx0 = lp_bound_sum(lp::kAX0_O5, sp, ep, qabs); bxr = lp_bound_sum(lp::kAXR_O5, sp, ep, qabs);
        bz = lp_bound_sum(lp::kAZ_O5, sp, ep, qabs);
    }
    const double ex = fabs(c.er_scale) * gs * (bx0 + rx * rx * bxr);
    const double ey = fabs(c.er_scale) * gs * rx * ry * bxr;
    const double ez = fabs(c.ez_scale) * gs * rx * bz;
    return ex * ex + ey * ey + ez * ez;
}

// Field of any model in double precision (test models included) at position
// (X, Y, Z) and retarded time d = tau - Z; with LO the retarded time is the
// unevaluated sum d + dl (the radial focus keeps the pair, the others add it).
template <int FIELD, bool WANT_B, class CFG, bool LO = false>
__device__ inline void field_f64(const CFG& c, double X, double Y, double Z, double d,
                                 double& ax, double& ay, double& az, double& bx, double& by,
                                 double& bz, double dl = 0.0)
{
    if constexpr (LO && !(FIELD == 1 || FIELD == 3 || FIELD == 5)) {
        d += dl;
    }
    if constexpr (FIELD == 11) {  // uniform static E, B
        ax = c.tE[0]; ay = c.tE[1]; az = c.tE[2];
        bx = c.tB[0]; by = c.tB[1]; bz = c.tB[2];
    } else if constexpr (FIELD == 10) {  // plane wave, x polarized
        const double s = d * c.inv_T0n;
        double sn, cs;
        fm::sincos_f64(d + c.phi0, &sn, &cs);
        const double e = c.a0 * fm::exp_fin_f64(-s * s) * cs;
        ax = e; ay = 0.0; az = 0.0;
        bx = 0.0; by = e; bz = 0.0;
    } else if constexpr (FIELD == 21 || FIELD == 23 || FIELD == 25) {
        lp_field_f64<FIELD - 20, WANT_B, CFG>(c, X, Y, Z, d, ax, ay, az, bx, by, bz);
    } else {
        rp_field_f64<FIELD, WANT_B, LO, CFG>(c, X, Y, Z, d, dl, ax, ay, az, bx, by);
        bz = 0.0;
    }
}

template <int FIELD, class CFG>
__device__ inline double bound2_f64(const CFG& c, double X, double Y, double Z)
{
    if constexpr (FIELD == 11)
        return c.tE[0] * c.tE[0] + c.tE[1] * c.tE[1] + c.tE[2] * c.tE[2];
    else if constexpr (FIELD == 10)
        return c.a0 * c.a0;
    else if constexpr (FIELD == 21 || FIELD == 23 || FIELD == 25)
        return lp_bound2<FIELD - 20, CFG>(c, X, Y, Z);
    else
        return rp_bound2<FIELD, CFG>(c, X, Y, Z);
}

// ---------------------------------------------------------------------------
// Static ADK tunnelling rate (the paper cites the semi-classical tunnelling
// model without printing a formula): l = m = 0, l* = n* - 1, in log space,
// per unit normalized time.  w = 0 when |a| = 0 or ln w < lnw_zero.
// ---------------------------------------------------------------------------
// Rate constants of one charge state, read from the configuration record at
// the state's index (from the kernel-argument segment in the single-
// configuration kernels, from LDS in the batched ones; picking them with
// static indices held all forty in scalar registers, which spilled).
struct AdkState {
    double c0, c1h, c2, a2thr, lnw_zero;
};

template <class CFG>
__device__ inline AdkState adk_state(const CFG& c, int s)
{
    return AdkState{c.adk_c0[s], c.adk_c1h[s], c.adk_c2[s], c.adk_a2thr[s], c.lnw_zero};
}

__device__ inline double adk_rate_n(const AdkState& st, double a2)
{
    // below 2^-960 the c2/|a| term alone puts ln w under any lnw_zero (c2 > 1e-30
    // for every state), so the rate is zero there either way
    if (!(a2 >= 0x1.0p-960)) return 0.0;
    const double l = st.c0 - st.c1h * fm::log_pos_f64(a2) - st.c2 * fm::rsqrt_mid_f64(a2);
    if (l < st.lnw_zero) return 0.0;
    return fm::exp_fin_f64(l);   // l >= lnw_zero > -745: no range guard needed
}

}  // namespace rpdla
