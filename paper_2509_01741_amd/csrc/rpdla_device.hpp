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

namespace rpdla {

constexpr int kMaxStates = 10;

// Per-configuration constants, built on the host (rpdla_api.hip) and passed
// by value to kernels or staged in LDS by the batched kernel.
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
    double tE[3], tB[3];         // normalized uniform test fields
    int32_t field, window;
    // tunnelling rate per normalized time for state k (index k-1):
    //   ln w = c0 - c1h ln|a|^2 - c2 / |a|,   w = 0 where ln w < lnw_zero
    double adk_c0[kMaxStates], adk_c1h[kMaxStates], adk_c2[kMaxStates];
    double adk_a2thr[kMaxStates];  // |a|^2 below which ln w < lnw_zero - 5 (exact skip)
    double lnw_zero;
    double gl_x[4], gl_w[4];       // Gauss-Legendre 4-point nodes / weights on [-1, 1]
    double rr_kappa;               // (2/3) k r_e: Landau-Lifshitz gamma^2 term, normalized
    double chi_eta;                // hbar omega / (m c^2): chi = eta gamma sqrt(Q)
    // controlled-step push: tolerances, largest step (normalized), constant-energy
    // tolerance and attempted-step budget per electron
    double ad_rtol, ad_atol, ad_hmax, ad_ktol;
    int64_t ad_max_steps;
};

// The subset of DevCfg the push needs (staged in LDS by the batched push).
struct PushCfg {
    double omega, k, inv_k, a0, inv_w0n2, inv_w0n, inv_zrn;
    double eps, e2, e3, e4, inv_T0n, phi0, hn, tb_n, ta_n, er_scale, ez_scale;
    double tE[3], tB[3];
    int32_t field, window;
};

__host__ __device__ inline PushCfg push_cfg_of(const DevCfg& c)
{
    PushCfg p;
    p.omega = c.omega; p.k = c.k; p.inv_k = c.inv_k; p.a0 = c.a0; p.inv_w0n2 = c.inv_w0n2;
    p.inv_w0n = c.inv_w0n; p.inv_zrn = c.inv_zrn; p.eps = c.eps; p.e2 = c.e2; p.e3 = c.e3;
    p.e4 = c.e4; p.inv_T0n = c.inv_T0n; p.phi0 = c.phi0; p.hn = c.hn; p.tb_n = c.tb_n; p.ta_n = c.ta_n;
    p.er_scale = c.er_scale; p.ez_scale = c.ez_scale;
    for (int i = 0; i < 3; ++i) { p.tE[i] = c.tE[i]; p.tB[i] = c.tB[i]; }
    p.field = c.field; p.window = c.window;
    return p;
}

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
// (C_n = Re Q_n, S_n = Im Q_n) come from repeated complex multiplication by q
// -- one sine/cosine and one exponential per evaluation, the Gouy phase
// carried by q.  Then
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

// Transverse / longitudinal factors shared by the double and mixed paths.
// Inputs: Q[n] for n = 2..8 (only the orders needed are read), r2 = rho^2.
template <int ORDER, typename T>
__device__ inline void rp_combine(const Cx<T>* Q, T r2, T eps, T e2, T e3, T e4,
                                  T& PE, T& PB, T& EZ)
{
    const T C2 = Q[2].re, S2 = Q[2].im, C3 = Q[3].re, S3 = Q[3].im;
    PE = C2;
    PB = C2;
    EZ = eps * (S2 - r2 * S3);
    if constexpr (ORDER >= 3) {
        const T C4 = Q[4].re, S4 = Q[4].im, C5 = Q[5].re, S5 = Q[5].im, S6 = Q[6].im;
        const T r4 = r2 * r2, r6 = r4 * r2;
        const T h = T(0.5), q = T(0.25);
        PE += e2 * (-h * C3 + r2 * C4 - q * r4 * C5);
        PB += e2 * (h * C3 + h * r2 * C4 - q * r4 * C5);
        EZ += e3 * (h * S3 + h * r2 * S4 - T(1.25) * r4 * S5 + q * r6 * S6);
        if constexpr (ORDER >= 5) {
            const T C6 = Q[6].re, C7 = Q[7].re, C8 = Q[8].re;
            const T r8 = r4 * r4;
            const T c38 = T(0.375), c132 = T(0.03125);
            PE += e4 * (-c38 * C4 - c38 * r2 * C5 + T(1.0625) * r4 * C6 - c38 * r6 * C7
                        + c132 * r8 * C8);
            PB += e4 * (c38 * C4 + c38 * r2 * C5 + T(0.1875) * r4 * C6 - q * r6 * C7
                        + c132 * r8 * C8);
        }
    }
}

// Complex amplitudes Q_2..Q_NMAX from the carrier (cs, sn), amplitude g, and q.
template <int ORDER, typename T>
__device__ inline void rp_amplitudes(T g, T cs, T sn, Cx<T> q, Cx<T>* Q)
{
    const Cx<T> q2 = cmul(q, q);
    Q[2] = cmul(Cx<T>{g * cs, g * sn}, q2);
    Q[3] = cmul(Q[2], q);
    if constexpr (ORDER >= 3) {
        Q[4] = cmul(Q[3], q);
        Q[5] = cmul(Q[4], q);
        Q[6] = cmul(Q[5], q);
        if constexpr (ORDER >= 5) {
            Q[7] = cmul(Q[6], q);
            Q[8] = cmul(Q[7], q);
        }
    }
}

// Double-precision field at normalized (X, Y, Z, tau).  WANT_B = false skips
// the magnetic field (ionization needs |E| only).
template <int ORDER, bool WANT_B, class CFG>
__device__ inline void rp_field_f64(const CFG& c, double X, double Y, double Z, double tau,
                                    double& ax, double& ay, double& az, double& bx, double& by)
{
    const double r2 = (X * X + Y * Y) * c.inv_w0n2;
    const double zeta = Z * c.inv_zrn;
    const double iD = fm::rcp_f64(1.0 + zeta * zeta);
    const double rD = r2 * iD;
    const double d = tau - Z;
    const double Psi = c.phi0 + d - rD * zeta;
    const double s = d * c.inv_T0n;
    const double g = c.a0 * fm::exp_f64(-rD - s * s);
    double sn, cs;
    fm::sincos_f64(Psi, &sn, &cs);
    Cx<double> Q[9];
    rp_amplitudes<ORDER, double>(g, cs, sn, Cx<double>{iD, zeta * iD}, Q);
    double PE, PB, EZ;
    rp_combine<ORDER, double>(Q, r2, c.eps, c.e2, c.e3, c.e4, PE, PB, EZ);
    const double pe = c.er_scale * PE * c.inv_w0n;
    ax = pe * X;
    ay = pe * Y;
    az = c.ez_scale * EZ;
    if constexpr (WANT_B) {
        const double pb = PB * c.inv_w0n;
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

// Field of any model in double precision (test models included).
template <int FIELD, bool WANT_B, class CFG>
__device__ inline void field_f64(const CFG& c, double X, double Y, double Z, double tau,
                                 double& ax, double& ay, double& az, double& bx, double& by,
                                 double& bz)
{
    if constexpr (FIELD == 11) {  // uniform static E, B
        ax = c.tE[0]; ay = c.tE[1]; az = c.tE[2];
        bx = c.tB[0]; by = c.tB[1]; bz = c.tB[2];
    } else if constexpr (FIELD == 10) {  // plane wave, x polarized
        const double d = tau - Z;
        const double s = d * c.inv_T0n;
        double sn, cs;
        fm::sincos_f64(d + c.phi0, &sn, &cs);
        const double e = c.a0 * fm::exp_f64(-s * s) * cs;
        ax = e; ay = 0.0; az = 0.0;
        bx = 0.0; by = e; bz = 0.0;
    } else {
        rp_field_f64<FIELD, WANT_B, CFG>(c, X, Y, Z, tau, ax, ay, az, bx, by);
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
    else
        return rp_bound2<FIELD, CFG>(c, X, Y, Z);
}

// ---------------------------------------------------------------------------
// Static ADK tunnelling rate (the paper cites the semi-classical tunnelling
// model without printing a formula): l = m = 0, l* = n* - 1, in log space,
// per unit normalized time.  w = 0 when |a| = 0 or ln w < lnw_zero.
// ---------------------------------------------------------------------------
// Rate constants of one charge state, picked out of the configuration record
// with static indices (no dynamic indexing into the record).
struct AdkState {
    double c0, c1h, c2, a2thr, lnw_zero;
};

template <class CFG>
__device__ inline AdkState adk_state(const CFG& c, int s)
{
    AdkState a{c.adk_c0[0], c.adk_c1h[0], c.adk_c2[0], c.adk_a2thr[0], c.lnw_zero};
#pragma unroll
    for (int i = 1; i < kMaxStates; ++i) {
        if (s == i) {
            a.c0 = c.adk_c0[i]; a.c1h = c.adk_c1h[i]; a.c2 = c.adk_c2[i]; a.a2thr = c.adk_a2thr[i];
        }
    }
    return a;
}

__device__ inline double adk_rate_n(const AdkState& st, double a2)
{
    if (!(a2 > 0.0)) return 0.0;
    const double l = st.c0 - st.c1h * log(a2) - st.c2 * rsqrt(a2);
    if (l < st.lnw_zero) return 0.0;
    return fm::exp_f64(l);
}

}  // namespace rpdla
