// rpdla_kernels.hpp -- HIP kernels for gfx950 (wave64): atom sampling,
// ionization times, the Newton-Lorentz push (double and mixed precision) and
// the energy-angle histogram.
#pragma once

#include "rpdla_device.hpp"

namespace rpdla {

constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr double kInvTwoPi = 0.15915494309189533576888376337251;

// ---------------------------------------------------------------------------
// Atom sampling: one lane per atom, structure-of-arrays output.
// r = R sqrt(u0), azimuth 2 pi u1, z = zh (2 u2 - 1)  (Sec. 2.1).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) sample_atoms_kernel(
    uint64_t seed, uint32_t cfg, uint64_t first_atom, int64_t n, double r_max, double z_half,
    double* __restrict__ x, double* __restrict__ y, double* __restrict__ z)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const U64x4 r = philox4x64(first_atom + (uint64_t)i, 0, 0, 0, seed, (uint64_t)cfg);
    const double rad = r_max * sqrt(u01(r.v[0]));
    double sn, cs;
    sincos(kTwoPi * u01(r.v[1]), &sn, &cs);
    x[i] = rad * cs;
    y[i] = rad * sn;
    z[i] = z_half * (2.0 * u01(r.v[2]) - 1.0);
}

// Annulus: r uniform in area between r_in and r_out (r = r_out exactly when
// r_in == r_out, a hollow-cylinder surface), azimuth and z as above.
__global__ void __launch_bounds__(256) sample_annulus_kernel(
    uint64_t seed, uint32_t cfg, uint64_t first_atom, int64_t n, double r_in, double r_out,
    double z_half, double* __restrict__ x, double* __restrict__ y, double* __restrict__ z)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const U64x4 r = philox4x64(first_atom + (uint64_t)i, 0, 0, 0, seed, (uint64_t)cfg);
    const double rad = (r_in == r_out) ? r_out
                                        : sqrt(r_in * r_in + u01(r.v[0]) * (r_out * r_out - r_in * r_in));
    double sn, cs;
    sincos(kTwoPi * u01(r.v[1]), &sn, &cs);
    x[i] = rad * cs;
    y[i] = rad * sn;
    z[i] = z_half * (2.0 * u01(r.v[2]) - 1.0);
}

// Laser phase at each birth, the phase defined under Eq. (2) of the paper
// (k z - omega t - 2 atan(z/z_r) + z r^2/(z_r w0^2 f^2), with the paper's
// carrier phase equal to minus this library's), in [0, 2 pi), and the radius
// of the parent ion (optional); NaN for unborn slots.
__global__ void __launch_bounds__(256) birth_phase_kernel(
    DevCfg c, int64_t n, const double* __restrict__ tb, const double* __restrict__ x,
    const double* __restrict__ y, const double* __restrict__ z, int spa,
    double* __restrict__ phase, double* __restrict__ r_birth)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const double t = tb[s];
    const int64_t a = s / spa;
    const bool born = t < __builtin_inf();
    if (r_birth) r_birth[s] = born ? sqrt(x[a] * x[a] + y[a] * y[a]) : __builtin_nan("");
    if (!born) { phase[s] = __builtin_nan(""); return; }
    const double X = x[a] * c.k, Y = y[a] * c.k, Z = z[a] * c.k;
    const double rho2 = (X * X + Y * Y) * c.inv_w0n2;
    const double zeta = Z * c.inv_zrn;
    double ph = Z - t * c.omega - 2.0 * atan(zeta) + zeta * rho2 / (1.0 + zeta * zeta) - c.phi0;
    ph = fmod(ph, kTwoPi);
    if (ph < 0.0) ph += kTwoPi;
    if (ph >= kTwoPi) ph -= kTwoPi;
    phase[s] = ph;
}

// ---------------------------------------------------------------------------
// Ionization.  One lane per atom.  Time axis in panels of width h from the
// window start; state s (charge state k_first + s) accumulates GL-4 panel
// integrals of its rate from the previous birth; at the panel where the sum
// reaches the Exp(1) threshold the crossing is solved by bracketed Newton.
// Panels where a rigorous bound keeps the rate negligible at every node are
// skipped: before each state's possible window and after it.
// ---------------------------------------------------------------------------
template <int FIELD, class CFG>
__device__ inline double emag2_f64(const CFG& c, double X, double Y, double Z, double d)
{
    double ax, ay, az, bx, by, bz;
    field_f64<FIELD, false, CFG>(c, X, Y, Z, d, ax, ay, az, bx, by, bz);
    return ax * ax + ay * ay + az * az;
}

// The field of an atom at rest reduced to its time dependence.  For the RP
// models every term of the series is g e^{i Psi} q^n times a polynomial in
// rho^2, so  Er/r ~ g Re(e^{i Psi} A_E),  Ez = g Im(e^{i Psi} A_Z)  with the
// complex position factors A_E = q^2 P_E(q), A_Z = q^2 P_Z(q) (the push's
// series coefficients regrouped by powers of q), g = a0 exp(-rho^2/D - s^2)
// and Psi = tau + psi_c: one sine/cosine and one exponential per time.
struct AtomGeom {
    double X, Y, Z;
    double r2, mrD, psi_c;
    double aer, aei, azr, azi;
};

template <int FIELD, class CFG>
__device__ inline AtomGeom atom_geom(const CFG& c, double X, double Y, double Z)
{
    AtomGeom a{X, Y, Z, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if constexpr (FIELD == 1 || FIELD == 3 || FIELD == 5) {
        const double r2 = (X * X + Y * Y) * c.inv_w0n2;
        const double zeta = Z * c.inv_zrn;
        const double iD = 1.0 / (1.0 + zeta * zeta);
        const double rD = r2 * iD;
        a.r2 = r2;
        a.mrD = -rD;
        a.psi_c = c.phi0 - rD * zeta;
        const Cx<double> q{iD, zeta * iD};
        const double r4 = r2 * r2, r6 = r4 * r2, r8 = r4 * r4;
        // P_E(q) = sum p_n q^n and P_Z(q) = sum z_n q^n, by Horner in q
        // Horner step: p <- p q + coefficient
        auto horner = [&q](Cx<double> p, double coef) {
            const Cx<double> t = cmul(p, q);
            return Cx<double>{t.re + coef, t.im};
        };
        Cx<double> pe{1.0, 0.0}, pz{c.eps, 0.0};
        if constexpr (FIELD == 1) {
            pz = horner(Cx<double>{-c.eps * r2, 0.0}, c.eps);
        } else {
            double p[7] = {1.0, -0.5 * c.e2, c.e2 * r2, -0.25 * c.e2 * r4, 0.0, 0.0, 0.0};
            if constexpr (FIELD == 5) {
                p[2] += -0.375 * c.e4;
                p[3] += -0.375 * c.e4 * r2;
                p[4] = 1.0625 * c.e4 * r4;
                p[5] = -0.375 * c.e4 * r6;
                p[6] = 0.03125 * c.e4 * r8;
            }
            const double z[5] = {c.eps, -c.eps * r2 + 0.5 * c.e3, 0.5 * c.e3 * r2,
                                 -1.25 * c.e3 * r4, 0.25 * c.e3 * r6};
            constexpr int NE = (FIELD == 5) ? 7 : 4;
            pe = Cx<double>{p[NE - 1], 0.0};
#pragma unroll
            for (int n = NE - 2; n >= 0; --n) pe = horner(pe, p[n]);
            pz = Cx<double>{z[4], 0.0};
#pragma unroll
            for (int n = 3; n >= 0; --n) pz = horner(pz, z[n]);
        }
        const Cx<double> q2 = cmul(q, q);
        const Cx<double> ae = cmul(q2, pe), az = cmul(q2, pz);
        a.aer = ae.re; a.aei = ae.im; a.azr = az.re; a.azi = az.im;
    }
    return a;
}

template <int FIELD, class CFG>
__device__ inline double emag2_atom(const CFG& c, const AtomGeom& a, double d)
{
    if constexpr (FIELD == 1 || FIELD == 3 || FIELD == 5) {
        const double s = d * c.inv_T0n;
        const double g = c.a0 * fm::exp_fin_f64(a.mrD - s * s);
        // the sign (-1)^n of the half-angle form cancels in the squares
        double sg, kp;
        fm::cis_half2_f64(d, a.psi_c, &sg, &kp);
        const double cs = fma(-sg, sg, 1.0), sn = sg * kp;
        const double et = c.er_scale * g * (cs * a.aer - sn * a.aei);
        const double ez = c.ez_scale * g * (sn * a.azr + cs * a.azi);
        return et * et * a.r2 + ez * ez;
    } else {
        return emag2_f64<FIELD>(c, a.X, a.Y, a.Z, d);
    }
}

template <int FIELD, class CFG>
__device__ inline double rate_at(const CFG& c, const AdkState& st, const AtomGeom& a, double d)
{
    return adk_rate_n(st, emag2_atom<FIELD>(c, a, d));
}

// GL-4 estimate of the integral of the rate over [a, b]; the nodes are
// evaluated one after another (one field evaluation live at a time).
template <int FIELD, class CFG>
__device__ inline double gl4_integral(const CFG& c, const AdkState& st, const AtomGeom& ag,
                                      double a, double b)
{
    const double h = 0.5 * (b - a), m = 0.5 * (a + b);
    double acc = 0.0;
#pragma unroll 1
    for (int i = 0; i < 4; ++i) acc += c.gl_w[i] * rate_at<FIELD>(c, st, ag, m + h * c.gl_x[i]);
    return h * acc;
}

template <int FIELD, class CFG>
__device__ double solve_crossing(const CFG& c, const AdkState& st, const AtomGeom& ag, double lo,
                                 double hi, double target, double Ghi)
{
    if (!(target > 0.0)) return lo;
    double tl = lo, th = hi;
    double t = lo + (hi - lo) * (target / Ghi);
    if (!(t > tl && t < th)) t = 0.5 * (tl + th);
    for (int it = 0; it < 100; ++it) {
        const double gd = gl4_integral<FIELD>(c, st, ag, lo, t) - target;
        if (gd == 0.0) return t;
        if (gd > 0.0) th = t; else tl = t;
        const double tol = ldexp(fmax(fabs(t), kTwoPi), -40);
        const double w = rate_at<FIELD>(c, st, ag, t);
        double tn = __builtin_nan("");
        if (w > 0.0) {
            const double dlt = gd / w;
            if (fabs(dlt) <= tol) return t - dlt;
            tn = t - dlt;
        }
        if (!(tn > tl && tn < th)) tn = 0.5 * (tl + th);
        const double step = fabs(tn - t);
        t = tn;
        if (step <= tol) break;
    }
    return t;
}

// Panel range [j_lo, j_hi] outside which the state's ln w lies below the skip
// level (adk_a2thr) at every node.
template <class CFG>
__device__ inline bool state_window(const CFG& c, const AdkState& st, double bound2, double Zc,
                                    double tau_s, double h, int32_t M, int32_t& j_lo, int32_t& j_hi)
{
    const double thr = st.a2thr;
    if (!(bound2 >= thr)) return false;            // never reaches a nonzero rate
    if (c.field == 11) { j_lo = 0; j_hi = M - 1; return true; }
    const double smax = sqrt(0.5 * log(bound2 / thr));
    const double half = smax / c.inv_T0n;          // in normalized time
    const double lo = floor((Zc - half - tau_s) / h) - 1.0;
    const double hi = ceil((Zc + half - tau_s) / h) + 1.0;
    j_lo = lo < 0.0 ? 0 : (lo > (double)(M - 1) ? M - 1 : (int32_t)lo);
    j_hi = hi > (double)(M - 1) ? M - 1 : (hi < 0.0 ? 0 : (int32_t)hi);
    return true;
}

// Upper bound of what the panel loop below can add up for state st over the
// panels j0..j1 (the first one from d_from): a panel's GL-4 estimate is at
// most its width times the largest rate at its nodes, and the rate is at
// most the ADK rate at the largest |a|^2 the field bound allows there,
// |a|^2 <= b2 exp(-2 s^2) (lb2 = ln b2), capped at the |a|^2 where the rate
// itself peaks.  Panels go in groups of kBoundGroup (one optical period);
// each group is charged its width times that rate at its smallest |s|.  When
// twice this bound stays below the state's threshold the loop could not reach
// it: the state, and so every later one, is never born, which is what
// integrating all the panels would give.  never_reaches() answers that.  It
// takes the group nearest the envelope peak (s = 0) first, the largest term,
// and stops as soon as the sum passes half the threshold, so a state that
// will be born costs one or two groups.
constexpr int32_t kBoundGroup = 200;

// Edges of group g (0-based) of panels j0..j1, as the panel loop forms its
// panel edges: from d_from or panel j0 + g kBoundGroup to the start of the
// next group or the end of panel j1.
__device__ inline void bound_group(int32_t g, int32_t groups, int32_t j0, int32_t j1, int32_t M,
                                   double d_s, double d_e, double h, double d_from, double& da,
                                   double& db)
{
    da = (g == 0) ? d_from : d_s + (double)(j0 + g * kBoundGroup) * h;
    db = (g + 1 < groups) ? d_s + (double)(j0 + (g + 1) * kBoundGroup) * h
                          : ((j1 == M - 1) ? d_e : d_s + (double)(j1 + 1) * h);
}

template <class CFG>
__device__ inline double bound_group_rate(const CFG& c, const AdkState& st, double lb2, double la2pk,
                                          double da, double db)
{
    const double smin = (da <= 0.0 && db >= 0.0) ? 0.0 : fmin(fabs(da), fabs(db)) * c.inv_T0n;
    const double la2 = fmin(lb2 - 2.0 * smin * smin, la2pk);
    const double lw = st.c0 - st.c1h * la2 - st.c2 * fm::exp_f64(-0.5 * la2);
    return (db - da) * fm::exp_f64(lw);
}

template <class CFG>
__device__ inline bool never_reaches(const CFG& c, const AdkState& st, double lb2, double d_s,
                                     double d_e, double h, int32_t M, int32_t j0, int32_t j1,
                                     double d_from, double target)
{
    // ln |a|^2 where ln w = c0 - c1h ln|a|^2 - c2 |a|^-1 peaks
    const double la2pk = (st.c1h > 0.0) ? 2.0 * fm::log_pos_f64(st.c2 / (2.0 * st.c1h))
                                         : __builtin_inf();
    const int32_t groups = (j1 - j0) / kBoundGroup + 1;
    // the group holding d = 0, or the one nearest to it
    const double jpk = floor(-d_s / h) - (double)j0;
    const int32_t gpk = jpk <= 0.0 ? 0
                      : (jpk >= (double)(groups - 1) * kBoundGroup ? groups - 1
                                                                   : (int32_t)jpk / kBoundGroup);
    double da, db;
    bound_group(gpk, groups, j0, j1, M, d_s, d_e, h, d_from, da, db);
    double sum = bound_group_rate(c, st, lb2, la2pk, da, db);
    if (!(2.0 * sum < target)) return false;
#pragma unroll 1
    for (int32_t g = 0; g < groups; ++g) {
        if (g == gpk) continue;
        bound_group(g, groups, j0, j1, M, d_s, d_e, h, d_from, da, db);
        sum += bound_group_rate(c, st, lb2, la2pk, da, db);
        if (!(2.0 * sum < target)) return false;
    }
    return true;
}

// Birth times of one atom (index `atom`, normalized position X, Y, Z) for
// states k_first..k_first+K-1, written to out[0..K) in seconds.  The atom is
// at rest, so its field depends on time only through the retarded time
// d = tau - Z: the panels, nodes and crossings are all taken in d (the same
// grid as in tau, shifted by Z), so the carrier phase is formed from d itself
// and the birth time tau = d + Z is rounded once, at the output.
template <int FIELD, class CFG>
__device__ void ionize_atom(const CFG& c, uint64_t seed, uint32_t cfg, uint64_t atom, double X,
                            double Y, double Z, int k_first, int K, double* __restrict__ out)
{
    for (int s = 0; s < K; ++s) out[s] = __builtin_inf();
    const double dz = (c.window == 0) ? 0.0 : -Z;   // window start relative to arrival
    const double d_s = dz - c.tb_n, d_e = dz + c.ta_n;
    const double h = c.hn;
    // panels in the window (below 2^31: the host limits window / dt to 2e9)
    const int32_t M = (int32_t)ceil((d_e - d_s) / h);
    const double b2 = bound2_f64<FIELD>(c, X, Y, Z);
    const double Zc = 0.0;  // the envelope peaks at d = 0 for the pulse models

    int s = 0;
    double target = -log(uniform_j(seed, cfg, atom, k_first + 2));
    // states with a zero threshold are born where they start
    while (s < K && !(target > 0.0)) {
        out[s] = (d_s + Z) * c.inv_omega;
        ++s;
        if (s < K) target = -log(uniform_j(seed, cfg, atom, k_first + s + 2));
    }
    if (s >= K) return;
    AdkState st = adk_state(c, k_first - 1 + s);
    int32_t j_lo, j_hi;
    if (!state_window(c, st, b2, Zc, d_s, h, M, j_lo, j_hi)) return;
    // the envelope bound holds for the pulse models (not the static field)
    if (FIELD != 11 &&
        never_reaches(c, st, fm::log_pos_f64(b2), d_s, d_e, h, M, j_lo, j_hi, d_s + (double)j_lo * h, target))
        return;
    const AtomGeom ag = atom_geom<FIELD>(c, X, Y, Z);
    double I = 0.0;
    double tstart = d_s;
    for (int32_t j = j_lo; j < M; ++j) {
        if (j > j_hi) break;
        const double a = d_s + (double)j * h;
        const double b = (j == M - 1) ? d_e : d_s + (double)(j + 1) * h;
        bool done = false;
        while (true) {
            const double lo = (tstart > a) ? tstart : a;
            const double seg = gl4_integral<FIELD>(c, st, ag, lo, b);
            if (I + seg < target) { I += seg; break; }
            const double t = solve_crossing<FIELD>(c, st, ag, lo, b, target - I, seg);
            out[s] = (t + Z) * c.inv_omega;
            ++s;
            if (s >= K) { done = true; break; }
            target = -log(uniform_j(seed, cfg, atom, k_first + s + 2));
            I = 0.0;
            tstart = t;
            st = adk_state(c, k_first - 1 + s);
            int32_t nlo, nhi;
            if (!state_window(c, st, b2, Zc, d_s, h, M, nlo, nhi)) {
                if (!(target > 0.0)) { j_hi = M - 1; continue; }
                done = true;
                break;
            }
            j_hi = (target > 0.0) ? nhi : M - 1;
            if (FIELD != 11 && target > 0.0) {
                const int32_t j0 = nlo > j ? nlo : j;
                const double d0 = nlo > j ? d_s + (double)nlo * h : t;
                if (never_reaches(c, st, fm::log_pos_f64(b2), d_s, d_e, h, M, j0, j_hi, d0, target)) {
                    done = true;
                    break;
                }
            }
            if (target > 0.0 && nlo > j) {
                // before its window the new state's ln w stays below the
                // skip level at every node, the same bound that starts the
                // first state at its window: resume at the window's first panel
                j = nlo - 1;
                break;
            }
        }
        if (done) break;
    }
}

// Wave-cooperative refill: lanes with need == true get consecutive queue
// indices (called by every lane of the wave; -1 for the other lanes).
__device__ inline int64_t queue_take(unsigned long long* queue, bool need)
{
    const uint64_t m = __ballot(need);
    if (m == 0) return -1;
    const int lane = __lane_id();
    const int leader = __ffsll((unsigned long long)m) - 1;
    unsigned long long base = 0;
    if (lane == leader) base = atomicAdd(queue, (unsigned long long)__popcll(m));
    base = __shfl(base, leader);
    const int rank = __popcll(m & ((1ull << lane) - 1ull));
    return need ? (int64_t)(base + (unsigned long long)rank) : -1;
}

// Lane i ionizes atom order[i] (atom i without an order).  An order that
// groups atoms of similar work in the same wave keeps the lanes of a wave
// busy for the same number of panels; the results do not depend on it.
template <int FIELD>
__global__ void __launch_bounds__(256, 3) ionize_kernel(
    DevCfg c, uint64_t seed, uint32_t cfg, uint64_t first_atom, int64_t n,
    const double* __restrict__ x, const double* __restrict__ y, const double* __restrict__ z,
    int k_first, int k_last, double* __restrict__ t_birth, const uint32_t* __restrict__ order)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t a = order ? (int64_t)order[i] : i;
    const int K = k_last - k_first + 1;
    ionize_atom<FIELD>(c, seed, cfg, first_atom + (uint64_t)a, x[a] * c.k, y[a] * c.k,
                       z[a] * c.k, k_first, K, t_birth + a * K);
}

// Work key of each atom for that order: first the number of its states that
// the rate bound (never_reaches) does not rule out from the window start --
// those the panel loop may integrate; the thresholds are random, so atoms of
// one field strength differ in it -- then the bound of its peak |a|^2 (the
// states' windows, and so the panels an atom integrates, grow with it), as
// the top bits of a non-negative float, which order like the value.
template <int FIELD>
__global__ void __launch_bounds__(256) ionize_key_kernel(DevCfg c, uint64_t seed, uint32_t cfg,
                                                         uint64_t first_atom, int64_t n,
                                                         const double* __restrict__ x,
                                                         const double* __restrict__ y,
                                                         const double* __restrict__ z, int k_first,
                                                         int k_last, uint32_t* __restrict__ key,
                                                         uint32_t* __restrict__ idx)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double X = x[i] * c.k, Y = y[i] * c.k, Z = z[i] * c.k;
    const double b2 = bound2_f64<FIELD>(c, X, Y, Z);
    uint32_t open = 0;
    if (FIELD != 11) {
        const double dz = (c.window == 0) ? 0.0 : -Z;
        const double d_s = dz - c.tb_n, d_e = dz + c.ta_n;
        const double h = c.hn;
        const int32_t M = (int32_t)ceil((d_e - d_s) / h);
        const double lb2 = fm::log_pos_f64(b2);
        for (int k = k_first; k <= k_last; ++k) {
            const double target = -log(uniform_j(seed, cfg, first_atom + (uint64_t)i, k + 2));
            if (!(target > 0.0)) { ++open; continue; }
            const AdkState st = adk_state(c, k - 1);
            int32_t j_lo, j_hi;
            if (!state_window(c, st, b2, 0.0, d_s, h, M, j_lo, j_hi)) break;
            if (never_reaches(c, st, lb2, d_s, d_e, h, M, j_lo, j_hi, d_s + (double)j_lo * h, target))
                break;
            ++open;
        }
    }
    const float b2f = (float)b2;
    key[i] = (open << 27) | (__float_as_uint(b2f > 0.0f ? b2f : 0.0f) >> 4);
    idx[i] = (uint32_t)i;
}

// ---------------------------------------------------------------------------
// Push.  One electron per lane: state (X, u) advanced by classical RK4 with
// fixed step h from its birth to the end of its atom's window (steps start at
// tau0 + n h, the last one ends on the window end).  The fields depend on
// time only through the retarded time D = tau - Z, which the state carries as
// a seventh variable (dD/dtau = 1 - u_z/gamma, D = tau0 - Z0 at birth): RK4
// is linear in its stage slopes, so in exact arithmetic D equals tau - Z at
// every stage, while in floating point the carrier phase is resolved to the
// rounding of D itself rather than that of tau and Z separately (each up to
// ~1e3 over the window).
// ---------------------------------------------------------------------------
template <int FIELD, class CFG>
__device__ inline void rhs_f64(const CFG& c, double d, double dl, double X, double Y, double Z,
                               double ux, double uy, double uz, double& dX, double& dY,
                               double& dZ, double& dux, double& duy, double& duz)
{
    const double ig = fm::rsqrt_ge1_f64(1.0 + ux * ux + uy * uy + uz * uz);
    dX = ux * ig; dY = uy * ig; dZ = uz * ig;
    if constexpr (FIELD == 1 || FIELD == 3 || FIELD == 5) {
        // radial field: a = (pe X, pe Y, az), b = pb (-Y, X, 0), so
        // a + beta x b = ((pe - beta_z pb) X, (pe - beta_z pb) Y,
        //                 az + pb (beta_x X + beta_y Y))
        double pe, pb, az;
        rp_field_parts_f64<FIELD, true>(c, X, Y, Z, d, dl, pe, pb, az);
        const double f = fma(-dZ, pb, pe);
        dux = -f * X;
        duy = -f * Y;
        duz = -fma(pb, fma(dY, Y, dX * X), az);
    } else {
        double ax, ay, az, bx, by, bz;
        field_f64<FIELD, true, CFG>(c, X, Y, Z, d + dl, ax, ay, az, bx, by, bz);
        dux = -(ax + dY * bz - dZ * by);
        duy = -(ay + dZ * bx - dX * bz);
        duz = -(az + dX * by - dY * bx);
    }
}

// The state is accumulated with compensated (Kahan) summation: over the
// ~3e4 steps of a trajectory the rounding of plain double accumulation,
// above all of the position, is amplified to more than 1e-8 of the final
// energy for a few electrons in a thousand; the compensation terms cX..cuz
// carry what each addition lost into the next one.
struct ElecF64 {
    double X, Y, Z, ux, uy, uz, tau0, taue;
    double D;                                  // retarded time tau - Z
    double cX, cY, cZ, cux, cuy, cuz, cD;
    int64_t n, N;
};

constexpr double kLightSpeed = 299792458.0;            // m/s, exact
constexpr double kInvLightSpeed = 1.0 / 299792458.0;

__device__ inline void kahan_add_f64(double& s, double& comp, double v)
{
    const double y = v - comp;
    const double t = s + y;
    comp = (t - s) - y;
    s = t;
}

// Set up an electron born at rest at t0 [s] at atom position (x, y, z) [m].
// Returns false (invalid slot) for a birth more than one step before the
// window start, which also bounds the step count of every lane.
template <class CFG>
__device__ inline bool elec_init(const CFG& c, ElecF64& e, double t0, double x, double y, double z)
{
    e.X = x * c.k; e.Y = y * c.k; e.Z = z * c.k;
    e.ux = e.uy = e.uz = 0.0;
    e.cX = e.cY = e.cZ = e.cux = e.cuy = e.cuz = e.cD = 0.0;
    e.tau0 = t0 * c.omega;
    // D = omega (t0 - z0/c), the quotient z0/c carried with its remainder so
    // that the retarded time is formed to the rounding of its own value
    const double zc = z * kInvLightSpeed;
    const double zr = fma(-zc, kLightSpeed, z);
    e.D = ((t0 - zc) - zr * kInvLightSpeed) * c.omega;
    const double tz = (c.window == 0) ? e.Z : 0.0;
    e.taue = tz + c.ta_n;
    e.n = 0;
    e.N = 0;
    if (!(e.tau0 >= tz - c.tb_n - c.hn)) return false;
    e.N = (int64_t)ceil((e.taue - e.tau0) / c.hn);
    return true;
}

template <int FIELD, class CFG>
__device__ inline void elec_step(const CFG& c, ElecF64& e)
{
    const double h = c.hn;
    const double ta = e.tau0 + (double)e.n * h;
    const double hs = (e.n == e.N - 1) ? (e.taue - ta) : h;
    const double hh = 0.5 * hs;
    double kX, kY, kZ, kx, ky, kz, aX, aY, aZ, ax, ay, az;
    rhs_f64<FIELD>(c, e.D, -e.cD, e.X, e.Y, e.Z, e.ux, e.uy, e.uz, kX, kY, kZ, kx, ky, kz);
    aX = kX; aY = kY; aZ = kZ; ax = kx; ay = ky; az = kz;
    rhs_f64<FIELD>(c, e.D, fma(hh, 1.0 - kZ, -e.cD), e.X + hh * kX, e.Y + hh * kY,
                   e.Z + hh * kZ, e.ux + hh * kx, e.uy + hh * ky, e.uz + hh * kz, kX, kY, kZ, kx,
                   ky, kz);
    aX += 2.0 * kX; aY += 2.0 * kY; aZ += 2.0 * kZ;
    ax += 2.0 * kx; ay += 2.0 * ky; az += 2.0 * kz;
    rhs_f64<FIELD>(c, e.D, fma(hh, 1.0 - kZ, -e.cD), e.X + hh * kX, e.Y + hh * kY,
                   e.Z + hh * kZ, e.ux + hh * kx, e.uy + hh * ky, e.uz + hh * kz, kX, kY, kZ, kx,
                   ky, kz);
    aX += 2.0 * kX; aY += 2.0 * kY; aZ += 2.0 * kZ;
    ax += 2.0 * kx; ay += 2.0 * ky; az += 2.0 * kz;
    rhs_f64<FIELD>(c, e.D, fma(hs, 1.0 - kZ, -e.cD), e.X + hs * kX, e.Y + hs * kY,
                   e.Z + hs * kZ, e.ux + hs * kx, e.uy + hs * ky, e.uz + hs * kz, kX, kY, kZ, kx,
                   ky, kz);
    const double w6 = hs * (1.0 / 6.0);
    const double sZ = aZ + kZ;
    kahan_add_f64(e.X, e.cX, w6 * (aX + kX));
    kahan_add_f64(e.Y, e.cY, w6 * (aY + kY));
    kahan_add_f64(e.Z, e.cZ, w6 * sZ);
    kahan_add_f64(e.ux, e.cux, w6 * (ax + kx));
    kahan_add_f64(e.uy, e.cuy, w6 * (ay + ky));
    kahan_add_f64(e.uz, e.cuz, w6 * (az + kz));
    // the weighted slopes of D sum to 6 - sZ
    kahan_add_f64(e.D, e.cD, w6 * (6.0 - sZ));
    ++e.n;
}

template <class CFG>
__device__ inline void elec_final(const CFG& c, const ElecF64& e, double& ux, double& uy,
                                  double& uz, double& xf, double& yf, double& zf)
{
    ux = e.ux; uy = e.uy; uz = e.uz;
    xf = e.X * c.inv_k; yf = e.Y * c.inv_k; zf = e.Z * c.inv_k;
}

// ---------------------------------------------------------------------------
// Radiation reaction (Eq. (3)) and the quantum parameter (Eqs. (4)-(5)).  In
// normalized units the gamma^2 Landau-Lifshitz term is
//   du/dtau = -kappa gamma u Q,   Q = (a + beta x b)^2 - (beta . a)^2,
// kappa = (2/3) k r_e, and chi = eta gamma sqrt(Q), eta = hbar omega/(m c^2).
// ElecRR<RR> pushes with the term on (RR) or off and keeps the largest
// gamma^2 Q met at its step starts (chi^2 / eta^2).
// ---------------------------------------------------------------------------
template <bool RR>
struct ElecRR : ElecF64 {
    double g2q;
};

// Right-hand side with the radiation term; returns gamma^2 Q at the state.
template <int FIELD, bool RR, class CFG>
__device__ inline double rhs_rr_f64(const CFG& c, double d, double dl, double X, double Y, double Z,
                                    double ux, double uy, double uz, double& dX, double& dY,
                                    double& dZ, double& dux, double& duy, double& duz)
{
    double ax, ay, az, bx, by, bz;
    field_f64<FIELD, true, CFG, true>(c, X, Y, Z, d, ax, ay, az, bx, by, bz, dl);
    const double ig = fm::rsqrt_ge1_f64(1.0 + ux * ux + uy * uy + uz * uz);
    dX = ux * ig; dY = uy * ig; dZ = uz * ig;
    const double fx = ax + (dY * bz - dZ * by);
    const double fy = ay + (dZ * bx - dX * bz);
    const double fz = az + (dX * by - dY * bx);
    const double ba = dX * ax + dY * ay + dZ * az;
    double q = fx * fx + fy * fy + fz * fz - ba * ba;
    q = q > 0.0 ? q : 0.0;
    dux = -fx; duy = -fy; duz = -fz;
    if (RR) {
        const double s = c.rr_kappa * q / ig;     // kappa gamma Q
        dux -= s * ux; duy -= s * uy; duz -= s * uz;
    }
    return q / (ig * ig);
}

template <class CFG, bool RR>
__device__ inline bool elec_init(const CFG& c, ElecRR<RR>& e, double t0, double x, double y,
                                 double z)
{
    e.g2q = 0.0;
    return elec_init(c, static_cast<ElecF64&>(e), t0, x, y, z);
}

template <int FIELD, class CFG, bool RR>
__device__ inline void elec_step(const CFG& c, ElecRR<RR>& e)
{
    const double h = c.hn;
    const double ta = e.tau0 + (double)e.n * h;
    const double hs = (e.n == e.N - 1) ? (e.taue - ta) : h;
    const double hh = 0.5 * hs;
    double kX, kY, kZ, kx, ky, kz, aX, aY, aZ, ax, ay, az;
    const double g2q = rhs_rr_f64<FIELD, RR>(c, e.D, -e.cD, e.X, e.Y, e.Z, e.ux, e.uy, e.uz, kX,
                                             kY, kZ, kx, ky, kz);
    e.g2q = g2q > e.g2q ? g2q : e.g2q;
    aX = kX; aY = kY; aZ = kZ; ax = kx; ay = ky; az = kz;
    rhs_rr_f64<FIELD, RR>(c, e.D, fma(hh, 1.0 - kZ, -e.cD), e.X + hh * kX, e.Y + hh * kY,
                          e.Z + hh * kZ, e.ux + hh * kx, e.uy + hh * ky, e.uz + hh * kz, kX, kY,
                          kZ, kx, ky, kz);
    aX += 2.0 * kX; aY += 2.0 * kY; aZ += 2.0 * kZ;
    ax += 2.0 * kx; ay += 2.0 * ky; az += 2.0 * kz;
    rhs_rr_f64<FIELD, RR>(c, e.D, fma(hh, 1.0 - kZ, -e.cD), e.X + hh * kX, e.Y + hh * kY,
                          e.Z + hh * kZ, e.ux + hh * kx, e.uy + hh * ky, e.uz + hh * kz, kX, kY,
                          kZ, kx, ky, kz);
    aX += 2.0 * kX; aY += 2.0 * kY; aZ += 2.0 * kZ;
    ax += 2.0 * kx; ay += 2.0 * ky; az += 2.0 * kz;
    rhs_rr_f64<FIELD, RR>(c, e.D, fma(hs, 1.0 - kZ, -e.cD), e.X + hs * kX, e.Y + hs * kY,
                          e.Z + hs * kZ, e.ux + hs * kx, e.uy + hs * ky, e.uz + hs * kz, kX, kY,
                          kZ, kx, ky, kz);
    const double w6 = hs * (1.0 / 6.0);
    const double sZ = aZ + kZ;
    kahan_add_f64(e.X, e.cX, w6 * (aX + kX));
    kahan_add_f64(e.Y, e.cY, w6 * (aY + kY));
    kahan_add_f64(e.Z, e.cZ, w6 * sZ);
    kahan_add_f64(e.ux, e.cux, w6 * (ax + kx));
    kahan_add_f64(e.uy, e.cuy, w6 * (ay + ky));
    kahan_add_f64(e.uz, e.cuz, w6 * (az + kz));
    kahan_add_f64(e.D, e.cD, w6 * (6.0 - sZ));
    ++e.n;
}


// ---------------------------------------------------------------------------
// Controlled-step push (Sec. 1, Sec. 2.1: fifth-order Runge-Kutta with a
// controlled step, run until the kinetic energy is constant).  Dormand-Prince
// 5(4): seven stages, the fifth-order result carried, the last stage reused
// as the next first one.  One call of elec_step is one attempted step:
//   error = max_i |y5_i - y4_i| / (atol + rtol max(|y_i|, |y5_i|)) over
//           (X, Y, Z, u) in normalized units; accept when <= 1;
//   next step h min(5, max(0.2, 0.9 err^(-1/5))), capped at h_max and at the
//   window end; first step dt;
//   stop at the window end or at the first accepted step end, at least 0.999
//   optical period (2 pi) after the previous check, where gamma changed by at
//   most k_tol relative (the margin keeps steps commensurate with the period
//   from making every check a rounding tie); over the step budget, or when a
//   step's error is not a number, the electron is NaN.
// ---------------------------------------------------------------------------
namespace dp {
constexpr double c2 = 1.0 / 5.0, c3 = 3.0 / 10.0, c4 = 4.0 / 5.0, c5 = 8.0 / 9.0;
constexpr double a21 = 1.0 / 5.0;
constexpr double a31 = 3.0 / 40.0, a32 = 9.0 / 40.0;
constexpr double a41 = 44.0 / 45.0, a42 = -56.0 / 15.0, a43 = 32.0 / 9.0;
constexpr double a51 = 19372.0 / 6561.0, a52 = -25360.0 / 2187.0, a53 = 64448.0 / 6561.0,
                 a54 = -212.0 / 729.0;
constexpr double a61 = 9017.0 / 3168.0, a62 = -355.0 / 33.0, a63 = 46732.0 / 5247.0,
                 a64 = 49.0 / 176.0, a65 = -5103.0 / 18656.0;
// fifth-order weights (b2 = 0, b7 = 0) and fifth minus fourth order
constexpr double b1 = 35.0 / 384.0, b3 = 500.0 / 1113.0, b4 = 125.0 / 192.0,
                 b5 = -2187.0 / 6784.0, b6 = 11.0 / 84.0;
constexpr double e1 = b1 - 5179.0 / 57600.0, e3 = b3 - 7571.0 / 16695.0,
                 e4 = b4 - 393.0 / 640.0, e5 = b5 + 92097.0 / 339200.0,
                 e6 = b6 - 187.0 / 2100.0, e7 = -1.0 / 40.0;
}  // namespace dp

struct ElecDP {
    double y[6];          // X, Y, Z, ux, uy, uz
    double k1[6];         // derivative at y (valid once `fresh` is false)
    double tau, h, taue, g_ref, t_ref;
    int64_t n, N;         // N = 1 while the electron runs, n = 1 when done
    long long acc, rej;
    bool fresh, failed;
};

template <class CFG>
__device__ inline bool elec_init(const CFG& c, ElecDP& e, double t0, double x, double y, double z)
{
    e.y[0] = x * c.k; e.y[1] = y * c.k; e.y[2] = z * c.k;
    e.y[3] = e.y[4] = e.y[5] = 0.0;
    e.tau = t0 * c.omega;
    const double tz = (c.window == 0) ? e.y[2] : 0.0;
    e.taue = tz + c.ta_n;
    e.h = c.hn;
    e.g_ref = 1.0;
    e.t_ref = e.tau;
    e.acc = e.rej = 0;
    e.fresh = true;
    e.failed = false;
    e.n = 0;
    e.N = 0;
    if (!(e.tau >= tz - c.tb_n - c.hn)) return false;
    e.N = (e.taue > e.tau) ? 1 : 0;
    return true;
}

template <int FIELD, class CFG>
__device__ inline void dp_rhs(const CFG& c, double tau, const double* y, double* k)
{
    rhs_f64<FIELD>(c, tau - y[2], 0.0, y[0], y[1], y[2], y[3], y[4], y[5], k[0], k[1], k[2], k[3],
                   k[4], k[5]);
}

template <int FIELD, class CFG>
__device__ inline void elec_step(const CFG& c, ElecDP& e)
{
    using namespace dp;
    if (e.fresh) {
        dp_rhs<FIELD>(c, e.tau, e.y, e.k1);
        e.fresh = false;
    }
    if (e.acc + e.rej >= c.ad_max_steps) {
        e.failed = true;
        e.n = e.N;
        return;
    }
    double hs = e.h < c.ad_hmax ? e.h : c.ad_hmax;
    bool last = false;
    if (hs >= e.taue - e.tau) { hs = e.taue - e.tau; last = true; }
    double k2[6], k3[6], k4[6], k5[6], k6[6], k7[6], yt[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) yt[i] = e.y[i] + hs * (a21 * e.k1[i]);
    dp_rhs<FIELD>(c, e.tau + c2 * hs, yt, k2);
#pragma unroll
    for (int i = 0; i < 6; ++i) yt[i] = e.y[i] + hs * (a31 * e.k1[i] + a32 * k2[i]);
    dp_rhs<FIELD>(c, e.tau + c3 * hs, yt, k3);
#pragma unroll
    for (int i = 0; i < 6; ++i) yt[i] = e.y[i] + hs * (a41 * e.k1[i] + a42 * k2[i] + a43 * k3[i]);
    dp_rhs<FIELD>(c, e.tau + c4 * hs, yt, k4);
#pragma unroll
    for (int i = 0; i < 6; ++i)
        yt[i] = e.y[i] + hs * (a51 * e.k1[i] + a52 * k2[i] + a53 * k3[i] + a54 * k4[i]);
    dp_rhs<FIELD>(c, e.tau + c5 * hs, yt, k5);
#pragma unroll
    for (int i = 0; i < 6; ++i)
        yt[i] = e.y[i] + hs * (a61 * e.k1[i] + a62 * k2[i] + a63 * k3[i] + a64 * k4[i] +
                               a65 * k5[i]);
    dp_rhs<FIELD>(c, e.tau + hs, yt, k6);
    double y5[6];
#pragma unroll
    for (int i = 0; i < 6; ++i)
        y5[i] = e.y[i] + hs * (b1 * e.k1[i] + b3 * k3[i] + b4 * k4[i] + b5 * k5[i] + b6 * k6[i]);
    dp_rhs<FIELD>(c, e.tau + hs, y5, k7);
    double err = 0.0;
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        const double d = fabs(hs * (e1 * e.k1[i] + e3 * k3[i] + e4 * k4[i] + e5 * k5[i] +
                                    e6 * k6[i] + e7 * k7[i]));
        const double ya = fabs(e.y[i]), yb = fabs(y5[i]);
        const double r = d / (c.ad_atol + c.ad_rtol * (ya > yb ? ya : yb));
        err = (r > err || r != r) ? r : err;
    }
    if (err != err) {            // the step produced no number: give up on this electron
        e.failed = true;
        e.n = e.N;
        return;
    }
    if (err <= 1.0) {
        e.tau = last ? e.taue : e.tau + hs;
#pragma unroll
        for (int i = 0; i < 6; ++i) { e.y[i] = y5[i]; e.k1[i] = k7[i]; }
        ++e.acc;
        if (last) { e.n = e.N; return; }
        if (e.tau - e.t_ref >= 0.999 * (2.0 * 3.14159265358979323846)) {
            const double g = sqrt(1.0 + e.y[3] * e.y[3] + e.y[4] * e.y[4] + e.y[5] * e.y[5]);
            if (fabs(g - e.g_ref) <= c.ad_ktol * g) { e.n = e.N; return; }
            e.g_ref = g;
            e.t_ref = e.tau;
        }
    } else {
        ++e.rej;
    }
    double fac = (err == 0.0) ? 5.0 : 0.9 * pow(err, -0.2);
    fac = fac > 5.0 ? 5.0 : (fac < 0.2 ? 0.2 : fac);
    e.h = hs * fac;
}

template <class CFG>
__device__ inline void elec_final(const CFG& c, const ElecDP& e, double& ux, double& uy,
                                  double& uz, double& xf, double& yf, double& zf)
{
    const double q = __builtin_nan("");
    ux = e.failed ? q : e.y[3]; uy = e.failed ? q : e.y[4]; uz = e.failed ? q : e.y[5];
    xf = e.failed ? q : e.y[0] * c.inv_k;
    yf = e.failed ? q : e.y[1] * c.inv_k;
    zf = e.failed ? q : e.y[2] * c.inv_k;
}

// ---------------------------------------------------------------------------
// Mixed precision: the field and the RK4 stage arithmetic in float; time,
// position and the carrier phase in double.  At each step start the retarded
// time tau - Z is formed in double and reduced to turns in [-1/2, 1/2] (the
// hardware sine/cosine take turns); the four stages then take the transverse
// position, zeta, the phase and the envelope argument as float offsets from
// that start -- the field needs them only to float precision, and the
// retarded time advances by h (1 - beta_z) over a stage of length h.  The
// momentum is kept in float with a Kahan compensation term, the position in
// double.
// ---------------------------------------------------------------------------

// Field arguments at the step start, in float (phase and envelope from the
// double retarded time).
struct MixedBase {
    float X, Y;        // transverse position
    float zeta;        // Z / (k z_r)
    float ph;          // (tau - Z) / (2 pi), reduced to [-1/2, 1/2]
    float s;           // (tau - Z) / (omega tau0)
    float izr, it0;    // 1/(k z_r), 1/(omega tau0)
};

template <class CFG>
__device__ inline MixedBase mixed_base(const CFG& c, double tau, double X, double Y, double Z)
{
    const double d = tau - Z;
    double turns = d * kInvTwoPi;
    turns -= rint(turns);
    MixedBase b;
    b.X = (float)X; b.Y = (float)Y;
    b.zeta = (float)(Z * c.inv_zrn);
    b.ph = (float)turns;
    b.s = (float)(d * c.inv_T0n);
    b.izr = (float)c.inv_zrn;
    b.it0 = (float)c.inv_T0n;
    return b;
}

// Field arguments of a stage at offset hk from the step start, reached with
// the slopes (kX, kY, kZ); dd is the retarded-time offset hk (1 - kZ).
struct MixedArgs {
    float X, Y, zeta, dd, s;
};

template <bool FIRST>
__device__ inline MixedArgs mixed_args(const MixedBase& b, float hk, float kX, float kY, float kZ)
{
    MixedArgs a;
    if constexpr (FIRST) {
        a.X = b.X; a.Y = b.Y; a.zeta = b.zeta; a.dd = 0.f; a.s = b.s;
    } else {
        a.X = fmaf(hk, kX, b.X);
        a.Y = fmaf(hk, kY, b.Y);
        a.zeta = fmaf(hk * kZ, b.izr, b.zeta);
        a.dd = fmaf(-hk, kZ, hk);
        a.s = fmaf(a.dd, b.it0, b.s);
    }
    return a;
}

template <int ORDER, class CFG>
__device__ inline void rp_field_parts_mixed(const CFG& c, const MixedBase& b, const MixedArgs& a,
                                            float& pe, float& pb, float& az)
{
    const float r2 = (a.X * a.X + a.Y * a.Y) * (float)c.inv_w0n2;
    const float zeta = a.zeta;
    const float iD = __builtin_amdgcn_rcpf(1.0f + zeta * zeta);
    const float rD = r2 * iD;
    const float ph = fmaf(a.dd + fmaf(-rD, zeta, (float)c.phi0), (float)kInvTwoPi, b.ph);
    const float g = (float)c.a0 * __builtin_amdgcn_exp2f(-(rD + a.s * a.s) * 1.4426950408889634f);
    const float sn = __builtin_amdgcn_sinf(ph), cs = __builtin_amdgcn_cosf(ph);
    const float gi = g * (iD * iD);
    float PE, PB, EZe;
    rp_brackets<ORDER, float>(gi * cs, gi * sn, zeta, rD, (float)c.e2 * iD, PE, PB, EZe);
    pe = (float)c.er_w * PE;
    pb = PB * (float)c.inv_w0n;
    az = (float)c.ez_e * EZe;
}

template <int FIELD, class CFG>
__device__ inline void field_mixed(const CFG& c, const MixedBase& b, const MixedArgs& a,
                                   float& ax, float& ay, float& az, float& bx, float& by,
                                   float& bz)
{
    static_assert(FIELD < 20, "the linearly polarized focus has no mixed form");
    if constexpr (FIELD == 11) {
        ax = (float)c.tE[0]; ay = (float)c.tE[1]; az = (float)c.tE[2];
        bx = (float)c.tB[0]; by = (float)c.tB[1]; bz = (float)c.tB[2];
    } else if constexpr (FIELD == 10) {
        const float ph = fmaf(a.dd + (float)c.phi0, (float)kInvTwoPi, b.ph);
        const float e = (float)c.a0 * __builtin_amdgcn_exp2f(-a.s * a.s * 1.4426950408889634f)
                        * __builtin_amdgcn_cosf(ph);
        ax = e; ay = 0.f; az = 0.f; bx = 0.f; by = e; bz = 0.f;
    } else {
        float pe, pb;
        rp_field_parts_mixed<FIELD>(c, b, a, pe, pb, az);
        ax = pe * a.X; ay = pe * a.Y;
        bx = -pb * a.Y; by = pb * a.X;
        bz = 0.f;
    }
}

template <int FIELD, bool FIRST, class CFG>
__device__ inline void rhs_mixed(const CFG& c, const MixedBase& b, float hk, float& dX, float& dY,
                                 float& dZ, float ux, float uy, float uz, float& dux, float& duy,
                                 float& duz)
{
    // (dX, dY, dZ) come in as the previous stage's slopes and leave as this one's
    const MixedArgs a = mixed_args<FIRST>(b, hk, dX, dY, dZ);
    const float ig = __builtin_amdgcn_rsqf(1.0f + ux * ux + uy * uy + uz * uz);
    dX = ux * ig; dY = uy * ig; dZ = uz * ig;
    if constexpr (FIELD == 1 || FIELD == 3 || FIELD == 5) {
        // radial field: the force from its radial and axial parts, as in rhs_f64
        float pe, pb, az;
        rp_field_parts_mixed<FIELD>(c, b, a, pe, pb, az);
        const float f = fmaf(-dZ, pb, pe);
        dux = -f * a.X;
        duy = -f * a.Y;
        duz = -fmaf(pb, fmaf(dY, a.Y, dX * a.X), az);
    } else {
        float ax, ay, az, bx, by, bz;
        field_mixed<FIELD, CFG>(c, b, a, ax, ay, az, bx, by, bz);
        dux = -(ax + dY * bz - dZ * by);
        duy = -(ay + dZ * bx - dX * bz);
        duz = -(az + dX * by - dY * bx);
    }
}

__device__ inline void kahan_add(float& s, float& comp, float v)
{
    const float y = v - comp;
    const float t = s + y;
    comp = (t - s) - y;
    s = t;
}

struct ElecMixed {
    double X, Y, Z, tau0, taue;
    float ux, uy, uz, cx, cy, cz;
    int64_t n, N;
};

template <class CFG>
__device__ inline bool elec_init(const CFG& c, ElecMixed& e, double t0, double x, double y, double z)
{
    e.X = x * c.k; e.Y = y * c.k; e.Z = z * c.k;
    e.ux = e.uy = e.uz = 0.f; e.cx = e.cy = e.cz = 0.f;
    e.tau0 = t0 * c.omega;
    const double tz = (c.window == 0) ? e.Z : 0.0;
    e.taue = tz + c.ta_n;
    e.n = 0;
    e.N = 0;
    if (!(e.tau0 >= tz - c.tb_n - c.hn)) return false;
    e.N = (int64_t)ceil((e.taue - e.tau0) / c.hn);
    return true;
}

template <int FIELD, class CFG>
__device__ inline void elec_step(const CFG& c, ElecMixed& e)
{
    const double h = c.hn;
    const double ta = e.tau0 + (double)e.n * h;
    const double hsd = (e.n == e.N - 1) ? (e.taue - ta) : h;
    const float hs = (float)hsd, hh = 0.5f * hs;
    const MixedBase b = mixed_base(c, ta, e.X, e.Y, e.Z);
    float kX, kY, kZ, kx, ky, kz, aX, aY, aZ, ax, ay, az;
    rhs_mixed<FIELD, true>(c, b, 0.f, kX, kY, kZ, e.ux, e.uy, e.uz, kx, ky, kz);
    aX = kX; aY = kY; aZ = kZ; ax = kx; ay = ky; az = kz;
    rhs_mixed<FIELD, false>(c, b, hh, kX, kY, kZ, e.ux + hh * kx, e.uy + hh * ky, e.uz + hh * kz,
                            kx, ky, kz);
    aX += 2.f * kX; aY += 2.f * kY; aZ += 2.f * kZ;
    ax += 2.f * kx; ay += 2.f * ky; az += 2.f * kz;
    rhs_mixed<FIELD, false>(c, b, hh, kX, kY, kZ, e.ux + hh * kx, e.uy + hh * ky, e.uz + hh * kz,
                            kx, ky, kz);
    aX += 2.f * kX; aY += 2.f * kY; aZ += 2.f * kZ;
    ax += 2.f * kx; ay += 2.f * ky; az += 2.f * kz;
    rhs_mixed<FIELD, false>(c, b, hs, kX, kY, kZ, e.ux + hs * kx, e.uy + hs * ky, e.uz + hs * kz,
                            kx, ky, kz);
    const double w6d = hsd * (1.0 / 6.0);
    const float w6 = hs * (1.0f / 6.0f);
    e.X += w6d * (double)(aX + kX); e.Y += w6d * (double)(aY + kY); e.Z += w6d * (double)(aZ + kZ);
    kahan_add(e.ux, e.cx, w6 * (ax + kx));
    kahan_add(e.uy, e.cy, w6 * (ay + ky));
    kahan_add(e.uz, e.cz, w6 * (az + kz));
    ++e.n;
}

template <class CFG>
__device__ inline void elec_final(const CFG& c, const ElecMixed& e, double& ux, double& uy,
                                  double& uz, double& xf, double& yf, double& zf)
{
    ux = (double)e.ux; uy = (double)e.uy; uz = (double)e.uz;
    xf = e.X * c.inv_k; yf = e.Y * c.inv_k; zf = e.Z * c.inv_k;
}

// ---------------------------------------------------------------------------
// Persistent push over one configuration.  A lane whose electron has reached
// its window end writes it out and takes the next slot from a global counter
// (one atomic per wave per refill, ranks from the ballot), so lanes stay busy
// however uneven the step counts are.  Unborn slots are written as NaN when
// taken.
// ---------------------------------------------------------------------------
struct PushIO {
    const double* tb; const double* x0; const double* y0; const double* z0;
    int32_t spa; int64_t n_slots;
    double* ux; double* uy; double* uz; double* xf; double* yf; double* zf;
    unsigned long long* queue;
    double* chi = nullptr;           // largest chi (radiation-reaction push), optional
    double* t_stop = nullptr;        // stop time [s] (controlled-step push), optional
    long long* n_acc = nullptr;      // accepted / rejected steps (controlled-step push)
    long long* n_rej = nullptr;
};

// Electron forms with outputs beyond momentum and position.
template <class E> struct HasExtra { static constexpr bool value = false; };
template <bool RR> struct HasExtra<ElecRR<RR>> { static constexpr bool value = true; };
template <> struct HasExtra<ElecDP> { static constexpr bool value = true; };

template <bool EXTRA>
__device__ inline void write_nan(const PushIO& io, int64_t j)
{
    const double q = __builtin_nan("");
    io.ux[j] = q; io.uy[j] = q; io.uz[j] = q; io.xf[j] = q; io.yf[j] = q; io.zf[j] = q;
    if (EXTRA) {
        if (io.chi) io.chi[j] = q;
        if (io.t_stop) io.t_stop[j] = q;
        if (io.n_acc) io.n_acc[j] = 0;
        if (io.n_rej) io.n_rej[j] = 0;
    }
}

// Per-electron extra outputs: nothing for the plain forms, chi for ElecRR,
// stop time and step counts for ElecDP.
template <class CFG, class E>
__device__ inline void elec_extra(const CFG&, const E&, const PushIO&, int64_t) {}

template <class CFG, bool RR>
__device__ inline void elec_extra(const CFG& c, const ElecRR<RR>& e, const PushIO& io, int64_t j)
{
    if (io.chi) io.chi[j] = c.chi_eta * sqrt(e.g2q);
}

template <class CFG>
__device__ inline void elec_extra(const CFG& c, const ElecDP& e, const PushIO& io, int64_t j)
{
    if (io.t_stop) io.t_stop[j] = e.failed ? __builtin_nan("") : e.tau * c.inv_omega;
    if (io.n_acc) io.n_acc[j] = e.acc;
    if (io.n_rej) io.n_rej[j] = e.rej;
}

// The single-configuration push splits its slots into kQueueParts contiguous
// parts, one counter each (kQueueStride words apart, one 128-byte line per
// counter).  A wave draws from the part of the XCD it runs on (the hardware
// XCC_ID register), so the slots of one part are read and written through one
// XCD's L2, where neighbouring slots share cache lines; lanes that find that
// part used up go on to the next parts in turn.
constexpr int kQueueParts = 8;
constexpr int kQueueStride = 16;
constexpr int kQueueWords = kQueueParts * kQueueStride;

__device__ inline int xcd_id()
{
    // hwreg(HW_REG_XCC_ID, 0, 4): id 20, offset 0, size 4
    return __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & (kQueueParts - 1);
}

// Wave-cooperative refill from the parts of [0, n): lanes with need == true
// get an index, or -1 when every part is used up (a part's counter only
// grows, so a part once used up stays so).
__device__ inline int64_t queue_take_xcd(unsigned long long* queue, int64_t n, bool need)
{
    const int home = xcd_id();
    int64_t got = -1;
    bool want = need;
#pragma unroll 1
    for (int m = 0; m < kQueueParts; ++m) {
        if (__ballot(want) == 0) break;
        const int part = (home + m) & (kQueueParts - 1);
        const int64_t j = queue_take(queue + part * kQueueStride, want);
        const int64_t lo = (n * part) >> 3, hi = (n * (part + 1)) >> 3;   // n / 8 parts
        if (want && j >= 0 && lo + j < hi) {
            got = lo + j;
            want = false;
        }
    }
    return got;
}

// Waves per SIMD each electron form is compiled for (its register budget):
// FP64 RK4 4 (5 needs a few spills and measured no faster), mixed 6 (lands
// at 7 without spills, 1-5% faster than 5), controlled-step unbounded (six
// stored stages, 2 waves).
template <class E> struct ElecWaves { static constexpr int value = 4; };
template <> struct ElecWaves<ElecMixed> { static constexpr int value = 7; };
template <> struct ElecWaves<ElecDP> { static constexpr int value = 1; };

template <int FIELD, class ELEC>
__global__ void __launch_bounds__(256, ElecWaves<ELEC>::value) push_kernel(DevCfg c, PushIO io)
{
    int64_t idx = -1;
    bool exhausted = false;
    ELEC e;
    e.n = e.N = 0;
    while (true) {
        // refill lanes without an electron (unborn slots are consumed here)
        while (true) {
            const bool need = (idx < 0) && !exhausted;
            if (__ballot(need) == 0) break;
            const int64_t j = queue_take_xcd(io.queue, io.n_slots, need);
            if (need && j < 0) exhausted = true;
            if (need && j >= 0) {
                const double t0 = io.tb[j];
                if (!(t0 < __builtin_inf())) {
                    write_nan<HasExtra<ELEC>::value>(io, j);
                } else {
                    const int64_t a = j / io.spa;
                    if (!elec_init(c, e, t0, io.x0[a], io.y0[a], io.z0[a])) {
                        write_nan<HasExtra<ELEC>::value>(io, j);
                        continue;
                    }
                    idx = j;
                    if (e.N <= 0) {
                        elec_final(c, e, io.ux[j], io.uy[j], io.uz[j], io.xf[j], io.yf[j],
                                   io.zf[j]);
                        elec_extra(c, e, io, j);
                        idx = -1;
                    }
                }
            }
        }
        if (__ballot(idx >= 0) == 0) break;
        if (idx >= 0) {
            elec_step<FIELD>(c, e);
            if (e.n == e.N) {
                elec_final(c, e, io.ux[idx], io.uy[idx], io.uz[idx], io.xf[idx], io.yf[idx],
                           io.zf[idx]);
                elec_extra(c, e, io, idx);
                idx = -1;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Histogram.  Each lane computes its bin key; lanes of a wave that share a
// key are merged (leader takes the key, ballot finds the matches, one atomic
// per distinct key); the six tallies are ballot-counted per wave.
// ---------------------------------------------------------------------------
struct HistArgs {
    int32_t nE, nA, angle;
    double lo, width;
    double mec2;  // electron rest energy [MeV]
};

// Bin key of one electron: >= 0 histogram cell index, or a negative tally code
// -(tally+1) for tallies 2..5; dir returned separately (0 fwd, 1 bwd, -1 none).
__device__ inline int64_t bin_key(const HistArgs& H, double tb, double ux, double uy, double uz,
                                  int& tally, int& dir)
{
#pragma clang fp contract(off)
    dir = -1;
    if (!(tb < __builtin_inf())) { tally = 4; return -1; }
    if (isnan(ux) || isnan(uy) || isnan(uz)) { tally = 5; return -1; }
    const double up2 = ux * ux + uy * uy;
    const double u2 = (ux * ux + uy * uy) + uz * uz;
    const double K = H.mec2 * u2 / (sqrt(1.0 + u2) + 1.0);
    dir = (uz > 0.0) ? 0 : 1;
    const double fe = floor((log10(K) - H.lo) / H.width);
    if (!(fe >= 0.0)) { tally = 2; return -1; }
    if (fe >= (double)H.nE) { tally = 3; return -1; }
    double fa;
    const double pi = 3.14159265358979323846;
    if (H.angle == 0) fa = floor(atan2(sqrt(up2), uz) / pi * (double)H.nA);
    else fa = floor((atan2(uy, ux) + pi) / (2.0 * pi) * (double)H.nA);
    int ia = (int)fa;
    ia = ia > H.nA - 1 ? H.nA - 1 : (ia < 0 ? 0 : ia);
    tally = -1;
    return ((int64_t)dir * H.nE + (int64_t)fe) * H.nA + ia;
}

// Add 1 at counter[key] for every lane with key >= 0, merging equal keys
// across the wave first: the lowest pending lane's key is broadcast, the
// lanes holding it are counted by ballot and one atomic adds the count.
// Called by every lane of the wave.
__device__ inline void wave_merge_add(int64_t key, unsigned long long* __restrict__ counter)
{
    const int lane = __lane_id();
    bool pending = key >= 0;
    while (true) {
        const uint64_t act = __ballot(pending);
        if (act == 0) break;
        const int leader = __ffsll((unsigned long long)act) - 1;
        const int64_t lk = __shfl(key, leader);
        const uint64_t same = __ballot(pending && key == lk);
        if (lane == leader) atomicAdd(&counter[lk], (unsigned long long)__popcll(same));
        if (pending && key == lk) pending = false;
    }
}

__device__ inline void wave_hist_commit(int64_t key, int tally, int dir,
                                        unsigned long long* __restrict__ counts,
                                        unsigned long long* __restrict__ tallies)
{
    const int lane = __lane_id();
    wave_merge_add(key, counts);
    // tallies: 0 fwd, 1 bwd, 2 below, 3 above, 4 unborn, 5 NaN
    const uint64_t t0 = __ballot(dir == 0), t1 = __ballot(dir == 1);
    const uint64_t t2 = __ballot(tally == 2), t3 = __ballot(tally == 3);
    const uint64_t t4 = __ballot(tally == 4), t5 = __ballot(tally == 5);
    if (lane == 0) {
        if (t0) atomicAdd(&tallies[0], (unsigned long long)__popcll(t0));
        if (t1) atomicAdd(&tallies[1], (unsigned long long)__popcll(t1));
        if (t2) atomicAdd(&tallies[2], (unsigned long long)__popcll(t2));
        if (t3) atomicAdd(&tallies[3], (unsigned long long)__popcll(t3));
        if (t4) atomicAdd(&tallies[4], (unsigned long long)__popcll(t4));
        if (t5) atomicAdd(&tallies[5], (unsigned long long)__popcll(t5));
    }
}

__global__ void __launch_bounds__(256) histogram_kernel(
    HistArgs H, int64_t n, const double* __restrict__ tb, const double* __restrict__ ux,
    const double* __restrict__ uy, const double* __restrict__ uz,
    unsigned long long* __restrict__ counts, unsigned long long* __restrict__ tallies)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    // wave-uniform trip count so every lane takes part in the ballots
    const int64_t base0 = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63);
    for (int64_t b = base0; b < n; b += stride) {
        const int64_t i = b + __lane_id();
        int64_t key = -1;
        int tally = -1, dir = -1;
        if (i < n) key = bin_key(H, tb[i], ux[i], uy[i], uz[i], tally, dir);
        wave_hist_commit(key, tally, dir, counts, tallies);
    }
}

// Two-dimensional forward/backward histogram: pair i adds 1 at
// counts[dir][ia][ib], dir 0 if uz > 0 else 1, ia = floor((a - a_lo)/wa),
// ib likewise; tallies[0] counts pairs outside the ranges, tallies[1] pairs
// with a NaN.  Same arithmetic, without contraction, as the definition.
struct Hist2dArgs {
    double a_lo, wa, b_lo, wb;
    int32_t na, nb;
};

__global__ void __launch_bounds__(256) histogram2d_kernel(
    Hist2dArgs H, int64_t n, const double* __restrict__ a, const double* __restrict__ b,
    const double* __restrict__ uz, unsigned long long* __restrict__ counts,
    unsigned long long* __restrict__ tallies)
{
#pragma clang fp contract(off)
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t base0 = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63);
    for (int64_t w = base0; w < n; w += stride) {
        const int64_t i = w + __lane_id();
        int64_t key = -1;
        int tally = -1;
        if (i < n) {
            const double av = a[i], bv = b[i], u = uz[i];
            if (isnan(av) || isnan(bv) || isnan(u)) {
                tally = 1;
            } else {
                const double fa = floor((av - H.a_lo) / H.wa);
                const double fb = floor((bv - H.b_lo) / H.wb);
                if (fa >= 0.0 && fa < (double)H.na && fb >= 0.0 && fb < (double)H.nb)
                    key = ((int64_t)(u > 0.0 ? 0 : 1) * H.na + (int64_t)fa) * H.nb + (int64_t)fb;
                else
                    tally = 0;
            }
        }
        wave_merge_add(key, counts);
        const uint64_t t0 = __ballot(tally == 0), t1 = __ballot(tally == 1);
        if (__lane_id() == 0) {
            if (t0) atomicAdd(&tallies[0], (unsigned long long)__popcll(t0));
            if (t1) atomicAdd(&tallies[1], (unsigned long long)__popcll(t1));
        }
    }
}

// Per-electron outputs: kinetic energy m c^2 u^2/(gamma + 1) [MeV], polar
// angle atan2(|u_perp|, u_z), azimuth atan2(u_y, u_x), forward flag u_z > 0.
// NaN momenta give NaN energy and angles and flag -1.
__global__ void __launch_bounds__(256) epilogue_kernel(
    int64_t n, double mec2, const double* __restrict__ ux, const double* __restrict__ uy,
    const double* __restrict__ uz, double* __restrict__ K, double* __restrict__ theta,
    double* __restrict__ psi, int32_t* __restrict__ fwd)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double x = ux[i], y = uy[i], z = uz[i];
    const double up2 = x * x + y * y;
    const double u2 = up2 + z * z;
    K[i] = mec2 * u2 / (sqrt(1.0 + u2) + 1.0);
    theta[i] = atan2(sqrt(up2), z);
    psi[i] = atan2(y, x);
    fwd[i] = (isnan(x) || isnan(y) || isnan(z)) ? -1 : (z > 0.0 ? 1 : 0);
}

__global__ void zero_u64_kernel(unsigned long long* p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

}  // namespace rpdla
