/*
 * rpdla.h -- C ABI of the MI355X (gfx950) library for the ionization-seeded
 * direct-laser-acceleration Monte Carlo of arXiv 2509.01741 ("Forward and
 * backward electron acceleration by radially polarized ultra-intense laser
 * focus seeded by field ionization of high charge states of neon").
 *
 * The path: neon atoms sampled over the focal volume (Sec. 2.1 "Ionization"),
 * field-ionized charge state by charge state with a semi-classical tunnelling
 * rate (Sec. 1, Sec. 2.1), every freed electron born at rest and pushed
 * through the radially polarized focus (Eqs. (1)-(2) and B_theta, with the
 * w0/z_r corrections of Sec. 2.1) by the Newton-Lorentz equations
 * (Eqs. (7)-(14)), then binned by final energy ((gamma-1) m c^2, text after
 * Eq. (14)) and emission angle, split forward / backward (Sec. 2.2).
 *
 * Conventions for every entry point:
 *   - SI units unless stated.
 *   - Array arguments are DEVICE pointers owned by the caller (for example
 *     torch tensors' data_ptr()).  The library never frees them and keeps no
 *     reference after the call has been enqueued.  Struct arguments
 *     (rpdla_laser, rpdla_hist_spec) are HOST pointers read during the call.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     Work is enqueued asynchronously on it; the call returns after
 *     validation and enqueue.  Faults inside kernels surface at the caller's
 *     next synchronization.
 *   - Every entry point validates its arguments before enqueueing anything
 *     and returns RPDLA_EINVAL (nothing enqueued) on bad input;
 *     rpdla_last_error() then holds a thread-local description.
 *   - No C++ exception crosses the ABI.  Calls are reentrant; two calls on
 *     different streams may run concurrently.
 *   - Random numbers: Philox4x64-10 (Salmon et al., SC'11) with key
 *     (seed, cfg_id) and counter (atom index, j/4, 0, 0), word j%4, mapped to
 *     (m+1) 2^-53 with m the top 53 bits.  Stream j = 0, 1, 2 places the atom;
 *     j = k + 2 is the Exp(1) threshold -ln u of charge state k.  Any atom
 *     range therefore gives the same numbers however the ensemble is split.
 */
#ifndef RPDLA_H
#define RPDLA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RPDLA_OK = 0,
    RPDLA_EINVAL = -1,       /* invalid argument; nothing enqueued            */
    RPDLA_ERANGE = -2,       /* size out of the supported range                */
    RPDLA_EHIP = -3,         /* HIP runtime error at launch / allocation       */
    RPDLA_ENOMEM = -4,       /* workspace too small or allocation failed       */
    RPDLA_EUNSUPPORTED = -5  /* combination not implemented                    */
} rpdla_status;

/* Field model.  RP_O1/O3/O5: radially polarized TM01 focus truncated at
 * order 1, 3, 5 of the series in eps = w0/z_r (order 1 is Eqs. (1)-(2) of
 * Sec. 2.1 with the Maxwell-consistent Ez sign; orders 3 and 5 are the
 * non-paraxial corrections the same section names).  LP_O1/O3/O5: the
 * linearly polarized focus of Sec. 2.2's comparison (Fig. 4), polarized along
 * x: the same Lax series psi = psi0 + eps^2 psi2 + eps^4 psi4 (truncated
 * after psi0, psi2, psi4) under the vector potential x^ (i A/omega) psi
 * e^{i(omega t - k z + phi0)}, fields from E = -grad phi - dA/dt (Lorenz
 * gauge) and B = curl A, times the same envelope; A is the peak field at the
 * focus, so the amplitude from intensity gives peak intensity I.  Double
 * precision forms only (RPDLA_EUNSUPPORTED for the mixed push and for
 * rpdla_birth_phase).  The rest are test models: PLANE_LP,
 * Ex = A env cos(omega t - k z + phi0), By = Ex/c; UNIFORM_EB, static fields
 * test_E, test_B. */
typedef enum {
    RPDLA_RP_O1 = 1, RPDLA_RP_O3 = 3, RPDLA_RP_O5 = 5,
    RPDLA_PLANE_LP = 10, RPDLA_UNIFORM_EB = 11,
    RPDLA_LP_O1 = 21, RPDLA_LP_O3 = 23, RPDLA_LP_O5 = 25
} rpdla_field;

typedef enum { RPDLA_FP64 = 0, RPDLA_MIXED = 1 } rpdla_precision;

/* Integration window of an atom at axial position z: ARRIVAL,
 * [z/c - t_before, z/c + t_after] (around the pulse's arrival at the atom);
 * LAB, [-t_before, t_after]. */
typedef enum { RPDLA_WIN_ARRIVAL = 0, RPDLA_WIN_LAB = 1 } rpdla_window;

typedef enum { RPDLA_ANG_POLAR = 0, RPDLA_ANG_AZIMUTH = 1 } rpdla_angle;

/* One laser configuration (SI).  Filled by rpdla_laser_init_*, then editable. */
typedef struct {
    double lambda;      /* wavelength [m]                                          */
    double w0;          /* waist radius r0 [m]; z_r = k w0^2 / 2                   */
    double tau_fwhm;    /* intensity FWHM [s]; envelope exp(-(t-z/c)^2/tau0^2),
                           tau0 = tau_fwhm / sqrt(2 ln 2)                          */
    double amp;         /* A, the E0 of Eq. (1) [V/m]                              */
    double phi0;        /* carrier phase: cos(omega t - k z + ... + phi0)          */
    int32_t field;      /* rpdla_field                                             */
    int32_t window;     /* rpdla_window                                            */
    double t_before;    /* window start before the reference time [s]; default 5 tau */
    double t_after;     /* window end after the reference time [s]; default 10 tau */
    double dt;          /* RK4 step and ionization panel width [s]; default T/200  */
    double ez_scale;    /* multiplies Ez (Sec. 2.2, Fig. 9 study); default 1       */
    double er_scale;    /* multiplies Ex, Ey; default 1                            */
    double test_E[3];   /* UNIFORM_EB only [V/m]                                   */
    double test_B[3];   /* UNIFORM_EB only [T]                                     */
} rpdla_laser;

/* Energy-angle histogram layout: counts[dir][iE][iA], dir 0 forward (u_z > 0
 * at the end of the window), 1 backward; iE = floor((log10 K[MeV] -
 * logE_min_MeV) / width) with width = (logE_max - logE_min)/nE; iA over
 * [0, pi] (POLAR, atan2(|u_perp|, u_z)) or (-pi, pi] (AZIMUTH, atan2(u_y,
 * u_x), Sec. 2.2 Fig. 5), top edge folded into the last bin.  Energies
 * outside the range go to tallies, not to the edge bins. */
typedef struct {
    int32_t nE, nA;
    double logE_min_MeV, logE_max_MeV;
    int32_t angle;      /* rpdla_angle */
} rpdla_hist_spec;

/* Tallies, uint64[6]: 0 forward, 1 backward (born, finite), 2 below the energy
 * range, 3 above it, 4 unborn slots, 5 born slots with a NaN momentum. */
#define RPDLA_NTALLY 6

/* ------------------------------------------------------------------------
 * Laser set-up (host only, no device work).
 * Intensity: A = sqrt(2 I / (eps0 c)), the Gaussian-equivalent field Sec. 2.1
 * attaches to every quoted intensity (5e19 W/cm^2 -> 1.94e13 V/m).
 * Power: A = sqrt(8 P / (pi w0^2 eps0 c)), the order-1 beam's power.
 * Defaults: field RP_O5, window ARRIVAL, t_before 5 tau, t_after 10 tau,
 * dt = lambda/(200 c), phi0 0, unit scales.  EINVAL on non-positive input.
 * ------------------------------------------------------------------------ */
rpdla_status rpdla_laser_init_intensity(rpdla_laser* L, double lambda, double w0,
                                        double tau_fwhm, double I_W_cm2);
rpdla_status rpdla_laser_init_power(rpdla_laser* L, double lambda, double w0,
                                    double tau_fwhm, double P_W);

/* Rayleigh length z_r = k w0^2 / 2 [m] (definition under Eq. (2)). */
double rpdla_rayleigh(const rpdla_laser* L);

/* ------------------------------------------------------------------------
 * Atom sampling (Sec. 2.1: ions at rest, uniform in a cylinder about the
 * propagation axis, focus at the origin).  Atom i = first_atom + j:
 * r = r_max sqrt(u0), azimuth 2 pi u1, z = z_half (2 u2 - 1).
 * x, y, z: device double[n_atoms], written.  EINVAL: n_atoms < 0, null
 * pointers with n_atoms > 0, r_max or z_half negative or non-finite.
 * ------------------------------------------------------------------------ */
rpdla_status rpdla_sample_atoms(uint64_t seed, uint32_t cfg_id, uint64_t first_atom,
                                int64_t n_atoms, double r_max, double z_half,
                                double* x, double* y, double* z, void* stream);

/* Hollow / annular variant (Sec. 2.2, Fig. 8: ions uniform on the surface of
 * a hollow cylinder of radius 0..4 um): r uniform in area between r_in and
 * r_out, r = r_out exactly when r_in == r_out; same random streams as
 * rpdla_sample_atoms.  EINVAL unless 0 <= r_in <= r_out, z_half >= 0. */
rpdla_status rpdla_sample_atoms_annulus(uint64_t seed, uint32_t cfg_id, uint64_t first_atom,
                                        int64_t n_atoms, double r_in, double r_out,
                                        double z_half, double* x, double* y, double* z,
                                        void* stream);

/* ------------------------------------------------------------------------
 * Ionization times (Sec. 2.1 "Ionization": charge states freed one after
 * another, t0 the birth time).  For atom i (index first_atom + j, position
 * x[j], y[j], z[j]) and states k = k_first..k_last in order, state k is born
 * when the integral of the static ADK rate w_k(|E(x_i, t)|) since the previous
 * birth (the window start for k_first) reaches -ln u_{k+2}; the integral is
 * GL-4 on panels of width dt laid from the window start, the crossing solved
 * inside its panel by bracketed Newton.  ADK: l = m = 0, l* = n* - 1, neon
 * potentials, w = 0 where ln w[1/s] < -700.
 * t_birth: device double[n_atoms * K], K = k_last - k_first + 1, atom-major
 * (slot j*K + (k - k_first)), seconds, +INF where the state is not reached
 * in the window.  A state whose rate, bounded through the field's envelope,
 * cannot reach its threshold within the window is left unborn without
 * integrating its panels (the same result).  From 16384 atoms on, the atoms
 * are taken in an order that groups similar work in each wave (a sort by the
 * number of states that bound leaves open, then by the peak-field bound),
 * which needs stream-ordered scratch of about 16 bytes per atom
 * (hipMallocAsync / hipFreeAsync on `stream`); results do not depend on the
 * order.  EINVAL: bad
 * laser, 1 <= k_first <= k_last <= 10 violated, null pointers with
 * n_atoms > 0.
 * ------------------------------------------------------------------------ */
rpdla_status rpdla_ionize(const rpdla_laser* L, uint64_t seed, uint32_t cfg_id,
                          uint64_t first_atom, int64_t n_atoms, const double* x,
                          const double* y, const double* z, int32_t k_first,
                          int32_t k_last, double* t_birth, void* stream);

/* Laser phase and radius at each birth (Sec. 2.2, Figs. 6, 13, 14: the phase
 * of the laser coincident with the birth and the distance of the parent ion
 * from the axis), using the phase defined under Eq. (2):
 * k z - omega t - 2 atan(z/z_r) + z r^2 / (z_r w0^2 f^2) + phi0_paper, with
 * phi0_paper = -L->phi0, reduced to [0, 2 pi).  Slot s belongs to atom
 * s / slots_per_atom (positions x, y, z [m], device double[n_atoms]); t_birth
 * as from rpdla_ionize.  phase: device double[n_slots] out; r_birth: device
 * double[n_slots] out [m] or NULL; both NaN for unborn slots.  EINVAL: bad
 * laser, n_slots < 0, slots_per_atom < 1, null pointers with n_slots > 0. */
rpdla_status rpdla_birth_phase(const rpdla_laser* L, int64_t n_slots, const double* t_birth,
                               const double* x, const double* y, const double* z,
                               int32_t slots_per_atom, double* phase, double* r_birth,
                               void* stream);

/* ------------------------------------------------------------------------
 * Push (Eqs. (7)-(14), radiation reaction dropped as in the paper below
 * 5e22 W/cm^2).  Slot s belongs to atom s / slots_per_atom, whose position is
 * x0/y0/z0[s / slots_per_atom]; the electron starts at rest there at
 * t_birth[s] and is advanced by classical RK4 with fixed step dt (steps
 * start at t_birth + n dt, the last one ends on the window end) to the end
 * of its atom's window.  u = p/(m c).
 * Outputs, device double[n_slots]: ux, uy, uz and final position xf, yf, zf
 * [m]; all six NaN for unborn slots (t_birth = +INF or NaN) and for births
 * earlier than one step before the window start (invalid input; this also
 * bounds every lane's step count).
 * precision RPDLA_FP64: everything in double.  RPDLA_MIXED: field and RK4
 * stages in float; time, position and the carrier phase in double (phase
 * reduced to one turn before the float sine / cosine); momentum accumulated
 * in float with Kahan compensation.
 * EINVAL: bad laser, n_slots < 0, slots_per_atom < 1, null pointers with
 * n_slots > 0.  Uses a small stream-ordered device allocation (1 KiB) for its
 * work queue (RPDLA_EHIP if that fails): the slots are split into eight
 * contiguous parts with a counter each, and a wave draws from the part of the
 * XCD it runs on (the hardware XCC_ID register) before it moves on to the
 * others, so the slots of one part pass through one XCD's L2; results do not
 * depend on it.
 * ------------------------------------------------------------------------ */
rpdla_status rpdla_push(const rpdla_laser* L, int32_t precision, int64_t n_slots,
                        const double* t_birth, const double* x0, const double* y0,
                        const double* z0, int32_t slots_per_atom, double* ux, double* uy,
                        double* uz, double* xf, double* yf, double* zf, void* stream);

/* ------------------------------------------------------------------------
 * Allocation-free push, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, validation, kernels and results as rpdla_push;
 * it calls no hipMalloc / hipFree and no allocating library routine.  Its
 * work-queue counters live in a 1 KiB library-owned device array (one per
 * GPU, held until the process ends, its address looked up on the first call
 * on each device), cleared by a fill kernel at the start of every call.
 * Limit: n_slots <= 2^40 (RPDLA_ERANGE beyond).  Every call on one GPU uses
 * that GPU's array, so calls that overlap in time on one GPU (different
 * streams, or several host threads) race on the counters and give wrong
 * results: serialize them.  RPDLA_EHIP if the array's address cannot be
 * obtained.
 * ------------------------------------------------------------------------ */
rpdla_status rpdla_push_noalloc(const rpdla_laser* L, int32_t precision, int64_t n_slots,
                                const double* t_birth, const double* x0, const double* y0,
                                const double* z0, int32_t slots_per_atom, double* ux,
                                double* uy, double* uz, double* xf, double* yf, double* zf,
                                void* stream);

/* ------------------------------------------------------------------------
 * Push with the radiation term of Eq. (3) and the quantum parameter of
 * Eqs. (4)-(6) (Sec. 2.1).  Same slots, window, RK4 steps and outputs as
 * rpdla_push in RPDLA_FP64, with
 *   radiation_reaction = 1: the gamma^2 Landau-Lifshitz term added to the
 *     Lorentz force, -(e^4 gamma^2 / (6 pi eps0 m^2 c^5)) v [(E + v x B)^2 -
 *     (v.E)^2/c^2] (SI form of Eq. (3), whose printed coefficient is read as
 *     the Gaussian 2 e^4 gamma^2 / (3 m^2 c^5));
 *   radiation_reaction = 0: the plain Lorentz force.
 * chi_max: device double[n_slots] out, or NULL: per electron the largest
 * chi = (gamma / E_cr) sqrt((E + v x B)^2 - (v.E)^2/c^2), E_cr = m^2 c^3 /
 * (e hbar), over the starts of its RK4 steps (0 if it takes none, NaN for
 * unborn and invalid slots).  The classical radiation parameter of Eq. (6)
 * is Rc = alpha a0 chi, a0 = e A / (m c omega).
 * EINVAL: bad laser, radiation_reaction not 0 or 1, n_slots < 0,
 * slots_per_atom < 1, null pointers (other than chi_max) with n_slots > 0.
 * Uses a small stream-ordered device allocation for its work queue.
 * ------------------------------------------------------------------------ */
rpdla_status rpdla_push_rr(const rpdla_laser* L, int32_t radiation_reaction, int64_t n_slots,
                           const double* t_birth, const double* x0, const double* y0,
                           const double* z0, int32_t slots_per_atom, double* ux, double* uy,
                           double* uz, double* xf, double* yf, double* zf, double* chi_max,
                           void* stream);

/* ------------------------------------------------------------------------
 * Controlled-step push (Sec. 1 and Sec. 2.1: a fifth-order Runge-Kutta method
 * with a controlled, attosecond-range step, electrons followed until their
 * kinetic energy is constant).  Same slots, window, birth rules and outputs
 * as rpdla_push (FP64), integrated with the Dormand-Prince 5(4) pair: the
 * fifth-order result is carried, the last stage reused as the next first.
 * A step's error is the largest over (k x, k y, k z, ux, uy, uz) of
 * |y5 - y4| / (atol + rtol max(|y_n|, |y_n+1|)); accepted when <= 1; the
 * next step is h min(5, max(0.2, 0.9 err^(-1/5))), at most h_max and never
 * past the window end; the first step is L->dt.  The electron stops at the
 * window end, or at the first accepted step end at least 0.999 optical period
 * after the previous check where gamma changed by at most k_tol (relative;
 * k_tol < 0: never early).  More than max_steps attempted steps, or a step
 * whose error estimate is not a number: NaN outputs.
 * t_stop: device double[n_slots] out [s] or NULL (NaN for unborn, invalid or
 * failed slots); steps_accepted / steps_rejected: device int64[n_slots] out
 * or NULL (0 for unborn slots).
 * EINVAL: bad laser, NULL A, rtol or atol negative or both 0, non-finite
 * h_max or k_tol, max_steps < 1, n_slots < 0, slots_per_atom < 1, null
 * pointers (other than the optional outputs) with n_slots > 0.  Uses a small
 * stream-ordered device allocation for its work queue.
 * ------------------------------------------------------------------------ */
typedef struct {
    double rtol, atol;    /* error tolerances (dimensionless); e.g. 1e-9, 1e-9   */
    double h_max;         /* largest step [s]; <= 0: 10 L->dt                    */
    double k_tol;         /* constant-energy tolerance; e.g. 1e-10; < 0: never   */
    int64_t max_steps;    /* attempted steps allowed per electron (>= 1)         */
} rpdla_adaptive;

rpdla_status rpdla_push_adaptive(const rpdla_laser* L, const rpdla_adaptive* A, int64_t n_slots,
                                 const double* t_birth, const double* x0, const double* y0,
                                 const double* z0, int32_t slots_per_atom, double* ux, double* uy,
                                 double* uz, double* xf, double* yf, double* zf, double* t_stop,
                                 int64_t* steps_accepted, int64_t* steps_rejected, void* stream);

/* ------------------------------------------------------------------------
 * Per-electron outputs (text after Eq. (14); Sec. 2.2, Fig. 5): kinetic
 * energy K = m c^2 u^2 / (gamma + 1) [MeV] (= (gamma - 1) m c^2 without
 * cancellation), polar emission angle theta = atan2(|u_perp|, u_z), azimuth
 * psi = atan2(u_y, u_x), forward flag 1 if u_z > 0 else 0 (-1 for NaN momenta,
 * e.g. unborn slots, whose K, theta, psi are NaN).
 * ux, uy, uz: device double[n] in; K_MeV, theta, psi: device double[n] out;
 * fwd: device int32[n] out.  EINVAL: n < 0, null pointers with n > 0.
 * ------------------------------------------------------------------------ */
rpdla_status rpdla_epilogue(int64_t n, const double* ux, const double* uy, const double* uz,
                            double* K_MeV, double* theta, double* psi, int32_t* fwd,
                            void* stream);

/* ------------------------------------------------------------------------
 * Energy-angle histogram of n_slots electrons (see rpdla_hist_spec).
 * t_birth (to recognise unborn slots), ux, uy, uz: device double[n_slots].
 * counts: device uint64[2 * nE * nA] and tallies: device uint64[6], both
 * ACCUMULATED into (clear them first for a fresh histogram).  Wave-level
 * aggregation before the global atomics.  EINVAL: nE, nA < 1, min >= max,
 * null pointers.
 * ------------------------------------------------------------------------ */
rpdla_status rpdla_histogram(int64_t n_slots, const double* t_birth, const double* ux,
                             const double* uy, const double* uz, const rpdla_hist_spec* spec,
                             uint64_t* counts, uint64_t* tallies, void* stream);

/* Two-dimensional histogram of pairs (a[i], b[i]) split by the direction of
 * final motion: the birth phase x birth radius maps of forward and backward
 * electrons (Sec. 2.2, Figs. 13, 14) or a birth variable against the final
 * energy (Fig. 6).  Pair i adds 1 at counts[dir][ia][ib], dir 0 if uz[i] > 0
 * else 1, ia = floor((a - a_lo) / ((a_hi - a_lo) / na)), ib likewise, each
 * bin half-open [lo, lo + width); tallies[0] counts pairs outside either range,
 * tallies[1] pairs with a NaN in a, b or uz (unborn slots).  a, b, uz: device
 * double[n]; counts: device uint64[2 * na * nb], tallies: device uint64[2],
 * both ACCUMULATED into.  EINVAL: na, nb < 1, lo >= hi or non-finite, null
 * pointers; ERANGE: na * nb > 2^28. */
typedef struct {
    int32_t na, nb;
    double a_lo, a_hi, b_lo, b_hi;
} rpdla_hist2d_spec;

rpdla_status rpdla_histogram2d(int64_t n, const double* a, const double* b, const double* uz,
                               const rpdla_hist2d_spec* spec, uint64_t* counts, uint64_t* tallies,
                               void* stream);

/* ------------------------------------------------------------------------
 * Batched sweep: n_cfg laser configurations (host array cfgs[n_cfg]), each
 * with atoms_per_cfg atoms sampled uniformly in r < r_factor * w0,
 * |z| < z_r, RNG key (seed, cfg_base + c) for configuration c, charge states
 * k_first..k_last.  Atoms are processed in chunks of atoms_per_chunk per
 * configuration; each chunk runs sample -> ionize -> push -> histogram, the
 * push as ONE persistent launch over every configuration's electrons: every
 * configuration has its own work counter, each wave serves one configuration
 * at a time (its constants read with scalar loads from the configuration
 * table) and moves to another with work left when its own runs dry; lanes are
 * refilled as their electron finishes.
 * On a non-null stream that is not being captured, the chunk's launch
 * sequence is captured once in a hipGraph (the chunk index advances in device
 * memory) and replayed per chunk, one chunk included; graphs are cached per
 * argument set for the process lifetime (up to 32; further argument sets are
 * enqueued directly).  On the null stream or a capturing stream the launches
 * are enqueued directly.
 * counts: device uint64[n_cfg][2][nE][nA], tallies: device uint64[n_cfg][6],
 * accumulated; electron_steps: device uint64[n_cfg] (accumulated) receiving
 * the number of RK4 steps taken per configuration, or NULL.  The chunk's
 * final momenta are binned by a separate wave-merged histogram pass.
 * workspace: device memory of at least
 * rpdla_batched_workspace_bytes(n_cfg, atoms_per_chunk, k_first, k_last)
 * bytes, 256-byte aligned, owned by the caller, not touched by other work
 * until the stream reaches the end of this call.
 * EINVAL on bad configurations or sizes; RPDLA_ENOMEM when ws_bytes is too
 * small; RPDLA_EUNSUPPORTED for n_cfg > 64.
 * ------------------------------------------------------------------------ */
size_t rpdla_batched_workspace_bytes(int32_t n_cfg, int64_t atoms_per_chunk, int32_t k_first,
                                     int32_t k_last);

/* Where the last chunk's particle data sits in the workspace once
 * rpdla_run_batched has completed on its stream: byte offsets[7] of
 * x, y, z (double[n_cfg][atoms_per_chunk], m), t_birth, ux, uy, uz
 * (double[n_cfg][atoms_per_chunk][K], K = k_last - k_first + 1), atom a of
 * configuration c being atom chunk_start + a of that configuration.  Entries
 * past atoms_per_cfg in a partial last chunk, and the momenta of unborn
 * slots, are not written (stale).  The layout depends only on the sizes.
 * EINVAL: NULL offsets, invalid sizes. */
#define RPDLA_WS_NARRAYS 7
rpdla_status rpdla_batched_workspace_layout(int32_t n_cfg, int64_t atoms_per_chunk,
                                           int32_t k_first, int32_t k_last, size_t* offsets);
/* Number of chunk graphs the library holds (captured by rpdla_run_batched,
 * kept until the process ends, at most 32).  Host only, no device work. */
int32_t rpdla_batched_graphs(void);

rpdla_status rpdla_run_batched(const rpdla_laser* cfgs, int32_t n_cfg, uint64_t seed,
                               uint32_t cfg_base, int64_t atoms_per_cfg, int64_t atoms_per_chunk,
                               double r_factor, int32_t k_first, int32_t k_last,
                               int32_t precision, const rpdla_hist_spec* spec,
                               uint64_t* counts, uint64_t* tallies, uint64_t* electron_steps,
                               void* workspace, size_t ws_bytes, void* stream);

/* The chunks first_chunk .. first_chunk + n_chunks - 1 of the same stream
 * (n_chunks = -1: to its end), so that a long sweep can be run, timed or
 * checked in parts: chunk c covers atoms c * atoms_per_chunk onwards of every
 * configuration, exactly as in rpdla_run_batched, and counts, tallies and
 * electron_steps accumulate, so consecutive ranges add up to one whole call.
 * Arguments otherwise as rpdla_run_batched; EINVAL when the range leaves the
 * stream's cdiv(atoms_per_cfg, atoms_per_chunk) chunks. */
rpdla_status rpdla_run_batched_range(const rpdla_laser* cfgs, int32_t n_cfg, uint64_t seed,
                                     uint32_t cfg_base, int64_t atoms_per_cfg,
                                     int64_t atoms_per_chunk, int64_t first_chunk,
                                     int64_t n_chunks, double r_factor, int32_t k_first,
                                     int32_t k_last, int32_t precision,
                                     const rpdla_hist_spec* spec, uint64_t* counts,
                                     uint64_t* tallies, uint64_t* electron_steps,
                                     void* workspace, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Launch-shape autotuning.  Kernel kinds: 0 push, 1 ionize, 2 batched push.
 * A launch shape is the number of threads per block (64, 128, 192, 256) and,
 * for the persistent push kernels, a factor on the resident-block count of
 * the grid (1..8).  Shapes live in a process-wide table keyed by (kind,
 * field model, precision; ionize ignores precision), default 256 x 1, and
 * are read by every later launch.  Results never depend on the shape.
 *
 * rpdla_autotune samples a probe ensemble of n_atoms (64..2^24) for laser L
 * and states k_first..k_last, times ionize for each block size and the push
 * and the one-configuration batched push for each block size x grid factor
 * 1, 2 (one untimed call before each timed one, HIP events on `stream`),
 * stores the fastest shapes, and writes a JSON report of all timings to
 * `report` (host buffer of report_len bytes, NUL-terminated, may be NULL).
 * It allocates and frees its own probe buffers (hipMalloc) and synchronizes
 * `stream` before returning.  rpdla_set_launch_shape / rpdla_get_launch_shape
 * store / read one entry (for example to re-apply a saved report).
 * ------------------------------------------------------------------------ */
rpdla_status rpdla_autotune(const rpdla_laser* L, int32_t precision, int64_t n_atoms,
                            int32_t k_first, int32_t k_last, char* report, size_t report_len,
                            void* stream);
rpdla_status rpdla_set_launch_shape(int32_t kernel, int32_t field, int32_t precision,
                                    int32_t block, int32_t grid_factor);
rpdla_status rpdla_get_launch_shape(int32_t kernel, int32_t field, int32_t precision,
                                    int32_t* block, int32_t* grid_factor);

/* Resources and occupancy of one kernel (kinds as above; field 1, 3, 5, 10 or
 * 11; precision RPDLA_FP64 or RPDLA_MIXED, ignored for ionize) on the current
 * device, at its current launch shape: vector registers per lane (*vgprs),
 * private scratch bytes per lane (*scratch_bytes, nonzero only when registers
 * spill) and resident waves per SIMD (*waves_per_simd, from the runtime's
 * occupancy query; a CU has four SIMDs).  The batched push is sized with the
 * per-configuration step counters of 64 configurations in LDS.  Field 21, 23
 * or 25 (linear focus) is accepted for the FP64 forms.  Host pointers, all
 * non-NULL; RPDLA_EINVAL
 * otherwise, RPDLA_EHIP when the runtime query fails. */
rpdla_status rpdla_kernel_occupancy(int32_t kernel, int32_t field, int32_t precision,
                                    int32_t* vgprs, int32_t* scratch_bytes,
                                    double* waves_per_simd);

/* Status text and the calling thread's last error detail (never NULL). */
const char* rpdla_status_string(rpdla_status s);
const char* rpdla_last_error(void);

/* Library version string. */
const char* rpdla_version(void);

#ifdef __cplusplus
}
#endif

#endif /* RPDLA_H */
