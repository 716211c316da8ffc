// rpdla_api.hip -- host side of the C ABI declared in include/rpdla.h:
// argument validation, the per-configuration constants in normalized units,
// kernel dispatch and launch shapes.
#include <hip/hip_runtime.h>
#include <hipcub/device/device_radix_sort.hpp>

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include <type_traits>

#include "rpdla.h"
#include "rpdla_kernels.hpp"
#include "rpdla_batched.hpp"

// Scratch of the allocation-free push (rpdla_push_noalloc): its work-queue
// counters (one per queue part, each on its own 128-byte line), 1 KiB.  Each
// GPU holds its own copy until the process ends.
constexpr int kScratchWords = rpdla::kQueueWords;
static_assert(rpdla::kQueueParts == 8, "queue_take_xcd splits the slots with a shift by 3");
static __device__ __align__(256) unsigned long long scratch[kScratchWords];

namespace {

using rpdla::DevCfg;

// CODATA 2018 (SI).
constexpr double kC = 299792458.0;
constexpr double kQe = 1.602176634e-19;
constexpr double kMe = 9.1093837015e-31;
constexpr double kEps0 = 8.8541878128e-12;
constexpr double kMeC2MeV = 0.51099895000;
constexpr double kEa = 5.14220674763e11;       // atomic unit of field [V/m]
constexpr double kTauA = 2.4188843265857e-17;  // atomic unit of time [s]
constexpr double kEhEv = 27.211386245988;      // Hartree [eV]
constexpr double kPi = 3.14159265358979323846;
constexpr double kHbar = 1.054571817e-34;        // reduced Planck constant [J s]
// Ionization panels are skipped where a rigorous bound keeps ln w (per unit
// normalized time) below this level: over a window of at most 1e5 normalized
// time units the skipped part of any survival integral is below 1e5 e^-80
// = 2e-30, far under the rounding of the integrals (targets -ln u >= 1e-16).
constexpr double kLnwSkip = -80.0;

// Neon ionization potentials Ne^(k-1)+ -> Ne^k+ [eV] (NIST ASD).
constexpr double kNeIpEv[10] = {21.564540, 40.96297, 63.4233, 97.1900, 126.247,
                                157.934,   207.271,  239.0970, 1195.80784, 1362.19911};

// Largest slot count of one push call.
constexpr int64_t kMaxPushSlots = (int64_t)1 << 40;
// Below this many atoms the ionization runs in the caller's order (sorting
// the atoms by work would cost more than it saves).
constexpr int64_t kIonizeSortMin = 16384;

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

thread_local std::string g_err;

rpdla_status fail(rpdla_status s, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

#define RPDLA_HIP(call)                                                                  \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess) return fail(RPDLA_EHIP, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

bool is_fin(double v) { return isfinite(v) != 0; }

// Linearly polarized focus (orders 1, 3, 5): double-precision forms only.
bool is_lp(int field) { return field == RPDLA_LP_O1 || field == RPDLA_LP_O3 || field == RPDLA_LP_O5; }

rpdla_status check_laser(const rpdla_laser* L)
{
    if (!L) return fail(RPDLA_EINVAL, "laser is NULL");
    if (!(is_fin(L->lambda) && L->lambda > 0)) return fail(RPDLA_EINVAL, "lambda must be > 0");
    if (!(is_fin(L->w0) && L->w0 > 0)) return fail(RPDLA_EINVAL, "w0 must be > 0");
    if (!(is_fin(L->tau_fwhm) && L->tau_fwhm > 0)) return fail(RPDLA_EINVAL, "tau_fwhm must be > 0");
    if (!(is_fin(L->amp) && L->amp >= 0)) return fail(RPDLA_EINVAL, "amp must be >= 0");
    if (!(is_fin(L->dt) && L->dt > 0)) return fail(RPDLA_EINVAL, "dt must be > 0");
    if (!(is_fin(L->t_before) && is_fin(L->t_after) && L->t_before > 0 && L->t_after > 0))
        return fail(RPDLA_EINVAL, "window must contain the pulse peak (t_before, t_after > 0)");
    if (!(is_fin(L->phi0) && is_fin(L->ez_scale) && is_fin(L->er_scale)))
        return fail(RPDLA_EINVAL, "phi0 and the field scales must be finite");
    const int f = L->field;
    if (!(f == RPDLA_RP_O1 || f == RPDLA_RP_O3 || f == RPDLA_RP_O5 || f == RPDLA_PLANE_LP ||
          f == RPDLA_UNIFORM_EB || is_lp(f)))
        return fail(RPDLA_EINVAL, "unknown field model %d", f);
    if (!(L->window == RPDLA_WIN_ARRIVAL || L->window == RPDLA_WIN_LAB))
        return fail(RPDLA_EINVAL, "unknown window %d", L->window);
    for (int i = 0; i < 3; ++i)
        if (!(is_fin(L->test_E[i]) && is_fin(L->test_B[i])))
            return fail(RPDLA_EINVAL, "test fields must be finite");
    const double panels = (L->t_before + L->t_after) / L->dt;
    if (!(panels < 2.0e9)) return fail(RPDLA_ERANGE, "window / dt = %.3g steps is too many", panels);
    return RPDLA_OK;
}

// Rate ln w[normalized] = c0 - c1h ln a2 - c2 a2^(-1/2); |a|^2 where it first
// reaches `level` on its rising branch (INF if it never does).
double adk_threshold_a2(double c0, double c1h, double c2, double level)
{
    auto f = [&](double la2) { return c0 - c1h * la2 - c2 * exp(-0.5 * la2); };
    double hi = (c1h > 0) ? 2.0 * log(0.5 * c2 / c1h) : 300.0;  // ln a2 at the rate's peak
    if (hi > 300.0) hi = 300.0;
    if (f(hi) < level) return INFINITY;
    double lo = -300.0;
    if (f(lo) >= level) return 0.0;
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (f(mid) < level) lo = mid; else hi = mid;
    }
    return exp(lo);
}

DevCfg make_cfg(const rpdla_laser* L)
{
    DevCfg c;
    memset(&c, 0, sizeof c);
    const double k = 2.0 * kPi / L->lambda;
    const double om = kC * k;
    const double w0n = k * L->w0;
    const double zrn = 0.5 * w0n * w0n;  // k z_r, z_r = k w0^2 / 2
    const double tau0 = L->tau_fwhm / sqrt(2.0 * log(2.0));
    c.omega = om; c.inv_omega = 1.0 / om;
    c.k = k; c.inv_k = 1.0 / k;
    c.a0 = kQe * L->amp / (kMe * kC * om);
    c.inv_w0n2 = 1.0 / (w0n * w0n);
    c.inv_w0n = 1.0 / w0n;
    c.inv_zrn = 1.0 / zrn;
    c.eps = 2.0 / w0n;
    c.e2 = c.eps * c.eps; c.e3 = c.e2 * c.eps; c.e4 = c.e2 * c.e2;
    c.inv_T0n = 1.0 / (om * tau0);
    c.phi0 = L->phi0;
    c.hn = om * L->dt;
    c.tb_n = om * L->t_before;
    c.ta_n = om * L->t_after;
    c.er_scale = L->er_scale; c.ez_scale = L->ez_scale;
    c.er_w = c.er_scale * c.inv_w0n; c.ez_e = c.ez_scale * c.eps;
    c.a0_w = c.a0 * c.inv_w0n; c.ez_2 = 2.0 * c.ez_scale;
    for (int i = 0; i < 3; ++i) {
        c.tE[i] = kQe * L->test_E[i] / (kMe * kC * om);
        c.tB[i] = kQe * L->test_B[i] / (kMe * om);
    }
    c.field = L->field; c.window = L->window;
    // tunnelling constants: F [a.u.] = |a| fconv
    const double fconv = (kMe * kC * om / kQe) / kEa;
    c.lnw_zero = -700.0 - log(om);
    for (int s = 0; s < rpdla::kMaxStates; ++s) {
        const double Ip = kNeIpEv[s] / kEhEv;
        const double Z = (double)(s + 1);
        const double ns = Z / sqrt(2.0 * Ip);
        const double F0 = pow(2.0 * Ip, 1.5);
        const double lnC2 = 2.0 * ns * log(2.0) - log(ns) - lgamma(2.0 * ns);
        c.adk_c0[s] = lnC2 + log(Ip / kTauA) + (2.0 * ns - 1.0) * (log(2.0 * F0) - log(fconv)) - log(om);
        c.adk_c1h[s] = 0.5 * (2.0 * ns - 1.0);
        c.adk_c2[s] = 2.0 * F0 / (3.0 * fconv);
        c.adk_a2thr[s] = adk_threshold_a2(c.adk_c0[s], c.adk_c1h[s], c.adk_c2[s], kLnwSkip);
    }
    const double ga = sqrt(3.0 / 7.0 - 2.0 / 7.0 * sqrt(6.0 / 5.0));
    const double gb = sqrt(3.0 / 7.0 + 2.0 / 7.0 * sqrt(6.0 / 5.0));
    const double wa = (18.0 + sqrt(30.0)) / 36.0, wb = (18.0 - sqrt(30.0)) / 36.0;
    c.gl_x[0] = -gb; c.gl_x[1] = -ga; c.gl_x[2] = ga; c.gl_x[3] = gb;
    c.gl_w[0] = wb; c.gl_w[1] = wa; c.gl_w[2] = wa; c.gl_w[3] = wb;
    const double re = kQe * kQe / (4.0 * kPi * kEps0 * kMe * kC * kC);   // classical radius
    c.rr_kappa = 2.0 / 3.0 * k * re;
    c.chi_eta = kHbar * om / (kMe * kC * kC);
    c.ad_rtol = 1e-9; c.ad_atol = 1e-9; c.ad_hmax = 10.0 * c.hn; c.ad_ktol = 1e-10;
    c.ad_max_steps = 10000000;
    return c;
}

void laser_defaults(rpdla_laser* L, double lambda, double w0, double tau)
{
    memset(L, 0, sizeof *L);
    L->lambda = lambda; L->w0 = w0; L->tau_fwhm = tau;
    L->phi0 = 0.0;
    L->field = RPDLA_RP_O5;
    L->window = RPDLA_WIN_ARRIVAL;
    L->t_before = 5.0 * tau;
    L->t_after = 10.0 * tau;
    L->dt = lambda / kC / 200.0;
    L->ez_scale = 1.0; L->er_scale = 1.0;
}

int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Launch shapes, per (kernel kind, field model, precision): threads per block
// and, for persistent kernels, resident blocks per CU times grid_factor.
// Filled by rpdla_autotune / rpdla_set_launch_shape; default 256 x 1.
struct Shape { int block = 256; int grid_factor = 1; };
std::mutex g_shape_mu;
std::map<int, Shape> g_shapes;
int shape_key(int kind, int field, int prec) { return (kind * 64 + field) * 4 + prec; }
Shape get_shape(int kind, int field, int prec)
{
    std::lock_guard<std::mutex> lk(g_shape_mu);
    auto it = g_shapes.find(shape_key(kind, field, prec));
    return it == g_shapes.end() ? Shape() : it->second;
}

// Persistent grid: resident blocks (occupancy query) x grid_factor, capped by the work.
template <typename K>
int persistent_blocks(K kernel, int64_t work_items, int block, int grid_factor, size_t lds = 0)
{
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 1;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, lds) != hipSuccess || per_cu < 1)
        per_cu = 1;
    int64_t blocks = (int64_t)cus * per_cu * grid_factor;
    const int64_t need = cdiv(work_items, block);
    if (need < blocks) blocks = need;
    return (int)(blocks < 1 ? 1 : blocks);
}

constexpr int kKindPush = 0, kKindIonize = 1, kKindBatchPush = 2;

template <int FIELD>
rpdla_status launch_ionize(const DevCfg& c, uint64_t seed, uint32_t cfg, uint64_t first,
                           int64_t n, const double* x, const double* y, const double* z, int kf,
                           int kl, double* tb, hipStream_t st)
{
    const int bs = get_shape(kKindIonize, FIELD, 0).block;
    if (n < kIonizeSortMin || n > (int64_t)INT32_MAX) {
        hipLaunchKernelGGL(rpdla::ionize_kernel<FIELD>, dim3((unsigned)cdiv(n, bs)), dim3(bs), 0,
                           st, c, seed, cfg, first, n, x, y, z, kf, kl, tb,
                           (const uint32_t*)nullptr);
        RPDLA_HIP(hipGetLastError());
        return RPDLA_OK;
    }
    // atoms ordered by their work key (radix sort of key/index pairs), so that
    // each wave holds atoms of similar work; stream-ordered scratch
    size_t sort_bytes = 0;
    RPDLA_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, sort_bytes, (const uint32_t*)nullptr,
                                                 (uint32_t*)nullptr, (const uint32_t*)nullptr,
                                                 (uint32_t*)nullptr, (int)n, 0, 32, st));
    const size_t arr = align256((size_t)n * sizeof(uint32_t));
    char* buf = nullptr;
    RPDLA_HIP(hipMallocAsync((void**)&buf, 4 * arr + sort_bytes, st));
    uint32_t* key_in = (uint32_t*)buf;
    uint32_t* key_out = (uint32_t*)(buf + arr);
    uint32_t* idx_in = (uint32_t*)(buf + 2 * arr);
    uint32_t* idx_out = (uint32_t*)(buf + 3 * arr);
    rpdla_status r = RPDLA_OK;
    hipLaunchKernelGGL(rpdla::ionize_key_kernel<FIELD>, dim3((unsigned)cdiv(n, 256)), dim3(256), 0,
                       st, c, seed, cfg, first, n, x, y, z, kf, kl, key_in, idx_in);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess)
        e = hipcub::DeviceRadixSort::SortPairs(buf + 4 * arr, sort_bytes, key_in, key_out, idx_in,
                                               idx_out, (int)n, 0, 32, st);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(rpdla::ionize_kernel<FIELD>, dim3((unsigned)cdiv(n, bs)), dim3(bs), 0,
                           st, c, seed, cfg, first, n, x, y, z, kf, kl, tb,
                           (const uint32_t*)idx_out);
        e = hipGetLastError();
    }
    if (e != hipSuccess) r = fail(RPDLA_EHIP, "ionize: %s", hipGetErrorString(e));
    const hipError_t fe = hipFreeAsync(buf, st);
    if (r != RPDLA_OK) return r;
    if (fe != hipSuccess) return fail(RPDLA_EHIP, "hipFreeAsync: %s", hipGetErrorString(fe));
    return RPDLA_OK;
}

template <int FIELD>
rpdla_status launch_push(const DevCfg& c, int prec, const rpdla::PushIO& io, hipStream_t st)
{
    const Shape sh = get_shape(kKindPush, FIELD, prec);
    if (prec == RPDLA_FP64) {
        auto* kern = rpdla::push_kernel<FIELD, rpdla::ElecF64>;
        const int g = persistent_blocks(kern, io.n_slots, sh.block, sh.grid_factor);
        hipLaunchKernelGGL(kern, dim3(g), dim3(sh.block), 0, st, c, io);
    } else if constexpr (FIELD < 20) {
        auto* kern = rpdla::push_kernel<FIELD, rpdla::ElecMixed>;
        const int g = persistent_blocks(kern, io.n_slots, sh.block, sh.grid_factor);
        hipLaunchKernelGGL(kern, dim3(g), dim3(sh.block), 0, st, c, io);
    } else {
        return fail(RPDLA_EUNSUPPORTED, "the linearly polarized focus has no mixed form");
    }
    RPDLA_HIP(hipGetLastError());
    return RPDLA_OK;
}

template <int FIELD>
rpdla_status launch_push_rr(const DevCfg& c, bool rr, const rpdla::PushIO& io, hipStream_t st)
{
    const Shape sh = get_shape(kKindPush, FIELD, RPDLA_FP64);
    if (rr) {
        auto* kern = rpdla::push_kernel<FIELD, rpdla::ElecRR<true>>;
        const int g = persistent_blocks(kern, io.n_slots, sh.block, sh.grid_factor);
        hipLaunchKernelGGL(kern, dim3(g), dim3(sh.block), 0, st, c, io);
    } else {
        auto* kern = rpdla::push_kernel<FIELD, rpdla::ElecRR<false>>;
        const int g = persistent_blocks(kern, io.n_slots, sh.block, sh.grid_factor);
        hipLaunchKernelGGL(kern, dim3(g), dim3(sh.block), 0, st, c, io);
    }
    RPDLA_HIP(hipGetLastError());
    return RPDLA_OK;
}

template <int FIELD>
rpdla_status launch_push_dp(const DevCfg& c, const rpdla::PushIO& io, hipStream_t st)
{
    const Shape sh = get_shape(kKindPush, FIELD, RPDLA_FP64);
    auto* kern = rpdla::push_kernel<FIELD, rpdla::ElecDP>;
    const int g = persistent_blocks(kern, io.n_slots, sh.block, sh.grid_factor);
    hipLaunchKernelGGL(kern, dim3(g), dim3(sh.block), 0, st, c, io);
    RPDLA_HIP(hipGetLastError());
    return RPDLA_OK;
}

// Checks shared by rpdla_push and rpdla_push_noalloc (nothing is enqueued).
rpdla_status check_push_args(const rpdla_laser* L, int32_t precision, int64_t n_slots,
                             const double* t_birth, const double* x0, const double* y0,
                             const double* z0, int32_t slots_per_atom, double* ux, double* uy,
                             double* uz, double* xf, double* yf, double* zf)
{
    rpdla_status st = check_laser(L);
    if (st != RPDLA_OK) return st;
    if (!(precision == RPDLA_FP64 || precision == RPDLA_MIXED))
        return fail(RPDLA_EINVAL, "unknown precision %d", precision);
    if (n_slots < 0) return fail(RPDLA_EINVAL, "n_slots < 0");
    if (slots_per_atom < 1) return fail(RPDLA_EINVAL, "slots_per_atom < 1");
    if (n_slots == 0) return RPDLA_OK;
    if (!t_birth || !x0 || !y0 || !z0 || !ux || !uy || !uz || !xf || !yf || !zf)
        return fail(RPDLA_EINVAL, "null pointer");
    if (n_slots > kMaxPushSlots) return fail(RPDLA_ERANGE, "n_slots too large");
    return RPDLA_OK;
}

// Clear the work counters q[kQueueWords] (a fill kernel, no memset node) and
// launch the persistent push that draws slots from them.
rpdla_status enqueue_push(const rpdla_laser* L, int32_t precision, int64_t n_slots,
                          const double* t_birth, const double* x0, const double* y0,
                          const double* z0, int32_t slots_per_atom, double* ux, double* uy,
                          double* uz, double* xf, double* yf, double* zf, unsigned long long* q,
                          hipStream_t s)
{
    const DevCfg c = make_cfg(L);
    hipLaunchKernelGGL(rpdla::zero_u64_kernel, dim3(1), dim3(rpdla::kQueueWords), 0, s, q,
                       (int64_t)rpdla::kQueueWords);
    RPDLA_HIP(hipGetLastError());
    rpdla::PushIO io{t_birth, x0, y0, z0, slots_per_atom, n_slots, ux, uy, uz, xf, yf, zf, q};
    switch (L->field) {
    case 1: return launch_push<1>(c, precision, io, s);
    case 3: return launch_push<3>(c, precision, io, s);
    case 5: return launch_push<5>(c, precision, io, s);
    case 10: return launch_push<10>(c, precision, io, s);
    case 21: return launch_push<21>(c, precision, io, s);
    case 23: return launch_push<23>(c, precision, io, s);
    case 25: return launch_push<25>(c, precision, io, s);
    default: return launch_push<11>(c, precision, io, s);
    }
}

// Device address of this device's copy of `scratch`, looked up once per
// device (with that device current) and kept for the process lifetime.  The
// array's name is only a host-side stand-in: kernels and copies get this
// address.
std::mutex g_scratch_mu;
std::vector<unsigned long long*> g_scratch_ptr;

rpdla_status scratch_address(unsigned long long** out)
{
    int dev = 0;
    RPDLA_HIP(hipGetDevice(&dev));
    if (dev < 0) return fail(RPDLA_EHIP, "hipGetDevice returned %d", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if ((size_t)dev >= g_scratch_ptr.size()) g_scratch_ptr.resize((size_t)dev + 1, nullptr);
    if (!g_scratch_ptr[(size_t)dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(RPDLA_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_scratch_ptr[(size_t)dev] = (unsigned long long*)p;
    }
    *out = g_scratch_ptr[(size_t)dev];
    return RPDLA_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* rpdla_version(void) { return "rpdla 0.1 (gfx950)"; }

const char* rpdla_status_string(rpdla_status s)
{
    switch (s) {
    case RPDLA_OK: return "ok";
    case RPDLA_EINVAL: return "invalid argument";
    case RPDLA_ERANGE: return "size out of range";
    case RPDLA_EHIP: return "HIP runtime error";
    case RPDLA_ENOMEM: return "out of memory / workspace too small";
    case RPDLA_EUNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

const char* rpdla_last_error(void) { return g_err.c_str(); }

rpdla_status rpdla_laser_init_intensity(rpdla_laser* L, double lambda, double w0, double tau,
                                        double I_W_cm2)
{
    if (!L) return fail(RPDLA_EINVAL, "laser is NULL");
    if (!(lambda > 0 && w0 > 0 && tau > 0 && I_W_cm2 >= 0 && is_fin(lambda) && is_fin(w0) &&
          is_fin(tau) && is_fin(I_W_cm2)))
        return fail(RPDLA_EINVAL, "lambda, w0, tau must be > 0 and I >= 0");
    laser_defaults(L, lambda, w0, tau);
    L->amp = sqrt(2.0 * I_W_cm2 * 1.0e4 / (kEps0 * kC));
    return RPDLA_OK;
}

rpdla_status rpdla_laser_init_power(rpdla_laser* L, double lambda, double w0, double tau, double P_W)
{
    if (!L) return fail(RPDLA_EINVAL, "laser is NULL");
    if (!(lambda > 0 && w0 > 0 && tau > 0 && P_W >= 0 && is_fin(lambda) && is_fin(w0) &&
          is_fin(tau) && is_fin(P_W)))
        return fail(RPDLA_EINVAL, "lambda, w0, tau must be > 0 and P >= 0");
    laser_defaults(L, lambda, w0, tau);
    L->amp = sqrt(8.0 * P_W / (kPi * w0 * w0 * kEps0 * kC));
    return RPDLA_OK;
}

double rpdla_rayleigh(const rpdla_laser* L)
{
    if (!L) return NAN;
    const double k = 2.0 * kPi / L->lambda;
    return 0.5 * k * L->w0 * L->w0;
}

rpdla_status rpdla_sample_atoms(uint64_t seed, uint32_t cfg_id, uint64_t first_atom, int64_t n,
                                double r_max, double z_half, double* x, double* y, double* z,
                                void* stream)
{
    if (n < 0) return fail(RPDLA_EINVAL, "n_atoms < 0");
    if (!(is_fin(r_max) && is_fin(z_half) && r_max >= 0 && z_half >= 0))
        return fail(RPDLA_EINVAL, "r_max and z_half must be finite and >= 0");
    if (n == 0) return RPDLA_OK;
    if (!x || !y || !z) return fail(RPDLA_EINVAL, "null output pointer");
    if (n > ((int64_t)1 << 40)) return fail(RPDLA_ERANGE, "n_atoms too large");
    hipLaunchKernelGGL(rpdla::sample_atoms_kernel, dim3((unsigned)cdiv(n, 256)), dim3(256), 0,
                       (hipStream_t)stream, seed, cfg_id, first_atom, n, r_max, z_half, x, y, z);
    RPDLA_HIP(hipGetLastError());
    return RPDLA_OK;
}

rpdla_status rpdla_sample_atoms_annulus(uint64_t seed, uint32_t cfg_id, uint64_t first_atom,
                                        int64_t n, double r_in, double r_out, double z_half,
                                        double* x, double* y, double* z, void* stream)
{
    if (n < 0) return fail(RPDLA_EINVAL, "n_atoms < 0");
    if (!(is_fin(r_in) && is_fin(r_out) && is_fin(z_half) && r_in >= 0 && r_out >= r_in && z_half >= 0))
        return fail(RPDLA_EINVAL, "need 0 <= r_in <= r_out and z_half >= 0, finite");
    if (n == 0) return RPDLA_OK;
    if (!x || !y || !z) return fail(RPDLA_EINVAL, "null output pointer");
    if (n > ((int64_t)1 << 40)) return fail(RPDLA_ERANGE, "n_atoms too large");
    hipLaunchKernelGGL(rpdla::sample_annulus_kernel, dim3((unsigned)cdiv(n, 256)), dim3(256), 0,
                       (hipStream_t)stream, seed, cfg_id, first_atom, n, r_in, r_out, z_half, x, y, z);
    RPDLA_HIP(hipGetLastError());
    return RPDLA_OK;
}

rpdla_status rpdla_birth_phase(const rpdla_laser* L, int64_t n_slots, const double* t_birth,
                               const double* x, const double* y, const double* z,
                               int32_t slots_per_atom, double* phase, double* r_birth,
                               void* stream)
{
    rpdla_status st = check_laser(L);
    if (st != RPDLA_OK) return st;
    if (n_slots < 0) return fail(RPDLA_EINVAL, "n_slots < 0");
    if (slots_per_atom < 1) return fail(RPDLA_EINVAL, "slots_per_atom < 1");
    if (n_slots == 0) return RPDLA_OK;
    if (!t_birth || !x || !y || !z || !phase) return fail(RPDLA_EINVAL, "null pointer");
    if (is_lp(L->field))
        return fail(RPDLA_EUNSUPPORTED, "the birth phase is the radial focus's carrier phase");
    const DevCfg c = make_cfg(L);
    hipLaunchKernelGGL(rpdla::birth_phase_kernel, dim3((unsigned)cdiv(n_slots, 256)), dim3(256), 0,
                       (hipStream_t)stream, c, n_slots, t_birth, x, y, z, slots_per_atom, phase,
                       r_birth);
    RPDLA_HIP(hipGetLastError());
    return RPDLA_OK;
}

rpdla_status rpdla_ionize(const rpdla_laser* L, uint64_t seed, uint32_t cfg_id, uint64_t first_atom,
                          int64_t n, const double* x, const double* y, const double* z,
                          int32_t k_first, int32_t k_last, double* t_birth, void* stream)
{
    rpdla_status st = check_laser(L);
    if (st != RPDLA_OK) return st;
    if (!(1 <= k_first && k_first <= k_last && k_last <= 10))
        return fail(RPDLA_EINVAL, "need 1 <= k_first <= k_last <= 10 (got %d..%d)", k_first, k_last);
    if (n < 0) return fail(RPDLA_EINVAL, "n_atoms < 0");
    if (n == 0) return RPDLA_OK;
    if (!x || !y || !z || !t_birth) return fail(RPDLA_EINVAL, "null pointer");
    if (n > ((int64_t)1 << 36)) return fail(RPDLA_ERANGE, "n_atoms too large");
    const DevCfg c = make_cfg(L);
    hipStream_t s = (hipStream_t)stream;
    switch (L->field) {
    case 1: return launch_ionize<1>(c, seed, cfg_id, first_atom, n, x, y, z, k_first, k_last, t_birth, s);
    case 3: return launch_ionize<3>(c, seed, cfg_id, first_atom, n, x, y, z, k_first, k_last, t_birth, s);
    case 5: return launch_ionize<5>(c, seed, cfg_id, first_atom, n, x, y, z, k_first, k_last, t_birth, s);
    case 10: return launch_ionize<10>(c, seed, cfg_id, first_atom, n, x, y, z, k_first, k_last, t_birth, s);
    case 21: return launch_ionize<21>(c, seed, cfg_id, first_atom, n, x, y, z, k_first, k_last, t_birth, s);
    case 23: return launch_ionize<23>(c, seed, cfg_id, first_atom, n, x, y, z, k_first, k_last, t_birth, s);
    case 25: return launch_ionize<25>(c, seed, cfg_id, first_atom, n, x, y, z, k_first, k_last, t_birth, s);
    default: return launch_ionize<11>(c, seed, cfg_id, first_atom, n, x, y, z, k_first, k_last, t_birth, s);
    }
}

rpdla_status rpdla_push(const rpdla_laser* L, int32_t precision, int64_t n_slots,
                        const double* t_birth, const double* x0, const double* y0, const double* z0,
                        int32_t slots_per_atom, double* ux, double* uy, double* uz, double* xf,
                        double* yf, double* zf, void* stream)
{
    rpdla_status st = check_push_args(L, precision, n_slots, t_birth, x0, y0, z0, slots_per_atom,
                                      ux, uy, uz, xf, yf, zf);
    if (st != RPDLA_OK || n_slots == 0) return st;
    hipStream_t s = (hipStream_t)stream;
    unsigned long long* q = nullptr;
    RPDLA_HIP(hipMallocAsync((void**)&q, rpdla::kQueueWords * sizeof(unsigned long long), s));
    st = enqueue_push(L, precision, n_slots, t_birth, x0, y0, z0, slots_per_atom, ux, uy, uz, xf,
                      yf, zf, q, s);
    hipError_t fe = hipFreeAsync(q, s);
    if (st != RPDLA_OK) return st;
    if (fe != hipSuccess) return fail(RPDLA_EHIP, "hipFreeAsync: %s", hipGetErrorString(fe));
    return RPDLA_OK;
}

rpdla_status rpdla_push_noalloc(const rpdla_laser* L, int32_t precision, int64_t n_slots,
                                const double* t_birth, const double* x0, const double* y0,
                                const double* z0, int32_t slots_per_atom, double* ux, double* uy,
                                double* uz, double* xf, double* yf, double* zf, void* stream)
{
    rpdla_status st = check_push_args(L, precision, n_slots, t_birth, x0, y0, z0, slots_per_atom,
                                      ux, uy, uz, xf, yf, zf);
    if (st != RPDLA_OK || n_slots == 0) return st;
    unsigned long long* q = nullptr;
    st = scratch_address(&q);
    if (st != RPDLA_OK) return st;
    return enqueue_push(L, precision, n_slots, t_birth, x0, y0, z0, slots_per_atom, ux, uy, uz,
                        xf, yf, zf, q, (hipStream_t)stream);
}

rpdla_status rpdla_push_rr(const rpdla_laser* L, int32_t radiation_reaction, int64_t n_slots,
                           const double* t_birth, const double* x0, const double* y0,
                           const double* z0, int32_t slots_per_atom, double* ux, double* uy,
                           double* uz, double* xf, double* yf, double* zf, double* chi_max,
                           void* stream)
{
    rpdla_status st = check_laser(L);
    if (st != RPDLA_OK) return st;
    if (radiation_reaction != 0 && radiation_reaction != 1)
        return fail(RPDLA_EINVAL, "radiation_reaction must be 0 or 1");
    if (n_slots < 0) return fail(RPDLA_EINVAL, "n_slots < 0");
    if (slots_per_atom < 1) return fail(RPDLA_EINVAL, "slots_per_atom < 1");
    if (n_slots == 0) return RPDLA_OK;
    if (!t_birth || !x0 || !y0 || !z0 || !ux || !uy || !uz || !xf || !yf || !zf)
        return fail(RPDLA_EINVAL, "null pointer");
    if (n_slots > ((int64_t)1 << 40)) return fail(RPDLA_ERANGE, "n_slots too large");
    const DevCfg c = make_cfg(L);
    hipStream_t s = (hipStream_t)stream;
    unsigned long long* q = nullptr;
    RPDLA_HIP(hipMallocAsync((void**)&q, rpdla::kQueueWords * sizeof(unsigned long long), s));
    hipLaunchKernelGGL(rpdla::zero_u64_kernel, dim3(1), dim3(rpdla::kQueueWords), 0, s, q,
                       (int64_t)rpdla::kQueueWords);
    rpdla::PushIO io{t_birth, x0, y0, z0, slots_per_atom, n_slots, ux, uy, uz, xf, yf, zf, q,
                     chi_max};
    const bool rr = radiation_reaction == 1;
    switch (L->field) {
    case 1: st = launch_push_rr<1>(c, rr, io, s); break;
    case 3: st = launch_push_rr<3>(c, rr, io, s); break;
    case 5: st = launch_push_rr<5>(c, rr, io, s); break;
    case 10: st = launch_push_rr<10>(c, rr, io, s); break;
    case 21: st = launch_push_rr<21>(c, rr, io, s); break;
    case 23: st = launch_push_rr<23>(c, rr, io, s); break;
    case 25: st = launch_push_rr<25>(c, rr, io, s); break;
    default: st = launch_push_rr<11>(c, rr, io, s); break;
    }
    hipError_t fe = hipFreeAsync(q, s);
    if (st != RPDLA_OK) return st;
    if (fe != hipSuccess) return fail(RPDLA_EHIP, "hipFreeAsync: %s", hipGetErrorString(fe));
    return RPDLA_OK;
}

rpdla_status rpdla_push_adaptive(const rpdla_laser* L, const rpdla_adaptive* A, int64_t n_slots,
                                 const double* t_birth, const double* x0, const double* y0,
                                 const double* z0, int32_t slots_per_atom, double* ux, double* uy,
                                 double* uz, double* xf, double* yf, double* zf, double* t_stop,
                                 int64_t* steps_accepted, int64_t* steps_rejected, void* stream)
{
    rpdla_status st = check_laser(L);
    if (st != RPDLA_OK) return st;
    if (!A) return fail(RPDLA_EINVAL, "adaptive settings are NULL");
    if (!(is_fin(A->rtol) && is_fin(A->atol) && A->rtol >= 0.0 && A->atol >= 0.0 &&
          A->rtol + A->atol > 0.0))
        return fail(RPDLA_EINVAL, "need rtol, atol >= 0, not both 0");
    if (!(is_fin(A->h_max) && is_fin(A->k_tol))) return fail(RPDLA_EINVAL, "h_max, k_tol not finite");
    if (A->max_steps < 1) return fail(RPDLA_EINVAL, "max_steps < 1");
    if (n_slots < 0) return fail(RPDLA_EINVAL, "n_slots < 0");
    if (slots_per_atom < 1) return fail(RPDLA_EINVAL, "slots_per_atom < 1");
    if (n_slots == 0) return RPDLA_OK;
    if (!t_birth || !x0 || !y0 || !z0 || !ux || !uy || !uz || !xf || !yf || !zf)
        return fail(RPDLA_EINVAL, "null pointer");
    if (n_slots > ((int64_t)1 << 40)) return fail(RPDLA_ERANGE, "n_slots too large");
    DevCfg c = make_cfg(L);
    c.ad_rtol = A->rtol;
    c.ad_atol = A->atol;
    c.ad_hmax = A->h_max > 0.0 ? A->h_max * c.omega : 10.0 * c.hn;
    c.ad_ktol = A->k_tol;
    c.ad_max_steps = A->max_steps;
    hipStream_t s = (hipStream_t)stream;
    unsigned long long* q = nullptr;
    RPDLA_HIP(hipMallocAsync((void**)&q, rpdla::kQueueWords * sizeof(unsigned long long), s));
    hipLaunchKernelGGL(rpdla::zero_u64_kernel, dim3(1), dim3(rpdla::kQueueWords), 0, s, q,
                       (int64_t)rpdla::kQueueWords);
    rpdla::PushIO io{t_birth, x0, y0, z0, slots_per_atom, n_slots, ux, uy, uz, xf, yf, zf, q};
    io.t_stop = t_stop;
    io.n_acc = (long long*)steps_accepted;
    io.n_rej = (long long*)steps_rejected;
    switch (L->field) {
    case 1: st = launch_push_dp<1>(c, io, s); break;
    case 3: st = launch_push_dp<3>(c, io, s); break;
    case 5: st = launch_push_dp<5>(c, io, s); break;
    case 10: st = launch_push_dp<10>(c, io, s); break;
    case 21: st = launch_push_dp<21>(c, io, s); break;
    case 23: st = launch_push_dp<23>(c, io, s); break;
    case 25: st = launch_push_dp<25>(c, io, s); break;
    default: st = launch_push_dp<11>(c, io, s); break;
    }
    hipError_t fe = hipFreeAsync(q, s);
    if (st != RPDLA_OK) return st;
    if (fe != hipSuccess) return fail(RPDLA_EHIP, "hipFreeAsync: %s", hipGetErrorString(fe));
    return RPDLA_OK;
}

rpdla_status rpdla_epilogue(int64_t n, const double* ux, const double* uy, const double* uz,
                            double* K_MeV, double* theta, double* psi, int32_t* fwd, void* stream)
{
    if (n < 0) return fail(RPDLA_EINVAL, "n < 0");
    if (n == 0) return RPDLA_OK;
    if (!ux || !uy || !uz || !K_MeV || !theta || !psi || !fwd) return fail(RPDLA_EINVAL, "null pointer");
    hipLaunchKernelGGL(rpdla::epilogue_kernel, dim3((unsigned)cdiv(n, 256)), dim3(256), 0,
                       (hipStream_t)stream, n, kMeC2MeV, ux, uy, uz, K_MeV, theta, psi, fwd);
    RPDLA_HIP(hipGetLastError());
    return RPDLA_OK;
}

rpdla_status rpdla_histogram(int64_t n, const double* t_birth, const double* ux, const double* uy,
                             const double* uz, const rpdla_hist_spec* spec, uint64_t* counts,
                             uint64_t* tallies, void* stream)
{
    if (!spec) return fail(RPDLA_EINVAL, "spec is NULL");
    if (spec->nE < 1 || spec->nA < 1) return fail(RPDLA_EINVAL, "nE, nA must be >= 1");
    if (!(is_fin(spec->logE_min_MeV) && is_fin(spec->logE_max_MeV) &&
          spec->logE_min_MeV < spec->logE_max_MeV))
        return fail(RPDLA_EINVAL, "need logE_min < logE_max");
    if (!(spec->angle == RPDLA_ANG_POLAR || spec->angle == RPDLA_ANG_AZIMUTH))
        return fail(RPDLA_EINVAL, "unknown angle mode");
    if ((int64_t)spec->nE * spec->nA > ((int64_t)1 << 28)) return fail(RPDLA_ERANGE, "too many bins");
    if (n < 0) return fail(RPDLA_EINVAL, "n_slots < 0");
    if (!counts || !tallies) return fail(RPDLA_EINVAL, "null output pointer");
    if (n == 0) return RPDLA_OK;
    if (!t_birth || !ux || !uy || !uz) return fail(RPDLA_EINVAL, "null input pointer");
    rpdla::HistArgs H;
    H.nE = spec->nE; H.nA = spec->nA; H.angle = spec->angle;
    H.lo = spec->logE_min_MeV;
    H.width = (spec->logE_max_MeV - spec->logE_min_MeV) / (double)spec->nE;
    H.mec2 = kMeC2MeV;
    int64_t blocks = cdiv(n, 256);
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(rpdla::histogram_kernel, dim3((unsigned)blocks), dim3(256), 0,
                       (hipStream_t)stream, H, n, t_birth, ux, uy, uz,
                       (unsigned long long*)counts, (unsigned long long*)tallies);
    RPDLA_HIP(hipGetLastError());
    return RPDLA_OK;
}

}  // extern "C"

// ===========================================================================
// Batched sweep
// ===========================================================================
namespace {


struct WsLayout {
    size_t cfg, geo, ctl, x, y, z, tb, ux, uy, uz, total;
};

WsLayout ws_layout(int n_cfg, int64_t apc, int K)
{
    WsLayout w;
    size_t off = 0;
    const size_t na = (size_t)n_cfg * (size_t)apc;
    w.cfg = off; off += align256((size_t)n_cfg * sizeof(DevCfg));
    w.geo = off; off += align256((size_t)n_cfg * 2 * sizeof(double));
    w.ctl = off; off += align256(sizeof(rpdla::BatchCtl));
    w.x = off; off += align256(na * sizeof(double));
    w.y = off; off += align256(na * sizeof(double));
    w.z = off; off += align256(na * sizeof(double));
    w.tb = off; off += align256(na * (size_t)K * sizeof(double));
    w.ux = off; off += align256(na * (size_t)K * sizeof(double));
    w.uy = off; off += align256(na * (size_t)K * sizeof(double));
    w.uz = off; off += align256(na * (size_t)K * sizeof(double));
    w.total = off;
    return w;
}

std::mutex g_graph_mu;
std::vector<std::pair<std::string, hipGraphExec_t>> g_graphs;  // small cache, process lifetime
// Graphs are never destroyed while the process runs (a replay may still be in
// flight on its stream); once this many argument sets have been captured,
// further ones are enqueued directly, without a graph.
constexpr size_t kMaxGraphs = 32;

template <int FIELD, class ELEC>
rpdla_status run_batched_impl(const rpdla::BatchArgs& A, int64_t n_chunks, hipStream_t s)
{
    const size_t lds_i = (size_t)A.n_cfg * sizeof(DevCfg);
    const size_t lds_p = (size_t)A.n_cfg * sizeof(unsigned long long);
    auto* kpush = rpdla::batch_push_kernel<FIELD, ELEC>;
    auto* kion = rpdla::batch_ionize_kernel<FIELD>;
    const Shape sh = get_shape(kKindBatchPush, FIELD, std::is_same<ELEC, rpdla::ElecMixed>::value);
    const int64_t slots = (int64_t)A.n_cfg * A.apc * A.K;
    const int64_t grid_p = persistent_blocks(kpush, slots, sh.block, sh.grid_factor, lds_p);
    const unsigned grid_a = (unsigned)cdiv((int64_t)A.n_cfg * A.apc, 256);
    int64_t grid_h = cdiv(slots, 256);
    if (grid_h > 8192) grid_h = 8192;

    auto enqueue_chunk = [&](hipStream_t st) -> rpdla_status {
        hipLaunchKernelGGL(rpdla::batch_zero_queue_kernel, dim3(1), dim3(64), 0, st, A.ctl);
        hipLaunchKernelGGL(rpdla::batch_sample_kernel, dim3(grid_a), dim3(256), 0, st, A);
        hipLaunchKernelGGL(kion, dim3(grid_a), dim3(256), lds_i, st, A);
        hipLaunchKernelGGL(kpush, dim3((unsigned)grid_p), dim3(sh.block), lds_p, st, A, A.cfgs);
        hipLaunchKernelGGL(rpdla::batch_hist_kernel, dim3((unsigned)grid_h), dim3(256), 0, st, A);
        hipLaunchKernelGGL(rpdla::batch_advance_kernel, dim3(1), dim3(64), 0, st, A.ctl);
        RPDLA_HIP(hipGetLastError());
        return RPDLA_OK;
    };

    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (s != nullptr) RPDLA_HIP(hipStreamIsCapturing(s, &cap));
    if (s == nullptr || cap != hipStreamCaptureStatusNone) {
        for (int64_t i = 0; i < n_chunks; ++i) {
            rpdla_status r = enqueue_chunk(s);
            if (r != RPDLA_OK) return r;
        }
        return RPDLA_OK;
    }
    // one chunk captured as a graph (kernel arguments fixed; the chunk index
    // lives in device memory and advances inside the graph), replayed per chunk
    std::string key(reinterpret_cast<const char*>(&A), sizeof A);
    const int tag[2] = {FIELD, (int)sizeof(ELEC)};
    key.append(reinterpret_cast<const char*>(tag), sizeof tag);
    key.append(reinterpret_cast<const char*>(&s), sizeof s);
    key.append(reinterpret_cast<const char*>(&grid_p), sizeof grid_p);
    key.append(reinterpret_cast<const char*>(&sh), sizeof sh);
    hipGraphExec_t exec = nullptr;
    bool full = false;
    {
        std::lock_guard<std::mutex> lk(g_graph_mu);
        for (auto& kv : g_graphs)
            if (kv.first == key) { exec = kv.second; break; }
        full = g_graphs.size() >= kMaxGraphs;
    }
    if (!exec && full) {
        for (int64_t i = 0; i < n_chunks; ++i) {
            rpdla_status r = enqueue_chunk(s);
            if (r != RPDLA_OK) return r;
        }
        return RPDLA_OK;
    }
    if (!exec) {
        hipGraph_t graph = nullptr;
        RPDLA_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        rpdla_status r = enqueue_chunk(s);
        hipError_t ee = hipStreamEndCapture(s, &graph);
        if (r != RPDLA_OK) return r;
        if (ee != hipSuccess) return fail(RPDLA_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(ee));
        hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ie != hipSuccess) return fail(RPDLA_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(ie));
        std::lock_guard<std::mutex> lk(g_graph_mu);
        g_graphs.emplace_back(key, exec);
    }
    for (int64_t i = 0; i < n_chunks; ++i) RPDLA_HIP(hipGraphLaunch(exec, s));
    return RPDLA_OK;
}

}  // namespace

extern "C" {

size_t rpdla_batched_workspace_bytes(int32_t n_cfg, int64_t atoms_per_chunk, int32_t k_first,
                                     int32_t k_last)
{
    if (n_cfg < 1 || atoms_per_chunk < 1 || k_first < 1 || k_last < k_first || k_last > 10) return 0;
    return ws_layout(n_cfg, atoms_per_chunk, k_last - k_first + 1).total;
}

rpdla_status rpdla_batched_workspace_layout(int32_t n_cfg, int64_t atoms_per_chunk,
                                           int32_t k_first, int32_t k_last, size_t* offsets)
{
    if (!offsets) return fail(RPDLA_EINVAL, "offsets is NULL");
    if (n_cfg < 1 || atoms_per_chunk < 1 || k_first < 1 || k_last < k_first || k_last > 10)
        return fail(RPDLA_EINVAL, "invalid sizes");
    const WsLayout w = ws_layout(n_cfg, atoms_per_chunk, k_last - k_first + 1);
    const size_t o[RPDLA_WS_NARRAYS] = {w.x, w.y, w.z, w.tb, w.ux, w.uy, w.uz};
    for (int i = 0; i < RPDLA_WS_NARRAYS; ++i) offsets[i] = o[i];
    return RPDLA_OK;
}

int32_t rpdla_batched_graphs(void)
{
    std::lock_guard<std::mutex> lk(g_graph_mu);
    return (int32_t)g_graphs.size();
}

rpdla_status rpdla_run_batched(const rpdla_laser* cfgs, int32_t n_cfg, uint64_t seed,
                               uint32_t cfg_base, int64_t atoms_per_cfg, int64_t atoms_per_chunk,
                               double r_factor, int32_t k_first, int32_t k_last, int32_t precision,
                               const rpdla_hist_spec* spec, uint64_t* counts, uint64_t* tallies,
                               uint64_t* electron_steps, void* workspace, size_t ws_bytes,
                               void* stream)
{
    return rpdla_run_batched_range(cfgs, n_cfg, seed, cfg_base, atoms_per_cfg, atoms_per_chunk, 0,
                                   -1, r_factor, k_first, k_last, precision, spec, counts, tallies,
                                   electron_steps, workspace, ws_bytes, stream);
}

rpdla_status rpdla_run_batched_range(const rpdla_laser* cfgs, int32_t n_cfg, uint64_t seed,
                                     uint32_t cfg_base, int64_t atoms_per_cfg,
                                     int64_t atoms_per_chunk, int64_t first_chunk,
                                     int64_t n_chunks_run, double r_factor, int32_t k_first,
                                     int32_t k_last, int32_t precision,
                                     const rpdla_hist_spec* spec, uint64_t* counts,
                                     uint64_t* tallies, uint64_t* electron_steps,
                                     void* workspace, size_t ws_bytes, void* stream)
{
    if (!cfgs) return fail(RPDLA_EINVAL, "cfgs is NULL");
    if (n_cfg < 1) return fail(RPDLA_EINVAL, "n_cfg must be >= 1");
    if (n_cfg > 64) return fail(RPDLA_EUNSUPPORTED, "at most 64 configurations per call");
    for (int c = 0; c < n_cfg; ++c) {
        rpdla_status st = check_laser(&cfgs[c]);
        if (st != RPDLA_OK) return fail(st, "configuration %d: %s", c, g_err.c_str());
        if (cfgs[c].field != cfgs[0].field)
            return fail(RPDLA_EINVAL, "all configurations must use the same field model");
    }
    if (!(precision == RPDLA_FP64 || precision == RPDLA_MIXED))
        return fail(RPDLA_EINVAL, "unknown precision %d", precision);
    if (precision == RPDLA_MIXED && is_lp(cfgs[0].field))
        return fail(RPDLA_EUNSUPPORTED, "the linearly polarized focus has no mixed form");
    if (!(1 <= k_first && k_first <= k_last && k_last <= 10))
        return fail(RPDLA_EINVAL, "need 1 <= k_first <= k_last <= 10");
    if (atoms_per_cfg < 0) return fail(RPDLA_EINVAL, "atoms_per_cfg < 0");
    if (atoms_per_chunk < 1) return fail(RPDLA_EINVAL, "atoms_per_chunk must be >= 1");
    if (!(is_fin(r_factor) && r_factor >= 0)) return fail(RPDLA_EINVAL, "r_factor must be >= 0");
    if (!spec || spec->nE < 1 || spec->nA < 1 ||
        !(is_fin(spec->logE_min_MeV) && is_fin(spec->logE_max_MeV) &&
          spec->logE_min_MeV < spec->logE_max_MeV) ||
        !(spec->angle == RPDLA_ANG_POLAR || spec->angle == RPDLA_ANG_AZIMUTH))
        return fail(RPDLA_EINVAL, "invalid histogram spec");
    if ((int64_t)n_cfg * spec->nE * spec->nA > ((int64_t)1 << 28))
        return fail(RPDLA_ERANGE, "too many histogram bins");
    if (!counts || !tallies || !workspace) return fail(RPDLA_EINVAL, "null pointer");
    const int64_t n_total = cdiv(atoms_per_cfg, atoms_per_chunk);
    const int64_t n_chunks = n_chunks_run < 0 ? n_total - first_chunk : n_chunks_run;
    if (first_chunk < 0 || first_chunk > n_total || n_chunks < 0 || n_chunks > n_total - first_chunk)
        return fail(RPDLA_EINVAL, "chunks [%lld, %lld) outside the stream's %lld chunks",
                    (long long)first_chunk, (long long)(first_chunk + n_chunks),
                    (long long)n_total);
    if (((uintptr_t)workspace & 255) != 0) return fail(RPDLA_EINVAL, "workspace must be 256-byte aligned");
    const int K = k_last - k_first + 1;
    if ((double)n_cfg * (double)atoms_per_chunk * K > 1.0e12)
        return fail(RPDLA_ERANGE, "chunk too large");
    const WsLayout w = ws_layout(n_cfg, atoms_per_chunk, K);
    if (ws_bytes < w.total)
        return fail(RPDLA_ENOMEM, "workspace %zu bytes < required %zu", ws_bytes, w.total);
    hipStream_t s = (hipStream_t)stream;
    char* base = (char*)workspace;
    rpdla::BatchArgs A;
    memset(&A, 0, sizeof A);
    A.cfgs = (const DevCfg*)(base + w.cfg);
    A.geo = (const double*)(base + w.geo);
    A.n_cfg = n_cfg;
    A.seed = seed;
    A.cfg_base = cfg_base;
    A.atoms_per_cfg = atoms_per_cfg;
    A.apc = atoms_per_chunk;
    A.k_first = k_first;
    A.K = K;
    A.x = (double*)(base + w.x); A.y = (double*)(base + w.y); A.z = (double*)(base + w.z);
    A.tb = (double*)(base + w.tb);
    A.ux = (double*)(base + w.ux); A.uy = (double*)(base + w.uy); A.uz = (double*)(base + w.uz);
    A.ctl = (rpdla::BatchCtl*)(base + w.ctl);
    A.H.nE = spec->nE; A.H.nA = spec->nA; A.H.angle = spec->angle;
    A.H.lo = spec->logE_min_MeV;
    A.H.width = (spec->logE_max_MeV - spec->logE_min_MeV) / (double)spec->nE;
    A.H.mec2 = kMeC2MeV;
    A.counts = (unsigned long long*)counts;
    A.tallies = (unsigned long long*)tallies;
    A.steps = (unsigned long long*)electron_steps;
    // configuration table: written by tiny kernels (arguments copied at launch)
    for (int c = 0; c < n_cfg; ++c) {
        const DevCfg dc = make_cfg(&cfgs[c]);
        const double rmax = r_factor * cfgs[c].w0;
        const double zh = rpdla_rayleigh(&cfgs[c]);
        hipLaunchKernelGGL(rpdla::batch_set_cfg_kernel, dim3(1), dim3(64), 0, s, dc, rmax, zh,
                           (DevCfg*)(base + w.cfg), (double*)(base + w.geo), c);
    }
    hipLaunchKernelGGL(rpdla::batch_reset_kernel, dim3(1), dim3(64), 0, s, A.ctl,
                       (unsigned long long)first_chunk);
    RPDLA_HIP(hipGetLastError());
    if (n_chunks == 0) return RPDLA_OK;
    const bool mixed = precision == RPDLA_MIXED;
    switch (cfgs[0].field) {
    case 1: return mixed ? run_batched_impl<1, rpdla::ElecMixed>(A, n_chunks, s)
                         : run_batched_impl<1, rpdla::ElecF64>(A, n_chunks, s);
    case 3: return mixed ? run_batched_impl<3, rpdla::ElecMixed>(A, n_chunks, s)
                         : run_batched_impl<3, rpdla::ElecF64>(A, n_chunks, s);
    case 5: return mixed ? run_batched_impl<5, rpdla::ElecMixed>(A, n_chunks, s)
                         : run_batched_impl<5, rpdla::ElecF64>(A, n_chunks, s);
    case 10: return mixed ? run_batched_impl<10, rpdla::ElecMixed>(A, n_chunks, s)
                          : run_batched_impl<10, rpdla::ElecF64>(A, n_chunks, s);
    case 21: return run_batched_impl<21, rpdla::ElecF64>(A, n_chunks, s);
    case 23: return run_batched_impl<23, rpdla::ElecF64>(A, n_chunks, s);
    case 25: return run_batched_impl<25, rpdla::ElecF64>(A, n_chunks, s);
    default: return mixed ? run_batched_impl<11, rpdla::ElecMixed>(A, n_chunks, s)
                          : run_batched_impl<11, rpdla::ElecF64>(A, n_chunks, s);
    }
}

}  // extern "C"

// ===========================================================================
// Launch-shape autotuning
// ===========================================================================
namespace {

struct DevBuf {
    void* p = nullptr;
    ~DevBuf() { if (p) (void)hipFree(p); }
};

// Time one enqueue of `fn` on stream s (after one untimed call), in ms.
template <class F>
rpdla_status time_ms(hipStream_t s, F fn, float* ms)
{
    rpdla_status st = fn();
    if (st != RPDLA_OK) return st;
    hipEvent_t a, b;
    RPDLA_HIP(hipEventCreate(&a));
    RPDLA_HIP(hipEventCreate(&b));
    RPDLA_HIP(hipEventRecord(a, s));
    st = fn();
    RPDLA_HIP(hipEventRecord(b, s));
    RPDLA_HIP(hipEventSynchronize(b));
    RPDLA_HIP(hipEventElapsedTime(ms, a, b));
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return st;
}

void set_shape(int kind, int field, int prec, Shape sh)
{
    std::lock_guard<std::mutex> lk(g_shape_mu);
    g_shapes[shape_key(kind, field, prec)] = sh;
}

}  // namespace

extern "C" {

rpdla_status rpdla_set_launch_shape(int32_t kernel, int32_t field, int32_t precision, int32_t block,
                                    int32_t grid_factor)
{
    if (kernel < 0 || kernel > 2) return fail(RPDLA_EINVAL, "kernel must be 0 (push), 1 (ionize) or 2 (batched push)");
    if (!(field == 1 || field == 3 || field == 5 || field == 10 || field == 11))
        return fail(RPDLA_EINVAL, "unknown field model %d", field);
    if (!(precision == RPDLA_FP64 || precision == RPDLA_MIXED)) return fail(RPDLA_EINVAL, "unknown precision");
    if (!(block == 64 || block == 128 || block == 192 || block == 256))
        return fail(RPDLA_EINVAL, "block must be 64, 128, 192 or 256");
    if (grid_factor < 1 || grid_factor > 8) return fail(RPDLA_EINVAL, "grid_factor must be 1..8");
    set_shape(kernel, field, kernel == kKindIonize ? 0 : precision, Shape{block, grid_factor});
    return RPDLA_OK;
}

rpdla_status rpdla_get_launch_shape(int32_t kernel, int32_t field, int32_t precision, int32_t* block,
                                    int32_t* grid_factor)
{
    if (!block || !grid_factor) return fail(RPDLA_EINVAL, "null pointer");
    if (kernel < 0 || kernel > 2) return fail(RPDLA_EINVAL, "unknown kernel");
    const Shape sh = get_shape(kernel, field, kernel == kKindIonize ? 0 : precision);
    *block = sh.block;
    *grid_factor = sh.grid_factor;
    return RPDLA_OK;
}

rpdla_status rpdla_autotune(const rpdla_laser* L, int32_t precision, int64_t n_atoms, int32_t k_first,
                            int32_t k_last, char* report, size_t report_len, void* stream)
{
    rpdla_status st = check_laser(L);
    if (st != RPDLA_OK) return st;
    if (!(precision == RPDLA_FP64 || precision == RPDLA_MIXED)) return fail(RPDLA_EINVAL, "unknown precision");
    if (!(1 <= k_first && k_first <= k_last && k_last <= 10)) return fail(RPDLA_EINVAL, "bad charge-state range");
    if (n_atoms < 64 || n_atoms > (1 << 24)) return fail(RPDLA_ERANGE, "probe size must be 64..2^24 atoms");
    hipStream_t s = (hipStream_t)stream;
    const int K = k_last - k_first + 1;
    const int64_t ns = n_atoms * K;
    DevBuf bx, by, bz, btb, bo[6], bcnt, btal, bws;
    RPDLA_HIP(hipMalloc(&bx.p, n_atoms * 8)); RPDLA_HIP(hipMalloc(&by.p, n_atoms * 8));
    RPDLA_HIP(hipMalloc(&bz.p, n_atoms * 8)); RPDLA_HIP(hipMalloc(&btb.p, ns * 8));
    for (auto& b : bo) RPDLA_HIP(hipMalloc(&b.p, ns * 8));
    double* x = (double*)bx.p; double* y = (double*)by.p; double* z = (double*)bz.p;
    double* tb = (double*)btb.p;
    double* o[6];
    for (int i = 0; i < 6; ++i) o[i] = (double*)bo[i].p;
    st = rpdla_sample_atoms(0x5eedull, 0xA070u, 0, n_atoms, 2.0 * L->w0, rpdla_rayleigh(L), x, y, z, stream);
    if (st != RPDLA_OK) return st;
    const int field = L->field;
    const int blocks[3] = {64, 128, 256};
    std::string js = "{\"field\": " + std::to_string(field) + ", \"precision\": " + std::to_string(precision) +
                     ", \"atoms\": " + std::to_string(n_atoms);
    // ionize: threads per block
    {
        const Shape keep = get_shape(kKindIonize, field, 0);
        float best = 1e30f; Shape bsh = keep;
        js += ", \"ionize_ms\": {";
        for (int bi = 0; bi < 3; ++bi) {
            set_shape(kKindIonize, field, 0, Shape{blocks[bi], 1});
            float ms = 0;
            st = time_ms(s, [&] { return rpdla_ionize(L, 0x5eedull, 0xA070u, 0, n_atoms, x, y, z,
                                                      k_first, k_last, tb, stream); }, &ms);
            if (st != RPDLA_OK) { set_shape(kKindIonize, field, 0, keep); return st; }
            js += (bi ? ", \"" : "\"") + std::to_string(blocks[bi]) + "x1\": " + std::to_string(ms);
            if (ms < best) { best = ms; bsh = Shape{blocks[bi], 1}; }
        }
        set_shape(kKindIonize, field, 0, bsh);
        js += "}, \"ionize_best\": \"" + std::to_string(bsh.block) + "x1\"";
    }
    // push: threads per block x persistent grid factor
    {
        const Shape keep = get_shape(kKindPush, field, precision);
        float best = 1e30f; Shape bsh = keep;
        js += ", \"push_ms\": {";
        bool firstc = true;
        for (int bi = 0; bi < 3; ++bi) {
            for (int gf = 1; gf <= 2; ++gf) {
                set_shape(kKindPush, field, precision, Shape{blocks[bi], gf});
                float ms = 0;
                st = time_ms(s, [&] { return rpdla_push(L, precision, ns, tb, x, y, z, K, o[0], o[1], o[2],
                                                        o[3], o[4], o[5], stream); }, &ms);
                if (st != RPDLA_OK) { set_shape(kKindPush, field, precision, keep); return st; }
                js += (firstc ? "\"" : ", \"") + std::to_string(blocks[bi]) + "x" + std::to_string(gf) +
                      "\": " + std::to_string(ms);
                firstc = false;
                if (ms < best) { best = ms; bsh = Shape{blocks[bi], gf}; }
            }
        }
        set_shape(kKindPush, field, precision, bsh);
        js += "}, \"push_best\": \"" + std::to_string(bsh.block) + "x" + std::to_string(bsh.grid_factor) + "\"";
    }
    // batched push (one configuration through the batched path)
    {
        rpdla_hist_spec sp{64, 36, -3.0, 4.0, RPDLA_ANG_POLAR};
        const size_t wsb = rpdla_batched_workspace_bytes(1, n_atoms, k_first, k_last);
        RPDLA_HIP(hipMalloc(&bws.p, wsb));
        RPDLA_HIP(hipMalloc(&bcnt.p, 2 * 64 * 36 * 8));
        RPDLA_HIP(hipMalloc(&btal.p, 6 * 8));
        const Shape keep = get_shape(kKindBatchPush, field, precision);
        float best = 1e30f; Shape bsh = keep;
        js += ", \"batched_push_ms\": {";
        bool firstc = true;
        for (int bi = 0; bi < 3; ++bi) {
            for (int gf = 1; gf <= 2; ++gf) {
                set_shape(kKindBatchPush, field, precision, Shape{blocks[bi], gf});
                float ms = 0;
                st = time_ms(s, [&] {
                    return rpdla_run_batched(L, 1, 0x5eedull, 0xA070u, n_atoms, n_atoms, 2.0, k_first, k_last,
                                             precision, &sp, (uint64_t*)bcnt.p, (uint64_t*)btal.p, nullptr,
                                             bws.p, wsb, stream);
                }, &ms);
                if (st != RPDLA_OK) { set_shape(kKindBatchPush, field, precision, keep); return st; }
                js += (firstc ? "\"" : ", \"") + std::to_string(blocks[bi]) + "x" + std::to_string(gf) +
                      "\": " + std::to_string(ms);
                firstc = false;
                if (ms < best) { best = ms; bsh = Shape{blocks[bi], gf}; }
            }
        }
        set_shape(kKindBatchPush, field, precision, bsh);
        js += "}, \"batched_push_best\": \"" + std::to_string(bsh.block) + "x" + std::to_string(bsh.grid_factor) + "\"";
    }
    RPDLA_HIP(hipStreamSynchronize(s));
    js += "}";
    if (report && report_len > 0) {
        const size_t m = js.size() < report_len - 1 ? js.size() : report_len - 1;
        memcpy(report, js.data(), m);
        report[m] = 0;
    }
    return RPDLA_OK;
}

rpdla_status rpdla_histogram2d(int64_t n, const double* a, const double* b, const double* uz,
                               const rpdla_hist2d_spec* spec, uint64_t* counts, uint64_t* tallies,
                               void* stream)
{
    if (!spec) return fail(RPDLA_EINVAL, "spec is NULL");
    if (spec->na < 1 || spec->nb < 1) return fail(RPDLA_EINVAL, "na, nb must be >= 1");
    if (!(is_fin(spec->a_lo) && is_fin(spec->a_hi) && spec->a_lo < spec->a_hi &&
          is_fin(spec->b_lo) && is_fin(spec->b_hi) && spec->b_lo < spec->b_hi))
        return fail(RPDLA_EINVAL, "need finite a_lo < a_hi and b_lo < b_hi");
    if ((int64_t)spec->na * spec->nb > ((int64_t)1 << 28)) return fail(RPDLA_ERANGE, "too many bins");
    if (n < 0) return fail(RPDLA_EINVAL, "n < 0");
    if (!counts || !tallies) return fail(RPDLA_EINVAL, "null output pointer");
    if (n == 0) return RPDLA_OK;
    if (!a || !b || !uz) return fail(RPDLA_EINVAL, "null input pointer");
    rpdla::Hist2dArgs H;
    H.a_lo = spec->a_lo;
    H.wa = (spec->a_hi - spec->a_lo) / (double)spec->na;
    H.b_lo = spec->b_lo;
    H.wb = (spec->b_hi - spec->b_lo) / (double)spec->nb;
    H.na = spec->na;
    H.nb = spec->nb;
    int64_t blocks = cdiv(n, 256);
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(rpdla::histogram2d_kernel, dim3((unsigned)blocks), dim3(256), 0,
                       (hipStream_t)stream, H, n, a, b, uz, (unsigned long long*)counts,
                       (unsigned long long*)tallies);
    RPDLA_HIP(hipGetLastError());
    return RPDLA_OK;
}

}  // extern "C"

// ===========================================================================
// Kernel resources and occupancy
// ===========================================================================
namespace {

template <typename K>
rpdla_status kernel_info(K kern, int block, size_t lds, int32_t* vgprs, int32_t* scratch,
                         double* waves)
{
    hipFuncAttributes fa;
    RPDLA_HIP(hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(kern)));
    int per_cu = 0;
    RPDLA_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, block, lds));
    *vgprs = fa.numRegs;
    *scratch = (int32_t)fa.localSizeBytes;
    *waves = (double)per_cu * (double)(block / 64) / 4.0;   // four SIMDs per CU
    return RPDLA_OK;
}

template <int FIELD>
rpdla_status field_kernel_info(int kind, bool mixed, int32_t* v, int32_t* s, double* w)
{
    const Shape sh = get_shape(kind, FIELD, kind == kKindIonize ? 0 : (mixed ? 1 : 0));
    if (kind == kKindIonize)
        return kernel_info(rpdla::ionize_kernel<FIELD>, sh.block, 0, v, s, w);
    if constexpr (FIELD > 20) {
        if (mixed) return fail(RPDLA_EUNSUPPORTED, "the linearly polarized focus has no mixed form");
        const size_t lds = (size_t)rpdla::kMaxCfg * sizeof(unsigned long long);
        return kind == kKindPush
                   ? kernel_info(rpdla::push_kernel<FIELD, rpdla::ElecF64>, sh.block, 0, v, s, w)
                   : kernel_info(rpdla::batch_push_kernel<FIELD, rpdla::ElecF64>, sh.block, lds, v, s, w);
    } else {
    if (kind == kKindPush)
        return mixed ? kernel_info(rpdla::push_kernel<FIELD, rpdla::ElecMixed>, sh.block, 0, v, s, w)
                     : kernel_info(rpdla::push_kernel<FIELD, rpdla::ElecF64>, sh.block, 0, v, s, w);
    const size_t lds = (size_t)rpdla::kMaxCfg * sizeof(unsigned long long);
    return mixed ? kernel_info(rpdla::batch_push_kernel<FIELD, rpdla::ElecMixed>, sh.block, lds, v, s, w)
                 : kernel_info(rpdla::batch_push_kernel<FIELD, rpdla::ElecF64>, sh.block, lds, v, s, w);
    }
}

}  // namespace

extern "C" {

rpdla_status rpdla_kernel_occupancy(int32_t kernel, int32_t field, int32_t precision, int32_t* vgprs,
                                    int32_t* scratch_bytes, double* waves_per_simd)
{
    if (!vgprs || !scratch_bytes || !waves_per_simd) return fail(RPDLA_EINVAL, "null pointer");
    if (kernel < 0 || kernel > 2) return fail(RPDLA_EINVAL, "kernel must be 0 (push), 1 (ionize) or 2 (batched push)");
    if (!(precision == RPDLA_FP64 || precision == RPDLA_MIXED)) return fail(RPDLA_EINVAL, "unknown precision");
    const bool mixed = precision == RPDLA_MIXED;
    switch (field) {
    case 1: return field_kernel_info<1>(kernel, mixed, vgprs, scratch_bytes, waves_per_simd);
    case 3: return field_kernel_info<3>(kernel, mixed, vgprs, scratch_bytes, waves_per_simd);
    case 5: return field_kernel_info<5>(kernel, mixed, vgprs, scratch_bytes, waves_per_simd);
    case 10: return field_kernel_info<10>(kernel, mixed, vgprs, scratch_bytes, waves_per_simd);
    case 11: return field_kernel_info<11>(kernel, mixed, vgprs, scratch_bytes, waves_per_simd);
    case 21: return field_kernel_info<21>(kernel, mixed, vgprs, scratch_bytes, waves_per_simd);
    case 23: return field_kernel_info<23>(kernel, mixed, vgprs, scratch_bytes, waves_per_simd);
    case 25: return field_kernel_info<25>(kernel, mixed, vgprs, scratch_bytes, waves_per_simd);
    default: return fail(RPDLA_EINVAL, "unknown field model %d", field);
    }
}

}  // extern "C"
