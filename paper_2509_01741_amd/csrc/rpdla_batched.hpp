// rpdla_batched.hpp -- parameter sweeps in one pass per atom chunk: sampling
// and ionization over every configuration's atoms, then ONE persistent push
// launch over every configuration's electrons (per-configuration work
// counters, each wave serving one configuration at a time from an LDS table,
// lanes refilled as their electron finishes, so uneven step counts across
// wavelengths and powers balance themselves), then one binning pass over the
// chunk's final momenta into per-configuration energy-angle histograms.
#pragma once

#include "rpdla_kernels.hpp"

namespace rpdla {

constexpr int kMaxCfg = 64;

struct BatchCtl {
    unsigned long long chunk;            // index of the chunk being processed
    unsigned long long queue[kMaxCfg];   // per-configuration push work counters
};

struct BatchArgs {
    const DevCfg* cfgs;        // device table [n_cfg]
    const double* geo;         // [n_cfg][2]: sampling radius, half length [m]
    int32_t n_cfg;
    uint64_t seed;
    uint32_t cfg_base;         // RNG key of configuration c is (seed, cfg_base + c)
    int64_t atoms_per_cfg, apc;  // atoms per configuration, atoms per chunk
    int32_t k_first, K;
    double* x; double* y; double* z;  // [n_cfg * apc]
    double* tb;                       // [n_cfg * apc * K]
    double* ux; double* uy; double* uz;  // final momenta [n_cfg * apc * K]
    BatchCtl* ctl;
    HistArgs H;
    unsigned long long* counts;       // [n_cfg][2 nE nA]
    unsigned long long* tallies;      // [n_cfg][6]
    unsigned long long* steps;        // [n_cfg] electron-steps taken, or null
};

__global__ void batch_set_cfg_kernel(DevCfg c, double r_max, double z_half, DevCfg* table,
                                     double* geo, int idx)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        table[idx] = c;
        geo[2 * idx] = r_max;
        geo[2 * idx + 1] = z_half;
    }
}

__global__ void batch_reset_kernel(BatchCtl* ctl, unsigned long long first_chunk)
{
    if (blockIdx.x == 0) {
        if (threadIdx.x == 0) ctl->chunk = first_chunk;
        if (threadIdx.x < kMaxCfg) ctl->queue[threadIdx.x] = 0ull;
    }
}

__global__ void batch_zero_queue_kernel(BatchCtl* ctl)
{
    if (blockIdx.x == 0 && threadIdx.x < kMaxCfg) ctl->queue[threadIdx.x] = 0ull;
}

__global__ void batch_advance_kernel(BatchCtl* ctl)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) ctl->chunk += 1ull;
}

// Atoms of this chunk for every configuration, configuration-major.
__global__ void __launch_bounds__(256) batch_sample_kernel(BatchArgs A)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)A.n_cfg * A.apc) return;
    const int c = (int)(i / A.apc);
    const int64_t a = i - (int64_t)c * A.apc;
    const int64_t first = (int64_t)A.ctl->chunk * A.apc;
    if (first + a >= A.atoms_per_cfg) return;
    const U64x4 r = philox4x64((uint64_t)(first + a), 0, 0, 0, A.seed, (uint64_t)(A.cfg_base + c));
    const double rad = A.geo[2 * c] * sqrt(u01(r.v[0]));
    double sn, cs;
    sincos(kTwoPi * u01(r.v[1]), &sn, &cs);
    A.x[i] = rad * cs;
    A.y[i] = rad * sn;
    A.z[i] = A.geo[2 * c + 1] * (2.0 * u01(r.v[2]) - 1.0);
}

template <int FIELD>
__global__ void __launch_bounds__(256, 2) batch_ionize_kernel(BatchArgs A)
{
    extern __shared__ double lds_raw[];
    DevCfg* s_cfg = reinterpret_cast<DevCfg*>(lds_raw);
    {
        const int nwords = A.n_cfg * (int)(sizeof(DevCfg) / sizeof(double));
        const double* src = reinterpret_cast<const double*>(A.cfgs);
        for (int w = threadIdx.x; w < nwords; w += blockDim.x) lds_raw[w] = src[w];
    }
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)A.n_cfg * A.apc) return;
    const int c = (int)(i / A.apc);
    const int64_t a = i - (int64_t)c * A.apc;
    const int64_t first = (int64_t)A.ctl->chunk * A.apc;
    if (first + a >= A.atoms_per_cfg) return;
    const DevCfg& cf = s_cfg[c];
    ionize_atom<FIELD>(cf, A.seed, A.cfg_base + (uint32_t)c, (uint64_t)(first + a), A.x[i] * cf.k,
                       A.y[i] * cf.k, A.z[i] * cf.k, A.k_first, A.K, A.tb + i * A.K);
}

// One persistent launch over n_cfg * apc * K slots.  Slot j belongs to
// configuration j / (apc K) and atom (j / K) % apc of the chunk.  Every
// configuration has its own work counter, and a wave works on ONE
// configuration at a time: it starts on configuration (wave id mod n_cfg),
// refills its lanes from that configuration's counter, and when the counter
// is exhausted lets its lanes finish and moves on to the next configuration
// that still has work.  The wave's configuration index is therefore uniform,
// and its constants are read from the configuration table (a separate
// read-only kernel argument) with scalar loads at a uniform address, so they
// never occupy vector registers and the compiler can reload instead of
// spilling them.  The step's vector registers hold electron state only.  Final
// momenta go to the chunk's u arrays (NaN for invalid births; unborn and
// inactive slots are not written).
// Register budgets: as the single push, except that the mixed form keeps 6
// waves (its queue switching needs a few more registers than 7 waves leave).
template <class E> struct BatchWaves { static constexpr int value = ElecWaves<E>::value; };
template <> struct BatchWaves<ElecMixed> { static constexpr int value = 6; };

template <int FIELD, class ELEC>
__global__ void __launch_bounds__(256, BatchWaves<ELEC>::value) batch_push_kernel(
    BatchArgs A, const DevCfg* __restrict__ cfgs)
{
    extern __shared__ unsigned long long s_steps[];   // [n_cfg] steps taken in this block
    const int ncfg = A.n_cfg;
    for (int w = threadIdx.x; w < ncfg; w += blockDim.x) s_steps[w] = 0ull;
    __syncthreads();

    const int64_t per_cfg = A.apc * A.K;
    const int64_t first = (int64_t)A.ctl->chunk * A.apc;
    const int wave = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    int cw = __builtin_amdgcn_readfirstlane(wave % ncfg);
    int64_t idx = -1;
    bool draining = false;
    ELEC e;
    e.n = e.N = 0;
    while (true) {
        if (!draining) {
            while (true) {
                const bool need = idx < 0;
                if (__ballot(need) == 0) break;
                const int64_t j = queue_take(&A.ctl->queue[cw], need);
                bool dry = false;
                if (need) {
                    if (j >= per_cfg) {
                        dry = true;
                    } else {
                        const int64_t a = j / A.K;
                        const int64_t js = (int64_t)cw * per_cfg + j;
                        const double t0 = A.tb[js];
                        if (first + a < A.atoms_per_cfg && t0 < __builtin_inf()) {
                            const int64_t ia = (int64_t)cw * A.apc + a;
                            if (elec_init(cfgs[cw], e, t0, A.x[ia], A.y[ia], A.z[ia])) {
                                if (e.N > 0) {
                                    idx = js;
                                    atomicAdd(&s_steps[cw], (unsigned long long)e.N);
                                } else {
                                    double ux, uy, uz, xf, yf, zf;
                                    elec_final(cfgs[cw], e, ux, uy, uz, xf, yf, zf);
                                    A.ux[js] = ux; A.uy[js] = uy; A.uz[js] = uz;
                                }
                            } else {
                                const double q = __builtin_nan("");
                                A.ux[js] = q; A.uy[js] = q; A.uz[js] = q;
                            }
                        }
                    }
                }
                if (__ballot(dry) != 0) { draining = true; break; }
            }
        }
        if (__ballot(idx >= 0) == 0) {
            if (!draining) continue;
            // this configuration is exhausted: move to the next one with work
            int next = -1;
            for (int k = 1; k <= ncfg && next < 0; ++k) {
                const int c2 = (cw + k) % ncfg;
                const unsigned long long taken = atomicAdd(&A.ctl->queue[c2], 0ull);
                if ((int64_t)taken < per_cfg) next = c2;
            }
            if (next < 0) break;
            cw = __builtin_amdgcn_readfirstlane(next);
            draining = false;
            continue;
        }
        if (idx >= 0) {
            elec_step<FIELD>(cfgs[cw], e);
            if (e.n == e.N) {
                double ux, uy, uz, xf, yf, zf;
                elec_final(cfgs[cw], e, ux, uy, uz, xf, yf, zf);
                A.ux[idx] = ux; A.uy[idx] = uy; A.uz[idx] = uz;
                idx = -1;
            }
        }
    }
    if (A.steps) {
        __syncthreads();
        for (int w = threadIdx.x; w < ncfg; w += blockDim.x)
            if (s_steps[w]) atomicAdd(&A.steps[w], s_steps[w]);
    }
}

// Bin the chunk's electrons into their configuration's histogram: one lane
// per slot; bins and tallies merged across the wave (one atomic per distinct
// key).  Tallies as in rpdla_histogram; inactive atoms of a partial chunk are
// skipped.
__global__ void __launch_bounds__(256) batch_hist_kernel(BatchArgs A)
{
    const int64_t per_cfg = A.apc * A.K;
    const int64_t n_slots = (int64_t)A.n_cfg * per_cfg;
    const int64_t first = (int64_t)A.ctl->chunk * A.apc;
    const int64_t nbins = 2ll * A.H.nE * A.H.nA;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t base0 = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63);
    for (int64_t b = base0; b < n_slots; b += stride) {
        const int64_t j = b + __lane_id();
        int64_t key = -1, tkey = -1, dkey = -1;
        if (j < n_slots) {
            const int c = (int)(j / per_cfg);
            const int64_t a = (j - (int64_t)c * per_cfg) / A.K;
            if (first + a < A.atoms_per_cfg) {
                int tally = -1, dir = -1;
                const double t0 = A.tb[j];
                const bool born = t0 < __builtin_inf();
                key = bin_key(A.H, t0, born ? A.ux[j] : 0.0, born ? A.uy[j] : 0.0,
                              born ? A.uz[j] : 0.0, tally, dir);
                if (key >= 0) key += (int64_t)c * nbins;
                if (tally >= 2) tkey = (int64_t)c * 6 + tally;
                if (dir >= 0) dkey = (int64_t)c * 6 + dir;
            }
        }
        wave_merge_add(key, A.counts);
        wave_merge_add(tkey, A.tallies);
        wave_merge_add(dkey, A.tallies);
    }
}

}  // namespace rpdla
