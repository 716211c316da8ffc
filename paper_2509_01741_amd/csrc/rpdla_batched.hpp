// rpdla_batched.hpp -- parameter sweeps in one pass per atom chunk: sampling
// and ionization over every configuration's atoms, then ONE persistent push
// launch over every configuration's electrons with a single global work
// queue (lanes refilled as their electron finishes, so uneven step counts
// across wavelengths and powers balance themselves), the configuration table
// staged in LDS and the energy-angle binning fused into the push epilogue.
#pragma once

#include "rpdla_kernels.hpp"

namespace rpdla {

struct BatchCtl {
    unsigned long long chunk;  // index of the chunk being processed
    unsigned long long queue;  // push work counter of the current chunk
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
    BatchCtl* ctl;
    HistArgs H;
    unsigned long long* counts;       // [n_cfg][2 nE nA]
    unsigned long long* tallies;      // [n_cfg][6]
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

__global__ void batch_reset_kernel(BatchCtl* ctl)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) { ctl->chunk = 0ull; ctl->queue = 0ull; }
}

__global__ void batch_zero_queue_kernel(BatchCtl* ctl)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) ctl->queue = 0ull;
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
__global__ void __launch_bounds__(256) batch_ionize_kernel(BatchArgs A)
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
// configuration j / (apc K) and atom (j / K) % apc of the chunk.
template <int FIELD, class ELEC>
__global__ void __launch_bounds__(256) batch_push_kernel(BatchArgs A)
{
    extern __shared__ double lds_raw[];
    const int ncfg = A.n_cfg;
    PushCfg* s_pc = reinterpret_cast<PushCfg*>(lds_raw);
    unsigned long long* s_tal = reinterpret_cast<unsigned long long*>(s_pc + ncfg);
    for (int w = threadIdx.x; w < ncfg; w += blockDim.x) s_pc[w] = push_cfg_of(A.cfgs[w]);
    for (int w = threadIdx.x; w < ncfg * 6; w += blockDim.x) s_tal[w] = 0ull;
    __syncthreads();

    const int64_t per_cfg = A.apc * A.K;
    const int64_t n_slots = (int64_t)ncfg * per_cfg;
    const int64_t first = (int64_t)A.ctl->chunk * A.apc;
    const int64_t nbins = 2ll * A.H.nE * A.H.nA;
    int64_t idx = -1;
    int ci = 0;
    bool exhausted = false;
    ELEC e;
    e.n = e.N = 0;
    while (true) {
        while (true) {
            const bool need = (idx < 0) && !exhausted;
            if (__ballot(need) == 0) break;
            const int64_t j = queue_take(&A.ctl->queue, need);
            if (need) {
                if (j >= n_slots) {
                    exhausted = true;
                } else {
                    const int c = (int)(j / per_cfg);
                    const int64_t a = (j - (int64_t)c * per_cfg) / A.K;
                    if (first + a < A.atoms_per_cfg) {
                        const double t0 = A.tb[j];
                        if (!(t0 < __builtin_inf())) {
                            atomicAdd(&s_tal[c * 6 + 4], 1ull);
                        } else {
                            const int64_t ia = (int64_t)c * A.apc + a;
                            if (elec_init(s_pc[c], e, t0, A.x[ia], A.y[ia], A.z[ia])) {
                                ci = c;
                                idx = j;
                            } else {
                                atomicAdd(&s_tal[c * 6 + 5], 1ull);
                            }
                        }
                    }
                }
            }
        }
        if (__ballot(idx >= 0) == 0) break;
        bool finished = false;
        if (idx >= 0) {
            if (e.n < e.N) elec_step<FIELD>(s_pc[ci], e);
            finished = (e.n >= e.N);
        }
        if (__ballot(finished) != 0) {
            int64_t key = -1;
            int tally = -1, dir = -1;
            if (finished) {
                double ux, uy, uz, xf, yf, zf;
                elec_final(s_pc[ci], e, ux, uy, uz, xf, yf, zf);
                key = bin_key(A.H, 0.0, ux, uy, uz, tally, dir);
                if (key >= 0) key += (int64_t)ci * nbins;
                if (dir >= 0) atomicAdd(&s_tal[ci * 6 + dir], 1ull);
                if (tally >= 2) atomicAdd(&s_tal[ci * 6 + tally], 1ull);
                idx = -1;
            }
            // merge equal bins across the wave, one global atomic per bin
            bool pending = key >= 0;
            while (true) {
                const uint64_t act = __ballot(pending);
                if (act == 0) break;
                const int leader = __ffsll((unsigned long long)act) - 1;
                const int64_t lk = __shfl(key, leader);
                const uint64_t same = __ballot(pending && key == lk);
                if (__lane_id() == leader) atomicAdd(&A.counts[lk], (unsigned long long)__popcll(same));
                if (pending && key == lk) pending = false;
            }
        }
    }
    __syncthreads();
    for (int w = threadIdx.x; w < ncfg * 6; w += blockDim.x)
        if (s_tal[w]) atomicAdd(&A.tallies[w], s_tal[w]);
}

}  // namespace rpdla
