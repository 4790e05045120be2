// Kernels of the native MD engine (Sec. 5.4, "Native MD engine": GPU-resident
// time stepping, velocity Verlet for NVE and BAOAB for Langevin dynamics).
//
// Units: positions A, velocities A/fs, forces eV/A, masses amu, time fs;
// a = F / m * 9.648533212e-3 A/fs^2.
//
//   NVE (velocity Verlet):  B(dt/2) A(dt) | forces | B(dt/2)
//   Langevin (BAOAB):       B(dt/2) A(dt/2) O(dt) A(dt/2) | forces | B(dt/2)
//   with B: v += h a,  A: x += h v,  O: v = c1 v + c2 sqrt(kT / m) xi,
//   c1 = exp(-gamma dt), c2 = sqrt(1 - c1^2).
//
// The Gaussian numbers xi of atom a at step s come from one block of the
// counter-based generator Philox4x64-10 (Salmon, Moraes, Dror and Shaw,
// "Parallel random numbers: as easy as 1, 2, 3", SC'11) with counter
// (a + 1, s, 0, 0) and key (seed, 0): its four 64-bit words give uniforms
// u_k = ((w_k >> 40) + 1/2) 2^-24 in (0, 1), and Box-Muller gives
//   xi_x = rho0 cos(2 pi u1), xi_y = rho0 sin(2 pi u1), xi_z = rho2 cos(2 pi u3),
//   rho_k = sqrt(-2 ln u_k).
// A run replayed from the same state therefore draws the same noise.
//
// Neighbour-list rebuilds are decided on the device (by the fused front
// kernel of small systems, by the cell-binning kernel of the neighbour
// builder for larger periodic boxes of up to 8,192 cells, else by
// k_md_decide), so the host enqueues whole runs without waiting: the later
// list build kernels read the decision through a gate word and do nothing on
// steps without a rebuild.
#include "nnp_internal.hpp"
#include "md_internal.hpp"

namespace nnp {
namespace {

constexpr int kFirstThreads = 256;

// First part of the step; the two largest squared displacements of each
// block go to d2_part[2 block], d2_part[2 block + 1] (one write per block, no
// contended atomics).
template <bool kLangevin>
__global__ __launch_bounds__(kFirstThreads) void k_md_first(int n, float* __restrict__ pos, float* __restrict__ vel,
                                                           const float* __restrict__ F,
                                                           const float* __restrict__ inv_mass, const MdStepConst c,
                                                           uint64_t step, const float* __restrict__ ref,
                                                           float* __restrict__ d2_part) {
    __shared__ float s_m[kFirstThreads / kWave][2];
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    float m1 = 0.f, m2 = 0.f;
    if (a < n) m1 = md_first_atom<kLangevin>(a, pos, vel, F, inv_mass, c, step, ref);
    top2_wave(m1, m2);
    if (lane_id() == 0) {
        s_m[threadIdx.x / kWave][0] = m1;
        s_m[threadIdx.x / kWave][1] = m2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 1; q < kFirstThreads / kWave; ++q) top2_merge(m1, m2, s_m[q][0], s_m[q][1]);
        d2_part[2 * blockIdx.x] = m1;
        d2_part[2 * blockIdx.x + 1] = m2;
    }
}

// Rebuild decision for this step from the blocks' displacements (large
// systems whose binning does not take it; small ones decide in the fused
// front kernel of the neighbour builder).  One block.
__global__ __launch_bounds__(256) void k_md_decide(const MdState* cur_st, MdState* nxt,
                                                   const float* __restrict__ d2_part, int n_parts, int rebuild_every,
                                                   float trig_len) {
    __shared__ float s_m[256 / kWave][2];
    MdState cur{};
    if (threadIdx.x == 0) cur = *cur_st;
    float m1 = 0.f, m2 = 0.f;
    for (int q = threadIdx.x; q < n_parts; q += 256) top2_merge(m1, m2, d2_part[2 * q], d2_part[2 * q + 1]);
    top2_wave(m1, m2);
    if (lane_id() == 0) {
        s_m[threadIdx.x / kWave][0] = m1;
        s_m[threadIdx.x / kWave][1] = m2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 1; q < 256 / kWave; ++q) top2_merge(m1, m2, s_m[q][0], s_m[q][1]);
        md_decide(nxt, cur, m1, m2, rebuild_every, trig_len);
    }
}

// On rebuild steps: wrap into the box (periodic) and take the new reference.
__global__ void k_md_wrap_ref(int n, float* pos, float* ref, BoxConst bx, const MdState* st) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= n || st->gate == 0) return;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        float x = pos[3 * a + k];
        if (bx.periodic) {
            x = md_wrap_coord(x, bx.L[k]);
            pos[3 * a + k] = x;
        }
        ref[3 * a + k] = x;
    }
}

// Force gather (gather_row_force: the same per-atom sum as the plain path's
// k_force_gather), the last half kick and per-block float64 kinetic energies
// (eV), in one kernel.  With kEnergy the structure energy is summed in
// float64 by the first ne = ceil(n / kEChunk) blocks, which are dispatched
// before the gather blocks: block k sums the atoms of chunk k (per-thread
// sums in ascending atom order, then a fixed tree) into part[k]; the block
// that finishes last (an integer ticket) adds the parts in ascending order.
// The order of every addition is fixed, so the energy does not depend on
// scheduling.
constexpr int kBackThreads = 256, kBackAtoms = kBackThreads / kGatherLanes;
constexpr int kEChunk = 4096;
static_assert(kEChunk % kBackThreads == 0, "whole energy chunks per thread");

__device__ __forceinline__ double block_sum(double v, double* red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int st = kBackThreads / 2; st >= 1; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    return red[0];
}

template <bool kEnergy>
__global__ __launch_bounds__(kBackThreads) void k_md_back(int n, int ne, const RowsView rows,
                                                         const int32_t* __restrict__ rev, const float4* __restrict__ G,
                                                         const float4* __restrict__ Gown, float* __restrict__ F, float* __restrict__ vel,
                                                         const float* __restrict__ inv_mass, float dt, double* ke_part,
                                                         const MdEnergyIn E) {
    __shared__ double red[kBackThreads];
    __shared__ double s_se[kMaxSpecies];
    __shared__ int last;
    int blk = blockIdx.x;
    if (kEnergy) {
        if (blk < ne) {
            // a thread's kEPer atoms: every load first, then the sum in
            // ascending atom order (the self energies from LDS)
            constexpr int kEPer = kEChunk / kBackThreads;
            if (threadIdx.x < kMaxSpecies) s_se[threadIdx.x] = E.se[threadIdx.x];
            const int base = blk * kEChunk;
            const int stop = min(n, base + kEChunk);
            int pr[kEPer], sp[kEPer];
            float ea[kEPer];
#pragma unroll
            for (int u = 0; u < kEPer; ++u) {
                const int a = base + (int)threadIdx.x + u * kBackThreads;
                const bool in = a < stop;
                pr[u] = in ? E.prow[a] : -1;
                sp[u] = in ? E.species[a] : 0;
                ea[u] = in ? E.E_at[a] : 0.f;
            }
            __syncthreads();   // s_se
            double acc = 0.0;
#pragma unroll
            for (int u = 0; u < kEPer; ++u)
                if (pr[u] >= 0) acc += (double)ea[u] + s_se[sp[u]];   // a grouped atom has a valid species
            const double tot = block_sum(acc, red);
            if (ne == 1) {
                if (threadIdx.x == 0) *E.e_pot = tot;
                return;
            }
            if (threadIdx.x == 0) {
                E.part[blk] = tot;
                __threadfence();                                   // the part before the ticket
                last = atomicAdd(E.ticket, 1u) == (unsigned)(ne - 1);
            }
            __syncthreads();
            if (!last) return;
            __threadfence();                                       // every part after the last ticket
            if (threadIdx.x == 0) {
                double e = 0.0;
                for (int q = 0; q < ne; ++q) e += __hip_atomic_load(&E.part[q], __ATOMIC_RELAXED,
                                                                    __HIP_MEMORY_SCOPE_AGENT);
                *E.e_pot = e;
                *E.ticket = 0u;                                    // ready for the next step
            }
            return;
        }
        blk -= ne;
    }
    const int a = blk * kBackAtoms + threadIdx.x / kGatherLanes;
    const int sub = threadIdx.x % kGatherLanes;
    const float3 fs = gather_row_force(rows, rev, G, Gown, a, n, sub);
    double ke = 0.0;
    if (a < n && sub == 0) {
        const float f[3] = {fs.x, fs.y, fs.z};
        const float im = inv_mass[a];
        const float kick = 0.5f * dt * kAccUnit * im;
        double v2 = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            F[3 * a + k] = f[k];
            const float v = vel[3 * a + k] + kick * f[k];
            vel[3 * a + k] = v;
            v2 += (double)v * v;
        }
        ke = 0.5 * v2 / ((double)im * (double)kAccUnit);
    }
    if (!ke_part) return;
    const double tot = block_sum(ke, red);
    if (threadIdx.x == 0) ke_part[blk] = tot;
}

// log row: {potential energy, kinetic energy}, both float64, fixed order
__global__ void k_md_log(int nparts, const double* ke_part, const double* e_pot, double* row) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double ke = 0.0;
    for (int q = 0; q < nparts; ++q) ke += ke_part[q];
    row[0] = *e_pot;
    row[1] = ke;
}

__global__ void k_md_inv_mass(int n, const float* masses, float* inv_mass, unsigned* flags) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= n) return;
    const float m = masses[a];
    if (!(m > 0.f) || !isfinite(m)) {
        set_flag(flags, NNP_FLAG_NONFINITE);
        inv_mass[a] = 0.f;
        return;
    }
    inv_mass[a] = 1.f / m;
}

}  // namespace

int md_first_parts(int n) { return ceil_div(n > 0 ? n : 1, kFirstThreads); }

hipError_t md_launch_first(int n, float* pos, float* vel, const float* F, const float* inv_mass, const MdStepConst& c,
                           uint64_t step, const float* ref, float* d2_part, bool langevin, hipStream_t s) {
    const int nb = md_first_parts(n);
    if (langevin) k_md_first<true><<<nb, kFirstThreads, 0, s>>>(n, pos, vel, F, inv_mass, c, step, ref, d2_part);
    else k_md_first<false><<<nb, kFirstThreads, 0, s>>>(n, pos, vel, F, inv_mass, c, step, ref, d2_part);
    return hipGetLastError();
}

hipError_t md_launch_decide(const MdState* cur, MdState* nxt, const float* d2_part, int n_parts, int rebuild_every,
                            float trig_len, hipStream_t s) {
    k_md_decide<<<1, 256, 0, s>>>(cur, nxt, d2_part, n_parts, rebuild_every, trig_len);
    return hipGetLastError();
}

hipError_t md_launch_wrap_ref(int n, float* pos, float* ref, const BoxConst& bx, const MdState* st, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_md_wrap_ref<<<ceil_div(n, 256), 256, 0, s>>>(n, pos, ref, bx, st);
    return hipGetLastError();
}

int md_ke_parts(int n) { return ceil_div(n > 0 ? n : 1, kBackAtoms); }

int md_energy_parts(int n) { return ceil_div(n > 0 ? n : 1, kEChunk); }

hipError_t md_launch_back(int n, const RowsView& rows, const float4* G, const float4* Gown, float* F,
                          const MdBack& b, const MdEnergyIn* e, hipStream_t s) {
    if (b.fuse_energy && e) {
        const int ne = md_energy_parts(n);
        if (ne > 1 && (!e->part || !e->ticket)) return hipErrorInvalidValue;
        k_md_back<true><<<md_ke_parts(n) + ne, kBackThreads, 0, s>>>(n, ne, rows, rows.rev, G, Gown, F, b.vel,
                                                                     b.inv_mass, b.dt, b.ke_part, *e);
    } else {
        k_md_back<false><<<md_ke_parts(n), kBackThreads, 0, s>>>(n, 0, rows, rows.rev, G, Gown, F, b.vel,
                                                                 b.inv_mass, b.dt, b.ke_part, MdEnergyIn{});
    }
    return hipGetLastError();
}

hipError_t md_launch_log(int n, const double* ke_part, const double* e_pot, double* row, hipStream_t s) {
    k_md_log<<<1, 64, 0, s>>>(md_ke_parts(n), ke_part, e_pot, row);
    return hipGetLastError();
}

hipError_t md_launch_inv_mass(int n, const float* masses, float* inv_mass, unsigned* flags, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_md_inv_mass<<<ceil_div(n, 256), 256, 0, s>>>(n, masses, inv_mass, flags);
    return hipGetLastError();
}

}  // namespace nnp
