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
// Neighbour-list rebuilds are decided on the device (k_md_decide), so the
// host enqueues whole runs without waiting: the list build kernels read the
// decision through a gate word and do nothing on steps without a rebuild.
#include "nnp_internal.hpp"
#include "md_internal.hpp"

namespace nnp {
namespace {

constexpr int kFirstThreads = 256;

// First part of the step; the largest squared displacement of each block
// goes to d2_part[block] (one write per block, no contended atomics).
template <bool kLangevin>
__global__ __launch_bounds__(kFirstThreads) void k_md_first(int n, float* __restrict__ pos, float* __restrict__ vel,
                                                           const float* __restrict__ F,
                                                           const float* __restrict__ inv_mass, const MdStepConst c,
                                                           uint64_t step, const float* __restrict__ ref,
                                                           float* __restrict__ d2_part) {
    __shared__ float s_max[kFirstThreads / kWave];
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    float d2 = 0.f;
    if (a < n) d2 = md_first_atom<kLangevin>(a, pos, vel, F, inv_mass, c, step, ref);
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) d2 = fmaxf(d2, shfl_xor(d2, m));
    if (lane_id() == 0) s_max[threadIdx.x / kWave] = d2;
    __syncthreads();
    if (threadIdx.x == 0) {
        float mx = s_max[0];
        for (int q = 1; q < kFirstThreads / kWave; ++q) mx = fmaxf(mx, s_max[q]);
        d2_part[blockIdx.x] = mx;
    }
}

// Rebuild decision for this step from the blocks' displacements (large
// systems; small ones decide in the fused front kernel of the neighbour
// builder).  One block.
__global__ __launch_bounds__(256) void k_md_decide(MdState* st, const float* __restrict__ d2_part, int n_parts,
                                                   int rebuild_every, float trigger2) {
    __shared__ float s_max[256 / kWave];
    MdState cur{};
    if (threadIdx.x == 0) cur = *st;
    float mx = 0.f;
    for (int q = threadIdx.x; q < n_parts; q += 256) mx = fmaxf(mx, d2_part[q]);
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) mx = fmaxf(mx, shfl_xor(mx, m));
    if (lane_id() == 0) s_max[threadIdx.x / kWave] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 1; q < 256 / kWave; ++q) mx = fmaxf(mx, s_max[q]);
        md_decide(st, cur, mx, rebuild_every, trigger2);
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
            const float L = bx.L[k];
            x -= L * floorf(x / L);
            if (x >= L) x -= L;
            if (x < 0.f) x = 0.f;
            pos[3 * a + k] = x;
        }
        ref[3 * a + k] = x;
    }
}

// Force gather (16 lanes per atom over its row, F_a = sum_j G_aj - G_ja, as
// in k_force_gather), the last half kick and per-block float64 kinetic
// energies (eV), in one kernel.  With kEnergy, one extra block (the last)
// sums the structure energy in float64 (per-thread sums in ascending atom
// order, then a fixed tree) while the others gather.
constexpr int kBackThreads = 256, kBackLanes = 32, kBackAtoms = kBackThreads / kBackLanes;

template <bool kEnergy>
__global__ __launch_bounds__(kBackThreads) void k_md_back(int n, const RowsView rows,
                                                         const int32_t* __restrict__ rev, const float4* __restrict__ G,
                                                         float* __restrict__ F, float* __restrict__ vel,
                                                         const float* __restrict__ inv_mass, float dt, double* ke_part,
                                                         const MdEnergyIn E) {
    __shared__ double red[kBackThreads];
    if (kEnergy && (int)blockIdx.x == (int)gridDim.x - 1) {
        double acc = 0.0;
        for (int a = threadIdx.x; a < n; a += kBackThreads)
            if (E.prow[a] >= 0) acc += (double)E.E_at[a] + E.se[E.species[a]];
        red[threadIdx.x] = acc;
        __syncthreads();
        for (int st = kBackThreads / 2; st >= 1; st >>= 1) {
            if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
            __syncthreads();
        }
        if (threadIdx.x == 0) *E.e_pot = red[0];
        return;
    }
    const int a = blockIdx.x * kBackAtoms + threadIdx.x / kBackLanes;
    const int sub = threadIdx.x % kBackLanes;
    float fx = 0.f, fy = 0.f, fz = 0.f;
    if (a < n) {
        const int b = rows.begin(a), e = rows.end(a);
        for (int p = b + sub; p < e; p += kBackLanes) {
            const int q = rev[p];
            const float4 gp = G[p], gq = G[q];
            fx += gp.x - gq.x;
            fy += gp.y - gq.y;
            fz += gp.z - gq.z;
        }
    }
#pragma unroll
    for (int m = kBackLanes / 2; m >= 1; m >>= 1) {
        fx += shfl_xor(fx, m);
        fy += shfl_xor(fy, m);
        fz += shfl_xor(fz, m);
    }
    double ke = 0.0;
    if (a < n && sub == 0) {
        const float f[3] = {fx, fy, fz};
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
    red[threadIdx.x] = ke;
    __syncthreads();
    for (int st = kBackThreads / 2; st >= 1; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) ke_part[blockIdx.x] = red[0];
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

hipError_t md_launch_decide(MdState* st, const float* d2_part, int n_parts, int rebuild_every, float trigger2,
                            hipStream_t s) {
    k_md_decide<<<1, 256, 0, s>>>(st, d2_part, n_parts, rebuild_every, trigger2);
    return hipGetLastError();
}

hipError_t md_launch_wrap_ref(int n, float* pos, float* ref, const BoxConst& bx, const MdState* st, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_md_wrap_ref<<<ceil_div(n, 256), 256, 0, s>>>(n, pos, ref, bx, st);
    return hipGetLastError();
}

int md_ke_parts(int n) { return ceil_div(n > 0 ? n : 1, kBackAtoms); }

hipError_t md_launch_back(int n, const RowsView& rows, const float4* G, float* F,
                          const MdBack& b, const MdEnergyIn* e, hipStream_t s) {
    MdEnergyIn E{};
    if (e) E = *e;
    if (b.fuse_energy && e)
        k_md_back<true><<<md_ke_parts(n) + 1, kBackThreads, 0, s>>>(n, rows, rows.rev, G, F, b.vel,
                                                                    b.inv_mass, b.dt, b.ke_part, E);
    else
        k_md_back<false><<<md_ke_parts(n), kBackThreads, 0, s>>>(n, rows, rows.rev, G, F, b.vel,
                                                                 b.inv_mass, b.dt, b.ke_part, E);
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
