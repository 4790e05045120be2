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

__device__ __forceinline__ void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1) {
    constexpr uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    constexpr uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += W0;
            k1 += W1;
        }
        const uint64_t lo0 = M0 * c[0], hi0 = __umul64hi(M0, c[0]);
        const uint64_t lo1 = M1 * c[2], hi1 = __umul64hi(M1, c[2]);
        const uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
    }
}

__device__ __forceinline__ float uniform24(uint64_t w) {
    return ((float)(uint32_t)(w >> 40) + 0.5f) * 5.9604644775390625e-8f;   // 2^-24
}

__device__ __forceinline__ void gauss3(uint64_t seed, uint64_t step, int a, float xi[3]) {
    uint64_t c[4] = {(uint64_t)a + 1, step, 0, 0};
    philox4x64_10(c, seed, 0);
    const float u0 = uniform24(c[0]), u1 = uniform24(c[1]), u2 = uniform24(c[2]), u3 = uniform24(c[3]);
    const float r0 = sqrtf(-2.f * logf(u0)), r2 = sqrtf(-2.f * logf(u2));
    const float t1 = 6.283185307179586f * u1, t3 = 6.283185307179586f * u3;
    xi[0] = r0 * cosf(t1);
    xi[1] = r0 * sinf(t1);
    xi[2] = r2 * cosf(t3);
}

template <bool kLangevin>
__global__ __launch_bounds__(256) void k_md_first(int n, float* __restrict__ pos, float* __restrict__ vel,
                                                 const float* __restrict__ F, const float* __restrict__ inv_mass,
                                                 const MdStepConst c, uint64_t step, const float* __restrict__ ref,
                                                 MdState* st) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    float d2 = 0.f;
    if (a < n) {
        const float im = inv_mass[a];
        const float kick = 0.5f * c.dt * kAccUnit * im;
        float x[3], v[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            v[k] = vel[3 * a + k] + kick * F[3 * a + k];
            x[k] = pos[3 * a + k];
        }
        if (kLangevin) {
            float xi[3];
            gauss3(c.seed, step, a, xi);
            const float sig = c.c2 * sqrtf(c.kT * kAccUnit * im);
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                x[k] += 0.5f * c.dt * v[k];
                v[k] = c.c1 * v[k] + sig * xi[k];
                x[k] += 0.5f * c.dt * v[k];
            }
        } else {
#pragma unroll
            for (int k = 0; k < 3; ++k) x[k] += c.dt * v[k];
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            vel[3 * a + k] = v[k];
            pos[3 * a + k] = x[k];
            const float d = x[k] - ref[3 * a + k];
            d2 += d * d;
        }
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) d2 = fmaxf(d2, shfl_xor(d2, m));
    if (lane_id() == 0 && d2 > 0.f) atomicMax((unsigned*)&st->max_d2, __float_as_uint(d2));
}

// Rebuild decision for this step: every `rebuild_every` steps, or earlier
// once an atom has moved more than trigger * skin / 2 since the last build.
__global__ void k_md_decide(MdState* st, int rebuild_every, float trigger2) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int since = st->since + 1;
    const bool due = since >= rebuild_every;
    const bool moved = trigger2 >= 0.f && st->max_d2 > trigger2;
    if (due || moved) {
        st->gate = 1;
        st->since = 0;
        st->rebuilds += 1;
        if (!due) st->early_rebuilds += 1;
    } else {
        st->gate = 0;
        st->since = since;
    }
    st->max_d2 = 0.f;
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

// Last half kick; optionally per-block float64 kinetic energies (eV).
__global__ __launch_bounds__(256) void k_md_last(int n, float* __restrict__ vel, const float* __restrict__ F,
                                                const float* __restrict__ inv_mass, float dt, double* ke_part) {
    __shared__ double red[256];
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    double ke = 0.0;
    if (a < n) {
        const float im = inv_mass[a];
        const float kick = 0.5f * dt * kAccUnit * im;
        double v2 = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const float v = vel[3 * a + k] + kick * F[3 * a + k];
            vel[3 * a + k] = v;
            v2 += (double)v * v;
        }
        ke = 0.5 * v2 / ((double)im * (double)kAccUnit);
    }
    if (!ke_part) return;
    red[threadIdx.x] = ke;
    __syncthreads();
    for (int s = 128; s >= 1; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
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

hipError_t md_launch_first(int n, float* pos, float* vel, const float* F, const float* inv_mass, const MdStepConst& c,
                           uint64_t step, const float* ref, MdState* st, bool langevin, hipStream_t s) {
    const int nb = ceil_div(n > 0 ? n : 1, 256);
    if (langevin) k_md_first<true><<<nb, 256, 0, s>>>(n, pos, vel, F, inv_mass, c, step, ref, st);
    else k_md_first<false><<<nb, 256, 0, s>>>(n, pos, vel, F, inv_mass, c, step, ref, st);
    return hipGetLastError();
}

hipError_t md_launch_decide(MdState* st, int rebuild_every, float trigger2, hipStream_t s) {
    k_md_decide<<<1, 64, 0, s>>>(st, rebuild_every, trigger2);
    return hipGetLastError();
}

hipError_t md_launch_wrap_ref(int n, float* pos, float* ref, const BoxConst& bx, const MdState* st, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_md_wrap_ref<<<ceil_div(n, 256), 256, 0, s>>>(n, pos, ref, bx, st);
    return hipGetLastError();
}

int md_ke_parts(int n) { return ceil_div(n > 0 ? n : 1, 256); }

hipError_t md_launch_last(int n, float* vel, const float* F, const float* inv_mass, float dt, double* ke_part,
                          hipStream_t s) {
    k_md_last<<<md_ke_parts(n), 256, 0, s>>>(n, vel, F, inv_mass, dt, ke_part);
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
