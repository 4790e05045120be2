// Forces from edge gradients, and the velocity-Verlet kernels.
//
// With G_ij = dE_i/dv_ij and v_ij = x_j + n L - x_i, the force on atom a is
//   F_a = -dE/dx_a = sum_{j in N(a)} (G_aj - G_ja),
// where G_ja sits at rev[p] of the pair a -> j (the list is symmetric) and
// the adjoint kernel has summed each row's own part.  Each atom's sum runs
// over its own row in a fixed order (gather_row_force), so no atomics are
// involved (Sec. 2.4: forces as the gradient of the total energy).
#include "nnp_internal.hpp"

namespace nnp {
namespace {

__global__ __launch_bounds__(256) void k_force_gather(int n, const RowsView rows,
                                                     const int32_t* __restrict__ rev, const float4* __restrict__ G,
                                                     const float4* __restrict__ Gown, float* __restrict__ F) {
    const int a = (blockIdx.x * blockDim.x + threadIdx.x) / kGatherLanes;
    const int sub = threadIdx.x % kGatherLanes;
    const float3 f = gather_row_force(rows, rev, G, Gown, a, n, sub);
    if (a < n && sub == 0) {
        F[3 * a] = f.x;
        F[3 * a + 1] = f.y;
        F[3 * a + 2] = f.z;
    }
}

__global__ void k_kick_drift(int n, float* pos, float* vel, const float* F, const float* inv_mass, float dt,
                             const float* ref, float* max_d2) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    float d2 = 0.f;
    if (a < n) {
        const float c = 0.5f * dt * kAccUnit * inv_mass[a];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            float v = vel[3 * a + k] + c * F[3 * a + k];
            vel[3 * a + k] = v;
            const float x = pos[3 * a + k] + dt * v;
            pos[3 * a + k] = x;
            if (ref) {
                const float d = x - ref[3 * a + k];
                d2 += d * d;
            }
        }
    }
    if (ref) {
        d2 = d2 <= INFINITY ? d2 : INFINITY;   // a non-finite displacement must trigger a rebuild
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) d2 = fmaxf(d2, shfl_xor(d2, m));
        if (lane_id() == 0 && d2 > 0.f) atomicMax((unsigned*)max_d2, __float_as_uint(d2));
    }
}

__global__ void k_kick(int n, float* vel, const float* F, const float* inv_mass, float dt) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= n) return;
    const float c = 0.5f * dt * kAccUnit * inv_mass[a];
#pragma unroll
    for (int k = 0; k < 3; ++k) vel[3 * a + k] += c * F[3 * a + k];
}

__global__ void k_wrap(int n, float* pos, float Lx, float Ly, float Lz) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= n) return;
    const float L[3] = {Lx, Ly, Lz};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        float x = pos[3 * a + k];
        x -= L[k] * floorf(x / L[k]);
        if (x >= L[k]) x -= L[k];
        if (x < 0.f) x = 0.f;
        pos[3 * a + k] = x;
    }
}

// Structure virials in float64 from per-centre virials: per-thread sums in
// ascending atom order, then a fixed tree (deterministic).  One block per
// structure; a single large structure is split into fixed chunks whose
// partial sums are added in order by one block.
constexpr int kVirThreads = 256;
constexpr int kVirChunk = 4096;

__device__ void block_sum9(double (&acc)[9], double (*red)[9]) {
    for (int k = 0; k < 9; ++k) red[threadIdx.x][k] = acc[k];
    __syncthreads();
    for (int st = kVirThreads / 2; st >= 1; st >>= 1) {
        if ((int)threadIdx.x < st)
            for (int k = 0; k < 9; ++k) red[threadIdx.x][k] += red[threadIdx.x + st][k];
        __syncthreads();
    }
}

__global__ __launch_bounds__(kVirThreads) void k_virial_mol(int n_mol, const int32_t* mstart, const int32_t* mend,
                                                           const float* Wat, double* out) {
    __shared__ double red[kVirThreads][9];
    const int m = blockIdx.x;
    double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int a = mstart[m] + threadIdx.x; a < mend[m]; a += kVirThreads)
        for (int k = 0; k < 9; ++k) acc[k] += (double)Wat[9 * (size_t)a + k];
    block_sum9(acc, red);
    if (threadIdx.x < 9) out[9 * (size_t)m + threadIdx.x] = red[0][threadIdx.x];
}

__global__ __launch_bounds__(kVirThreads) void k_virial_chunks(int n, const float* Wat, double* part) {
    __shared__ double red[kVirThreads][9];
    const int base = blockIdx.x * kVirChunk;
    const int end = min(n, base + kVirChunk);
    double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int a = base + threadIdx.x; a < end; a += kVirThreads)
        for (int k = 0; k < 9; ++k) acc[k] += (double)Wat[9 * (size_t)a + k];
    block_sum9(acc, red);
    if (threadIdx.x < 9) part[9 * (size_t)blockIdx.x + threadIdx.x] = red[0][threadIdx.x];
}

__global__ void k_virial_final(int nparts, const double* part, double* out) {
    if (threadIdx.x >= 9) return;
    double acc = 0.0;
    for (int q = 0; q < nparts; ++q) acc += part[9 * (size_t)q + threadIdx.x];
    out[threadIdx.x] = acc;
}

}  // namespace

size_t virial_partial_doubles(int n) { return 9 * (size_t)ceil_div(n > 0 ? n : 1, kVirChunk); }

// n_mol == 1: the whole range [0, n); otherwise mstart/mend hold each structure's atom range.
hipError_t launch_virial(int n, int n_mol, const int32_t* mstart, const int32_t* mend, const float* Wat, double* part,
                         double* virial, hipStream_t s) {
    if (n_mol <= 0) return hipSuccess;
    if (n_mol == 1) {
        const int nparts = ceil_div(n > 0 ? n : 1, kVirChunk);
        k_virial_chunks<<<nparts, kVirThreads, 0, s>>>(n, Wat, part);
        k_virial_final<<<1, 64, 0, s>>>(nparts, part, virial);
    } else {
        k_virial_mol<<<n_mol, kVirThreads, 0, s>>>(n_mol, mstart, mend, Wat, virial);
    }
    return hipGetLastError();
}

hipError_t launch_force_gather(int n, const RowsView& rows, const float4* G, const float4* Gown, float* F,
                               hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_force_gather<<<ceil_div((long)n * kGatherLanes, 256), 256, 0, s>>>(n, rows, rows.rev, G, Gown, F);
    return hipGetLastError();
}

hipError_t launch_kick_drift(int n, float* pos, float* vel, const float* F, const float* inv_mass, float dt,
                             const float* ref, float* max_d2, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_kick_drift<<<ceil_div(n, 256), 256, 0, s>>>(n, pos, vel, F, inv_mass, dt, ref, max_d2);
    return hipGetLastError();
}

hipError_t launch_kick(int n, float* vel, const float* F, const float* inv_mass, float dt, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_kick<<<ceil_div(n, 256), 256, 0, s>>>(n, vel, F, inv_mass, dt);
    return hipGetLastError();
}

hipError_t launch_wrap(int n, float* pos, const float* L, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_wrap<<<ceil_div(n, 256), 256, 0, s>>>(n, pos, L[0], L[1], L[2]);
    return hipGetLastError();
}

}  // namespace nnp
