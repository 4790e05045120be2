// Device state and launchers of the native MD engine (md.hip, md_engine.cpp).
#pragma once

#include "nnp_internal.hpp"

namespace nnp {

// Lives in device memory; read by the host only after a synchronisation.
// The engine keeps two: the decision of step s reads slot s mod 2 and writes
// slot (s + 1) mod 2, so that every block of a kernel can take the same
// decision from the old state while one of them records the new one.
struct MdState {
    int32_t gate;              // 1 on steps that rebuild the neighbour list
    int32_t since;             // steps since the last rebuild
    float max_d2;              // largest squared displacement since the last rebuild (at the last decision)
    int32_t pad;
    unsigned long long rebuilds;
    unsigned long long early_rebuilds;
};

struct MdStepConst {
    float dt;        // fs
    float c1, c2;    // exp(-gamma dt), sqrt(1 - c1^2)
    float kT;        // eV
    uint64_t seed;
};

// ---- device helpers shared by the integrator kernels (md.hip) and the fused
// front kernel of small systems (neighbors.hip)

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

// three Gaussian numbers of atom a at step `step`: Philox4x64-10 block with
// counter (a + 1, step, 0, 0), key (seed, 0), then Box-Muller
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

// First part of a step for atom a: velocity Verlet B(dt/2) A(dt), or BAOAB
// B(dt/2) A(dt/2) O A(dt/2).  Returns the squared displacement from ref
// (+inf if it is not finite, so that the list is rebuilt and the rebuild
// flags the coordinates).  md_first_load reads what the step needs, so that
// a thread with several atoms can issue every load before the first use;
// md_first_finish computes and stores.
struct MdAtomIn {
    float im, v[3], f[3], x[3], r[3];
};

__device__ __forceinline__ MdAtomIn md_first_load(int a, const float* __restrict__ pos,
                                                  const float* __restrict__ vel, const float* __restrict__ F,
                                                  const float* __restrict__ inv_mass, const float* __restrict__ ref) {
    MdAtomIn q;
    q.im = inv_mass[a];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        q.v[k] = vel[3 * a + k];
        q.f[k] = F[3 * a + k];
        q.x[k] = pos[3 * a + k];
        q.r[k] = ref[3 * a + k];
    }
    return q;
}

template <bool kLangevin>
__device__ __forceinline__ float md_first_finish(int a, const MdAtomIn& q, float* __restrict__ pos,
                                                 float* __restrict__ vel, const MdStepConst& c, uint64_t step,
                                                 float* xout = nullptr) {
    const float kick = 0.5f * c.dt * kAccUnit * q.im;
    float x[3], v[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        v[k] = q.v[k] + kick * q.f[k];
        x[k] = q.x[k];
    }
    if (kLangevin) {
        float xi[3];
        gauss3(c.seed, step, a, xi);
        const float sig = c.c2 * sqrtf(c.kT * kAccUnit * q.im);
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
    float d2 = 0.f;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        vel[3 * a + k] = v[k];
        pos[3 * a + k] = x[k];
        if (xout) xout[k] = x[k];
        const float d = x[k] - q.r[k];
        d2 += d * d;
    }
    return d2 <= INFINITY ? d2 : INFINITY;
}

template <bool kLangevin>
__device__ __forceinline__ float md_first_atom(int a, float* __restrict__ pos, float* __restrict__ vel,
                                               const float* __restrict__ F, const float* __restrict__ inv_mass,
                                               const MdStepConst& c, uint64_t step, const float* __restrict__ ref,
                                               float* xout = nullptr) {
    return md_first_finish<kLangevin>(a, md_first_load(a, pos, vel, F, inv_mass, ref), pos, vel, c, step, xout);
}

// The two largest squared displacements of a set of atoms (m1 >= m2):
// adding one atom, merging two disjoint sets, and the whole wave.
__device__ __forceinline__ void top2_add(float& m1, float& m2, float x) {
    m2 = fmaxf(m2, fminf(m1, x));
    m1 = fmaxf(m1, x);
}
__device__ __forceinline__ void top2_merge(float& m1, float& m2, float n1, float n2) {
    m2 = fmaxf(fminf(m1, n1), fmaxf(m2, n2));
    m1 = fmaxf(m1, n1);
}
__device__ __forceinline__ void top2_wave(float& m1, float& m2) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        const float n1 = shfl_xor(m1, m), n2 = shfl_xor(m2, m);
        top2_merge(m1, m2, n1, n2);
    }
}

// Rebuild decision (one thread): every rebuild_every steps, or earlier once
// the two largest displacements since the last build, d1 + d2, exceed
// trig_len = trigger * skin (trig_len < 0: no displacement check).  A pair
// outside the list was at least r_list = Rc + skin apart at the build and
// its distance has since shrunk by at most d_i + d_j <= d1 + d2, so no pair
// can come within Rc before the check fires (the Verlet-list bound).  cur is
// the state before this step's decision; the new state is written whole to
// nxt unless nxt is null.
__device__ __forceinline__ int md_decide(MdState* nxt, const MdState& cur, float m1, float m2, int rebuild_every,
                                         float trig_len) {
    const int since = cur.since + 1;
    const bool due = since >= rebuild_every;
    const bool moved = trig_len >= 0.f && !(sqrtf(m1) + sqrtf(m2) <= trig_len);   // NaN rebuilds
    const int gate = due || moved ? 1 : 0;
    if (nxt) {
        MdState o = cur;
        o.gate = gate;
        o.since = gate ? 0 : since;
        o.max_d2 = m1;
        if (gate) {
            o.rebuilds = cur.rebuilds + 1;
            if (!due) o.early_rebuilds = cur.early_rebuilds + 1;
        }
        *nxt = o;
    }
    return gate;
}

// One coordinate wrapped into [0, L) on a rebuild step (the same arithmetic
// wherever the engine wraps).
__device__ __forceinline__ float md_wrap_coord(float x, float L) {
    x -= L * floorf(x / L);
    if (x >= L) x -= L;
    if (x < 0.f) x = 0.f;
    return x;
}

// The rebuild decision and the wrap of a step, taken by the cell-binning
// kernel of the neighbour builder (periodic boxes binned and scanned in one
// kernel): every block reduces d2_part to the same two largest
// displacements and decides; block 0 records the new state in nxt; on
// rebuild steps each atom is wrapped into the box and becomes its own
// displacement reference.
struct MdFront {
    const MdState* cur;     // state before this step's decision
    MdState* nxt;           // state after it
    const float* d2_part;   // [2 n_parts] per-block two largest squared displacements
    int n_parts;
    int rebuild_every;
    float trig_len;
    float* pos;             // the positions being binned (wrapped in place)
    float* ref;             // displacement reference (written on rebuild steps)
};

// Energy fused into the last kernel of a step: what it needs.
struct MdEnergyIn {
    const int32_t* prow;      // grouped row of each atom (< 0: no network energy)
    const int32_t* species;
    const float* E_at;        // network energies in atom order
    double se[kMaxSpecies];   // self energies
    double* e_pot;            // [1]
    double* part;             // [md_energy_parts(n)] chunk sums (unused for one chunk)
    unsigned* ticket;         // zero between launches (the last block resets it)
};

// Second part of a step: force gather, B(dt/2), per-block kinetic energies.
struct MdBack {
    float* vel;
    const float* inv_mass;
    float dt;
    double* ke_part;          // [md_ke_parts(n)] or null
    bool fuse_energy;         // sum the structure energy in the same kernel
    double* e_part;           // [md_energy_parts(n)] chunk sums of the structure energy
    unsigned* e_ticket;       // one word, zero between launches
};

// d2_part: [2 md_first_parts(n)] per-block two largest squared displacements
int md_first_parts(int n);
hipError_t md_launch_first(int n, float* pos, float* vel, const float* F, const float* inv_mass, const MdStepConst& c,
                           uint64_t step, const float* ref, float* d2_part, bool langevin, hipStream_t s);
hipError_t md_launch_decide(const MdState* cur, MdState* nxt, const float* d2_part, int n_parts, int rebuild_every,
                            float trig_len, hipStream_t s);
hipError_t md_launch_wrap_ref(int n, float* pos, float* ref, const BoxConst& bx, const MdState* st, hipStream_t s);
int md_ke_parts(int n);
int md_energy_parts(int n);
hipError_t md_launch_back(int n, const RowsView& rows, const float4* G, const float4* Gown, float* F,
                          const MdBack& b, const MdEnergyIn* e, hipStream_t s);
// neighbors.hip: the fused front of a step for small systems
bool md_front_fits(int n, const float* box_host, float r_list);
nnp_status launch_md_front(int n, float* pos, float* vel, const float* F, const float* inv_mass, const MdStepConst& c,
                           uint64_t step, float* ref, const MdState* cur, MdState* nxt, int rebuild_every,
                           float trig_len, bool langevin, const float* box_host, float r_list, void* ws,
                           size_t ws_bytes, unsigned* flags, hipStream_t s);
// neighbors.hip: whether build_neighbors can take an MdFront (the binning
// and scan of this box run as one kernel)
bool md_front_fuses(int n, const float* box_host, float r_list);
hipError_t md_launch_log(int n, const double* ke_part, const double* e_pot, double* row, hipStream_t s);
hipError_t md_launch_inv_mass(int n, const float* masses, float* inv_mass, unsigned* flags, hipStream_t s);

}  // namespace nnp
