// Device state and launchers of the native MD engine (md.hip, md_engine.cpp).
#pragma once

#include "nnp_internal.hpp"

namespace nnp {

// Lives in device memory; read by the host only after a synchronisation.
struct MdState {
    int32_t gate;              // 1 on steps that rebuild the neighbour list
    int32_t since;             // steps since the last rebuild
    float max_d2;              // largest squared displacement since the last rebuild (this step)
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

hipError_t md_launch_first(int n, float* pos, float* vel, const float* F, const float* inv_mass, const MdStepConst& c,
                           uint64_t step, const float* ref, MdState* st, bool langevin, hipStream_t s);
hipError_t md_launch_decide(MdState* st, int rebuild_every, float trigger2, hipStream_t s);
hipError_t md_launch_wrap_ref(int n, float* pos, float* ref, const BoxConst& bx, const MdState* st, hipStream_t s);
int md_ke_parts(int n);
hipError_t md_launch_last(int n, float* vel, const float* F, const float* inv_mass, float dt, double* ke_part,
                          hipStream_t s);
hipError_t md_launch_log(int n, const double* ke_part, const double* e_pot, double* row, hipStream_t s);
hipError_t md_launch_inv_mass(int n, const float* masses, float* inv_mass, unsigned* flags, hipStream_t s);

}  // namespace nnp
