// Internal declarations shared by the HIP translation units of libnnp.
// gfx950 (CDNA4) only: wave64, MFMA, 160 KB LDS per CU.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nnp.h"

namespace nnp {

constexpr int kWave = 64;
constexpr int kMaxSpecies = 8;
constexpr int kMaxLayers = 8;
constexpr int kTileM = 64;          // rows per MLP tile (atoms of one species)
constexpr int kNr = 16;             // radial shells the AEV kernels are written for
constexpr int kNa = 4;              // angular radial shells
constexpr int kNz = 8;              // angle sections
constexpr float kAccUnit = 9.648533212e-3f;   // eV / (A amu) -> A / fs^2

// AEV hyper-parameters as kernels see them (passed by value).
struct AevConst {
    int ns;              // species
    int radial_dim;      // ns * 16
    int dim;             // radial_dim + ns(ns+1)/2 * 32
    int stride;          // dim rounded up to a multiple of 64
    float rc_r, eta_r, rc_a, eta_a, zeta, pr, cs;
    float pi_rc_r, pi_rc_a;   // pi / Rc
    float shf_r[kNr];
    float shf_a[kNa];
    float cos_z[kNz];
    float sin_z[kNz];
    float hcos_z[kNz];   // cos_z / 2 and sin_z / 2 (exact halves)
    float hsin_z[kNz];
};

// Orthorhombic box as kernels see it (periodic == 0: open boundaries).
struct BoxConst {
    int periodic;
    float L[3];
};

// Per-species, per-layer weight pointers for the MLP kernels.
struct MlpPtrs {
    const float* W[kMaxSpecies][kMaxLayers];        // [Np][Kp]  (out x in), fp32, padded
    const float* WT[kMaxSpecies][kMaxLayers];       // [Kp][Np]  (in x out), fp32, padded
    const uint16_t* Wb[kMaxSpecies][kMaxLayers];    // bf16 copies
    const uint16_t* WTb[kMaxSpecies][kMaxLayers];
    const float* b[kMaxSpecies][kMaxLayers];        // [Np]
    const float* head_w[kMaxSpecies];               // last layer weights [Kp_last]
    float head_b[kMaxSpecies];                      // last bias + self energy (fp32)
};

}  // namespace nnp

struct nnp_model {
    int device;
    nnp_precision precision;
    nnp::AevConst aev;
    int n_layers;                     // including the 1-wide head
    int widths[nnp::kMaxLayers + 1];
    int wpad[nnp::kMaxLayers + 1];    // widths padded to multiples of 64 (head: 1)
    float celu_alpha;
    double self_energy[nnp::kMaxSpecies];
    double head_bias64[nnp::kMaxSpecies];
    void* dev_weights;                // one allocation for every packed weight
    size_t dev_weights_bytes;
    nnp::MlpPtrs ptrs;
    unsigned* flags;                  // device sticky error flags
    void* host_stage;                 // pinned host staging for synchronous reads
    bool fused;                       // widths match the fused 1008-256-192-160-1 kernel
    bool force_unfused;               // use the per-layer GEMM path (testing / comparison)
    int n_nets;                       // networks of the ensemble (1: a single network)
    void* fused_dev;                  // fragment-ordered weight packs, biases, head weights of every network
    void* fused_tab;                  // device tables of per-network pointers (float32 and bfloat16 forms)
    const void* fused_tab_fp32;
    const void* fused_tab_bf16;
    struct nnp_prof* prof;            // per-stage event timing (host side)
};

namespace nnp {

// ---------------------------------------------------------------- wave helpers

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ unsigned long long ballot(bool p) { return __ballot(p); }

// number of set lanes below the calling lane in mask
__device__ __forceinline__ int rank_below(unsigned long long mask) {
    return __popcll(mask & ((1ull << lane_id()) - 1ull));
}

__device__ __forceinline__ float shfl(float v, int src) { return __shfl(v, src, kWave); }
__device__ __forceinline__ int shfl(int v, int src) { return __shfl(v, src, kWave); }
__device__ __forceinline__ float shfl_xor(float v, int m) { return __shfl_xor(v, m, kWave); }
__device__ __forceinline__ double shfl_xor(double v, int m) { return __shfl_xor(v, m, kWave); }
__device__ __forceinline__ int shfl_xor(int v, int m) { return __shfl_xor(v, m, kWave); }

// Make LDS writes of this wave visible to its other lanes.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ void set_flag(unsigned* flags, unsigned bit) {
    atomicOr(flags, bit);
}

// Round-to-nearest-even float32 -> bfloat16 bits.
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
    // gfx950 converts in hardware (v_cvt_pk_bf16_f32: round to nearest even,
    // NaN stays NaN)
    return __builtin_bit_cast(uint16_t, (__bf16)f);
}

__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

inline int ceil_div(long a, long b) { return (int)((a + b - 1) / b); }

}  // namespace nnp

// ---------------------------------------------------------------- launchers (host)

namespace nnp {

struct SelfE {
    double e[kMaxSpecies];
};

struct MlpWs {
    int32_t* bcount;     // [blocks][8]
    int32_t* boff;       // [blocks][8]
    int32_t* meta;       // [32]: counts[8], padded offsets[9]
    int32_t* prow;       // [n] atom -> grouped row
    int32_t* row_atom;   // [rows_max] grouped row -> atom (-1: padding)
    // [n] species present in each atom's environment (bits 0-7 within the
    // radial cutoff, 8-15 within the angular cutoff), from the AEV kernel;
    // null: treat every feature as possibly non-zero
    uint32_t* amask;
    int rows_max;
};

// Per-stage timing hooks (no-ops unless nnp_profile_enable(model, 1)).
void prof_begin(nnp_model* m, int stage, hipStream_t s);
void prof_end(nnp_model* m, int stage, hipStream_t s);

// Optional capacity clamp of an exclusive scan (capacity < 0: none).
struct ScanClamp {
    int64_t capacity;
    int64_t* need;       // device: the largest total seen (atomic max), or null
    unsigned* flags;     // device: NNP_FLAG_CAPACITY on overflow
};
hipError_t launch_exclusive_scan_i32(const int32_t* in, int32_t* out, int64_t* total_out, int n,
                                     int64_t* block_tmp, hipStream_t s, const int32_t* gate = nullptr,
                                     const ScanClamp* clamp = nullptr);
size_t scan_tmp_elems(int n);

size_t neighbors_ws_bytes(int32_t n_atoms, int32_t n_mol, const float* box_host, float r_list);
// sync == false: no pair-count readback (the caller guarantees the capacity),
// device flags go to flags_override (or the model's flags if null).
// rows_out: stop at the builder's fixed-stride rows (in ws) and describe them
// there instead of compacting into nl (its CSR arrays are not touched; the
// reverse index is left to the caller).
struct RowsView;
struct MdFront;
// front (MD engine, with gate = &front->nxt->gate): the step's rebuild
// decision and wrap, taken by the binning kernel (md_front_fuses)
nnp_status build_neighbors(nnp_model* model, int32_t n, const float* pos, const int32_t* mol, int32_t n_mol,
                           const float* box_host, float r_list, nnp_nlist* nl, int64_t* n_pairs_host, void* ws,
                           size_t ws_bytes, hipStream_t s, bool sync = true, unsigned* flags_override = nullptr,
                           const int32_t* gate = nullptr, int64_t* need_pairs = nullptr, bool cells_ready = false,
                           RowsView* rows_out = nullptr, const MdFront* front = nullptr);
struct MdBack;
struct MdEnergyIn;
// Options of the MD engine's calls: skip the species grouping (species and
// workspace unchanged since the last call) and replace the energy sum and
// force gather by the engine's fused last kernel.
struct EfOpts {
    bool skip_group = false;
    bool skip_energy = false;   // no structure energies (e_mol untouched)
    const MdBack* md = nullptr;
    // fixed-stride rows in place of nl's CSR arrays (nl->capacity must cover
    // n * NNP_MAX_ROW); their reverse index is written to rev_out by the AEV
    // kernel while gate is null or *gate != 0
    const RowsView* rows = nullptr;
    int32_t* rev_out = nullptr;
    const int32_t* gate = nullptr;
    bool no_profile = false;    // record no stage events (they may allocate)
    // the structure ranges of mol, already built and checked (by the list
    // build, neighbors_mol_ranges); the energy sum then takes them as they are
    int32_t* mol_start = nullptr;
    int32_t* mol_end = nullptr;
};
// The structure ranges a build with mol left in its workspace.
nnp_status neighbors_mol_ranges(void* ws, int32_t n, int32_t n_mol, const float* box_host, float r_list,
                                int32_t** start, int32_t** end);
// nnp_energy_forces with an explicit device flags word (n_pairs of nl is not checked)
nnp_status energy_forces_impl(nnp_model* m, int32_t n, const float* pos, const int32_t* species, const int32_t* mol,
                              int32_t n_mol, const float* box_host, const nnp_nlist* nl, double* e_mol, float* e_atom,
                              float* forces, void* ws, size_t ws_bytes, hipStream_t s, unsigned* flags,
                              double* virial = nullptr, float* atom_virial = nullptr, const EfOpts* opts = nullptr,
                              double* e_mol_net = nullptr);
nnp_status read_and_clear_flags(nnp_model* m, hipStream_t s, uint32_t* out, int64_t* total_dev,
                                int64_t* total_host);

// Neighbour rows as the kernels read them: the ABI's CSR list, or the
// builder's fixed-stride rows (the MD engine), where row i holds count[i]
// pairs at i * NNP_MAX_ROW and each image shift is packed into one int32
// ((x & 0xff) | (y & 0xff) << 8 | (z & 0xff) << 16).
struct RowsView {
    const int32_t* row_ptr;        // CSR, or null for fixed-stride rows
    const int32_t* count;          // fixed-stride rows
    const int32_t* col;
    const int8_t* shift;           // CSR: int8 [pairs][3]
    const int32_t* shift_packed;   // fixed-stride rows
    const int32_t* rev;            // slot of the reverse pair
    __device__ __forceinline__ int begin(int i) const { return row_ptr ? row_ptr[i] : i * NNP_MAX_ROW; }
    __device__ __forceinline__ int end(int i) const {
        return row_ptr ? row_ptr[i + 1] : i * NNP_MAX_ROW + count[i];
    }
    __device__ __forceinline__ void shift3(int p, float& x, float& y, float& z) const {
        if (row_ptr) {
            x = (float)shift[3 * p];
            y = (float)shift[3 * p + 1];
            z = (float)shift[3 * p + 2];
        } else {
            const int v = shift_packed[p];
            x = (float)(int8_t)(v & 0xff);
            y = (float)(int8_t)((v >> 8) & 0xff);
            z = (float)(int8_t)((v >> 16) & 0xff);
        }
    }
};

// Force on atom a from the edge gradients (Sec. 2.4: forces as the gradient
// of the total energy), F_a = sum_j G_aj - G_ja: the own part sum_j G_aj
// comes summed by the adjoint kernel (Gown[a]), the reverse part G_ja is
// read at rev[p] by kGatherLanes lanes striding over the row, then summed by
// a fixed butterfly.  A lane takes its slots kGatherBatch at a time: every
// reverse index of a batch is loaded before any gradient, so that its loads
// are in flight together (one slot at a time, each slot cost two dependent
// memory latencies); each lane still adds its slots in ascending order.  The
// plain path's gather and the MD engine's last kernel both use it, so the two
// give the same forces bit for bit at the same positions.
constexpr int kGatherLanes = 8;
constexpr int kGatherBatch = 16;

__device__ __forceinline__ float3 gather_row_force(const RowsView& rows, const int32_t* __restrict__ rev,
                                                   const float4* __restrict__ G, const float4* __restrict__ Gown,
                                                   int a, int n, int sub) {
    float fx = 0.f, fy = 0.f, fz = 0.f;
    float4 own = make_float4(0.f, 0.f, 0.f, 0.f);
    if (a < n) {
        if (sub == 0) own = Gown[a];
        const int b = rows.begin(a), e = rows.end(a);
        for (int p0 = b + sub; p0 < e; p0 += kGatherBatch * kGatherLanes) {
            int q[kGatherBatch];
#pragma unroll
            for (int u = 0; u < kGatherBatch; ++u) {
                const int p = p0 + u * kGatherLanes;
                q[u] = p < e ? rev[p] : -1;   // a slot's reverse index is >= 0
            }
            float4 gq[kGatherBatch];
#pragma unroll
            for (int u = 0; u < kGatherBatch; ++u) gq[u] = q[u] >= 0 ? G[q[u]] : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
            for (int u = 0; u < kGatherBatch; ++u) {
                if (q[u] < 0) continue;
                fx += gq[u].x;
                fy += gq[u].y;
                fz += gq[u].z;
            }
        }
    }
#pragma unroll
    for (int m = kGatherLanes / 2; m >= 1; m >>= 1) {
        fx += shfl_xor(fx, m);
        fy += shfl_xor(fy, m);
        fz += shfl_xor(fz, m);
    }
    return make_float3(own.x - fx, own.y - fy, own.z - fz);   // lane sub == 0 of the atom
}

inline RowsView rows_csr(const nnp_nlist* nl) {
    RowsView r{};
    r.row_ptr = nl->row_ptr;
    r.col = nl->col;
    r.shift = nl->shift;
    r.rev = nl->rev;
    return r;
}

// rev_out (fixed-stride rows only, may be null): the reverse index of each
// row, written while gate is null or *gate != 0 (the rows were rebuilt)
// amask_out (may be null): each atom's species-presence mask (MlpWs::amask)
hipError_t launch_aev_fwd(const AevConst& P, int n, const float* pos, const int32_t* species, const BoxConst& bx,
                          const RowsView& rows, const int32_t* out_row, void* out, bool bf16, unsigned* flags,
                          hipStream_t s, int32_t* rev_out = nullptr, const int32_t* gate = nullptr,
                          uint32_t* amask_out = nullptr);
// G: one edge gradient per list slot; Gown: per atom, the sum of its own
// row's edge gradients (the own part of the force)
hipError_t launch_aev_bwd(const AevConst& P, int n, const float* pos, const int32_t* species, const BoxConst& bx,
                          const RowsView& rows, const int32_t* g_row, const float* g, float4* G, float4* Gown,
                          float* atom_virial, unsigned* flags, hipStream_t s);

hipError_t launch_species_group(const nnp_model* m, int n, const int32_t* species, const MlpWs& W, unsigned* flags,
                                hipStream_t s);
hipError_t launch_zero_pad_rows(const MlpWs& W, int stride, void* aev, bool bf16, hipStream_t s);
hipError_t launch_mlp(const nnp_model* m, const MlpWs& W, const void* aev, bool aev_bf16, float* const* h,
                      float* g_out, float* E_row, float* E_atomo, hipStream_t s);
bool fused_mlp_shape(const int* widths, int n_layers, int ns);
size_t fused_net_bytes();
bool mlp_split(const nnp_model* m, int n_atoms);
void fused_net_entry(void* out, int ns, const char* const* packs, const float* const* b1, const float* const* b2,
                     const float* const* b3, const float* const* w4, const float* b4, bool bf16);
hipError_t launch_mlp_ensemble(const nnp_model* m, const MlpWs& W, const void* aev, float* g_out, float* E_row,
                               float* E_atomo, int n_atoms, void* d1_scratch, float* E_net, float* E_atom_net,
                               hipStream_t s);
size_t pack_fused_species(char* dst, bool bf16, const float* W1, const float* W2, const float* W3, int n_in, int n3);
uint16_t host_bf16_bits(float f);
hipError_t launch_mlp_fused(const nnp_model* m, const MlpWs& W, const void* aev, float* g_out, float* E_row,
                            float* E_atomo, int n_atoms, hipStream_t s);
hipError_t launch_permute_rows_bf16(const int32_t* prow, int n, int stride, const float* src, uint16_t* dst,
                                    hipStream_t s);
// ranges_ready: mstart / mend already hold the checked structure ranges of mol
hipError_t launch_energy(int n, int n_mol, const int32_t* mol, const int32_t* species, const SelfE& se,
                         int32_t* mstart, int32_t* mend, bool ranges_ready, const MlpWs& W, const float* E_at,
                         double* e_mol, float* e_atom, unsigned* flags, hipStream_t s);
hipError_t launch_permute_rows(bool to_grouped, const int32_t* prow, int n, int stride, const float* src, float* dst,
                               hipStream_t s);
hipError_t launch_gather_e(const int32_t* prow, int n, const int32_t* species, const SelfE& se, const float* E_row,
                           float* e_atom, hipStream_t s);

size_t virial_partial_doubles(int n);
hipError_t launch_virial(int n, int n_mol, const int32_t* mstart, const int32_t* mend, const float* Wat, double* part,
                         double* virial, hipStream_t s);
hipError_t launch_force_gather(int n, const RowsView& rows, const float4* G, const float4* Gown,
                               float* F, hipStream_t s);
hipError_t launch_kick_drift(int n, float* pos, float* vel, const float* F, const float* inv_mass, float dt,
                             const float* ref, float* max_d2, hipStream_t s);
hipError_t launch_kick(int n, float* vel, const float* F, const float* inv_mass, float dt, hipStream_t s);
hipError_t launch_wrap(int n, float* pos, const float* L, hipStream_t s);

}  // namespace nnp
