// extern "C" entry points of libnnp (declared in include/nnp.h): argument
// checks, workspace carving, weight packing and kernel sequencing.  Every
// step of the computation runs in the HIP kernels of this library.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <vector>

#include "md_internal.hpp"
#include "nnp_internal.hpp"

using namespace nnp;

namespace {

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
inline int round_up(int x, int m) { return (x + m - 1) / m * m; }

uint16_t host_bf16(float f) { return nnp::host_bf16_bits(f); }

std::mutex g_stage_mutex;

}  // namespace

// Fixed device scratch of nnp_energy_forces_static (callers that cannot
// allocate).  In host code this name is only a stand-in for the symbol: the
// device address comes from hipGetSymbolAddress, once per device, and only
// that address is ever handed to kernels or runtime calls.
static __device__ __align__(256) char scratch[NNP_STATIC_SCRATCH_BYTES];

namespace {

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_addr[kMaxScratchDevices] = {};

// the device address of `scratch` on `device` (which must be current),
// resolved on the first call for that device
nnp_status scratch_address(int device, void** out) {
    if (device < 0 || device >= kMaxScratchDevices) return NNP_E_ARG;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_addr[device]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return NNP_E_HIP;
        g_scratch_addr[device] = p;
    }
    *out = g_scratch_addr[device];
    return NNP_OK;
}

}  // namespace

struct nnp_prof {
    bool enabled = false;
    uint32_t mask = 0;        // stages timed while enabled
    std::mutex mu;
    std::vector<hipEvent_t> free_events;
    struct Pair { hipEvent_t a, b; int stage; };
    std::vector<Pair> pending;
    hipEvent_t open[NNP_N_STAGES] = {};
    double ms[NNP_N_STAGES] = {};
    int64_t cnt[NNP_N_STAGES] = {};

    hipEvent_t take() {
        if (!free_events.empty()) {
            hipEvent_t e = free_events.back();
            free_events.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
    void drain() {
        for (auto& p : pending) {
            float t = 0.f;
            if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&t, p.a, p.b) == hipSuccess) {
                ms[p.stage] += t;
                cnt[p.stage] += 1;
            }
            free_events.push_back(p.a);
            free_events.push_back(p.b);
        }
        pending.clear();
    }
    ~nnp_prof() {
        drain();
        for (auto e : free_events) (void)hipEventDestroy(e);
        for (auto e : open)
            if (e) (void)hipEventDestroy(e);
    }
};

namespace nnp {

void prof_begin(nnp_model* m, int stage, hipStream_t s) {
    nnp_prof* p = m->prof;
    if (!p || !p->enabled || !((p->mask >> stage) & 1u)) return;
    std::lock_guard<std::mutex> lock(p->mu);
    if (p->pending.size() > 16384) p->drain();
    hipEvent_t e = p->take();
    if (!e) return;
    if (p->open[stage]) p->free_events.push_back(p->open[stage]);
    p->open[stage] = e;
    (void)hipEventRecord(e, s);
}

void prof_end(nnp_model* m, int stage, hipStream_t s) {
    nnp_prof* p = m->prof;
    if (!p || !p->enabled || !((p->mask >> stage) & 1u)) return;
    std::lock_guard<std::mutex> lock(p->mu);
    hipEvent_t a = p->open[stage];
    if (!a) return;
    hipEvent_t b = p->take();
    if (!b) return;
    (void)hipEventRecord(b, s);
    p->pending.push_back({a, b, stage});
    p->open[stage] = nullptr;
}

}  // namespace nnp

namespace {

struct EfWs {
    MlpWs mw;
    int32_t* mstart;
    int32_t* mend;
    void* aev;          // [rows_max][stride] float32-sized (bf16 rows use the first half)
    float* g;           // [rows_max][stride] float32 dE/dAEV (its own buffer: tiles run concurrently)
    float* h[kMaxLayers];
    float* E_row;
    float* E_at;        // network energies in atom order
    float4* G;      // edge gradients dE/dv_ij, one (x, y, z, 0) per list slot
    float4* Gown;       // per atom, the sum of its row's edge gradients
    float* Wat;         // per-centre virials [n][9] when the caller passes none
    double* vpart;      // chunk partials of the structure virial
    void* d1;           // ensembles: per-network dE/dh1 [n_nets][rows_max][256]
    float* E_net;       // ensembles: per-network energies [n_nets][rows_max]
    float* E_at_net;    // ensembles: per-network atomic energies [n_nets][n]
    size_t end;
};

EfWs ef_layout(const nnp_model* m, int n, int64_t cap, char* base) {
    EfWs W;
    std::memset(&W, 0, sizeof(W));
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o = align256(o + bytes); return base ? (void*)(base + r) : nullptr; };
    const int nn = n > 0 ? n : 1;
    const int nb = ceil_div(nn, 1024);
    const int rows_max = round_up(nn, kTileM) + m->aev.ns * kTileM;
    W.mw.rows_max = rows_max;
    W.mw.bcount = (int32_t*)take(sizeof(int32_t) * nb * kMaxSpecies);
    W.mw.boff = (int32_t*)take(sizeof(int32_t) * nb * kMaxSpecies);
    W.mw.meta = (int32_t*)take(sizeof(int32_t) * 32);
    W.mw.prow = (int32_t*)take(sizeof(int32_t) * nn);
    W.mw.row_atom = (int32_t*)take(sizeof(int32_t) * rows_max);
    W.mw.amask = (uint32_t*)take(sizeof(uint32_t) * nn);
    W.mstart = (int32_t*)take(sizeof(int32_t) * (nn + 1));
    W.mend = (int32_t*)take(sizeof(int32_t) * (nn + 1));
    W.aev = take(sizeof(float) * (size_t)rows_max * m->aev.stride);
    W.g = (float*)take(sizeof(float) * (size_t)rows_max * m->aev.stride);
    for (int l = 0; l + 1 < m->n_layers; ++l) W.h[l] = (float*)take(sizeof(float) * (size_t)rows_max * m->wpad[l + 1]);
    W.E_row = (float*)take(sizeof(float) * rows_max);
    W.E_at = (float*)take(sizeof(float) * nn);
    const int64_t c = cap > 0 ? cap : 1;
    W.G = (float4*)take(sizeof(float4) * c);
    W.Gown = (float4*)take(sizeof(float4) * nn);
    W.Wat = (float*)take(sizeof(float) * 9 * (size_t)nn);
    W.vpart = (double*)take(sizeof(double) * virial_partial_doubles(nn));
    if (mlp_split(m, nn)) {
        W.d1 = take(sizeof(float) * (size_t)m->n_nets * rows_max * 256);
        W.E_net = (float*)take(sizeof(float) * (size_t)m->n_nets * rows_max);
        W.E_at_net = (float*)take(sizeof(float) * (size_t)m->n_nets * nn);
    }
    W.end = o;
    return W;
}

BoxConst box_const(const float* box_host) {
    BoxConst b;
    b.periodic = box_host != nullptr;
    for (int k = 0; k < 3; ++k) b.L[k] = box_host ? box_host[k] : 0.f;
    return b;
}

SelfE self_e(const nnp_model* m) {
    SelfE s;
    for (int k = 0; k < kMaxSpecies; ++k) s.e[k] = m->self_energy[k];
    return s;
}

nnp_status hip_status(hipError_t e) { return e == hipSuccess ? NNP_OK : NNP_E_HIP; }

}  // namespace

namespace nnp {

uint16_t host_bf16_bits(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

nnp_status read_and_clear_flags(nnp_model* m, hipStream_t s, uint32_t* out, int64_t* total_dev, int64_t* total_host) {
    std::lock_guard<std::mutex> lock(g_stage_mutex);
    char* st = (char*)m->host_stage;
    if (hipMemcpyAsync(st, m->flags, sizeof(unsigned), hipMemcpyDeviceToHost, s) != hipSuccess) return NNP_E_HIP;
    if (total_dev && hipMemcpyAsync(st + 8, total_dev, sizeof(int64_t), hipMemcpyDeviceToHost, s) != hipSuccess)
        return NNP_E_HIP;
    if (hipStreamSynchronize(s) != hipSuccess) return NNP_E_HIP;
    uint32_t fl;
    std::memcpy(&fl, st, 4);
    if (total_dev && total_host) std::memcpy(total_host, st + 8, 8);
    if (fl) {
        if (hipMemsetAsync(m->flags, 0, sizeof(unsigned), s) != hipSuccess) return NNP_E_HIP;
        if (hipStreamSynchronize(s) != hipSuccess) return NNP_E_HIP;
    }
    if (out) *out = fl;
    return NNP_OK;
}

}  // namespace nnp

nnp_status nnp::energy_forces_impl(nnp_model* m, int32_t n, const float* pos, const int32_t* species,
                                   const int32_t* mol, int32_t n_mol, const float* box_host, const nnp_nlist* nl,
                                   double* e_mol, float* e_atom, float* forces, void* ws, size_t ws_bytes,
                                   hipStream_t s, unsigned* flags, double* virial, float* atom_virial,
                                   const EfOpts* opts, double* e_mol_net) {
    if (!m || !nl || n < 0) return NNP_E_ARG;
    if (n > 0 && (!pos || !species)) return NNP_E_ARG;
    if (n_mol < 0 || (n > 0 && n_mol < 1) || n_mol > (n > 0 ? n : 1)) return NNP_E_ARG;
    if (n_mol > 0 && !e_mol) return NNP_E_ARG;
    if (nl->n_atoms != n) return NNP_E_ARG;
    if (box_host && (nl->r_list * 2.f > box_host[0] || nl->r_list * 2.f > box_host[1] || nl->r_list * 2.f > box_host[2]))
        return NNP_E_BOX;
    if (nl->r_list < m->aev.rc_r) return NNP_E_ARG;
    const EfWs need = ef_layout(m, n, nl->capacity, nullptr);
    if (!ws || ws_bytes < need.end) return NNP_E_ARG;
    const EfWs W = ef_layout(m, n, nl->capacity, (char*)ws);
    const BoxConst bx = box_const(box_host);
    const bool bf = m->precision == NNP_BF16_MLP;
    hipError_t e = hipSuccess;
    const MdBack* md = opts ? opts->md : nullptr;
    if (md && (!forces || virial || atom_virial)) return NNP_E_ARG;
    const RowsView rows = opts && opts->rows ? *opts->rows : rows_csr(nl);
    const bool timed = !(opts && opts->no_profile);
    auto pbeg = [&](int stage) { if (timed) prof_begin(m, stage, s); };
    auto pend = [&](int stage) { if (timed) prof_end(m, stage, s); };
    if (opts && opts->rows && nl->capacity < (int64_t)n * NNP_MAX_ROW) return NNP_E_ARG;
    if (n > 0 && !(opts && opts->skip_group)) {
        pbeg(NNP_STAGE_GROUP);
        e = launch_species_group(m, n, species, W.mw, flags, s);
        // the per-layer GEMMs read padding rows; the fused kernel keeps them to their own rows
        if (e == hipSuccess && !(m->fused && !m->force_unfused))
            e = launch_zero_pad_rows(W.mw, m->aev.stride, W.aev, bf, s);
        pend(NNP_STAGE_GROUP);
    }
    if (n > 0) {
        pbeg(NNP_STAGE_AEV);
        if (e == hipSuccess) e = launch_aev_fwd(m->aev, n, pos, species, bx, rows, W.mw.prow, W.aev, bf, flags, s,
                               opts ? opts->rev_out : nullptr, opts ? opts->gate : nullptr, W.mw.amask);
        pend(NNP_STAGE_AEV);
        pbeg(NNP_STAGE_MLP);
        const bool ens = mlp_split(m, n) && !(m->force_unfused && m->n_nets == 1);
        const bool fused_nets = ens || (m->fused && !m->force_unfused);
        if (e == hipSuccess) {
            if (ens)
                e = launch_mlp_ensemble(m, W.mw, W.aev, forces ? W.g : nullptr, W.E_row, W.E_at, n, W.d1, W.E_net,
                                        e_mol_net ? W.E_at_net : nullptr, s);
            else if (fused_nets)
                e = launch_mlp_fused(m, W.mw, W.aev, forces ? W.g : nullptr, W.E_row, W.E_at, n, s);
            else
                e = launch_mlp(m, W.mw, W.aev, bf, W.h, forces ? W.g : nullptr, W.E_row, W.E_at, s);
        }
        pend(NNP_STAGE_MLP);
    }
    if (!(md && md->fuse_energy) && !(opts && opts->skip_energy)) {
        pbeg(NNP_STAGE_ENERGY);
        {
            // the ranges of mol: the caller's (already checked), else built by the first sum
            const bool given = opts && opts->mol_start && opts->mol_end && mol;
            int32_t* ms = given ? opts->mol_start : W.mstart;
            int32_t* me = given ? opts->mol_end : W.mend;
            if (e == hipSuccess)
                e = launch_energy(n, n_mol, mol, species, self_e(m), ms, me, given, W.mw, W.E_at, e_mol, e_atom,
                                  flags, s);
            // ensembles: every network's structure energies (self energies included)
            for (int k = 0; e_mol_net && k < m->n_nets && e == hipSuccess && n > 0; ++k)
                e = launch_energy(n, n_mol, mol, species, self_e(m), ms, me, true, W.mw, W.E_at_net + (size_t)k * n,
                                  e_mol_net + (size_t)k * n_mol, nullptr, flags, s);
        }
        pend(NNP_STAGE_ENERGY);
    }
    if (e == hipSuccess && forces && n > 0) {
        pbeg(NNP_STAGE_AEV_ADJ);
        float* wat = virial || atom_virial ? (atom_virial ? atom_virial : W.Wat) : nullptr;
        e = launch_aev_bwd(m->aev, n, pos, species, bx, rows, W.mw.prow, W.g, W.G, W.Gown, wat, flags, s);
        pend(NNP_STAGE_AEV_ADJ);
        pbeg(NNP_STAGE_FORCES);
        if (e == hipSuccess) {
            if (md) {
                // engine: gather + last half kick (+ structure energy) in one kernel
                MdEnergyIn ein{};
                ein.prow = W.mw.prow;
                ein.species = species;
                ein.E_at = W.E_at;
                for (int k = 0; k < kMaxSpecies; ++k) ein.se[k] = m->self_energy[k];
                ein.e_pot = e_mol;
                ein.part = md->e_part;
                ein.ticket = md->e_ticket;
                e = md_launch_back(n, rows, W.G, W.Gown, forces, *md, &ein, s);
            } else {
                e = launch_force_gather(n, rows, W.G, W.Gown, forces, s);
            }
        }
        pend(NNP_STAGE_FORCES);
    }
    if (e == hipSuccess && virial)
        e = launch_virial(n, n_mol, W.mstart, W.mend, atom_virial ? atom_virial : W.Wat, W.vpart, virial, s);
    return hip_status(e);
}


extern "C" {

const char* nnp_status_str(nnp_status s) {
    switch (s) {
        case NNP_OK: return "ok";
        case NNP_E_ARG: return "invalid argument";
        case NNP_E_CAPACITY: return "neighbour-list capacity too small";
        case NNP_E_BOX: return "box side below twice the list cutoff";
        case NNP_E_NONFINITE: return "non-finite coordinates";
        case NNP_E_NOMEM: return "out of memory";
        case NNP_E_BUSY: return "no free request slot";
        case NNP_E_PENDING: return "request pending";
        case NNP_E_HIP: return "HIP runtime error";
        case NNP_E_ROW: return "neighbour row longer than supported";
        case NNP_E_SCRATCH: return "input larger than the fixed scratch of the allocation-free call";
    }
    return "unknown status";
}

nnp_status nnp_model_create(const nnp_aev_params* a, const nnp_mlp_params* p, nnp_precision precision,
                            nnp_model** out) {
    return nnp_model_create_ensemble(a, p, 1, precision, out);
}

nnp_status nnp_model_create_ensemble(const nnp_aev_params* a, const nnp_mlp_params* nets, int32_t n_nets,
                                     nnp_precision precision, nnp_model** out) {
    if (!a || !nets || !out || n_nets < 1 || n_nets > NNP_MAX_NETS) return NNP_E_ARG;
    const nnp_mlp_params* p = &nets[0];
    for (int k = 1; k < n_nets; ++k) {
        if (nets[k].n_layers != p->n_layers || !nets[k].widths || !nets[k].W || !nets[k].b) return NNP_E_ARG;
        for (int l = 0; l <= p->n_layers; ++l)
            if (nets[k].widths[l] != p->widths[l]) return NNP_E_ARG;
    }
    *out = nullptr;
    if (a->n_species < 1 || a->n_species > kMaxSpecies) return NNP_E_ARG;
    if (a->n_shf_r != kNr || a->n_shf_a != kNa || a->n_shf_z != kNz) return NNP_E_ARG;
    if (!a->shf_r || !a->shf_a || !a->shf_z) return NNP_E_ARG;
    if (!(a->rc_r > 0.f) || !(a->rc_a > 0.f) || a->rc_a > a->rc_r) return NNP_E_ARG;
    if (precision != NNP_FP32 && precision != NNP_BF16_MLP) return NNP_E_ARG;
    const int ns = a->n_species;
    const int L = p->n_layers;
    if (L < 2 || L > kMaxLayers || !p->widths || !p->W || !p->b) return NNP_E_ARG;
    const int dim = ns * kNr + ns * (ns + 1) / 2 * kNa * kNz;
    if (p->widths[0] != dim || p->widths[L] != 1) return NNP_E_ARG;
    for (int l = 1; l < L; ++l)
        if (p->widths[l] < 1 || p->widths[l] > 4096) return NNP_E_ARG;
    if (!(p->celu_alpha > 0.f)) return NNP_E_ARG;

    nnp_model* m = new nnp_model;
    std::memset(m, 0, sizeof(*m));
    if (hipGetDevice(&m->device) != hipSuccess) {
        delete m;
        return NNP_E_HIP;
    }
    {
        void* scratch_dev = nullptr;
        const nnp_status st = scratch_address(m->device, &scratch_dev);
        if (st != NNP_OK) {
            delete m;
            return st;
        }
    }
    m->precision = precision;
    AevConst& P = m->aev;
    P.ns = ns;
    P.radial_dim = ns * kNr;
    P.dim = dim;
    P.stride = round_up(dim, 64);
    P.rc_r = a->rc_r;
    P.eta_r = a->eta_r;
    P.rc_a = a->rc_a;
    P.eta_a = a->eta_a;
    P.zeta = a->zeta;
    P.pr = a->radial_prefactor;
    P.cs = a->cos_scale;
    P.pi_rc_r = (float)(M_PI / (double)a->rc_r);
    P.pi_rc_a = (float)(M_PI / (double)a->rc_a);
    for (int k = 0; k < kNr; ++k) P.shf_r[k] = a->shf_r[k];
    for (int k = 0; k < kNa; ++k) P.shf_a[k] = a->shf_a[k];
    for (int k = 0; k < kNz; ++k) {
        P.cos_z[k] = (float)std::cos((double)a->shf_z[k]);
        P.sin_z[k] = (float)std::sin((double)a->shf_z[k]);
        P.hcos_z[k] = 0.5f * P.cos_z[k];
        P.hsin_z[k] = 0.5f * P.sin_z[k];
    }
    m->n_layers = L;
    for (int l = 0; l <= L; ++l) {
        m->widths[l] = p->widths[l];
        m->wpad[l] = l == L ? 1 : round_up(p->widths[l], 64);
    }
    m->wpad[0] = P.stride;
    m->celu_alpha = p->celu_alpha;
    for (int s = 0; s < kMaxSpecies; ++s) m->self_energy[s] = (p->self_energy && s < ns) ? p->self_energy[s] : 0.0;

    // pack weights: per species, per hidden layer: W [Np][Kp], WT [Kp][Np] (fp32 + bf16), bias [Np];
    // head: w [Kp_last]
    std::vector<size_t> offW(ns * L), offWT(ns * L), offWb(ns * L), offWTb(ns * L), offB(ns * L), offH(ns);
    size_t o = 0;
    for (int s = 0; s < ns; ++s) {
        for (int l = 0; l + 1 < L; ++l) {
            const size_t nk = (size_t)m->wpad[l] * m->wpad[l + 1];
            offW[s * L + l] = o; o = align256(o + 4 * nk);
            offWT[s * L + l] = o; o = align256(o + 4 * nk);
            offWb[s * L + l] = o; o = align256(o + 2 * nk);
            offWTb[s * L + l] = o; o = align256(o + 2 * nk);
            offB[s * L + l] = o; o = align256(o + 4 * (size_t)m->wpad[l + 1]);
        }
        offH[s] = o; o = align256(o + 4 * (size_t)m->wpad[L - 1]);
    }
    std::vector<char> host(o, 0);
    for (int s = 0; s < ns; ++s) {
        for (int l = 0; l + 1 < L; ++l) {
            const int K = m->widths[l], N = m->widths[l + 1];
            const int Kp = m->wpad[l], Np = m->wpad[l + 1];
            const float* Wsrc = p->W[s * L + l];
            const float* bsrc = p->b[s * L + l];
            if (!Wsrc || !bsrc) { delete m; return NNP_E_ARG; }
            float* W = (float*)(host.data() + offW[s * L + l]);
            float* WT = (float*)(host.data() + offWT[s * L + l]);
            uint16_t* Wb = (uint16_t*)(host.data() + offWb[s * L + l]);
            uint16_t* WTb = (uint16_t*)(host.data() + offWTb[s * L + l]);
            float* B = (float*)(host.data() + offB[s * L + l]);
            for (int nI = 0; nI < N; ++nI) {
                for (int k = 0; k < K; ++k) {
                    const float v = Wsrc[(size_t)nI * K + k];
                    W[(size_t)nI * Kp + k] = v;
                    WT[(size_t)k * Np + nI] = v;
                    Wb[(size_t)nI * Kp + k] = host_bf16(v);
                    WTb[(size_t)k * Np + nI] = host_bf16(v);
                }
                B[nI] = bsrc[nI];
            }
        }
        const float* wh = p->W[s * L + L - 1];
        const float* bh = p->b[s * L + L - 1];
        if (!wh || !bh) { delete m; return NNP_E_ARG; }
        float* H = (float*)(host.data() + offH[s]);
        for (int k = 0; k < m->widths[L - 1]; ++k) H[k] = wh[k];
        m->ptrs.head_b[s] = bh[0];
    }
    if (hipMalloc(&m->dev_weights, o) != hipSuccess) { delete m; return NNP_E_NOMEM; }
    m->dev_weights_bytes = o;
    if (hipMemcpy(m->dev_weights, host.data(), o, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(m->dev_weights);
        delete m;
        return NNP_E_HIP;
    }
    char* d = (char*)m->dev_weights;
    for (int s = 0; s < ns; ++s) {
        for (int l = 0; l + 1 < L; ++l) {
            m->ptrs.W[s][l] = (const float*)(d + offW[s * L + l]);
            m->ptrs.WT[s][l] = (const float*)(d + offWT[s * L + l]);
            m->ptrs.Wb[s][l] = (const uint16_t*)(d + offWb[s * L + l]);
            m->ptrs.WTb[s][l] = (const uint16_t*)(d + offWTb[s * L + l]);
            m->ptrs.b[s][l] = (const float*)(d + offB[s * L + l]);
        }
        m->ptrs.head_w[s] = (const float*)(d + offH[s]);
    }
    m->fused = fused_mlp_shape(m->widths, L, ns);
    m->n_nets = n_nets;
    if (n_nets > 1 && !m->fused) {   // ensembles run on the fused kernels only
        nnp_model_destroy(m);
        return NNP_E_ARG;
    }
    if (m->fused) {
        // per network: float32 packs of every species, bfloat16 packs, then the
        // biases and head weights (b1 [256], b2 [192], b3 [192], w4 [192], zero padded)
        const size_t per = pack_fused_species(nullptr, false, nullptr, nullptr, nullptr, dim, m->widths[3]);
        const size_t perb = pack_fused_species(nullptr, true, nullptr, nullptr, nullptr, dim, m->widths[3]);
        const int hw[4] = {256, 192, 192, 192};
        size_t vec_bytes = 0;
        for (int k = 0; k < 4; ++k) vec_bytes += align256(sizeof(float) * hw[k]);
        const size_t net_bytes = (per + perb + vec_bytes) * ns;
        std::vector<char> hp(net_bytes * n_nets, 0);
        for (int k = 0; k < n_nets; ++k) {
            const nnp_mlp_params* q = &nets[k];
            char* nb = hp.data() + net_bytes * k;
            for (int s = 0; s < ns; ++s) {
                const float* W1 = q->W[s * L + 0];
                const float* W2 = q->W[s * L + 1];
                const float* W3 = q->W[s * L + 2];
                const float* w4 = q->W[s * L + 3];
                if (!W1 || !W2 || !W3 || !w4 || !q->b[s * L + 0] || !q->b[s * L + 1] || !q->b[s * L + 2] ||
                    !q->b[s * L + 3]) {
                    nnp_model_destroy(m);
                    return NNP_E_ARG;
                }
                pack_fused_species(nb + per * s, false, W1, W2, W3, dim, m->widths[3]);
                pack_fused_species(nb + per * ns + perb * s, true, W1, W2, W3, dim, m->widths[3]);
                char* v = nb + (per + perb) * ns + vec_bytes * s;
                const float* src[4] = {q->b[s * L + 0], q->b[s * L + 1], q->b[s * L + 2], w4};
                const int len[4] = {m->widths[1], m->widths[2], m->widths[3], m->widths[3]};
                for (int j = 0; j < 4; ++j) {
                    std::memcpy(v, src[j], sizeof(float) * len[j]);
                    v += align256(sizeof(float) * hw[j]);
                }
            }
        }
        if (hipMalloc(&m->fused_dev, hp.size()) != hipSuccess) { nnp_model_destroy(m); return NNP_E_NOMEM; }
        if (hipMemcpy(m->fused_dev, hp.data(), hp.size(), hipMemcpyHostToDevice) != hipSuccess) {
            nnp_model_destroy(m);
            return NNP_E_HIP;
        }
        // device tables: [n_nets] float32 entries, then [n_nets] bfloat16 entries
        const size_t eb = fused_net_bytes();
        std::vector<char> tab(eb * 2 * n_nets);
        for (int k = 0; k < n_nets; ++k) {
            const char* nb = (const char*)m->fused_dev + net_bytes * k;
            const char* pf[kMaxSpecies];
            const char* pb[kMaxSpecies];
            const float *b1[kMaxSpecies], *b2[kMaxSpecies], *b3[kMaxSpecies], *w4[kMaxSpecies];
            float b4[kMaxSpecies];
            for (int s = 0; s < ns; ++s) {
                pf[s] = nb + per * s;
                pb[s] = nb + per * ns + perb * s;
                const char* v = nb + (per + perb) * ns + vec_bytes * s;
                const float** dst[4] = {&b1[s], &b2[s], &b3[s], &w4[s]};
                for (int j = 0; j < 4; ++j) {
                    *dst[j] = (const float*)v;
                    v += align256(sizeof(float) * hw[j]);
                }
                b4[s] = nets[k].b[s * L + L - 1][0];
            }
            fused_net_entry(tab.data() + eb * k, ns, pf, b1, b2, b3, w4, b4, false);
            fused_net_entry(tab.data() + eb * (n_nets + k), ns, pb, b1, b2, b3, w4, b4, true);
        }
        if (hipMalloc(&m->fused_tab, tab.size()) != hipSuccess) { nnp_model_destroy(m); return NNP_E_NOMEM; }
        if (hipMemcpy(m->fused_tab, tab.data(), tab.size(), hipMemcpyHostToDevice) != hipSuccess) {
            nnp_model_destroy(m);
            return NNP_E_HIP;
        }
        m->fused_tab_fp32 = m->fused_tab;
        m->fused_tab_bf16 = (char*)m->fused_tab + eb * n_nets;
    }
    if (hipMalloc(&m->flags, 256) != hipSuccess) { nnp_model_destroy(m); return NNP_E_NOMEM; }
    if (hipMemset(m->flags, 0, 256) != hipSuccess) { nnp_model_destroy(m); return NNP_E_HIP; }
    if (hipHostMalloc(&m->host_stage, 256, 0) != hipSuccess) { nnp_model_destroy(m); return NNP_E_NOMEM; }
    *out = m;
    return NNP_OK;
}

void nnp_model_destroy(nnp_model* m) {
    if (!m) return;
    if (m->dev_weights) (void)hipFree(m->dev_weights);
    if (m->fused_dev) (void)hipFree(m->fused_dev);
    if (m->fused_tab) (void)hipFree(m->fused_tab);
    if (m->flags) (void)hipFree(m->flags);
    if (m->host_stage) (void)hipHostFree(m->host_stage);
    delete m->prof;
    delete m;
}

nnp_status nnp_model_set_precision(nnp_model* m, nnp_precision p) {
    if (!m || (p != NNP_FP32 && p != NNP_BF16_MLP)) return NNP_E_ARG;
    m->precision = p;
    return NNP_OK;
}

int32_t nnp_aev_dim(const nnp_model* m) { return m ? m->aev.dim : 0; }

int32_t nnp_model_fused_mlp(const nnp_model* m) { return m && m->fused && !m->force_unfused ? 1 : 0; }

nnp_status nnp_model_set_fused_mlp(nnp_model* m, int32_t allow) {
    if (!m || (allow == 0 && m->n_nets > 1)) return NNP_E_ARG;
    m->force_unfused = allow == 0;
    return NNP_OK;
}

nnp_status nnp_check(nnp_model* m, void* stream, uint32_t* flags) {
    if (!m) return NNP_E_ARG;
    uint32_t fl = 0;
    nnp_status st = read_and_clear_flags(m, (hipStream_t)stream, &fl, nullptr, nullptr);
    if (st != NNP_OK) return st;
    if (flags) *flags = fl;
    if (!fl) return NNP_OK;
    if (fl & NNP_FLAG_NONFINITE) return NNP_E_NONFINITE;
    if (fl & NNP_FLAG_ROW) return NNP_E_ROW;
    if (fl & NNP_FLAG_CAPACITY) return NNP_E_CAPACITY;
    return NNP_E_ARG;
}

size_t nnp_neighbors_workspace_bytes(int32_t n_atoms, int32_t n_mol, const float* box_host, float r_list) {
    if (n_atoms < 0) return 0;
    return neighbors_ws_bytes(n_atoms, n_mol, box_host, r_list);
}

nnp_status nnp_neighbors(nnp_model* m, int32_t n, const float* pos, const int32_t* mol, int32_t n_mol,
                         const float* box_host, float r_list, nnp_nlist* nl, int64_t* n_pairs_host, void* ws,
                         size_t ws_bytes, void* stream) {
    if (!m || !nl || n < 0 || (n > 0 && !pos) || !nl->row_ptr) return NNP_E_ARG;
    if (!(r_list > 0.f) || !std::isfinite(r_list)) return NNP_E_ARG;
    if (mol && n_mol < 1) return NNP_E_ARG;
    if (nl->capacity > 0 && (!nl->col || !nl->shift || !nl->rev)) return NNP_E_ARG;
    return build_neighbors(m, n, pos, mol, mol ? n_mol : 1, box_host, r_list, nl, n_pairs_host, ws, ws_bytes,
                           (hipStream_t)stream);
}

size_t nnp_workspace_bytes(const nnp_model* m, int32_t n_atoms, int64_t pair_capacity) {
    if (!m || n_atoms < 0) return 0;
    return ef_layout(m, n_atoms, pair_capacity, nullptr).end;
}

nnp_status nnp_energy_forces(nnp_model* m, int32_t n, const float* pos, const int32_t* species, const int32_t* mol,
                             int32_t n_mol, const float* box_host, const nnp_nlist* nl, double* e_mol, float* e_atom,
                             float* forces, void* ws, size_t ws_bytes, void* stream) {
    if (!m || !nl || n < 0) return NNP_E_ARG;
    if (nl->n_atoms != n || nl->n_pairs > nl->capacity) return NNP_E_ARG;
    return energy_forces_impl(m, n, pos, species, mol, n_mol, box_host, nl, e_mol, e_atom, forces, ws, ws_bytes,
                              (hipStream_t)stream, m->flags);
}

nnp_status nnp_energy_forces_static(nnp_model* m, int32_t n, const float* pos, const int32_t* species,
                                    const int32_t* mol, int32_t n_mol, const float* box_host, const nnp_nlist* nl,
                                    double* e_mol, float* e_atom, float* forces, void* stream) {
    if (!m || !nl || n < 0) return NNP_E_ARG;
    if (nl->n_atoms != n || nl->n_pairs > nl->capacity) return NNP_E_ARG;
    const size_t need = ef_layout(m, n, nl->capacity, nullptr).end;
    if (need > NNP_STATIC_SCRATCH_BYTES) return NNP_E_SCRATCH;
    void* ws = nullptr;
    const nnp_status st = scratch_address(m->device, &ws);   // resolved when the model was created
    if (st != NNP_OK) return st;
    EfOpts opts;
    opts.no_profile = true;
    return energy_forces_impl(m, n, pos, species, mol, n_mol, box_host, nl, e_mol, e_atom, forces, ws,
                              NNP_STATIC_SCRATCH_BYTES, (hipStream_t)stream, m->flags, nullptr, nullptr, &opts);
}

nnp_status nnp_energy_forces_virial(nnp_model* m, int32_t n, const float* pos, const int32_t* species,
                                    const int32_t* mol, int32_t n_mol, const float* box_host, const nnp_nlist* nl,
                                    double* e_mol, float* e_atom, float* forces, double* virial, float* atom_virial,
                                    void* ws, size_t ws_bytes, void* stream) {
    if (!m || !nl || n < 0 || !forces || !virial) return NNP_E_ARG;
    if (nl->n_atoms != n || nl->n_pairs > nl->capacity) return NNP_E_ARG;
    return energy_forces_impl(m, n, pos, species, mol, n_mol, box_host, nl, e_mol, e_atom, forces, ws, ws_bytes,
                              (hipStream_t)stream, m->flags, virial, atom_virial);
}

nnp_status nnp_energy_forces_ensemble(nnp_model* m, int32_t n, const float* pos, const int32_t* species,
                                      const int32_t* mol, int32_t n_mol, const float* box_host, const nnp_nlist* nl,
                                      double* e_mol, double* e_mol_net, float* e_atom, float* forces, void* ws,
                                      size_t ws_bytes, void* stream) {
    if (!m || !nl || n < 0 || m->n_nets < 2 || !e_mol_net) return NNP_E_ARG;
    if (nl->n_atoms != n || nl->n_pairs > nl->capacity) return NNP_E_ARG;
    return energy_forces_impl(m, n, pos, species, mol, n_mol, box_host, nl, e_mol, e_atom, forces, ws, ws_bytes,
                              (hipStream_t)stream, m->flags, nullptr, nullptr, nullptr, e_mol_net);
}

int32_t nnp_model_nets(const nnp_model* m) { return m ? m->n_nets : 0; }

nnp_status nnp_aev(nnp_model* m, int32_t n, const float* pos, const int32_t* species, const float* box_host,
                   const nnp_nlist* nl, float* aev_out, void* ws, size_t ws_bytes, void* stream) {
    (void)ws;
    (void)ws_bytes;
    if (!m || !nl || n < 0 || (n > 0 && (!pos || !species || !aev_out))) return NNP_E_ARG;
    if (nl->n_atoms != n) return NNP_E_ARG;
    return hip_status(launch_aev_fwd(m->aev, n, pos, species, box_const(box_host), rows_csr(nl), nullptr, aev_out, false,
                                     m->flags, (hipStream_t)stream));
}

nnp_status nnp_mlp(nnp_model* m, int32_t n, const int32_t* species, const float* aev_in, float* e_atom,
                   float* daev_out, void* ws, size_t ws_bytes, void* stream) {
    if (!m || n < 0 || (n > 0 && (!species || !aev_in || !e_atom))) return NNP_E_ARG;
    const EfWs need = ef_layout(m, n, 0, nullptr);
    if (!ws || ws_bytes < need.end) return NNP_E_ARG;
    if (n == 0) return NNP_OK;
    hipStream_t s = (hipStream_t)stream;
    const EfWs W = ef_layout(m, n, 0, (char*)ws);
    MlpWs dense = W.mw;
    dense.amask = nullptr;   // dE/dAEV of every feature is returned
    const bool fused = m->fused && (!m->force_unfused || m->n_nets > 1);
    const bool bfa = fused && m->precision == NNP_BF16_MLP;   // the fused BF16 kernels read bf16 rows
    void* rows = W.aev;
    hipError_t e = launch_species_group(m, n, species, W.mw, m->flags, s);
    if (e == hipSuccess) e = launch_zero_pad_rows(W.mw, m->aev.stride, rows, bfa, s);
    if (e == hipSuccess) {
        if (bfa) e = launch_permute_rows_bf16(W.mw.prow, n, m->aev.stride, aev_in, (uint16_t*)rows, s);
        else e = launch_permute_rows(true, W.mw.prow, n, m->aev.stride, aev_in, (float*)W.aev, s);
    }
    if (e == hipSuccess) {
        if (fused && mlp_split(m, n))
            e = launch_mlp_ensemble(m, dense, rows, daev_out ? W.g : nullptr, W.E_row, nullptr, n, W.d1, W.E_net,
                                    nullptr, s);
        else if (fused) e = launch_mlp_fused(m, dense, rows, daev_out ? W.g : nullptr, W.E_row, nullptr, n, s);
        else e = launch_mlp(m, W.mw, W.aev, false, W.h, daev_out ? W.g : nullptr, W.E_row, nullptr, s);
    }
    if (e == hipSuccess) e = launch_gather_e(W.mw.prow, n, species, self_e(m), W.E_row, e_atom, s);
    if (e == hipSuccess && daev_out) e = launch_permute_rows(false, W.mw.prow, n, m->aev.stride, W.g, daev_out, s);
    return hip_status(e);
}

nnp_status nnp_md_kick_drift(int32_t n, float* pos, float* vel, const float* forces, const float* inv_mass, float dt,
                             const float* ref_pos, float* max_disp2, void* stream) {
    if (n < 0 || (n > 0 && (!pos || !vel || !forces || !inv_mass)) || (ref_pos && !max_disp2)) return NNP_E_ARG;
    return hip_status(launch_kick_drift(n, pos, vel, forces, inv_mass, dt, ref_pos, max_disp2, (hipStream_t)stream));
}

nnp_status nnp_md_kick(int32_t n, float* vel, const float* forces, const float* inv_mass, float dt, void* stream) {
    if (n < 0 || (n > 0 && (!vel || !forces || !inv_mass))) return NNP_E_ARG;
    return hip_status(launch_kick(n, vel, forces, inv_mass, dt, (hipStream_t)stream));
}

nnp_status nnp_md_wrap(int32_t n, float* pos, const float* box_host, void* stream) {
    if (n < 0 || (n > 0 && !pos) || !box_host) return NNP_E_ARG;
    for (int k = 0; k < 3; ++k)
        if (!(box_host[k] > 0.f)) return NNP_E_ARG;
    return hip_status(launch_wrap(n, pos, box_host, (hipStream_t)stream));
}

nnp_status nnp_profile_enable_mask(nnp_model* m, uint32_t mask) {
    if (!m) return NNP_E_ARG;
    if (!m->prof) m->prof = new nnp_prof;
    std::lock_guard<std::mutex> lock(m->prof->mu);
    m->prof->drain();
    for (int k = 0; k < NNP_N_STAGES; ++k) {
        m->prof->ms[k] = 0.0;
        m->prof->cnt[k] = 0;
    }
    m->prof->mask = mask & ((1u << NNP_N_STAGES) - 1u);
    m->prof->enabled = m->prof->mask != 0;
    return NNP_OK;
}

nnp_status nnp_profile_enable(nnp_model* m, int enable) {
    return nnp_profile_enable_mask(m, enable ? (1u << NNP_N_STAGES) - 1u : 0u);
}

nnp_status nnp_profile_read(nnp_model* m, double* ms, int64_t* count) {
    if (!m || !m->prof) return NNP_E_ARG;
    std::lock_guard<std::mutex> lock(m->prof->mu);
    m->prof->drain();
    for (int k = 0; k < NNP_N_STAGES; ++k) {
        if (ms) ms[k] = m->prof->ms[k];
        if (count) count[k] = m->prof->cnt[k];
    }
    return NNP_OK;
}

}  // extern "C"
