// Native MD engine (Sec. 5.4, "Native MD engine": the whole time step stays on
// the GPU and the host only enqueues work).  One engine integrates one
// structure (periodic orthorhombic box or open) with velocity Verlet (NVE) or
// BAOAB Langevin dynamics (md.hip), rebuilding the neighbour list with a
// skin when the device decides to (Sec. 5.5: a list buffer and a rebuild
// every few steps).
//
// A run of K steps is enqueued in one go and synchronises once, at its end,
// to read the error flags.  The engine keeps the builder's fixed-stride rows
// (row i at i * NNP_MAX_ROW, sorted by neighbour) instead of a compacted
// list: a rebuild never needs the pair count, so nothing is read back and no
// capacity can run out (a row longer than NNP_MAX_ROW is an error, as for
// every list).  The reverse index of the rows is taken by the AEV kernel on
// rebuild steps.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "md_internal.hpp"
#include "nnp_internal.hpp"

using namespace nnp;

struct nnp_md {
    nnp_model* model = nullptr;
    int n = 0;
    nnp_md_params p{};
    BoxConst bx{};
    float box[3] = {0, 0, 0};
    float r_list = 0.f;
    MdStepConst c{};
    float trig_len = -1.f;     // trigger * skin, or -1 without a skin
    uint64_t step = 0;
    bool small = false;       // fused front / back kernels (md_front_fits)
    bool fuse_front = false;  // decision and wrap inside the binning kernel (md_front_fuses)
    bool grouped = false;     // species grouping in ws_ef is current
    // device state
    float *pos = nullptr, *vel = nullptr, *F = nullptr, *inv_mass = nullptr, *ref = nullptr;
    int32_t* species = nullptr;
    double* e_pot = nullptr;
    MdState* st = nullptr;    // [2]: step s decides from st[s % 2] into st[(s + 1) % 2]
    unsigned* flags = nullptr;
    double* ke_part = nullptr;
    float* d2_part = nullptr;   // per-block two largest displacements (general path)
    double* e_part = nullptr;   // chunk sums of the structure energy
    unsigned* e_ticket = nullptr;
    // energy log [log_cap][2]
    double* log = nullptr;
    int log_cap = 0;
    int log_rows = 0;
    // neighbour rows (in ws_nb), their reverse index (nl.rev) and workspaces;
    // nl carries the list's extent for the energy call
    nnp_nlist nl{};
    RowsView rows{};
    void* ws_nb = nullptr;
    size_t ws_nb_bytes = 0;
    void* ws_ef = nullptr;
    size_t ws_ef_bytes = 0;
    void* host = nullptr;     // pinned staging
};

namespace {

template <typename T>
hipError_t dmalloc(T** p, size_t count) {
    return hipMalloc((void**)p, sizeof(T) * (count > 0 ? count : 1));
}

nnp_status alloc_rows(nnp_md* md) {
    const int64_t capacity = (int64_t)md->n * NNP_MAX_ROW;
    md->nl.capacity = capacity;
    if (dmalloc(&md->nl.rev, (size_t)capacity) != hipSuccess) return NNP_E_NOMEM;
    // every reverse slot a valid index from the start (a slot of a row
    // emptied for overflowing may go unresolved by a build; that build is
    // flagged)
    if (hipMemset(md->nl.rev, 0, sizeof(int32_t) * (size_t)capacity) != hipSuccess) return NNP_E_HIP;
    md->ws_ef_bytes = nnp_workspace_bytes(md->model, md->n, capacity);
    if (hipMalloc(&md->ws_ef, md->ws_ef_bytes) != hipSuccess) return NNP_E_NOMEM;
    return NNP_OK;
}

nnp_status status_of_flags(unsigned fl) {
    if (fl & NNP_FLAG_NONFINITE) return NNP_E_NONFINITE;
    if (fl & NNP_FLAG_ROW) return NNP_E_ROW;
    return fl ? NNP_E_ARG : NNP_OK;
}

// One step.  Small systems (md_front_fits): a fused front kernel (first half
// step, displacement, rebuild decision, wrap and cell binning), the gated
// row kernel, AEV (with the reverse index on rebuild steps), networks, AEV
// adjoint, and a fused back kernel (force gather, last half kick and the
// float64 structure energy): six launches.  Larger systems use the general
// multi-kernel path for the front and the cell binning; up to 8,192 cells
// (md_front_fuses) the binning kernel also takes the rebuild decision and
// the wrap.  The potential energy is summed on every step, in the back
// kernel.
nnp_status enqueue_step(nnp_md* md, uint64_t step, hipStream_t s) {
    nnp_model* m = md->model;
    const bool langevin = md->p.integrator == NNP_MD_LANGEVIN;
    const float* bptr = md->bx.periodic ? md->box : nullptr;
    const MdState* cur = md->st + (step & 1);
    MdState* nxt = md->st + ((step + 1) & 1);
    MdFront front{};
    prof_begin(m, NNP_STAGE_INTEGRATE, s);
    hipError_t e = hipSuccess;
    if (md->small) {
        nnp_status st = launch_md_front(md->n, md->pos, md->vel, md->F, md->inv_mass, md->c, step, md->ref, cur, nxt,
                                        md->p.rebuild_every, md->trig_len, langevin, bptr, md->r_list, md->ws_nb,
                                        md->ws_nb_bytes, md->flags, s);
        if (st != NNP_OK) return st;
    } else {
        e = md_launch_first(md->n, md->pos, md->vel, md->F, md->inv_mass, md->c, step, md->ref, md->d2_part,
                            langevin, s);
        if (md->fuse_front) {
            front.cur = cur;
            front.nxt = nxt;
            front.d2_part = md->d2_part;
            front.n_parts = md_first_parts(md->n);
            front.rebuild_every = md->p.rebuild_every;
            front.trig_len = md->trig_len;
            front.pos = md->pos;
            front.ref = md->ref;
        } else {
            if (e == hipSuccess)
                e = md_launch_decide(cur, nxt, md->d2_part, md_first_parts(md->n), md->p.rebuild_every,
                                     md->trig_len, s);
            if (e == hipSuccess) e = md_launch_wrap_ref(md->n, md->pos, md->ref, md->bx, nxt, s);
        }
    }
    prof_end(m, NNP_STAGE_INTEGRATE, s);
    if (e != hipSuccess) return NNP_E_HIP;
    nnp_status st = build_neighbors(m, md->n, md->pos, nullptr, 1, bptr, md->r_list, &md->nl, nullptr, md->ws_nb,
                                    md->ws_nb_bytes, s, false, md->flags, &nxt->gate, nullptr, md->small,
                                    &md->rows, md->fuse_front ? &front : nullptr);
    if (st != NNP_OK) return st;
    md->rows.rev = md->nl.rev;
    const bool log = md->p.log_every > 0 && ((step + 1) % (uint64_t)md->p.log_every) == 0 &&
                     md->log_rows < md->log_cap;
    MdBack back{};
    back.vel = md->vel;
    back.inv_mass = md->inv_mass;
    back.dt = md->p.dt;
    back.ke_part = log ? md->ke_part : nullptr;
    back.fuse_energy = true;
    back.e_part = md->e_part;
    back.e_ticket = md->e_ticket;
    EfOpts opts;
    opts.skip_group = md->grouped;
    opts.md = &back;
    opts.rows = &md->rows;
    opts.rev_out = md->nl.rev;
    opts.gate = &nxt->gate;
    st = energy_forces_impl(m, md->n, md->pos, md->species, nullptr, 1, bptr, &md->nl, md->e_pot, nullptr, md->F,
                            md->ws_ef, md->ws_ef_bytes, s, md->flags, nullptr, nullptr, &opts);
    if (st != NNP_OK) return st;
    md->grouped = true;
    if (log) {
        prof_begin(m, NNP_STAGE_INTEGRATE, s);
        e = md_launch_log(md->n, md->ke_part, md->e_pot, md->log + 2 * (size_t)md->log_rows, s);
        md->log_rows += 1;
        prof_end(m, NNP_STAGE_INTEGRATE, s);
    }
    return e == hipSuccess ? NNP_OK : NNP_E_HIP;
}

// reads and clears the engine's flags
nnp_status read_flags(nnp_md* md, hipStream_t s, unsigned* fl) {
    if (hipMemcpyAsync(md->host, md->flags, sizeof(unsigned), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return NNP_E_HIP;
    std::memcpy(fl, md->host, sizeof(unsigned));
    if (*fl && hipMemsetAsync(md->flags, 0, sizeof(unsigned), s) != hipSuccess) return NNP_E_HIP;
    return NNP_OK;
}

}  // namespace

extern "C" {

nnp_status nnp_md_create(nnp_model* model, int32_t n, const float* pos, const float* vel, const int32_t* species,
                         const float* masses, const float* box_host, const nnp_md_params* params, void* stream,
                         nnp_md** out) {
    if (!model || !params || !out || n <= 0 || !pos || !vel || !species || !masses) return NNP_E_ARG;
    const nnp_md_params& p = *params;
    if (p.integrator != NNP_MD_NVE && p.integrator != NNP_MD_LANGEVIN) return NNP_E_ARG;
    if (!(p.dt > 0.f) || !std::isfinite(p.dt) || p.rebuild_every < 1 || !(p.skin >= 0.f) || p.log_every < 0 ||
        p.log_capacity < 0)
        return NNP_E_ARG;
    if (p.integrator == NNP_MD_LANGEVIN && (!(p.temperature >= 0.f) || !(p.friction >= 0.f))) return NNP_E_ARG;
    // every setting must keep the list complete between builds: with a skin
    // the displacement check is on (0 < trigger <= 1); without one the list
    // is rebuilt every step
    if (p.skin > 0.f ? !(p.trigger > 0.f && p.trigger <= 1.f) : p.rebuild_every != 1) return NNP_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    nnp_md* md = new nnp_md();
    md->model = model;
    md->n = n;
    md->p = p;
    md->bx.periodic = box_host != nullptr;
    for (int k = 0; k < 3; ++k) {
        md->box[k] = box_host ? box_host[k] : 0.f;
        md->bx.L[k] = md->box[k];
    }
    md->r_list = model->aev.rc_r + p.skin;
    md->small = md_front_fits(n, box_host, md->r_list);
    md->fuse_front = !md->small && md_front_fuses(n, box_host, md->r_list);
    if (box_host)
        for (int k = 0; k < 3; ++k)
            if (!(2.f * md->r_list <= box_host[k])) {
                delete md;
                return NNP_E_BOX;
            }
    md->trig_len = p.skin > 0.f ? p.trigger * p.skin : -1.f;
    md->c.dt = p.dt;
    md->c.seed = p.seed;
    if (p.integrator == NNP_MD_LANGEVIN) {
        const double c1 = std::exp(-(double)p.friction * 1e-3 * (double)p.dt);   // friction in 1/ps
        md->c.c1 = (float)c1;
        md->c.c2 = (float)std::sqrt(1.0 - c1 * c1);
        md->c.kT = (float)(8.617333262e-5 * (double)p.temperature);
    } else {
        md->c.c1 = 1.f;
        md->c.c2 = 0.f;
        md->c.kT = 0.f;
    }
    md->log_cap = p.log_every > 0 ? p.log_capacity : 0;
    const size_t v3 = 3 * (size_t)n;
    bool ok = dmalloc(&md->pos, v3) == hipSuccess && dmalloc(&md->vel, v3) == hipSuccess &&
              dmalloc(&md->F, v3) == hipSuccess && dmalloc(&md->ref, v3) == hipSuccess &&
              dmalloc(&md->inv_mass, (size_t)n) == hipSuccess && dmalloc(&md->species, (size_t)n) == hipSuccess &&
              dmalloc(&md->e_pot, 1) == hipSuccess && dmalloc(&md->st, 2) == hipSuccess &&
              dmalloc(&md->flags, 1) == hipSuccess && dmalloc(&md->ke_part, (size_t)md_ke_parts(n)) == hipSuccess &&
              dmalloc(&md->d2_part, 2 * (size_t)md_first_parts(n)) == hipSuccess &&
              dmalloc(&md->e_part, (size_t)md_energy_parts(n)) == hipSuccess && dmalloc(&md->e_ticket, 1) == hipSuccess &&
              dmalloc(&md->log, 2 * (size_t)(md->log_cap > 0 ? md->log_cap : 1)) == hipSuccess &&
              hipHostMalloc(&md->host, 64, hipHostMallocDefault) == hipSuccess;
    if (!ok) {
        nnp_md_destroy(md);
        return NNP_E_NOMEM;
    }
    md->ws_nb_bytes = nnp_neighbors_workspace_bytes(n, 1, box_host, md->r_list);
    if (hipMalloc(&md->ws_nb, md->ws_nb_bytes) != hipSuccess) {
        nnp_md_destroy(md);
        return NNP_E_NOMEM;
    }
    hipError_t e = hipMemcpyAsync(md->pos, pos, sizeof(float) * v3, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(md->vel, vel, sizeof(float) * v3, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(md->species, species, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipMemsetAsync(md->st, 0, 2 * sizeof(MdState), s);
    if (e == hipSuccess) e = hipMemsetAsync(md->flags, 0, sizeof(unsigned), s);
    if (e == hipSuccess) e = hipMemsetAsync(md->e_ticket, 0, sizeof(unsigned), s);
    if (e == hipSuccess) e = md_launch_inv_mass(n, masses, md->inv_mass, md->flags, s);
    // the starting configuration: wrapped, reference for displacements, list,
    // forces; step 0 decides from slot 0
    MdState st0{};
    st0.gate = 1;
    if (e == hipSuccess) e = hipMemcpyAsync(md->st, &st0, sizeof(MdState), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = md_launch_wrap_ref(n, md->pos, md->ref, md->bx, md->st, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        nnp_md_destroy(md);
        return NNP_E_HIP;
    }
    st0.gate = 0;
    st0.rebuilds = 1;
    nnp_status st = alloc_rows(md);
    if (st == NNP_OK)
        st = build_neighbors(model, n, md->pos, nullptr, 1, box_host, md->r_list, &md->nl, nullptr, md->ws_nb,
                             md->ws_nb_bytes, s, false, md->flags, nullptr, nullptr, false, &md->rows);
    md->rows.rev = md->nl.rev;
    if (st == NNP_OK &&
        hipMemcpyAsync(md->st, &st0, sizeof(MdState), hipMemcpyHostToDevice, s) != hipSuccess)
        st = NNP_E_HIP;
    if (st == NNP_OK) {
        EfOpts opts;
        opts.rows = &md->rows;
        opts.rev_out = md->nl.rev;
        st = energy_forces_impl(model, n, md->pos, md->species, nullptr, 1, box_host, &md->nl, md->e_pot, nullptr,
                                md->F, md->ws_ef, md->ws_ef_bytes, s, md->flags, nullptr, nullptr, &opts);
    }
    if (st == NNP_OK) md->grouped = true;
    if (st == NNP_OK) {
        unsigned fl = 0;
        st = read_flags(md, s, &fl);
        if (st == NNP_OK) st = status_of_flags(fl);
    }
    if (st != NNP_OK) {
        nnp_md_destroy(md);
        return st;
    }
    *out = md;
    return NNP_OK;
}

nnp_status nnp_md_run(nnp_md* md, int32_t n_steps, void* stream) {
    if (!md || n_steps < 0) return NNP_E_ARG;
    if (n_steps == 0) return NNP_OK;
    hipStream_t s = (hipStream_t)stream;
    // steps count once enqueued whole (the state slots and the noise
    // counters follow md->step), also when a later step or the flags fail
    for (int k = 0; k < n_steps; ++k) {
        const nnp_status st = enqueue_step(md, md->step, s);
        if (st != NNP_OK) return st;
        md->step += 1;
    }
    nnp_status st;
    unsigned fl = 0;
    st = read_flags(md, s, &fl);
    if (st != NNP_OK) return st;
    return fl ? status_of_flags(fl) : NNP_OK;
}

nnp_status nnp_md_get(nnp_md* md, float* pos, float* vel, float* forces, double* e_pot, void* stream) {
    if (!md) return NNP_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    const size_t v3 = sizeof(float) * 3 * (size_t)md->n;
    hipError_t e = hipSuccess;
    if (pos) e = hipMemcpyAsync(pos, md->pos, v3, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess && vel) e = hipMemcpyAsync(vel, md->vel, v3, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess && forces) e = hipMemcpyAsync(forces, md->F, v3, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess && e_pot) e = hipMemcpyAsync(e_pot, md->e_pot, sizeof(double), hipMemcpyDeviceToDevice, s);
    return e == hipSuccess ? NNP_OK : NNP_E_HIP;
}

nnp_status nnp_md_log(nnp_md* md, double* host_rows, int32_t max_rows, int32_t* n_rows, void* stream) {
    if (!md || !n_rows || max_rows < 0 || (max_rows > 0 && !host_rows)) return NNP_E_ARG;
    const int rows = md->log_rows < max_rows ? md->log_rows : max_rows;
    if (rows > 0) {
        hipStream_t s = (hipStream_t)stream;
        if (hipMemcpyAsync(host_rows, md->log, sizeof(double) * 2 * (size_t)rows, hipMemcpyDeviceToHost, s) !=
                hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return NNP_E_HIP;
    }
    *n_rows = rows;
    return NNP_OK;
}

nnp_status nnp_md_info(nnp_md* md, nnp_md_stats* out, void* stream) {
    if (!md || !out) return NNP_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    MdState st;   // the state after the last step's decision
    if (hipMemcpyAsync(md->host, md->st + (md->step & 1), sizeof(MdState), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return NNP_E_HIP;
    std::memcpy(&st, md->host, sizeof(MdState));
    out->steps = (int64_t)md->step;
    out->rebuilds = (int64_t)st.rebuilds;
    out->early_rebuilds = (int64_t)st.early_rebuilds;
    out->capacity = md->nl.capacity;
    out->r_list = md->r_list;
    return NNP_OK;
}

void nnp_md_destroy(nnp_md* md) {
    if (!md) return;
    void* bufs[] = {md->pos, md->vel, md->F, md->ref, md->inv_mass, md->species, md->e_pot, md->st, md->flags,
                    md->ke_part, md->d2_part, md->e_part, md->e_ticket, md->log, md->nl.rev, md->ws_ef, md->ws_nb};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    if (md->host) (void)hipHostFree(md->host);
    delete md;
}

}  // extern "C"
