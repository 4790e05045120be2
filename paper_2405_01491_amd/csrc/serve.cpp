// Continuous-batching server for single-structure energy + force requests.
//
// Requests (one open-boundary structure each; the same-batch rule of Sec. 2.1
// keeps structures independent, Sec. 2.4 batches them as concatenated atoms
// with a structure index) are admitted when a slot and room in the request
// arena are free.  A scheduler thread forms a launch from every queued
// request (FIFO, up to the launch's atom budget) as soon as one of
// `max_inflight` launch contexts is free, so requests arriving while others
// are on the GPU join the next launch, and up to `max_inflight` launches run
// concurrently on their own streams.  Each launch context owns persistent
// device buffers (inputs, neighbour list, workspace, outputs, error flags)
// and pinned host staging; the model weights stay resident.  A launch is:
// one host-to-device copy of the batch, the neighbour build (all pairs within
// each structure, kept as the builder's fixed-stride rows: no compaction, no
// host synchronisation), AEV (which also takes the rows' reverse index),
// species networks, adjoint, forces, and one device-to-host copy of
// energies, forces and flags, followed by an event the scheduler polls.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "nnp_internal.hpp"

using namespace nnp;

namespace {

constexpr int kMaxRequestAtoms = 256;     // rows stay below NNP_MAX_ROW
constexpr int kLaunchAtoms = 16384;       // atom budget of one launch
constexpr int kLaunchRequests = 1024;     // request budget of one launch

enum ReqState { kQueued = 0, kRunning = 1, kDone = 2, kFailed = 3 };

struct Req {
    int n = 0;
    size_t off = 0, bytes = 0;
    int state = kQueued;
    double energy = 0.0;
    std::vector<float> forces;
    nnp_status err = NNP_OK;
};

// first-fit allocator over [0, cap)
struct Arena {
    size_t cap = 0;
    std::map<size_t, size_t> free_;   // offset -> size
    void init(size_t c) {
        cap = c;
        free_.clear();
        if (c) free_[0] = c;
    }
    bool alloc(size_t bytes, size_t* off) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rem = it->second - bytes, noff = it->first + bytes;
                free_.erase(it);
                if (rem) free_[noff] = rem;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

// A launch's inputs and outputs in one buffer (device, and pinned host
// staging of the same layout), packed for its n atoms and nm requests:
//   positions [3n] f32 | species [n] i32 | structure index [n] i32 |
//   flags (8 bytes) | energies [nm] f64 | forces [3n] f32
// so that one copy takes the inputs and the zeroed flags word up, and one
// copy brings the flags, energies and forces back.
struct IoLayout {
    size_t sp, mol, flags, e, f, end;
};

IoLayout io_layout(int n, int nm) {
    IoLayout o;
    o.sp = 12 * (size_t)n;
    o.mol = 16 * (size_t)n;
    o.flags = (20 * (size_t)n + 7) & ~(size_t)7;
    o.e = o.flags + 8;
    o.f = o.e + 8 * (size_t)nm;
    o.end = o.f + 12 * (size_t)n;
    return o;
}

struct Launch {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    char* d_io = nullptr;         // IoLayout for kLaunchAtoms, kLaunchRequests
    char* h_io = nullptr;         // pinned, the same size
    nnp_nlist nl{};
    void* d_nbws = nullptr;
    size_t nbws_bytes = 0;
    void* d_ws = nullptr;
    size_t ws_bytes = 0;
    std::vector<uint64_t> tickets;
    std::vector<int> offsets;
    int n_atoms = 0;
    bool busy = false;
};

nnp_status flags_status(unsigned fl) {
    if (!fl) return NNP_OK;
    if (fl & NNP_FLAG_NONFINITE) return NNP_E_NONFINITE;
    if (fl & NNP_FLAG_ROW) return NNP_E_ROW;
    if (fl & NNP_FLAG_CAPACITY) return NNP_E_CAPACITY;
    return NNP_E_ARG;
}

}  // namespace

struct nnp_server {
    nnp_model* model = nullptr;
    int max_slots = 0, max_inflight = 0;
    int64_t pair_cap = 0;
    char* inbox = nullptr;       // pinned host request arena
    Arena arena;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<uint64_t> queue;
    std::unordered_map<uint64_t, Req> reqs;
    uint64_t next_ticket = 1;
    int admitted = 0;
    std::vector<Launch> launches;
    std::thread worker;
    bool stop = false;
    uint64_t completed = 0, n_launches = 0, batched = 0;
};

namespace {

void free_launch(Launch& L) {
    auto df = [](void* p) { if (p) (void)hipFree(p); };
    auto hf = [](void* p) { if (p) (void)hipHostFree(p); };
    if (L.stream) (void)hipStreamSynchronize(L.stream);
    df(L.d_io);
    df(L.nl.row_ptr); df(L.nl.col); df(L.nl.shift); df(L.nl.rev); df(L.d_nbws); df(L.d_ws);
    hf(L.h_io);
    if (L.done) (void)hipEventDestroy(L.done);
    if (L.stream) (void)hipStreamDestroy(L.stream);
    L = Launch();
}

bool alloc_launch(nnp_server* S, Launch& L) {
    const int A = kLaunchAtoms, R = kLaunchRequests;
    const int64_t P = S->pair_cap;
    bool ok = hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&L.done, hipEventDisableTiming) == hipSuccess;
    const size_t io = io_layout(A, R).end;   // the largest launch's layout
    ok = ok && hipMalloc(&L.d_io, io) == hipSuccess;
    // fixed-stride rows: only the reverse index lives outside the builder's workspace
    ok = ok && hipMalloc(&L.nl.rev, sizeof(int32_t) * P) == hipSuccess;
    L.nl.capacity = P;
    L.nbws_bytes = nnp_neighbors_workspace_bytes(A, R, nullptr, S->model->aev.rc_r);
    L.ws_bytes = nnp_workspace_bytes(S->model, A, P);
    ok = ok && hipMalloc(&L.d_nbws, L.nbws_bytes) == hipSuccess;
    ok = ok && hipMalloc(&L.d_ws, L.ws_bytes) == hipSuccess;
    ok = ok && hipHostMalloc(&L.h_io, io, 0) == hipSuccess;
    return ok;
}

// enqueue the whole launch on its stream (no host synchronisation)
nnp_status enqueue(nnp_server* S, Launch& L) {
    hipStream_t s = L.stream;
    const int n = L.n_atoms, nm = (int)L.tickets.size();
    const IoLayout o = io_layout(n, nm);
    std::memset(L.h_io + o.flags, 0, 8);
    if (hipMemcpyAsync(L.d_io, L.h_io, o.e, hipMemcpyHostToDevice, s) != hipSuccess) return NNP_E_HIP;
    const float* d_pos = (const float*)L.d_io;
    const int32_t* d_sp = (const int32_t*)(L.d_io + o.sp);
    const int32_t* d_mol = (const int32_t*)(L.d_io + o.mol);
    unsigned* d_flags = (unsigned*)(L.d_io + o.flags);
    RowsView rows{};
    nnp_status st = build_neighbors(S->model, n, d_pos, d_mol, nm, nullptr, S->model->aev.rc_r, &L.nl, nullptr,
                                    L.d_nbws, L.nbws_bytes, s, false, d_flags, nullptr, nullptr, false, &rows);
    if (st != NNP_OK) return st;
    rows.rev = L.nl.rev;
    EfOpts opts;
    opts.rows = &rows;
    opts.rev_out = L.nl.rev;   // taken by the AEV kernel (no gate: every launch builds its rows)
    // the structure ranges the list build made and checked serve the energy sum as well
    st = neighbors_mol_ranges(L.d_nbws, n, nm, nullptr, S->model->aev.rc_r, &opts.mol_start, &opts.mol_end);
    if (st != NNP_OK) return st;
    st = energy_forces_impl(S->model, n, d_pos, d_sp, d_mol, nm, nullptr, &L.nl, (double*)(L.d_io + o.e), nullptr,
                            (float*)(L.d_io + o.f), L.d_ws, L.ws_bytes, s, d_flags, nullptr, nullptr, &opts);
    if (st != NNP_OK) return st;
    bool ok = hipMemcpyAsync(L.h_io + o.flags, L.d_io + o.flags, o.end - o.flags, hipMemcpyDeviceToHost, s) ==
              hipSuccess;
    ok = ok && hipEventRecord(L.done, s) == hipSuccess;
    return ok ? NNP_OK : NNP_E_HIP;
}

// results of a finished launch into the requests (lock held)
void finish(nnp_server* S, Launch& L, nnp_status launch_err) {
    const IoLayout o = io_layout(L.n_atoms, (int)L.tickets.size());
    const double* h_e = (const double*)(L.h_io + o.e);
    const float* h_f = (const float*)(L.h_io + o.f);
    const nnp_status st = launch_err != NNP_OK ? launch_err : flags_status(*(const unsigned*)(L.h_io + o.flags));
    for (size_t k = 0; k < L.tickets.size(); ++k) {
        auto it = S->reqs.find(L.tickets[k]);
        if (it == S->reqs.end()) continue;
        Req& r = it->second;
        S->arena.release(r.off, r.bytes);   // request memory is held until its launch completes
        if (st == NNP_OK) {
            r.energy = h_e[k];
            r.forces.assign(h_f + 3 * (size_t)L.offsets[k], h_f + 3 * ((size_t)L.offsets[k] + r.n));
            r.state = kDone;
        } else {
            r.err = st;
            r.state = kFailed;
        }
    }
    S->completed += L.tickets.size();
    L.tickets.clear();
    L.offsets.clear();
    L.busy = false;
}

void worker_main(nnp_server* S) {
    (void)hipSetDevice(S->model->device);
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        bool any_busy = false, did = false;
        for (auto& L : S->launches) {
            if (!L.busy) continue;
            if (hipEventQuery(L.done) == hipSuccess) {
                finish(S, L, NNP_OK);
                did = true;
            } else {
                any_busy = true;
            }
        }
        if (S->stop) {
            if (!any_busy) break;
        } else if (!S->queue.empty()) {
            Launch* L = nullptr;
            for (auto& c : S->launches)
                if (!c.busy) { L = &c; break; }
            if (L) {
                // the queued requests that fit (FIFO), then packed into the
                // launch's pinned staging in its layout
                L->n_atoms = 0;
                while (!S->queue.empty() && (int)L->tickets.size() < kLaunchRequests) {
                    Req& r = S->reqs[S->queue.front()];
                    if (L->n_atoms + r.n > kLaunchAtoms) break;
                    L->tickets.push_back(S->queue.front());
                    L->offsets.push_back(L->n_atoms);
                    L->n_atoms += r.n;
                    r.state = kRunning;
                    S->queue.pop_front();
                }
                const IoLayout o = io_layout(L->n_atoms, (int)L->tickets.size());
                for (size_t m = 0; m < L->tickets.size(); ++m) {
                    const Req& r = S->reqs[L->tickets[m]];
                    const char* src = S->inbox + r.off;
                    const size_t a0 = (size_t)L->offsets[m];
                    std::memcpy(L->h_io + 12 * a0, src, sizeof(float) * 3 * r.n);
                    std::memcpy(L->h_io + o.sp + 4 * a0, src + sizeof(float) * 3 * r.n, sizeof(int32_t) * r.n);
                    int32_t* mol = (int32_t*)(L->h_io + o.mol) + a0;
                    for (int a = 0; a < r.n; ++a) mol[a] = (int32_t)m;
                }
                L->busy = true;
                S->n_launches += 1;
                S->batched += L->tickets.size();
                lk.unlock();
                const nnp_status st = enqueue(S, *L);
                lk.lock();
                if (st != NNP_OK) {
                    (void)hipStreamSynchronize(L->stream);
                    finish(S, *L, st);
                }
                did = true;
                any_busy = true;
            }
        }
        if (did) continue;
        if (any_busy) {
            lk.unlock();
            std::this_thread::yield();
            lk.lock();
        } else if (!S->stop) {
            S->cv.wait_for(lk, std::chrono::milliseconds(1));
        }
    }
}

}  // namespace

extern "C" {

nnp_status nnp_server_create(nnp_model* model, size_t arena_bytes, int32_t max_slots, int32_t max_inflight,
                             nnp_server** out) {
    if (!model || !out || max_slots < 1 || max_inflight < 1 || max_inflight > 4 || arena_bytes < 16 * 8)
        return NNP_E_ARG;
    *out = nullptr;
    nnp_server* S = new nnp_server;
    S->model = model;
    S->max_slots = max_slots;
    S->max_inflight = max_inflight;
    S->pair_cap = (int64_t)kLaunchAtoms * NNP_MAX_ROW;   // the slots of fixed-stride rows
    if (hipSetDevice(model->device) != hipSuccess || hipHostMalloc(&S->inbox, arena_bytes, 0) != hipSuccess) {
        delete S;
        return NNP_E_NOMEM;
    }
    S->arena.init(arena_bytes);
    S->launches.resize(max_inflight);
    for (auto& L : S->launches) {
        if (!alloc_launch(S, L)) {
            for (auto& M : S->launches) free_launch(M);
            (void)hipHostFree(S->inbox);
            delete S;
            return NNP_E_NOMEM;
        }
    }
    S->worker = std::thread(worker_main, S);
    *out = S;
    return NNP_OK;
}

nnp_status nnp_submit(nnp_server* S, int32_t n, const int32_t* species, const float* pos, uint64_t* ticket) {
    if (!S || !species || !pos || !ticket || n < 1 || n > kMaxRequestAtoms) return NNP_E_ARG;
    for (int a = 0; a < n; ++a) {
        if (species[a] < 0 || species[a] >= S->model->aev.ns) return NNP_E_ARG;
        if (!std::isfinite(pos[3 * a]) || !std::isfinite(pos[3 * a + 1]) || !std::isfinite(pos[3 * a + 2]))
            return NNP_E_NONFINITE;
    }
    const size_t bytes = (size_t)n * (3 * sizeof(float) + sizeof(int32_t));
    std::lock_guard<std::mutex> lock(S->mu);
    if (S->stop) return NNP_E_ARG;
    if (bytes > S->arena.cap) return NNP_E_ARG;
    if (S->admitted >= S->max_slots) return NNP_E_BUSY;
    size_t off = 0;
    if (!S->arena.alloc(bytes, &off)) return NNP_E_BUSY;
    std::memcpy(S->inbox + off, pos, sizeof(float) * 3 * n);
    std::memcpy(S->inbox + off + sizeof(float) * 3 * n, species, sizeof(int32_t) * n);
    const uint64_t t = S->next_ticket++;
    Req& r = S->reqs[t];
    r.n = n;
    r.off = off;
    r.bytes = bytes;
    r.state = kQueued;
    S->queue.push_back(t);
    S->admitted += 1;
    *ticket = t;
    S->cv.notify_one();
    return NNP_OK;
}

nnp_status nnp_poll(nnp_server* S, uint64_t ticket, double* energy, float* forces) {
    if (!S) return NNP_E_ARG;
    std::lock_guard<std::mutex> lock(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return NNP_E_ARG;
    Req& r = it->second;
    if (r.state == kQueued || r.state == kRunning) return NNP_E_PENDING;
    nnp_status st = NNP_OK;
    if (r.state == kDone) {
        if (energy) *energy = r.energy;
        if (forces) std::memcpy(forces, r.forces.data(), sizeof(float) * r.forces.size());
    } else {
        st = r.err;
    }
    S->reqs.erase(it);
    S->admitted -= 1;
    return st;
}

nnp_status nnp_server_stats(nnp_server* S, uint64_t* completed, uint64_t* launches, uint64_t* batched) {
    if (!S) return NNP_E_ARG;
    std::lock_guard<std::mutex> lock(S->mu);
    if (completed) *completed = S->completed;
    if (launches) *launches = S->n_launches;
    if (batched) *batched = S->batched;
    return NNP_OK;
}

void nnp_server_destroy(nnp_server* S) {
    if (!S) return;
    {
        std::lock_guard<std::mutex> lock(S->mu);
        S->stop = true;
        S->cv.notify_all();
    }
    if (S->worker.joinable()) S->worker.join();
    for (auto& L : S->launches) free_launch(L);
    if (S->inbox) (void)hipHostFree(S->inbox);
    delete S;
}

}  // extern "C"
