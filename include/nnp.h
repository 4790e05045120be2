/*
 * nnp.h -- C ABI of the MI355X (gfx950) AEV neural-network potential.
 *
 * The library evaluates energy and forces of a symmetry-function atomic
 * environment vector (AEV) potential with one multi-layer perceptron per
 * chemical species -- the ANI-2x-shaped model the FeNNol paper benchmarks
 * (Sec. 5, "Performance benchmarks"; model flow of Sec. 2.4: AEV, species
 * network, per-structure energy sum, forces by differentiation).
 *
 * Conventions for every entry point:
 *   - extern "C", C99 types, no exceptions cross the boundary; every call
 *     returns an nnp_status (or a size / pointer as documented).
 *   - "device" pointers are GPU memory owned by the caller (for example
 *     torch tensors); "host" pointers are CPU memory owned by the caller.
 *     The library owns only what a model or server allocates for itself.
 *   - Streams are passed as an opaque `void*` holding a hipStream_t
 *     (NULL = the default stream).  Work is enqueued on that stream only.
 *   - Units: Angstrom, eV, eV/Angstrom, femtosecond, amu.
 *   - Species are indices 0..n_species-1 (for ANI-2x: H, C, N, O, F, S, Cl).
 *   - Atoms of one structure are contiguous and `mol` (the structure index
 *     of every atom, Sec. 2.1: concatenated atoms plus a batch index) is
 *     non-decreasing; mol == NULL means every atom belongs to structure 0.
 *   - Argument errors detected on the host return immediately.  Errors only
 *     visible on the device (species out of range, a neighbour row longer
 *     than the kernels support, non-finite coordinates, a non-monotonic
 *     `mol`) set sticky flags in the model; they are reported by the next
 *     call that synchronises (nnp_neighbors, nnp_check) and cleared then.
 */
#ifndef NNP_H
#define NNP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    NNP_OK = 0,
    NNP_E_ARG = 1,        /* invalid argument (host-checked or device flag)       */
    NNP_E_CAPACITY = 2,   /* neighbour-list capacity too small; size reported     */
    NNP_E_BOX = 3,        /* a box side is below twice the list cutoff            */
    NNP_E_NONFINITE = 4,  /* NaN or Inf coordinates                               */
    NNP_E_NOMEM = 5,      /* device or host allocation failed / arena full        */
    NNP_E_BUSY = 6,       /* serving: no free request slot                        */
    NNP_E_PENDING = 7,    /* serving: the request has not completed yet           */
    NNP_E_HIP = 8,        /* a HIP runtime call failed                            */
    NNP_E_ROW = 9,        /* an atom has more neighbours than the kernels support */
    NNP_E_SCRATCH = 10    /* the call needs more than the fixed device scratch of
                             the allocation-free entry point                      */
} nnp_status;

typedef enum {
    NNP_FP32 = 0,         /* every stage in float32 (MLP on FP32 MFMA)            */
    NNP_BF16_MLP = 1      /* MLP matrix products take bfloat16 inputs on MFMA with
                             float32 accumulation; AEV, cutoffs, edge gradients and
                             forces stay float32; structure energies float64      */
} nnp_precision;

/* Device error flags (bit set), as returned by nnp_check. */
#define NNP_FLAG_SPECIES   0x1u   /* species index out of range                  */
#define NNP_FLAG_ROW       0x2u   /* neighbour row longer than NNP_MAX_ROW        */
#define NNP_FLAG_NONFINITE 0x4u   /* non-finite coordinate                        */
#define NNP_FLAG_MOL       0x8u   /* mol not non-decreasing or out of [0, n_mol) */
#define NNP_FLAG_SHIFT     0x10u  /* periodic image shift outside int8 range      */
#define NNP_FLAG_CAPACITY  0x20u  /* asynchronous list build exceeded its capacity */
#define NNP_FLAG_REVERSE   0x40u  /* a pair i -> j whose reverse j -> i is absent  */

/* Largest neighbour-row length (pairs within the list cutoff of one atom) the
 * AEV kernels accept.  Longer rows set NNP_FLAG_ROW and contribute nothing. */
#define NNP_MAX_ROW 256
/* Largest ensemble nnp_model_create_ensemble accepts. */
#define NNP_MAX_NETS 16
/* Largest number of neighbours within the angular cutoff of one atom. */
#define NNP_MAX_ANGULAR 96

typedef struct nnp_model nnp_model;     /* opaque: AEV parameters + packed weights */
typedef struct nnp_server nnp_server;   /* opaque: serving arena and scheduler     */

/* AEV hyper-parameters (Sec. 2.1 cosine switching function; Sec. 2.2 Gaussian
 * radial basis; App. A ANI angular basis).  Arrays are host memory, copied. */
typedef struct {
    int32_t n_species;        /* number of species (<= 8)                          */
    float rc_r;               /* radial cutoff Rc_R (5.1)                          */
    float eta_r;              /* radial Gaussian width eta_R (19.7)                */
    int32_t n_shf_r;          /* number of radial shells (16)                      */
    const float* shf_r;       /* [n_shf_r] radial shell centres R_k                */
    float rc_a;               /* angular cutoff Rc_A (3.5), rc_a <= rc_r           */
    float eta_a;              /* angular radial width eta_A (12.5)                 */
    float zeta;               /* angular exponent zeta (14.1); must exceed 1       */
    int32_t n_shf_a;          /* number of angular radial shells (4)               */
    int32_t n_shf_z;          /* number of angle sections (8)                      */
    const float* shf_a;       /* [n_shf_a] angular radial shell centres R_a        */
    const float* shf_z;       /* [n_shf_z] angle section centres theta_z           */
    float radial_prefactor;   /* factor on every radial term (0.25)                */
    float cos_scale;          /* cos(theta) is scaled by this before arccos (0.95) */
} nnp_aev_params;

/* Per-species MLP (Sec. 2.2, "Neural Networks": fully species-dependent
 * parameters).  widths[0] must equal the AEV length; widths[n_layers] must
 * be 1.  W[s*n_layers + l] is host float32 row-major [widths[l+1]][widths[l]];
 * b[s*n_layers + l] is [widths[l+1]].  Copied at model creation. */
typedef struct {
    int32_t n_layers;           /* 4 for 1008-256-192-160-1                        */
    const int32_t* widths;      /* [n_layers + 1]                                  */
    const float* const* W;      /* [n_species * n_layers]                          */
    const float* const* b;      /* [n_species * n_layers]                          */
    float celu_alpha;           /* CELU alpha (0.1)                                */
    const double* self_energy;  /* [n_species] added to every atomic energy, or NULL */
} nnp_mlp_params;

/* Caller-owned neighbour list (device memory): directed pairs i -> j of the
 * same structure with |v_ij| < r_list, v_ij = x_j + shift * box - x_i
 * (minimum image for periodic boxes).  Row i is col[row_ptr[i] ..
 * row_ptr[i+1]) sorted by ascending j.  rev[p] is the index of the reverse
 * pair j -> i.  Sec. 2.1, "Preprocessing Modules". */
typedef struct {
    int32_t* row_ptr;         /* [n_atoms + 1]                                     */
    int32_t* col;             /* [capacity]                                        */
    int8_t* shift;            /* [capacity][3] image shift in box vectors          */
    int32_t* rev;             /* [capacity]                                        */
    int64_t capacity;         /* entries available in col / shift / rev            */
    float r_list;             /* cutoff the list was built with (set by nnp_neighbors) */
    int32_t n_atoms;          /* set by nnp_neighbors                              */
    int64_t n_pairs;          /* set by nnp_neighbors                              */
} nnp_nlist;

/* ---------------------------------------------------------------- model */

/* Create a model on the current HIP device: validates the parameters, packs
 * the weights (float32 and bfloat16 copies, padded for MFMA tiles) into
 * device memory owned by the model.  *out receives the handle. */
nnp_status nnp_model_create(const nnp_aev_params* aev, const nnp_mlp_params* mlp,
                            nnp_precision precision, nnp_model** out);
/* An ensemble of n_nets networks on one shared AEV (ANI-2x is an ensemble
 * of eight networks; the paper's benchmarks evaluate the first one only,
 * Sec. 5.5).  nets[k] are complete network parameter sets with identical
 * widths, which must be 1008-256-192-160-1 (the fused kernels); self
 * energies come from nets[0].  Every entry point then works with the
 * ensemble-mean atomic energy E_i = (1/n_nets) sum_k E_i^k (+ self energy)
 * and its forces.  1 <= n_nets <= NNP_MAX_NETS; NNP_E_ARG otherwise. */
nnp_status nnp_model_create_ensemble(const nnp_aev_params* aev, const nnp_mlp_params* nets,
                                     int32_t n_nets, nnp_precision precision, nnp_model** out);
/* Networks of the model (1 for nnp_model_create). */
int32_t nnp_model_nets(const nnp_model* model);
void nnp_model_destroy(nnp_model* model);
/* Switch the precision form used by later nnp_energy_forces calls. */
nnp_status nnp_model_set_precision(nnp_model* model, nnp_precision precision);
const char* nnp_status_str(nnp_status status);
/* 1 if the species networks run as one fused kernel per tile (forward, head
 * and adjoint; available for the 1008-256-192-160-1 shape), 0 if they run
 * as one GEMM kernel per layer. */
int32_t nnp_model_fused_mlp(const nnp_model* model);
/* Allow (1) or forbid (0) the fused kernel; forbidding selects the per-layer
 * GEMM path (both compute the same function; used to compare them). */
nnp_status nnp_model_set_fused_mlp(nnp_model* model, int32_t allow);
/* Number of AEV features (1008 for ANI-2x) and padded row stride used by
 * nnp_aev (1024). */
int32_t nnp_aev_dim(const nnp_model* model);

/* Synchronise `stream`, read and clear the model's sticky device flags.
 * Returns NNP_OK if none is set, else the status of the first flag; *flags
 * (if non-NULL) receives the raw bit set. */
nnp_status nnp_check(nnp_model* model, void* stream, uint32_t* flags);

/* ---------------------------------------------------------------- neighbours */

/* Device workspace (bytes) nnp_neighbors needs for this system. */
size_t nnp_neighbors_workspace_bytes(int32_t n_atoms, int32_t n_mol, const float* box_host,
                                     float r_list);

/* Build the neighbour list of Sec. 2.1 with an integer cell list (periodic
 * box) or an all-pairs scan inside each structure (open boundaries).
 *   pos      device float32 [n_atoms][3]
 *   mol      device int32 [n_atoms] or NULL
 *   box_host host float32 [3] orthorhombic box sides, or NULL (open)
 *   r_list   list cutoff (model cutoff plus any skin)
 * The pair predicate is exact: coordinates are widened to float64,
 * d0 = x_j - x_i, n = -rint(d0 / L), d = d0 + n L, d2 = (dx^2 + dy^2) + dz^2
 * with every operation rounded (no fused multiply-add), pair kept iff
 * d2 < r_list^2 (r_list widened to float64).  The resulting pair set is
 * therefore identical bit for bit on any conforming implementation.
 * Synchronises `stream` once, to read the pair count: if it exceeds
 * nl->capacity the call returns NNP_E_CAPACITY, *n_pairs_host receives the
 * required size and the list contents are undefined (regrow and call again).
 * Returns NNP_E_BOX if any box side is below 2 r_list, NNP_E_NONFINITE for
 * non-finite coordinates, NNP_E_ARG for a bad `mol`. */
nnp_status nnp_neighbors(nnp_model* model, int32_t n_atoms, const float* pos, const int32_t* mol,
                         int32_t n_mol, const float* box_host, float r_list, nnp_nlist* nl,
                         int64_t* n_pairs_host, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------- energy and forces */

/* Device workspace (bytes) nnp_energy_forces / nnp_aev need for n_atoms
 * atoms and a neighbour list of pair_capacity entries. */
size_t nnp_workspace_bytes(const nnp_model* model, int32_t n_atoms, int64_t pair_capacity);

/* Energy and forces (Sec. 2.4): AEV of every atom from the list, species
 * network per atom, float64 sum of atomic energies per structure (ascending
 * atom order), forces F = -dE/dx through a hand-written adjoint of the
 * network, the AEV and the pair geometry.
 *   pos      device float32 [n_atoms][3]
 *   species  device int32 [n_atoms]
 *   mol      device int32 [n_atoms] or NULL; n_mol structures
 *   box_host host float32 [3] or NULL; must be the box the list was built for
 *   nl       list built by nnp_neighbors for these positions (a list built
 *            with a larger r_list, e.g. with a skin, is valid while no pair
 *            has moved inside the model cutoff unseen)
 *   e_mol    device float64 [n_mol]          (written)
 *   e_atom   device float32 [n_atoms] or NULL (written)
 *   forces   device float32 [n_atoms][3] or NULL (written)
 * Fully asynchronous on `stream`; never synchronises. */
nnp_status nnp_energy_forces(nnp_model* model, int32_t n_atoms, const float* pos,
                             const int32_t* species, const int32_t* mol, int32_t n_mol,
                             const float* box_host, const nnp_nlist* nl, double* e_mol,
                             float* e_atom, float* forces, void* ws, size_t ws_bytes,
                             void* stream);

/* nnp_energy_forces plus the virial (the stress-tensor output of the
 * energy/forces/virial call of Sec. 5.1).  With G_ij = dE_i/dv_ij the edge
 * gradient of the force adjoint,
 *   W = - sum over edges i -> j of v_ij (outer) G_ij      (eV),
 * which equals sum_a x_a (outer) F_a for an open structure and minus the
 * (transposed) derivative of E under a homogeneous strain of every edge
 * vector for a periodic one; pressure = (N k_B T + tr W / 3) / V.
 *   virial       device float64 [n_mol][3][3] row-major (written; required)
 *   atom_virial  device float32 [n_atoms][3][3] or NULL: the same sum over
 *                the edges leaving each atom (written)
 *   forces       required (the virial comes from the force adjoint)
 * Structure sums are float64 in ascending atom order (deterministic).
 * Other arguments, errors and asynchrony as nnp_energy_forces. */
nnp_status nnp_energy_forces_virial(nnp_model* model, int32_t n_atoms, const float* pos,
                                    const int32_t* species, const int32_t* mol, int32_t n_mol,
                                    const float* box_host, const nnp_nlist* nl, double* e_mol,
                                    float* e_atom, float* forces, double* virial,
                                    float* atom_virial, void* ws, size_t ws_bytes, void* stream);

/* nnp_energy_forces of an ensemble model (n_nets >= 2) that also writes
 * every network's structure energies (self energies included), the spread
 * of which estimates the model's uncertainty:
 *   e_mol_net  device float64 [n_nets][n_mol] (written; required)
 * e_mol, e_atom, forces as nnp_energy_forces (ensemble mean). */
nnp_status nnp_energy_forces_ensemble(nnp_model* model, int32_t n_atoms, const float* pos,
                                      const int32_t* species, const int32_t* mol, int32_t n_mol,
                                      const float* box_host, const nnp_nlist* nl, double* e_mol,
                                      double* e_mol_net, float* e_atom, float* forces, void* ws,
                                      size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------- allocation-free call */

/* Size of the fixed device scratch nnp_energy_forces_static works in. */
#define NNP_STATIC_SCRATCH_BYTES ((size_t)64 << 20)

/* nnp_energy_forces without a workspace argument, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  The intermediates of the call (grouped
 * features, dE/dAEV, hidden activations, edge gradients, energy partials)
 * live in one fixed scratch array of NNP_STATIC_SCRATCH_BYTES, which the
 * library holds on every device it runs on until the process ends; its
 * device address is resolved once per device when a model is created there.
 * The call allocates nothing (no hipMalloc, no hipFree, no allocating library
 * routine) and never synchronises.
 *   Arguments, layouts, ownership and the device-side error flags as
 *   nnp_energy_forces; inputs and outputs are still the caller's buffers.
 *   Returns NNP_E_SCRATCH, before anything is launched, if the call needs
 *   more than NNP_STATIC_SCRATCH_BYTES (nnp_workspace_bytes(model, n_atoms,
 *   nl->capacity) gives the need: about 5,000 atoms of water with a list
 *   sized to its pairs).
 *   Stage timing (nnp_profile_enable) is not recorded by this call.
 * Every call on a device shares that device's one scratch array, which keeps
 * the last call's contents (nothing in it needs to start at zero): calls
 * that overlap on one device (two streams, two threads) race, and the caller
 * must serialise them. */
nnp_status nnp_energy_forces_static(nnp_model* model, int32_t n_atoms, const float* pos,
                                    const int32_t* species, const int32_t* mol, int32_t n_mol,
                                    const float* box_host, const nnp_nlist* nl, double* e_mol,
                                    float* e_atom, float* forces, void* stream);

/* The AEV alone (the radial and angular features of Sec. 2.2 / App. A):
 * writes aev_out, device float32 [n_atoms][aev_stride] (aev_stride =
 * nnp_aev_dim rounded up to 1024; padding columns are zero), rows in atom
 * order.  Asynchronous. */
nnp_status nnp_aev(nnp_model* model, int32_t n_atoms, const float* pos, const int32_t* species,
                   const float* box_host, const nnp_nlist* nl, float* aev_out, void* ws,
                   size_t ws_bytes, void* stream);

/* The species networks alone on given features (Sec. 2.2): aev_in device
 * float32 [n_atoms][aev_stride]; writes e_atom [n_atoms] (float32, self
 * energy included) and, if non-NULL, daev_out [n_atoms][aev_stride] =
 * dE_i/dAEV_i.  Asynchronous. */
nnp_status nnp_mlp(nnp_model* model, int32_t n_atoms, const int32_t* species, const float* aev_in,
                   float* e_atom, float* daev_out, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------- molecular dynamics */

/* Velocity Verlet (the NVE integrator of the paper's native engine, Sec. 5.4):
 * first half: v += dt/2 * F * inv_mass * 9.648533212e-3; x += dt * v.  All
 * device float32: pos/vel/forces [n_atoms][3], inv_mass [n_atoms] (1/amu).
 * If ref_pos is non-NULL, the largest squared displacement from ref_pos is
 * folded into *max_disp2 (device float32, caller clears it). */
nnp_status nnp_md_kick_drift(int32_t n_atoms, float* pos, float* vel, const float* forces,
                             const float* inv_mass, float dt, const float* ref_pos,
                             float* max_disp2, void* stream);
/* Second half: v += dt/2 * F * inv_mass * 9.648533212e-3. */
nnp_status nnp_md_kick(int32_t n_atoms, float* vel, const float* forces, const float* inv_mass,
                       float dt, void* stream);
/* Wrap positions into [0, L) per dimension (periodic boxes, before a rebuild). */
nnp_status nnp_md_wrap(int32_t n_atoms, float* pos, const float* box_host, void* stream);

/* ---------------------------------------------------------------- native MD engine */

/* The paper's native engine (Sec. 5.4) keeps the whole time step on the GPU;
 * its benchmarks (Sec. 5.5) run Langevin dynamics at 300 K with a 0.5 fs
 * step and a neighbour-list buffer rebuilt every few steps.  An nnp_md owns
 * one structure's state (periodic orthorhombic box or open) in device memory
 * and advances it with:
 *   NNP_MD_NVE       velocity Verlet: B(dt/2) A(dt) | F | B(dt/2)
 *   NNP_MD_LANGEVIN  BAOAB: B(dt/2) A(dt/2) O A(dt/2) | F | B(dt/2), with
 *                    O: v = c1 v + sqrt((1 - c1^2) kT / m) xi, c1 = exp(-gamma dt)
 * B: v += h F/m (9.648533212e-3 converts eV/A/amu to A/fs^2), A: x += h v.
 * xi for atom a at step s (steps counted from 0 at creation) are three
 * Gaussian numbers from one Philox4x64-10 block (Salmon et al., SC'11) with
 * counter (a + 1, s, 0, 0) and key (seed, 0): with the block's words w_k,
 * u_k = ((w_k >> 40) + 1/2) 2^-24, xi = (rho0 cos 2pi u1, rho0 sin 2pi u1,
 * rho2 cos 2pi u3), rho_k = sqrt(-2 ln u_k).
 * The list (cutoff = radial cutoff + skin) is rebuilt, positions wrapped into
 * the box, every rebuild_every steps, and earlier as soon as the two largest
 * displacements since the last build sum to more than trigger * skin (the
 * Verlet-list bound: a pair outside the list was at least cutoff + skin
 * apart at the build and has since come closer by at most the sum of its
 * two atoms' displacements); the decision is taken on the device.  With a
 * skin, 0 < trigger <= 1 is required (1 is the exact bound); without one
 * (skin = 0), rebuild_every must be 1.  Other settings could let a pair
 * come within the cutoff unlisted and are rejected (NNP_E_ARG). */
typedef enum { NNP_MD_NVE = 0, NNP_MD_LANGEVIN = 1 } nnp_md_integrator;

typedef struct {
    nnp_md_integrator integrator;
    float dt;                 /* fs                                               */
    float temperature;        /* K (Langevin)                                     */
    float friction;           /* gamma in 1/ps (Langevin)                         */
    uint64_t seed;            /* key of the noise generator (Langevin)            */
    float skin;               /* A, added to the radial cutoff for the list       */
    int32_t rebuild_every;    /* >= 1                                             */
    float trigger;            /* early rebuild when d1 + d2 > trigger * skin      */
    int32_t log_every;        /* > 0: record (E_pot, E_kin) every log_every steps */
    int32_t log_capacity;     /* rows kept (later rows are dropped)               */
} nnp_md_params;

typedef struct {
    int64_t steps;            /* steps taken since creation                       */
    int64_t rebuilds;         /* list builds, the one at creation included        */
    int64_t early_rebuilds;   /* builds triggered by displacement                 */
    int64_t capacity;         /* list slots: n_atoms * NNP_MAX_ROW                */
    float r_list;
} nnp_md_stats;

typedef struct nnp_md nnp_md;

/* Create an engine for n_atoms atoms: pos, vel (A/fs) device float32
 * [n][3], species device int32 [n], masses device float32 [n] (amu, > 0),
 * box_host host float32 [3] or NULL.  Inputs are copied; the engine owns
 * its device memory, all of it allocated here: the list is kept as
 * fixed-stride rows of NNP_MAX_ROW slots per atom, so it never regrows.
 * Builds the list and the starting forces (synchronises once).  The model
 * must outlive it.  NNP_E_BOX if a box side is below 2 (cutoff + skin);
 * NNP_E_NONFINITE for non-finite positions or non-positive masses;
 * NNP_E_ROW if an atom has more than NNP_MAX_ROW neighbours. */
nnp_status nnp_md_create(nnp_model* model, int32_t n_atoms, const float* pos, const float* vel,
                         const int32_t* species, const float* masses, const float* box_host,
                         const nnp_md_params* params, void* stream, nnp_md** out);
/* Advance n_steps steps.  The steps are enqueued without waiting; the call
 * synchronises `stream` once at the end to read the error flags.  Errors
 * (the state is then that of a run that went on with the faulty values;
 * the step counter counts every step enqueued): NNP_E_NONFINITE, NNP_E_ROW
 * (a rebuild found an atom with more than NNP_MAX_ROW neighbours). */
nnp_status nnp_md_run(nnp_md* md, int32_t n_steps, void* stream);
/* Copy the current state into caller device buffers (any may be NULL):
 * pos, vel, forces float32 [n][3], e_pot float64 [1] (the potential energy
 * of the current positions: every step sums it).  Asynchronous. */
nnp_status nnp_md_get(nnp_md* md, float* pos, float* vel, float* forces, double* e_pot,
                      void* stream);
/* Copy up to max_rows logged rows {E_pot, E_kin} (eV, float64) to host
 * memory; *n_rows receives the count.  Synchronises. */
nnp_status nnp_md_log(nnp_md* md, double* host_rows, int32_t max_rows, int32_t* n_rows,
                      void* stream);
/* Counters (synchronises). */
nnp_status nnp_md_info(nnp_md* md, nnp_md_stats* out, void* stream);
void nnp_md_destroy(nnp_md* md);

/* ---------------------------------------------------------------- serving */

/* Continuous-batching server over one model (the model must outlive it).
 * Requests are single open-boundary structures of 1..256 atoms (Sec. 2.1:
 * structures of a batch never interact; Sec. 2.4: a batch is the
 * concatenation of its structures' atoms).  A request is admitted when a
 * slot is free and its inputs fit in the request arena; a scheduler thread
 * gathers every queued request (FIFO, up to 16384 atoms) into the next
 * launch as soon as one of `max_inflight` launch contexts is free, so
 * requests arriving while others are on the GPU join the next launch and
 * launches overlap on the device, each on its own stream with persistent
 * device buffers.
 *   arena_bytes  pinned host bytes for queued request inputs (16 B per atom)
 *   max_slots    most requests admitted and not yet polled to completion
 *   max_inflight launch contexts (1..4); each holds about 310 MB of device
 *   memory (measured for the 7-species FP32 model) */
nnp_status nnp_server_create(nnp_model* model, size_t arena_bytes, int32_t max_slots,
                             int32_t max_inflight, nnp_server** out);
/* Admit one request: host species [n_atoms] and float32 positions
 * [n_atoms][3] are copied (the caller may reuse its buffers on return);
 * *ticket receives a monotonically increasing id.  NNP_E_BUSY if no slot or
 * arena memory is free now (retry later); NNP_E_ARG for a request that can
 * never be served (size, species), NNP_E_NONFINITE for NaN/Inf positions. */
nnp_status nnp_submit(nnp_server* server, int32_t n_atoms, const int32_t* species,
                      const float* pos, uint64_t* ticket);
/* Non-blocking: NNP_E_PENDING until the request has completed; then copies
 * the float64 energy and float32 forces [n_atoms][3] (forces may be NULL)
 * to host memory and frees the slot (a ticket can be polled to completion
 * once; an unknown or already collected ticket gives NNP_E_ARG).  A request
 * whose launch raised a device flag completes with that flag's status. */
nnp_status nnp_poll(nnp_server* server, uint64_t ticket, double* energy, float* forces);
/* Counters: completed requests, launches issued, requests summed over launches. */
nnp_status nnp_server_stats(nnp_server* server, uint64_t* completed, uint64_t* launches,
                            uint64_t* batched_requests);
void nnp_server_destroy(nnp_server* server);

/* ---------------------------------------------------------------- stage timing */

/* Stages of nnp_neighbors / nnp_energy_forces / the MD kernels, for timing. */
enum {
    NNP_STAGE_NEIGHBORS = 0,   /* cell binning, row count, row fill + sort, reverse index */
    NNP_STAGE_GROUP = 1,       /* species grouping                                      */
    NNP_STAGE_AEV = 2,         /* AEV forward (one kernel)                               */
    NNP_STAGE_MLP = 3,         /* species networks, forward and adjoint                  */
    NNP_STAGE_ENERGY = 4,      /* float64 structure energies                            */
    NNP_STAGE_AEV_ADJ = 5,     /* AEV adjoint -> edge gradients (one kernel)             */
    NNP_STAGE_FORCES = 6,      /* force gather (one kernel)                              */
    NNP_STAGE_INTEGRATE = 7,   /* MD engine: integrator kernels and rebuild decision      */
    NNP_N_STAGES = 8
};

/* Enable (1) or disable (0) per-stage timing: while enabled, the library
 * records a pair of HIP events on the call's stream around every stage it
 * enqueues (a few microseconds of host overhead per stage; intended for one
 * stream at a time).  Enabling clears the accumulated times. */
nnp_status nnp_profile_enable(nnp_model* model, int enable);
/* As nnp_profile_enable, timing only the stages whose bit (1 << NNP_STAGE_x)
 * is set in mask (0 disables): fewer events in the stream when one stage's
 * kernel time is wanted inside a timed run. */
nnp_status nnp_profile_enable_mask(nnp_model* model, uint32_t mask);
/* Wait for the recorded events, add their elapsed times to the running
 * totals and return them: ms[NNP_N_STAGES] (milliseconds summed over
 * launches) and count[NNP_N_STAGES] (number of timed stage executions). */
nnp_status nnp_profile_read(nnp_model* model, double* ms, int64_t* count);

#ifdef __cplusplus
}
#endif
#endif /* NNP_H */
