// ANI atomic environment vector: forward and adjoint (one wave per atom).
//
// Definitions (Sec. 2.1 cosine switching function; Sec. 2.2 Gaussian radial
// encoding; App. A ANI angular basis; ANI AEV as used by the ANI_AEV module
// of Sec. 2.4):
//   radial   G[i][16 s + k]          = sum_{j: Z_j = s, r_ij < Rc_R}
//                                        p_R exp(-eta_R (r_ij - R_k)^2) fc_R(r_ij)
//   angular  G[i][D_R + 32 p + 8a + z] = sum_{j<k: r_ij, r_ik < Rc_A, pair(Z_j,Z_k) = p}
//                 2 ((1 + cos(theta' - theta_z)) / 2)^zeta
//                 exp(-eta_A ((r_ij + r_ik)/2 - R_a)^2) fc_A(r_ij) fc_A(r_ik)
//   with cos(theta' - theta_z) = u cos(theta_z) + sqrt(1 - u^2) sin(theta_z),
//   u = cos_scale * cos(theta_ijk).
//
// Work layout.  A wave owns one centre atom.  Each lane holds up to four
// slots of the atom's CSR row in registers (loaded once: one dependent-load
// chain per row), computes the float32 edge vectors, and the neighbours
// within each cutoff are grouped by species in LDS with a stable ballot sort.
//   forward:  radial sums with lanes as (shell k, quarter q) over each species
//             segment; angular sums per species-pair bin, one neighbour pair
//             per lane (8 angle factors, 4 radial factors) into a 64-pair LDS
//             tile, reduced by lanes as (shell, 4 angle sections, eighth of
//             the pairs).
//   adjoint:  radial gradient by the lane that holds the slot; angular pair
//             gradients one pair per lane into an LDS tile of up to 192
//             pairs, then summed per angular neighbour in a fixed order (one
//             pass over the tile, the same trip count for every lane).
// Every sum runs in a fixed order (no atomics), so results do not depend on
// scheduling or on the other atoms of a batch.
#include "nnp_internal.hpp"

namespace nnp {
namespace {

constexpr int kMaxR = NNP_MAX_ROW;        // CSR slots per row
constexpr int kQ = kMaxR / kWave;         // slots per lane
constexpr int kMaxA = NNP_MAX_ANGULAR;    // neighbours within the angular cutoff
constexpr int kWaves = 4;                 // waves (atoms) per block

__device__ __forceinline__ float cutoff_fc(float r, float pi_rc) { return 0.5f * __cosf(pi_rc * r) + 0.5f; }

// The hardware's own approximations (v_sqrt_f32, v_rcp_f32, v_log_f32,
// v_exp_f32, about 1 ulp each) without the library's denormal range
// handling: every argument here is a normal number or zero, and a result
// below the normal range is negligible next to the terms it is summed with.
__device__ __forceinline__ float hw_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float hw_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float hw_log2(float x) { return __builtin_amdgcn_logf(x); }
__device__ __forceinline__ float hw_exp2(float x) { return __builtin_amdgcn_exp2f(x); }

__device__ __forceinline__ int species_pair(int s, int t, int ns) {
    if (s > t) { int u = s; s = t; t = u; }
    return s * ns - (s * (s - 1)) / 2 + (t - s);
}

// (j, k) of the v-th unordered pair (j < k) of c <= NNP_MAX_ANGULAR items in
// row-major triangle order.  j is the largest integer with j (2c - j - 1) / 2
// <= v; the float root of that quadratic is exact up to the square root's
// rounding, so its truncation is off by at most one and one correction step
// each way gives j (checked exhaustively for every c and v, with the root
// perturbed by up to 4 ulp).  The products are below 2^24: 24-bit multiplies.
__device__ __forceinline__ void tri_decode(int v, int c, int& j, int& k) {
    const float tc = (float)(2 * c - 1);
    int jj = (int)((tc - hw_sqrt(fmaxf(tc * tc - 8.0f * (float)v, 0.f))) * 0.5f);
    jj = max(0, min(jj, c - 2));
    jj -= jj > 0 && (__mul24(jj, 2 * c - jj - 1) >> 1) > v;
    jj += jj + 1 <= c - 2 && (__mul24(jj + 1, 2 * c - jj - 2) >> 1) <= v;
    j = jj;
    k = jj + 1 + (v - (__mul24(jj, 2 * c - jj - 1) >> 1));
}

// base^zeta for base in [0, 1] (log2 0 = -inf gives 0; a base rounded below
// zero is clamped)
__device__ __forceinline__ float pow_zeta(float base, float zeta) { return hw_exp2(zeta * hw_log2(fmaxf(base, 0.f))); }

template <typename OutT>
__device__ __forceinline__ void store_out(OutT* p, float v);
template <>
__device__ __forceinline__ void store_out<float>(float* p, float v) { *p = v; }
template <>
__device__ __forceinline__ void store_out<uint16_t>(uint16_t* p, float v) { *p = f32_to_bf16(v); }

// Row slots of one atom, held in registers (slot = lane + 64 q).
struct Row {
    float vx[kQ], vy[kQ], vz[kQ], r2[kQ];
    int z[kQ];
    bool in_r[kQ], in_a[kQ];
    int b, len;
};

// Load row i (slots b .. e - 1) and classify every slot.  Returns false (and flags) if the
// row is longer than the kernels support.  kPacked: the builder's
// fixed-stride rows (packed image shifts), else the CSR list.  The loads are
// issued in two rounds with no wait among them: every slot's column and
// image shift, then every slot's neighbour position and species (a slot past
// the row's end reads the row's last entry), so a row costs two dependent
// memory round trips.  Slots past the row's end are discarded.
template <bool kPacked>
__device__ __forceinline__ bool load_row(Row& R, const AevConst& P, int i, int b, int e, const float* __restrict__ pos,
                                         const int32_t* __restrict__ species, const BoxConst& bx, const RowsView& rows,
                                         unsigned* flags) {
    const int l = lane_id();
    R.b = b;
    R.len = e - b;
    if (R.len > kMaxR) {
        if (l == 0) set_flag(flags, NNP_FLAG_ROW);
        return false;
    }
    const int last = e > b ? e - 1 : b;
    int pc[kQ], j[kQ], s0[kQ], s1[kQ], s2[kQ];
    bool valid[kQ];
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
        const int p = b + l + kWave * q;
        valid[q] = p < e;
        pc[q] = min(p, last);
    }
    // round 1: columns and shifts.  Fixed-stride rows load every group (a
    // slot past the row's end re-reads its last entry, or slot b of the
    // row's own fixed-stride space: no branch, so no wait between the
    // groups); CSR rows, whose shifts take three byte loads per slot and
    // whose slot b need not exist for an empty row, skip the groups past the
    // row's end (wave-uniform)
    const int nq = (R.len + kWave - 1) / kWave;
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
        j[q] = i;
        s0[q] = s1[q] = s2[q] = 0;
        if (kPacked || q < nq) {
            j[q] = rows.col[pc[q]];
            if (kPacked) {
                s0[q] = rows.shift_packed[pc[q]];
            } else {
                s0[q] = rows.shift[3 * pc[q]];
                s1[q] = rows.shift[3 * pc[q] + 1];
                s2[q] = rows.shift[3 * pc[q] + 2];
            }
        }
    }
    // round 2: neighbour positions and species (the group count passes
    // through readfirstlane, which keeps the compiler from merging each
    // group's two rounds into one block with a wait inside)
    const int nq2 = __builtin_amdgcn_readfirstlane(nq);
    float px[kQ], py[kQ], pz[kQ];
    int zz[kQ];
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
        px[q] = py[q] = pz[q] = 0.f;
        zz[q] = 0;
        if (kPacked || q < nq2) {
            const int jj = valid[q] ? j[q] : i;
            px[q] = pos[3 * jj];
            py[q] = pos[3 * jj + 1];
            pz[q] = pos[3 * jj + 2];
            zz[q] = species[jj];
        }
    }
    const float xi = pos[3 * i], yi = pos[3 * i + 1], zi = pos[3 * i + 2];
    const float rc_r2 = P.rc_r * P.rc_r, rc_a2 = P.rc_a * P.rc_a;
    const float Lx = bx.periodic ? bx.L[0] : 0.f, Ly = bx.periodic ? bx.L[1] : 0.f, Lz = bx.periodic ? bx.L[2] : 0.f;
    bool bad_species = false;
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
        R.vx[q] = R.vy[q] = R.vz[q] = R.r2[q] = 0.f;
        R.z[q] = 0;
        R.in_r[q] = R.in_a[q] = false;
        if (q >= nq2) continue;   // wave-uniform: a group past the row's end
        float sx, sy, sz;
        if (kPacked) {
            sx = (float)(int8_t)(s0[q] & 0xff);
            sy = (float)(int8_t)((s0[q] >> 8) & 0xff);
            sz = (float)(int8_t)((s0[q] >> 16) & 0xff);
        } else {
            sx = (float)s0[q];
            sy = (float)s1[q];
            sz = (float)s2[q];
        }
        const float vx = (px[q] - xi) + sx * Lx, vy = (py[q] - yi) + sy * Ly, vz = (pz[q] - zi) + sz * Lz;
        const float r2 = vx * vx + vy * vy + vz * vz;
        const bool ok_z = zz[q] >= 0 && zz[q] < P.ns;
        bad_species |= valid[q] && !ok_z;
        const bool use = valid[q] && ok_z;
        R.vx[q] = valid[q] ? vx : 0.f;
        R.vy[q] = valid[q] ? vy : 0.f;
        R.vz[q] = valid[q] ? vz : 0.f;
        R.r2[q] = valid[q] ? r2 : 0.f;
        R.z[q] = use ? zz[q] : 0;
        R.in_r[q] = use && r2 < rc_r2;
        R.in_a[q] = use && r2 < rc_a2;
    }
    if (bad_species) set_flag(flags, NNP_FLAG_SPECIES);
    return true;
}

// Stable positions of the slots in species-grouped lists (radial and angular).
// seg_r / seg_a receive the species offsets (ns + 1 entries); *present gets
// the wave-uniform masks of the species found inside the radial cutoff (bits
// 0-7) and inside the angular cutoff (bits 8-15).  Absent species cost no
// ballots.  Returns false if more than kMaxA neighbours fall inside the
// angular cutoff.
__device__ __forceinline__ bool group_species(const Row& R, int ns, int* pos_r, int* pos_a, int* seg_r,
                                              int* seg_a, unsigned* present, unsigned* flags) {
    const int l = lane_id();
    const int nq = (R.len + kWave - 1) / kWave;
    int bits = 0;
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
        if (q < nq && R.in_r[q]) bits |= 1 << R.z[q];
        if (q < nq && R.in_a[q]) bits |= 0x100 << R.z[q];
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) bits |= shfl_xor(bits, m);
    const unsigned mask = __builtin_amdgcn_readfirstlane((unsigned)bits);
    *present = mask;
    int off_r = 0, off_a = 0;
#pragma unroll
    for (int q = 0; q < kQ; ++q) pos_r[q] = pos_a[q] = -1;
    for (int s = 0; s < ns; ++s) {
        if (l == 0) {
            seg_r[s] = off_r;
            seg_a[s] = off_a;
        }
        if (!((mask >> s) & 1u)) continue;   // wave-uniform
#pragma unroll
        for (int q = 0; q < kQ; ++q) {
            if (q < nq) {
                const bool is = R.z[q] == s;
                const unsigned long long mr = ballot(R.in_r[q] && is);
                const unsigned long long ma = ballot(R.in_a[q] && is);
                if (R.in_r[q] && is) pos_r[q] = off_r + rank_below(mr);
                if (R.in_a[q] && is) pos_a[q] = off_a + rank_below(ma);
                off_r += __popcll(mr);
                off_a += __popcll(ma);
            }
        }
    }
    if (l == 0) {
        seg_r[ns] = off_r;
        seg_a[ns] = off_a;
    }
    if (off_a > kMaxA) {
        if (l == 0) set_flag(flags, NNP_FLAG_ROW);
        return false;
    }
    return true;
}

// ---------------------------------------------------------------- forward

constexpr int kMaxBins = kMaxSpecies * (kMaxSpecies + 1) / 2;   // species pairs

// Sum of v over the lanes l, l ^ 8, l ^ 16, l ^ 32, ... (the lanes that share
// l's bits 0-2): a DPP rotation within each 16-lane row for 8, then the
// gfx950 row and half swaps for 16 and 32.  Every lane receives the sum.
__device__ __forceinline__ float sum_over_rows_and_halves(float v, bool with8) {
    if (with8) v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x128, 0xf, 0xf, false));
    const auto h16 = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    v = __uint_as_float(h16[0]) + __uint_as_float(h16[1]);
    const auto h32 = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    return __uint_as_float(h32[0]) + __uint_as_float(h32[1]);
}

// v of lane l ^ x within the lane's quad (x = 1 or 2), by DPP
__device__ __forceinline__ float quad_xor(float v, int x) {
    return x == 1 ? __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xb1, 0xf, 0xf, false))
                  : __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4e, 0xf, 0xf, false));
}

// Sum of v over the 64 lanes (every lane receives it): the quad's lanes by
// DPP, then a row's four quads by two DPP rotations, then the row and half
// swaps.  A fixed order of additions.
__device__ __forceinline__ float wave_sum(float v) {
    v += quad_xor(v, 1);
    v += quad_xor(v, 2);
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x124, 0xf, 0xf, false));   // row_ror:4
    return sum_over_rows_and_halves(v, true);
}

// inclusive prefix sum over the 64 lanes
__device__ __forceinline__ int wave_inclusive_sum(int v) {
    const int l = lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const int u = __shfl_up(v, d, kWave);
        if (l >= d) v += u;
    }
    return v;
}

struct FwdLds {
    float4 au[kMaxA];          // angular list: unit vector, r
    float afc[kMaxA];
    // the radial list is read only before the angular pair tile is first
    // written, so the two share their space
    union {
        float2 rad[kMaxR];     // radial list: (r, fc), species-grouped
        struct {
            alignas(16) float f1[kWave][kNz];   // pair tile: 8 angle factors
            float f2[kWave][kNa];               // 4 radial factors times 2 fc fc
        } tile;
    };
    int seg_r[kMaxSpecies + 1];
    int seg_a[kMaxSpecies + 1];
    // species-pair bins that hold at least one pair, in bin order: the
    // offset of each bin's first pair in the packed pair sequence, and the
    // bin's index and species (p | s << 8 | t << 16)
    int bin_off[kMaxBins + 1];
    int bin_info[kMaxBins];
};

// (s, t), s <= t, of species-pair bin p in row-major triangle order
__device__ __forceinline__ void bin_species(int p, int ns, int& s, int& t) {
    s = 0;
    while (p >= ns - s) {
        p -= ns - s;
        ++s;
    }
    t = s + p;
}

template <typename OutT, bool kPacked>
__global__ __launch_bounds__(kWaves* kWave) void k_aev_fwd(
    const AevConst P, int n, const float* __restrict__ pos, const int32_t* __restrict__ species, const BoxConst bx,
    const RowsView rows, const int32_t* __restrict__ out_row, OutT* __restrict__ out, unsigned* flags,
    int32_t* __restrict__ rev_out, const int32_t* __restrict__ gate, uint32_t* __restrict__ amask) {
    __shared__ FwdLds lds[kWaves];
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);   // wave-uniform: the atom is a scalar
    const int l = lane_id();
    const int i = blockIdx.x * kWaves + w;
    if (i >= n) return;
    FwdLds& S = lds[w];
    // the row's extent and grouped row, loaded ahead of the rebuild gate
    const int rb = rows.begin(i), re = rows.end(i);
    const int row = out_row ? out_row[i] : i;
    // fixed-stride rows just rebuilt: the reverse index, found once per
    // unordered pair by the row of its lower index.  For a pair i -> j with
    // j > i, i's slot q in the row of j is found by bisection (rows are
    // sorted by neighbour) and both rev[p] = q and rev[q] = p are written;
    // the pairs with j < i are written by the row of j.  A lane searches the
    // rows of its pairs p and p + 64 side by side, so that the dependent
    // loads of the two searches are in flight together; a finished search
    // issues no load.  A pair i -> j, j > i, whose reverse is absent is
    // flagged and left pointing at itself.  (The builder's lists are
    // symmetric; only a row emptied for overflowing, which is flagged on its
    // own, leaves a slot of another row unresolved.)
    if (rev_out && (!gate || *gate)) {
        const int b = rb, e = re;
        bool missing = false;
        for (int p0 = b + l; p0 < e; p0 += 2 * kWave) {
            const int p1 = p0 + kWave;
            const bool two = p1 < e;
            const int j0 = rows.col[p0];
            const int j1 = two ? rows.col[p1] : j0;
            const bool s0 = j0 > i, s1 = two && j1 > i;
            const int e0 = rows.end(j0), e1 = two ? rows.end(j1) : e0;
            int lo0 = rows.begin(j0), hi0 = s0 ? e0 : lo0;
            int lo1 = rows.begin(j1), hi1 = s1 ? e1 : lo1;
            while (lo0 < hi0 || lo1 < hi1) {
                const int m0 = (lo0 + hi0) >> 1, m1 = (lo1 + hi1) >> 1;
                int c0 = 0, c1 = 0;
                if (lo0 < hi0) c0 = rows.col[m0];
                if (lo1 < hi1) c1 = rows.col[m1];
                if (lo0 < hi0) {
                    if (c0 < i) lo0 = m0 + 1; else hi0 = m0;
                }
                if (lo1 < hi1) {
                    if (c1 < i) lo1 = m1 + 1; else hi1 = m1;
                }
            }
            if (s0) {
                const bool f0 = lo0 < e0 && rows.col[lo0] == i;
                rev_out[p0] = f0 ? lo0 : p0;
                if (f0) rev_out[lo0] = p0;
                missing |= !f0;
            }
            if (s1) {
                const bool f1 = lo1 < e1 && rows.col[lo1] == i;
                rev_out[p1] = f1 ? lo1 : p1;
                if (f1) rev_out[lo1] = p1;
                missing |= !f1;
            }
        }
        if (missing) set_flag(flags, NNP_FLAG_REVERSE);
    }
    const int ns = P.ns;
    Row R;
    int pr_[kQ], pa_[kQ];
    unsigned present = 0;
    const bool loaded = load_row<kPacked>(R, P, i, rb, re, pos, species, bx, rows, flags);
    if (row < 0) return;   // atom without a grouped row (invalid species, flagged elsewhere)
    OutT* orow = out + (size_t)row * P.stride;
    if (!loaded || !group_species(R, ns, pr_, pa_, S.seg_r, S.seg_a, &present, flags)) {
        for (int c = l; c < P.stride; c += kWave) store_out(orow + c, 0.f);
        if (amask && l == 0) amask[i] = 0xffffu;
        return;
    }
    if (amask && l == 0) amask[i] = present;
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
        if (pr_[q] >= 0) {
            const float r = hw_sqrt(R.r2[q]);
            S.rad[pr_[q]] = make_float2(r, cutoff_fc(r, P.pi_rc_r));
            if (pa_[q] >= 0) {
                const float inv = r > 0.f ? hw_rcp(r) : 0.f;
                S.au[pa_[q]] = make_float4(R.vx[q] * inv, R.vy[q] * inv, R.vz[q] * inv, r);
                S.afc[pa_[q]] = cutoff_fc(r, P.pi_rc_a);
            }
        }
    }
    wave_sync();
    // exp(-eta x^2) as exp2(c x^2)
    const float c_r = -P.eta_r * 1.44269504088896341f, c_a = -P.eta_a * 1.44269504088896341f;
    // ---- radial: lane = (k, q); only the species present in the row
    {
        const int k = l & 15, q = l >> 4;
        const float rk = P.shf_r[k];
        for (unsigned m = present & 0xffu; m; m &= m - 1u) {
            const int s = __builtin_ctz(m);
            const int sb = S.seg_r[s], se = S.seg_r[s + 1];
            float acc = 0.f;
            for (int j = sb + q; j < se; j += 4) {
                const float2 e = S.rad[j];
                const float d = e.x - rk;
                acc += hw_exp2(c_r * d * d) * e.y;
            }
            acc = sum_over_rows_and_halves(acc, false);
            if (q == 0) store_out(orow + 16 * s + k, P.pr * acc);
        }
    }
    // ---- the bins that hold a pair: lane p counts bin p's pairs
    const int nbins = ns * (ns + 1) / 2;
    int bs_ = 0, bt_ = 0, cnt = 0;
    if (l < nbins) {
        bin_species(l, ns, bs_, bt_);
        const int cs_ = S.seg_a[bs_ + 1] - S.seg_a[bs_];
        cnt = bs_ == bt_ ? cs_ * (cs_ - 1) / 2 : cs_ * (S.seg_a[bt_ + 1] - S.seg_a[bt_]);
    }
    // packed order: the same-species bins first, then the mixed ones, so
    // that few tiles hold both kinds (their pair decodes differ)
    const unsigned long long binmask = ballot(cnt > 0);
    const unsigned long long same_m = ballot(cnt > 0 && bs_ == bt_);
    const int n_act = __popcll(binmask);
    if (cnt > 0) {
        const int rank = bs_ == bt_ ? rank_below(same_m) : __popcll(same_m) + rank_below(binmask & ~same_m);
        S.bin_off[rank] = cnt;   // the count for now; its offset below
        S.bin_info[rank] = l | (bs_ << 8) | (bt_ << 16);
    }
    wave_sync();
    const int cnt_r = l < n_act ? S.bin_off[l] : 0;
    const int incl = wave_inclusive_sum(cnt_r);
    const int total = __builtin_amdgcn_readlane(incl, kWave - 1);
    wave_sync();   // the radial list is read; its space becomes the pair tile
    if (l < n_act) S.bin_off[l] = incl - cnt_r;
    if (l == 0) S.bin_off[n_act] = total;
    wave_sync();
    // ---- angular: the pairs of every non-empty bin in one packed sequence,
    // 64 at a time, one per lane, into an LDS tile; then lane (ra, rz, rq)
    // sums f1[z] f2[ra] over the tile's pairs rq, rq + 8, ... of each bin for
    // the four angle sections z = 4 rz .. 4 rz + 3, carrying a bin's partial
    // sums into the next tile, and a butterfly over rq completes the bin
    const int ra = l & 3, rz = (l >> 2) & 1, rq = l >> 3;
    float acc[4] = {0.f, 0.f, 0.f, 0.f};
    int cb = 0;   // first bin not yet complete (wave-uniform)
    for (int u0 = 0; u0 < total; u0 += kWave) {
        const int u = u0 + l;
        if (u < total) {
            int b = cb;
            while (b + 1 < n_act && S.bin_off[b + 1] <= u) ++b;
            const int info = S.bin_info[b];
            const int s = (info >> 8) & 0xff, t = (info >> 16) & 0xff;
            const int v = u - S.bin_off[b];
            const int bs = S.seg_a[s];
            int ja, ka;
            if (s == t) {
                tri_decode(v, S.seg_a[s + 1] - bs, ja, ka);
                ja += bs;
                ka += bs;
            } else {
                // v = j' ct + k': the float quotient, corrected to the exact one
                const int bt = S.seg_a[t], ct = S.seg_a[t + 1] - bt;
                int qd = (int)((float)v * hw_rcp((float)ct));
                qd -= __mul24(qd, ct) > v;
                qd += __mul24(qd + 1, ct) <= v;
                ja = bs + qd;
                ka = bt + (v - __mul24(qd, ct));
            }
            const float4 A = S.au[ja], B = S.au[ka];
            float c = A.x * B.x + A.y * B.y + A.z * B.z;
            c = fminf(1.f, fmaxf(-1.f, c));
            const float uu = P.cs * c;
            const float sq = hw_sqrt(1.f - uu * uu);
            const float rbar = 0.5f * (A.w + B.w);
            const float w2 = 2.f * S.afc[ja] * S.afc[ka];
#pragma unroll
            for (int a = 0; a < kNa; ++a) {
                const float d = rbar - P.shf_a[a];
                S.tile.f2[l][a] = w2 * hw_exp2(c_a * d * d);
            }
#pragma unroll
            for (int z = 0; z < kNz; ++z)
                S.tile.f1[l][z] = pow_zeta(fmaf(uu, P.hcos_z[z], fmaf(sq, P.hsin_z[z], 0.5f)), P.zeta);
        }
        wave_sync();
        const int u1 = min(u0 + kWave, total);
        for (int b = cb; b < n_act; ++b) {
            const int off = __builtin_amdgcn_readfirstlane(S.bin_off[b]);
            if (off >= u1) break;
            const int end = __builtin_amdgcn_readfirstlane(S.bin_off[b + 1]);
            const int lo = max(off, u0) - u0, hi = min(end, u1) - u0;
            for (int m = lo + ((rq - lo) & 7); m < hi; m += 8) {
                const float4 f1v = *(const float4*)&S.tile.f1[m][4 * rz];
                const float f2v = S.tile.f2[m][ra];
                acc[0] += f1v.x * f2v;
                acc[1] += f1v.y * f2v;
                acc[2] += f1v.z * f2v;
                acc[3] += f1v.w * f2v;
            }
            if (end <= u1) {   // the bin is complete
                const int p = __builtin_amdgcn_readfirstlane(S.bin_info[b]) & 0xff;
#pragma unroll
                for (int x = 0; x < 4; ++x) acc[x] = sum_over_rows_and_halves(acc[x], true);
                if (rq == 0) {
                    OutT* o = orow + P.radial_dim + 32 * p + 8 * ra + 4 * rz;
#pragma unroll
                    for (int x = 0; x < 4; ++x) store_out(o + x, acc[x]);
                }
#pragma unroll
                for (int x = 0; x < 4; ++x) acc[x] = 0.f;
                cb = b + 1;
            }
        }
        wave_sync();
    }
    // ---- zeros for the 16-feature blocks not written above (species absent
    // from the row, bins without a pair, padding columns), 16 bytes per lane
    // store
    constexpr int kPer16 = 16 / (int)sizeof(OutT);       // features per 16-byte store
    const int nblk_r = ns, nblk = P.dim / 16;
    for (int c = l; c < P.stride / kPer16; c += kWave) {
        const int blk = (c * kPer16) >> 4;
        bool live;
        if (blk < nblk_r) live = (present >> blk) & 1u;
        else if (blk < nblk) live = (binmask >> ((blk - nblk_r) >> 1)) & 1ull;
        else live = false;
        if (!live) *(uint4*)(orow + c * kPer16) = make_uint4(0u, 0u, 0u, 0u);
    }
}

// ---------------------------------------------------------------- adjoint

constexpr int kPairTile = 3 * kWave;     // angular pairs held at once by the adjoint

struct BwdLds {
    float4 au[kMaxA];           // angular list: unit vector, r
    float afc[kMaxA], adfc[kMaxA];
    int azs[kMaxA];             // species | slot << 8
    union {
        float2 rl[kMaxR];       // first: radial list (r, species bits), then (dE/dr, -)
        float pb[kPairTile][6]; // pair tile: contributions to the two edges
        float ga[kMaxA][3];     // then: angular gradient per angular neighbour
    };
    unsigned char amap[kMaxR];  // slot -> angular index (255: none)
    int seg_r[kMaxSpecies + 1];
    int seg_a[kMaxSpecies + 1];
};

// kVir: also the per-centre virial W_i = -sum_j v_ij (outer) G_ij, row-major
// [n][9] (the strain derivative of E_i is -W_i transposed).
template <bool kVir, bool kPacked>
__global__ __launch_bounds__(kWaves* kWave, kVir ? 4 : 5) void k_aev_bwd(
    const AevConst P, int n, const float* __restrict__ pos, const int32_t* __restrict__ species, const BoxConst bx,
    const RowsView rows, const int32_t* __restrict__ g_row, const float* __restrict__ g, float4* __restrict__ G,
    float4* __restrict__ Gown, float* __restrict__ Wat, unsigned* flags) {
    __shared__ BwdLds lds[kWaves];
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);   // wave-uniform: the atom is a scalar
    const int l = lane_id();
    const int i = blockIdx.x * kWaves + w;
    if (i >= n) return;
    BwdLds& S = lds[w];
    const int ns = P.ns;
    Row R;
    int pr_[kQ], pa_[kQ];
    unsigned present = 0;
    const int row = g_row ? g_row[i] : i;
    const bool ok = load_row<kPacked>(R, P, i, rows.begin(i), rows.end(i), pos, species, bx, rows, flags) &&
                    group_species(R, ns, pr_, pa_, S.seg_r, S.seg_a, &present, flags) && row >= 0;
    if (!ok) {
        const int b = rows.begin(i), e = rows.end(i);
        for (int p = b + l; p < e; p += kWave) G[p] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (l == 0) Gown[i] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (kVir && l < 9) Wat[9 * (size_t)i + l] = 0.f;
        return;
    }
    // dE/dAEV of this atom, read where used (a species' 16 radial or a species
    // pair's 32 angular coefficients: one or two cache lines shared by the
    // lanes that need them)
    const float* __restrict__ grow = g + (size_t)row * P.stride;
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
        const int slot = l + kWave * q;
        if (slot < R.len) S.amap[slot] = 255;
    }
    // angular list entries; the radial list (r and species, species-grouped)
    float r_[kQ];
    const int nq = (R.len + kWave - 1) / kWave;
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
        r_[q] = 0.f;
        if (q >= nq) continue;   // wave-uniform: a group past the row's end
        r_[q] = hw_sqrt(R.r2[q]);
        if (pr_[q] >= 0) S.rl[pr_[q]] = make_float2(r_[q], __int_as_float(R.z[q]));
        if (pa_[q] >= 0) {
            const float r = r_[q];
            const float inv = r > 0.f ? hw_rcp(r) : 0.f;
            S.au[pa_[q]] = make_float4(R.vx[q] * inv, R.vy[q] * inv, R.vz[q] * inv, r);
            S.afc[pa_[q]] = cutoff_fc(r, P.pi_rc_a);
            S.adfc[pa_[q]] = -0.5f * P.pi_rc_a * __sinf(P.pi_rc_a * r);
            S.azs[pa_[q]] = R.z[q] | ((l + kWave * q) << 8);
        }
    }
    wave_sync();
    // ---- radial dE/dr, one radial-list entry per lane (the list holds only
    // the pairs within Rc_R, so the lanes are full up to its length):
    //   dE/dr = p_R sum_k g_k e_k (-2 eta_R (r - R_k) fc + fc')
    //         = p_R (-2 eta_R fc sum_k g_k e_k (r - R_k) + fc' sum_k g_k e_k)
    const float c_r = -P.eta_r * 1.44269504088896341f;   // exp(-eta x^2) = exp2(c_r x^2)
    const int n_r = S.seg_r[ns];
    for (int m = l; m < n_r; m += kWave) {
        const float2 e = S.rl[m];
        const float r = e.x;
        const float4* __restrict__ g4 = (const float4*)(grow + 16 * __float_as_int(e.y));
        float gk[kNr];
#pragma unroll
        for (int v = 0; v < kNr / 4; ++v) {
            const float4 q4 = g4[v];
            gk[4 * v] = q4.x;
            gk[4 * v + 1] = q4.y;
            gk[4 * v + 2] = q4.z;
            gk[4 * v + 3] = q4.w;
        }
        float a1 = 0.f, a2 = 0.f;
#pragma unroll
        for (int k = 0; k < kNr; ++k) {
            const float d = r - P.shf_r[k];
            const float ge = gk[k] * hw_exp2(c_r * d * d);
            a1 = fmaf(ge, d, a1);
            a2 += ge;
        }
        const float fc = cutoff_fc(r, P.pi_rc_r);
        const float dfc = -0.5f * P.pi_rc_r * __sinf(P.pi_rc_r * r);
        S.rl[m].x = P.pr * (-2.f * P.eta_r * fc * a1 + dfc * a2);
    }
    wave_sync();
    // ---- radial gradient of each slot: dE/dr times the unit vector
    float gx[kQ], gy[kQ], gz[kQ];
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
        gx[q] = gy[q] = gz[q] = 0.f;
        if (pr_[q] >= 0) {
            const float r = r_[q];
            const float dEdr = S.rl[pr_[q]].x;
            const float inv = r > 0.f ? hw_rcp(r) : 0.f;
            gx[q] = dEdr * R.vx[q] * inv;
            gy[q] = dEdr * R.vy[q] * inv;
            gz[q] = dEdr * R.vz[q] * inv;
        }
    }
    wave_sync();   // the radial list is read; its space becomes the pair tile
    // ---- angular: unordered pairs (j < k) of the species-grouped list in
    // triangle order, one per lane, into a tile of up to kPairTile pairs; then
    // every angular neighbour m sums its contributions from the tile in a
    // fixed order: pairs (j, m) by ascending j, then pairs (m, k) by ascending k
    const int n_a = S.seg_a[ns];
    const int total = n_a * (n_a - 1) / 2;
    const float c_a = -P.eta_a * 1.44269504088896341f, m2eta_a = -2.f * P.eta_a;
    const float zm1 = P.zeta - 1.f, l2hz = __log2f(0.5f * P.zeta);   // dF1/dw = 2^((zeta-1) log2 w + log2(zeta/2))
    float ax_[2] = {0.f, 0.f}, ay_[2] = {0.f, 0.f}, az_[2] = {0.f, 0.f};
    // lanes per angular neighbour in the per-neighbour sums: 4 up to 16
    // neighbours, 2 up to 32, else 1 (wave-uniform)
    const int lp = n_a <= 16 ? 2 : (n_a <= 32 ? 1 : 0);
    for (int c0 = 0; c0 < total; c0 += kPairTile) {
        const int c1 = min(c0 + kPairTile, total);
        for (int u0 = c0; u0 < c1; u0 += kWave) {
            const int u = u0 + l;
            if (u < c1) {
                int ja, ka;
                tri_decode(u, n_a, ja, ka);
                const float4 A = S.au[ja], B = S.au[ka];
                float c = A.x * B.x + A.y * B.y + A.z * B.z;
                c = fminf(1.f, fmaxf(-1.f, c));
                const float uu = P.cs * c;
                const float sq = hw_sqrt(1.f - uu * uu);
                const float rj = A.w, rk = B.w;
                const float rbar = 0.5f * (rj + rk);
                const float fj = S.afc[ja], fk = S.afc[ka];
                const float dfj = S.adfc[ja], dfk = S.adfc[ka];
                const int pp = species_pair(S.azs[ja] & 0xff, S.azs[ka] & 0xff, ns);
                // this bin's 32 coefficients, [a][z] (radial_dim is a multiple of 16)
            const float4* gp4 = (const float4*)(grow + P.radial_dim + 32 * pp);
            float gp[kNa * kNz];
#pragma unroll
            for (int v = 0; v < kNa * kNz / 4; ++v) {
                const float4 q4 = gp4[v];
                gp[4 * v] = q4.x;
                gp[4 * v + 1] = q4.y;
                gp[4 * v + 2] = q4.z;
                gp[4 * v + 3] = q4.w;
            }
                float F2[kNa], dF2[kNa];
#pragma unroll
                for (int a = 0; a < kNa; ++a) {
                    const float d = rbar - P.shf_a[a];
                    F2[a] = hw_exp2(c_a * d * d);
                    dF2[a] = m2eta_a * d * F2[a];
                }
                float Rz[kNa] = {0.f, 0.f, 0.f, 0.f};
                float sum_c = 0.f, Ssum = 0.f;
                const float us = uu * hw_rcp(sq);                 // u / sqrt(1 - u^2)
#pragma unroll
                for (int z = 0; z < kNz; ++z) {
                    // base^zeta and its derivative (zeta/2) base^(zeta-1), the factor
                    // folded into the exponent; base = 0 gives log2 = -inf and both 0
                    const float base = fmaxf(fmaf(uu, P.hcos_z[z], fmaf(sq, P.hsin_z[z], 0.5f)), 0.f);
                    const float lg = hw_log2(base);
                    const float F1 = hw_exp2(P.zeta * lg);
                    const float dF1 = hw_exp2(fmaf(zm1, lg, l2hz));
                    const float dwdu = P.cos_z[z] - us * P.sin_z[z];
                    float Q = 0.f;
#pragma unroll
                    for (int a = 0; a < kNa; ++a) {
                        const float gaz = gp[8 * a + z];
                        Q += gaz * F2[a];
                        Rz[a] += gaz * F1;
                    }
                    sum_c += Q * dF1 * dwdu;
                    Ssum += Q * F1;
                }
                float sum_r = 0.f;
#pragma unroll
                for (int a = 0; a < kNa; ++a) sum_r += Rz[a] * dF2[a];
                const float ff = 2.f * fj * fk;
                const float dEdc = ff * sum_c * P.cs;
                const float dEdrbar = ff * sum_r;
                const float sj = 0.5f * dEdrbar + 2.f * fk * Ssum * dfj;
                const float sk = 0.5f * dEdrbar + 2.f * fj * Ssum * dfk;
                const float ij = rj > 0.f ? hw_rcp(rj) : 0.f;
                const float ik = rk > 0.f ? hw_rcp(rk) : 0.f;
                // tile slot u - c0 < kPairTile: its offset by a 24-bit multiply
                float* pb = &S.pb[0][0] + __mul24(u - c0, 6);
                pb[0] = dEdc * (B.x - c * A.x) * ij + sj * A.x;
                pb[1] = dEdc * (B.y - c * A.y) * ij + sj * A.y;
                pb[2] = dEdc * (B.z - c * A.z) * ij + sj * A.z;
                pb[3] = dEdc * (A.x - c * B.x) * ik + sk * B.x;
                pb[4] = dEdc * (A.y - c * B.y) * ik + sk * B.y;
                pb[5] = dEdc * (A.z - c * B.z) * ik + sk * B.z;
            }
        }
        wave_sync();
        // lanes (m, part): the 2^lp lanes of neighbour m take every 2^lp-th
        // j, and their partial sums are combined after the last tile
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            if (q * kWave >= (n_a << lp)) break;   // wave-uniform
            const int m = (l >> lp) + q * kWave;
            const int Tm = __mul24(m, 2 * n_a - m - 1) >> 1;   // first pair (m, m + 1)
            for (int j = l & ((1 << lp) - 1); j + 1 < n_a; j += 1 << lp) {
                const bool before = j < m;              // pair (j, m), else pair (m, j + 1)
                const int Tj = __mul24(j, 2 * n_a - j - 1) >> 1;   // first pair (j, j + 1)
                const int t = before ? Tj + (m - j - 1) : Tm + (j - m);
                if (m < n_a && t >= c0 && t < c1) {
                    const float* e = &S.pb[0][0] + __mul24(t - c0, 6) + (before ? 3 : 0);
                    ax_[q] += e[0];
                    ay_[q] += e[1];
                    az_[q] += e[2];
                }
            }
        }
        wave_sync();
    }
    // the 2^lp partial sums of each neighbour (lanes adjacent in a quad)
    if (lp >= 1) {
        ax_[0] += quad_xor(ax_[0], 1);
        ay_[0] += quad_xor(ay_[0], 1);
        az_[0] += quad_xor(az_[0], 1);
    }
    if (lp >= 2) {
        ax_[0] += quad_xor(ax_[0], 2);
        ay_[0] += quad_xor(ay_[0], 2);
        az_[0] += quad_xor(az_[0], 2);
    }
    // the tile is dead: its space now holds the per-neighbour sums
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int m = (l >> lp) + q * kWave;
        if (m < n_a && (l & ((1 << lp) - 1)) == 0) {
            S.ga[m][0] = ax_[q];
            S.ga[m][1] = ay_[q];
            S.ga[m][2] = az_[q];
            S.amap[S.azs[m] >> 8] = (unsigned char)m;
        }
    }
    wave_sync();
    // ---- one value per row slot: radial part + angular part (zero outside Rc_R)
    // and the row's own sum, slots in order on each lane, then over the lanes
    float wv[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) wv[k] = 0.f;
    float ox = 0.f, oy = 0.f, oz = 0.f;
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
        const int slot = l + kWave * q;
        if (slot < R.len) {
            const int am = S.amap[slot];
            float x = gx[q], y = gy[q], z = gz[q];
            if (am != 255) {
                x += S.ga[am][0];
                y += S.ga[am][1];
                z += S.ga[am][2];
            }
            const int p = R.b + slot;
            G[p] = make_float4(x, y, z, 0.f);
            ox += x;
            oy += y;
            oz += z;
            if (kVir) {
                const float v[3] = {R.vx[q], R.vy[q], R.vz[q]}, G[3] = {x, y, z};
#pragma unroll
                for (int a = 0; a < 3; ++a)
#pragma unroll
                    for (int c = 0; c < 3; ++c) wv[3 * a + c] -= v[a] * G[c];
            }
        }
    }
    ox = wave_sum(ox);
    oy = wave_sum(oy);
    oz = wave_sum(oz);
    if (l == 0) Gown[i] = make_float4(ox, oy, oz, 0.f);
    if (kVir) {
#pragma unroll
        for (int k = 0; k < 9; ++k)
#pragma unroll
            for (int m = 32; m >= 1; m >>= 1) wv[k] += shfl_xor(wv[k], m);
        if (l < 9) {
            float o = 0.f;
#pragma unroll
            for (int k = 0; k < 9; ++k) o = l == k ? wv[k] : o;
            Wat[9 * (size_t)i + l] = o;
        }
    }
}

}  // namespace

hipError_t launch_aev_fwd(const AevConst& P, int n, const float* pos, const int32_t* species, const BoxConst& bx,
                          const RowsView& rows, const int32_t* out_row, void* out, bool bf16, unsigned* flags,
                          hipStream_t s, int32_t* rev_out, const int32_t* gate, uint32_t* amask_out) {
    if (n <= 0) return hipSuccess;
    const int grid = ceil_div(n, kWaves);
    const bool packed = rows.row_ptr == nullptr;
#define NNP_AEV_FWD(T, PK) \
    k_aev_fwd<T, PK><<<grid, kWaves * kWave, 0, s>>>(P, n, pos, species, bx, rows, out_row, (T*)out, flags, rev_out, \
                                                     gate, amask_out)
    if (bf16) {
        if (packed) NNP_AEV_FWD(uint16_t, true);
        else NNP_AEV_FWD(uint16_t, false);
    } else {
        if (packed) NNP_AEV_FWD(float, true);
        else NNP_AEV_FWD(float, false);
    }
#undef NNP_AEV_FWD
    return hipGetLastError();
}

hipError_t launch_aev_bwd(const AevConst& P, int n, const float* pos, const int32_t* species, const BoxConst& bx,
                          const RowsView& rows, const int32_t* g_row, const float* g, float4* G, float4* Gown,
                          float* atom_virial, unsigned* flags, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int grid = ceil_div(n, kWaves);
    const bool packed = rows.row_ptr == nullptr;
#define NNP_AEV_BWD(V, PK) \
    k_aev_bwd<V, PK><<<grid, kWaves * kWave, 0, s>>>(P, n, pos, species, bx, rows, g_row, g, G, Gown, atom_virial, flags)
    if (atom_virial) {
        if (packed) NNP_AEV_BWD(true, true);
        else NNP_AEV_BWD(true, false);
    } else {
        if (packed) NNP_AEV_BWD(false, true);
        else NNP_AEV_BWD(false, false);
    }
#undef NNP_AEV_BWD
    return hipGetLastError();
}

}  // namespace nnp
