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
// Layout of the work: a wave owns one centre atom.  It streams the atom's
// neighbour row (CSR, sorted by j) across its 64 lanes, computes edge
// vectors in float32, and stores the neighbours within each cutoff in LDS
// grouped by species (stable in j).  Radial sums use lanes as (shell k,
// quarter q); angular sums evaluate one neighbour pair per lane (8 angle
// factors + 4 radial factors, 32 products) into an LDS pair tile and reduce
// it per species-pair segment with lanes as (a, z) columns.  Every sum is
// taken in a fixed order, so results do not depend on scheduling.
//
// The adjoint recomputes the same neighbourhood, reads dE/dAEV of the atom
// into LDS and produces G_ij = dE_i / dv_ij for every slot of the row: the
// radial part per neighbour lane, the angular part per pair lane, gathered
// per neighbour in a fixed order (no atomics).
#include "nnp_internal.hpp"

namespace nnp {
namespace {

constexpr int kMaxR = NNP_MAX_ROW;        // neighbours within the list cutoff per atom
constexpr int kMaxA = NNP_MAX_ANGULAR;    // neighbours within the angular cutoff
constexpr int kWavesFwd = 2;
constexpr int kWavesBwd = 2;
constexpr int kPairStride = 33;           // 32 products + 1 pad (conflict-free)

struct Hood {
    // radial list (r < Rc_R), species-sorted
    float rr[kMaxR];
    float rfc[kMaxR];
    int rzs[kMaxR];        // species | (row slot offset << 8)
    // angular list (r < Rc_A), species-sorted, subset of the radial list
    float ax[kMaxA], ay[kMaxA], az[kMaxA];   // unit vectors
    float ar[kMaxA];
    float afc[kMaxA];
    int azs[kMaxA];        // species | (radial list index << 8)
    int sel[kMaxR];        // per row slot: species | in_r << 8 | in_a << 9 (decided once)
    int seg_r[kMaxSpecies + 1];
    int seg_a[kMaxSpecies + 1];
    int n_r, n_a, ok;
};

__device__ __forceinline__ float cutoff_fc(float r, float pi_rc) {
    return 0.5f * __cosf(pi_rc * r) + 0.5f;
}

// Stable species-grouped lists of the neighbours of atom i within the two
// cutoffs.  Returns false (and flags) if the row is longer than supported.
template <bool kBwd>
__device__ bool build_hood(Hood& H, const AevConst& P, int i, const float* pos, const int32_t* species,
                           const BoxConst bx, const int32_t* row_ptr, const int32_t* col, const int8_t* shift,
                           float* rux, float* ruy, float* ruz, float* rdfc, float* adfc, unsigned* flags) {
    const int l = lane_id();
    const int b = row_ptr[i], e = row_ptr[i + 1];
    const float xi = pos[3 * i], yi = pos[3 * i + 1], zi = pos[3 * i + 2];
    const float rc_r2 = P.rc_r * P.rc_r;
    const float rc_a2 = P.rc_a * P.rc_a;
    const bool periodic = bx.periodic != 0;
    const float Lx = bx.L[0], Ly = bx.L[1], Lz = bx.L[2];
    int cnt_r[kMaxSpecies], cnt_a[kMaxSpecies];
#pragma unroll
    for (int s = 0; s < kMaxSpecies; ++s) cnt_r[s] = cnt_a[s] = 0;
    if (e - b > kMaxR) {
        if (l == 0) set_flag(flags, NNP_FLAG_ROW);
        return false;
    }
    // pass 1: decide membership once per slot, count per species
    for (int t0 = b; t0 < e; t0 += kWave) {
        const int p = t0 + l;
        bool in_r = false, in_a = false;
        int z = 0;
        if (p < e) {
            const int j = col[p];
            z = species[j];
            float vx = pos[3 * j] - xi, vy = pos[3 * j + 1] - yi, vz = pos[3 * j + 2] - zi;
            if (periodic) {
                vx += (float)shift[3 * p] * Lx;
                vy += (float)shift[3 * p + 1] * Ly;
                vz += (float)shift[3 * p + 2] * Lz;
            }
            const float r2 = vx * vx + vy * vy + vz * vz;
            if (z < 0 || z >= P.ns) {
                set_flag(flags, NNP_FLAG_SPECIES);
                z = 0;
            } else {
                in_r = r2 < rc_r2;
                in_a = in_r && r2 < rc_a2;
            }
            H.sel[p - b] = z | (in_r ? 0x100 : 0) | (in_a ? 0x200 : 0);
        }
#pragma unroll
        for (int s = 0; s < kMaxSpecies; ++s) {
            cnt_r[s] += __popcll(ballot(in_r && z == s));
            cnt_a[s] += __popcll(ballot(in_a && z == s));
        }
    }
    wave_sync();
    int off_r[kMaxSpecies], off_a[kMaxSpecies];
    int accr = 0, acca = 0;
#pragma unroll
    for (int s = 0; s < kMaxSpecies; ++s) {
        off_r[s] = accr;
        off_a[s] = acca;
        accr += cnt_r[s];
        acca += cnt_a[s];
    }
    if (acca > kMaxA) {
        if (l == 0) set_flag(flags, NNP_FLAG_ROW);
        return false;
    }
    if (l <= kMaxSpecies) {
        int vr = accr, va = acca;
#pragma unroll
        for (int s = 0; s < kMaxSpecies; ++s)
            if (l == s) { vr = off_r[s]; va = off_a[s]; }
        H.seg_r[l] = vr;
        H.seg_a[l] = va;
    }
    if (l == 0) {
        H.n_r = accr;
        H.n_a = acca;
    }
    // pass 2: scatter into species-sorted positions (stable in j)
    for (int t0 = b; t0 < e; t0 += kWave) {
        const int p = t0 + l;
        bool in_r = false, in_a = false;
        int z = 0;
        float vx = 0.f, vy = 0.f, vz = 0.f, r = 0.f;
        if (p < e) {
            const int sl = H.sel[p - b];
            z = sl & 0xff;
            in_r = (sl & 0x100) != 0;
            in_a = (sl & 0x200) != 0;
            const int j = col[p];
            vx = pos[3 * j] - xi;
            vy = pos[3 * j + 1] - yi;
            vz = pos[3 * j + 2] - zi;
            if (periodic) {
                vx += (float)shift[3 * p] * Lx;
                vy += (float)shift[3 * p + 1] * Ly;
                vz += (float)shift[3 * p + 2] * Lz;
            }
            r = sqrtf(vx * vx + vy * vy + vz * vz);
        }
        int my_r = 0, my_a = 0;
#pragma unroll
        for (int s = 0; s < kMaxSpecies; ++s) {
            const unsigned long long mr = ballot(in_r && z == s);
            const unsigned long long ma = ballot(in_a && z == s);
            if (z == s) {
                my_r = off_r[s] + rank_below(mr);
                my_a = off_a[s] + rank_below(ma);
            }
            off_r[s] += __popcll(mr);
            off_a[s] += __popcll(ma);
        }
        const float inv_r = r > 0.f ? 1.0f / r : 0.f;
        if (in_r && my_r < kMaxR) {
            H.rr[my_r] = r;
            H.rfc[my_r] = cutoff_fc(r, P.pi_rc_r);
            H.rzs[my_r] = z | ((p - b) << 8);
            if (kBwd) {
                rux[my_r] = vx * inv_r;
                ruy[my_r] = vy * inv_r;
                ruz[my_r] = vz * inv_r;
                rdfc[my_r] = -0.5f * P.pi_rc_r * __sinf(P.pi_rc_r * r);
            }
        }
        if (in_a && my_a < kMaxA) {
            H.ax[my_a] = vx * inv_r;
            H.ay[my_a] = vy * inv_r;
            H.az[my_a] = vz * inv_r;
            H.ar[my_a] = r;
            H.afc[my_a] = cutoff_fc(r, P.pi_rc_a);
            H.azs[my_a] = z | (my_r << 8);
            if (kBwd) adfc[my_a] = -0.5f * P.pi_rc_a * __sinf(P.pi_rc_a * r);
        }
    }
    wave_sync();
    return true;
}

__device__ __forceinline__ int species_pair(int s, int t, int ns) {
    if (s > t) { int u = s; s = t; t = u; }
    return s * ns - (s * (s - 1)) / 2 + (t - s);
}

// (j, k) of the v-th unordered pair (j < k) of c items in row-major triangle order
__device__ __forceinline__ void tri_decode(int v, int c, int& j, int& k) {
    const float tc = (float)(2 * c - 1);
    int jj = (int)((tc - sqrtf(fmaxf(tc * tc - 8.0f * (float)v, 0.f))) * 0.5f);
    if (jj < 0) jj = 0;
    if (jj > c - 2) jj = c - 2;
    while (jj > 0 && (jj * (2 * c - jj - 1)) / 2 > v) --jj;
    while (jj + 1 <= c - 2 && ((jj + 1) * (2 * c - jj - 2)) / 2 <= v) ++jj;
    j = jj;
    k = jj + 1 + (v - (jj * (2 * c - jj - 1)) / 2);
}

__device__ __forceinline__ float pow_zeta(float base, float zeta) {
    return base > 0.f ? exp2f(zeta * __log2f(base)) : 0.f;
}

template <typename OutT>
__device__ __forceinline__ void store_out(OutT* p, float v);
template <>
__device__ __forceinline__ void store_out<float>(float* p, float v) { *p = v; }
template <>
__device__ __forceinline__ void store_out<uint16_t>(uint16_t* p, float v) { *p = f32_to_bf16(v); }

// ---------------------------------------------------------------- forward

template <typename OutT>
__global__ __launch_bounds__(kWavesFwd* kWave) void k_aev_fwd(
    const AevConst P, int n, const float* __restrict__ pos, const int32_t* __restrict__ species,
    const BoxConst bx, const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
    const int8_t* __restrict__ shift, const int32_t* __restrict__ out_row, OutT* __restrict__ out,
    unsigned* flags) {
    __shared__ Hood hood[kWavesFwd];
    __shared__ float pairs[kWavesFwd][kWave * kPairStride];
    __shared__ int pstart[kWavesFwd][40];    // pair-segment prefix over species pairs
    const int w = threadIdx.x / kWave;
    const int l = lane_id();
    const int i = blockIdx.x * kWavesFwd + w;
    if (i >= n) return;
    Hood& H = hood[w];
    const int row = out_row ? out_row[i] : i;
    if (row < 0) return;   // atom without a grouped row (invalid species, flagged elsewhere)
    OutT* orow = out + (size_t)row * P.stride;
    if (!build_hood<false>(H, P, i, pos, species, bx, row_ptr, col, shift, nullptr, nullptr, nullptr, nullptr,
                           nullptr, flags)) {
        for (int c = l; c < P.stride; c += kWave) store_out(orow + c, 0.f);
        return;
    }
    const int ns = P.ns;
    // ---- radial: lane = (k, q); species segments in order
    {
        const int k = l & 15, q = l >> 4;
        const float rk = P.shf_r[k];
        for (int s = 0; s < ns; ++s) {
            const int sb = H.seg_r[s], se = H.seg_r[s + 1];
            float acc = 0.f;
            for (int m = sb + q; m < se; m += 4) {
                const float d = H.rr[m] - rk;
                acc += __expf(-P.eta_r * d * d) * H.rfc[m];
            }
            acc += shfl_xor(acc, 16);
            acc += shfl_xor(acc, 32);
            if (q == 0) store_out(orow + 16 * s + k, P.pr * acc);
        }
    }
    // ---- angular
    const int n_sp = ns * (ns + 1) / 2;
    if (l == 0) {
        int acc = 0, p = 0;
        for (int s = 0; s < ns; ++s) {
            const int cs = H.seg_a[s + 1] - H.seg_a[s];
            for (int t = s; t < ns; ++t, ++p) {
                const int ct = H.seg_a[t + 1] - H.seg_a[t];
                pstart[w][p] = acc;
                acc += (s == t) ? cs * (cs - 1) / 2 : cs * ct;
            }
        }
        pstart[w][n_sp] = acc;
    }
    wave_sync();
    const int total = pstart[w][n_sp];
    float* T = pairs[w];
    const int col_az = l & 31, half = l >> 5;
    float acc = 0.f;
    int p_cur = 0;
    for (int u0 = 0;; u0 += kWave) {
        const int nvalid = min(kWave, total - u0);
        // phase 1: one pair per lane
        if (l < nvalid) {
            const int u = u0 + l;
            int lo = 0, hi = n_sp;   // last segment p with pstart[p] <= u
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (pstart[w][mid] <= u) lo = mid; else hi = mid;
            }
            const int p = lo;
            // species pair (s, t) of segment p
            int s = 0, rem = p;
            while (rem >= ns - s) { rem -= ns - s; ++s; }
            const int t = s + rem;
            const int v = u - pstart[w][p];
            int ja, ka;
            if (s == t) {
                const int c = H.seg_a[s + 1] - H.seg_a[s];
                tri_decode(v, c, ja, ka);
                ja += H.seg_a[s];
                ka += H.seg_a[s];
            } else {
                const int ct = H.seg_a[t + 1] - H.seg_a[t];
                ja = H.seg_a[s] + v / ct;
                ka = H.seg_a[t] + v % ct;
            }
            float c = H.ax[ja] * H.ax[ka] + H.ay[ja] * H.ay[ka] + H.az[ja] * H.az[ka];
            c = fminf(1.f, fmaxf(-1.f, c));
            const float uu = P.cs * c;
            const float sq = sqrtf(1.f - uu * uu);
            const float rbar = 0.5f * (H.ar[ja] + H.ar[ka]);
            const float w2 = 2.f * H.afc[ja] * H.afc[ka];
            float f2[kNa];
#pragma unroll
            for (int a = 0; a < kNa; ++a) {
                const float d = rbar - P.shf_a[a];
                f2[a] = w2 * __expf(-P.eta_a * d * d);
            }
#pragma unroll
            for (int z = 0; z < kNz; ++z) {
                const float base = 0.5f + 0.5f * (uu * P.cos_z[z] + sq * P.sin_z[z]);
                const float f1 = pow_zeta(base, P.zeta);
#pragma unroll
                for (int a = 0; a < kNa; ++a) T[l * kPairStride + 8 * a + z] = f1 * f2[a];
            }
        }
        wave_sync();
        // phase 2: lanes = (a z) columns x 2 halves; walk the segments of this chunk
        const int u1 = u0 + nvalid;
        const bool last = u0 + kWave >= total;
        while (p_cur < n_sp) {
            const int sb = pstart[w][p_cur], se = pstart[w][p_cur + 1];
            const int a0 = max(sb, u0) - u0, a1 = min(se, u1) - u0;
            if (a1 > a0) {
                const int mid = (a0 + a1 + 1) >> 1;
                const int lo = half ? mid : a0, hi = half ? a1 : mid;
                for (int m = lo; m < hi; ++m) acc += T[m * kPairStride + col_az];
            }
            if (se <= u1 || last) {
                const float tot = acc + shfl_xor(acc, 32);
                if (half == 0) store_out(orow + P.radial_dim + 32 * p_cur + col_az, tot);
                acc = 0.f;
                ++p_cur;
            } else {
                break;   // segment continues in the next chunk
            }
        }
        wave_sync();
        if (last) break;
    }
    for (int c = P.dim + l; c < P.stride; c += kWave) store_out(orow + c, 0.f);
}

// ---------------------------------------------------------------- adjoint

struct HoodB {
    Hood H;
    float rux[kMaxR], ruy[kMaxR], ruz[kMaxR], rdfc[kMaxR];
    float adfc[kMaxA];
    short loc[kMaxR];        // row slot -> radial list index (-1: none)
};

__global__ __launch_bounds__(kWavesBwd* kWave) void k_aev_bwd(
    const AevConst P, int n, const float* __restrict__ pos, const int32_t* __restrict__ species,
    const BoxConst bx, const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
    const int8_t* __restrict__ shift, const int32_t* __restrict__ g_row, const float* __restrict__ g,
    float* __restrict__ Gx, float* __restrict__ Gy, float* __restrict__ Gz, unsigned* flags) {
    __shared__ HoodB hb[kWavesBwd];
    __shared__ float gl[kWavesBwd][1280];
    __shared__ float pb[kWavesBwd][kWave * 7];
    const int w = threadIdx.x / kWave;
    const int l = lane_id();
    const int i = blockIdx.x * kWavesBwd + w;
    if (i >= n) return;
    HoodB& B = hb[w];
    Hood& H = B.H;
    const int b = row_ptr[i], e = row_ptr[i + 1];
    const bool ok = build_hood<true>(H, P, i, pos, species, bx, row_ptr, col, shift, B.rux, B.ruy, B.ruz,
                                     B.rdfc, B.adfc, flags);
    if (!ok) {
        for (int p = b + l; p < e; p += kWave) Gx[p] = Gy[p] = Gz[p] = 0.f;
        return;
    }
    const int row = g_row ? g_row[i] : i;
    if (row < 0) {
        for (int p = b + l; p < e; p += kWave) Gx[p] = Gy[p] = Gz[p] = 0.f;
        return;
    }
    const float* grow = g + (size_t)row * P.stride;
    for (int c = l; c < P.dim; c += kWave) gl[w][c] = grow[c];
    for (int c = l; c < e - b; c += kWave) B.loc[c] = -1;
    wave_sync();
    for (int m = l; m < H.n_r; m += kWave) B.loc[H.rzs[m] >> 8] = (short)m;
    wave_sync();
    const int n_r = H.n_r, n_a = H.n_a;
    // ---- radial part, one neighbour per lane (up to 4 per lane)
    float gx[4], gy[4], gz[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) gx[q] = gy[q] = gz[q] = 0.f;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int m = l + q * kWave;
        if (m < n_r) {
            const float r = H.rr[m], fc = H.rfc[m], dfc = B.rdfc[m];
            const int s = H.rzs[m] & 0xff;
            const float* gs = &gl[w][16 * s];
            float dEdr = 0.f;
#pragma unroll
            for (int k = 0; k < kNr; ++k) {
                const float d = r - P.shf_r[k];
                const float ek = __expf(-P.eta_r * d * d);
                dEdr += gs[k] * ek * (-2.f * P.eta_r * d * fc + dfc);
            }
            dEdr *= P.pr;
            gx[q] = dEdr * B.rux[m];
            gy[q] = dEdr * B.ruy[m];
            gz[q] = dEdr * B.ruz[m];
        }
    }
    // ---- angular part: unordered pairs in triangle order over the angular list
    const int ns = P.ns;
    const int total = n_a * (n_a - 1) / 2;
    // per angular neighbour owned by this lane (lane m and m + 64 -> up to 2)
    float ax_[2] = {0.f, 0.f}, ay_[2] = {0.f, 0.f}, az_[2] = {0.f, 0.f};
    int jptr[2] = {0, 0};
    float* PB = pb[w];
    for (int u0 = 0; u0 < total; u0 += kWave) {
        const int u = u0 + l;
        if (u < total) {
            int ja, ka;
            tri_decode(u, n_a, ja, ka);
            const float uxj = H.ax[ja], uyj = H.ay[ja], uzj = H.az[ja];
            const float uxk = H.ax[ka], uyk = H.ay[ka], uzk = H.az[ka];
            float c = uxj * uxk + uyj * uyk + uzj * uzk;
            c = fminf(1.f, fmaxf(-1.f, c));
            const float uu = P.cs * c;
            const float sq = sqrtf(1.f - uu * uu);
            const float rj = H.ar[ja], rk = H.ar[ka];
            const float rbar = 0.5f * (rj + rk);
            const float fj = H.afc[ja], fk = H.afc[ka];
            const float dfj = B.adfc[ja], dfk = B.adfc[ka];
            const int p = species_pair(H.azs[ja] & 0xff, H.azs[ka] & 0xff, ns);
            const float* gp = &gl[w][P.radial_dim + 32 * p];
            float F2[kNa], dF2[kNa];
#pragma unroll
            for (int a = 0; a < kNa; ++a) {
                const float d = rbar - P.shf_a[a];
                F2[a] = __expf(-P.eta_a * d * d);
                dF2[a] = -2.f * P.eta_a * d * F2[a];
            }
            float Rz[kNa] = {0.f, 0.f, 0.f, 0.f};   // sum_z g_az F1_z
            float sum_c = 0.f, S = 0.f;
            const float inv_sq = 1.f / sq;
#pragma unroll
            for (int z = 0; z < kNz; ++z) {
                const float base = 0.5f + 0.5f * (uu * P.cos_z[z] + sq * P.sin_z[z]);
                float F1 = 0.f, dF1 = 0.f;
                if (base > 0.f) {
                    const float lg = __log2f(base);
                    F1 = exp2f(P.zeta * lg);
                    dF1 = 0.5f * P.zeta * exp2f((P.zeta - 1.f) * lg);
                }
                const float dwdu = P.cos_z[z] - uu * P.sin_z[z] * inv_sq;
                float Q = 0.f;
#pragma unroll
                for (int a = 0; a < kNa; ++a) {
                    const float gaz = gp[8 * a + z];
                    Q += gaz * F2[a];
                    Rz[a] += gaz * F1;
                }
                sum_c += Q * dF1 * dwdu;
                S += Q * F1;
            }
            float sum_r = 0.f;
#pragma unroll
            for (int a = 0; a < kNa; ++a) sum_r += Rz[a] * dF2[a];
            const float ff = 2.f * fj * fk;
            const float dEdc = ff * sum_c * P.cs;
            const float dEdrbar = ff * sum_r;
            const float sj = 0.5f * dEdrbar + 2.f * fk * S * dfj;
            const float sk = 0.5f * dEdrbar + 2.f * fj * S * dfk;
            const float ij = rj > 0.f ? 1.f / rj : 0.f;
            const float ik = rk > 0.f ? 1.f / rk : 0.f;
            PB[l * 7 + 0] = dEdc * (uxk - c * uxj) * ij + sj * uxj;
            PB[l * 7 + 1] = dEdc * (uyk - c * uyj) * ij + sj * uyj;
            PB[l * 7 + 2] = dEdc * (uzk - c * uzj) * ij + sj * uzj;
            PB[l * 7 + 3] = dEdc * (uxj - c * uxk) * ik + sk * uxk;
            PB[l * 7 + 4] = dEdc * (uyj - c * uyk) * ik + sk * uyk;
            PB[l * 7 + 5] = dEdc * (uzj - c * uzk) * ik + sk * uzk;
        }
        wave_sync();
        // gather per angular neighbour, fixed order: first-element pairs, then second-element pairs
        const int u1 = min(u0 + kWave, total);
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int m = l + q * kWave;
            if (m < n_a) {
                // pairs (m, k>m): contiguous [tri(m), tri(m+1))
                const int t0 = m * (2 * n_a - m - 1) / 2, t1 = t0 + (n_a - m - 1);
                for (int t = max(t0, u0); t < min(t1, u1); ++t) {
                    ax_[q] += PB[(t - u0) * 7 + 0];
                    ay_[q] += PB[(t - u0) * 7 + 1];
                    az_[q] += PB[(t - u0) * 7 + 2];
                }
                // pairs (j<m, m): u_j = tri(j) + m - j - 1, increasing in j
                while (jptr[q] < m) {
                    const int jj = jptr[q];
                    const int t = jj * (2 * n_a - jj - 1) / 2 + (m - jj - 1);
                    if (t >= u1) break;
                    ax_[q] += PB[(t - u0) * 7 + 3];
                    ay_[q] += PB[(t - u0) * 7 + 4];
                    az_[q] += PB[(t - u0) * 7 + 5];
                    ++jptr[q];
                }
            }
        }
        wave_sync();
    }
    // ---- combine radial and angular parts and write one value per row slot
    // angular neighbours add to their radial entries: stage through LDS (reuse pair buffer)
    float* GA = pb[w];   // [kMaxA][3] fits in kWave*7 floats (448 >= 3*96 = 288)
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int m = l + q * kWave;
        if (m < n_a) {
            GA[3 * m] = ax_[q];
            GA[3 * m + 1] = ay_[q];
            GA[3 * m + 2] = az_[q];
        }
    }
    wave_sync();
    // radial entry -> angular entry map is implicit: angular entries store their radial index
    __shared__ short amap[kWavesBwd][kMaxR];
    for (int m = l; m < n_r; m += kWave) amap[w][m] = -1;
    wave_sync();
    for (int m = l; m < n_a; m += kWave) amap[w][H.azs[m] >> 8] = (short)m;
    wave_sync();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int m = l + q * kWave;
        if (m < n_r) {
            const int am = amap[w][m];
            if (am >= 0) {
                gx[q] += GA[3 * am];
                gy[q] += GA[3 * am + 1];
                gz[q] += GA[3 * am + 2];
            }
            const int slot = b + (H.rzs[m] >> 8);
            Gx[slot] = gx[q];
            Gy[slot] = gy[q];
            Gz[slot] = gz[q];
        }
    }
    for (int p = b + l; p < e; p += kWave)
        if (B.loc[p - b] < 0) Gx[p] = Gy[p] = Gz[p] = 0.f;
}

}  // namespace

hipError_t launch_aev_fwd(const AevConst& P, int n, const float* pos, const int32_t* species, const BoxConst& bx,
                          const nnp_nlist* nl, const int32_t* out_row, void* out, bool bf16, unsigned* flags,
                          hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int grid = ceil_div(n, kWavesFwd);
    if (bf16)
        k_aev_fwd<uint16_t><<<grid, kWavesFwd * kWave, 0, s>>>(P, n, pos, species, bx, nl->row_ptr, nl->col,
                                                               nl->shift, out_row, (uint16_t*)out, flags);
    else
        k_aev_fwd<float><<<grid, kWavesFwd * kWave, 0, s>>>(P, n, pos, species, bx, nl->row_ptr, nl->col,
                                                            nl->shift, out_row, (float*)out, flags);
    return hipGetLastError();
}

hipError_t launch_aev_bwd(const AevConst& P, int n, const float* pos, const int32_t* species, const BoxConst& bx,
                          const nnp_nlist* nl, const int32_t* g_row, const float* g, float* Gx, float* Gy, float* Gz,
                          unsigned* flags, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int grid = ceil_div(n, kWavesBwd);
    k_aev_bwd<<<grid, kWavesBwd * kWave, 0, s>>>(P, n, pos, species, bx, nl->row_ptr, nl->col, nl->shift, g_row,
                                                g, Gx, Gy, Gz, flags);
    return hipGetLastError();
}

}  // namespace nnp
