// Species networks (Sec. 2.2, "Neural Networks": one MLP per chemical
// species; Sec. 2.4: atomic energies from the AEV, summed per structure) and
// their adjoint dE/dAEV, on MFMA.
//
//   forward   h_l = CELU(W_l h_{l-1} + b_l), E = w_head . h_L + b_head + e_s
//   adjoint   d_L = w_head * CELU'(z_L), d_{l-1} = (W_l^T d_l) * CELU'(z_{l-1}),
//             dE/dAEV = W_1^T d_1,   CELU'(z) = 1 (z > 0), 1 + h/alpha (z <= 0)
//
// Atoms are grouped by species with a stable counting sort; every species
// segment is padded to a multiple of 64 rows so a 64-row tile never mixes
// species and every GEMM sees one weight matrix per tile.  GEMMs are
// 64x64-output tiles on 4 waves, each wave a 2x2 grid of 16x16 MFMA tiles:
// v_mfma_f32_16x16x4_f32 for the FP32 form, v_mfma_f32_16x16x32_bf16 with
// float32 accumulation for the BF16 form.  Bias + CELU (forward) and the
// CELU derivative (adjoint) are fused into the GEMM epilogues.
#include "nnp_internal.hpp"

namespace nnp {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

constexpr int kGroupBlock = 1024;     // atoms per block in the species sort

// ---------------------------------------------------------------- species grouping

__global__ __launch_bounds__(256) void k_species_count(const int32_t* species, int n, int ns, int32_t* bcount,
                                                      unsigned* flags) {
    __shared__ int cnt[kMaxSpecies];
    if (threadIdx.x < kMaxSpecies) cnt[threadIdx.x] = 0;
    __syncthreads();
    for (int k = 0; k < kGroupBlock / 256; ++k) {
        const int a = blockIdx.x * kGroupBlock + k * 256 + threadIdx.x;
        if (a < n) {
            const int s = species[a];
            if (s >= 0 && s < ns) atomicAdd(&cnt[s], 1);
            else set_flag(flags, NNP_FLAG_SPECIES);
        }
    }
    __syncthreads();
    if (threadIdx.x < kMaxSpecies) bcount[blockIdx.x * kMaxSpecies + threadIdx.x] = cnt[threadIdx.x];
}

// meta: [0..8) counts, [8..17) padded row offsets (poff[ns] = padded total)
__global__ void k_species_scan(const int32_t* bcount, int nb, int ns, int32_t* boff, int32_t* meta) {
    __shared__ int tot[kMaxSpecies];
    const int s = threadIdx.x;
    if (s < kMaxSpecies) {
        int acc = 0;
        for (int b = 0; b < nb; ++b) {
            boff[b * kMaxSpecies + s] = acc;
            acc += bcount[b * kMaxSpecies + s];
        }
        tot[s] = s < ns ? acc : 0;
    }
    __syncthreads();
    if (s == 0) {
        int off = 0;
        for (int q = 0; q < kMaxSpecies; ++q) {
            meta[q] = tot[q];
            meta[8 + q] = off;
            off += ((tot[q] + kTileM - 1) / kTileM) * kTileM;
        }
        meta[8 + kMaxSpecies] = off;
    }
}

__global__ void k_fill_i32(int32_t* p, int n, int32_t v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ __launch_bounds__(256) void k_species_rank(const int32_t* species, int n, int ns, const int32_t* boff,
                                                     const int32_t* meta, int32_t* prow, int32_t* row_atom) {
    __shared__ int wcnt[kGroupBlock / kWave][kMaxSpecies];
    const int w = threadIdx.x / kWave;     // 4 waves, 4 rounds of 256 atoms
    int rank_in[4], sp[4];
    for (int k = 0; k < 4; ++k) {
        const int a = blockIdx.x * kGroupBlock + k * 256 + threadIdx.x;
        const int s = a < n ? species[a] : -1;
        sp[k] = s;
        int r = 0;
        for (int q = 0; q < kMaxSpecies; ++q) {
            const unsigned long long m = ballot(s == q);
            if (s == q) r = rank_below(m);
            if (lane_id() == 0) wcnt[k * 4 + w][q] = __popcll(m);
        }
        rank_in[k] = r;
    }
    __syncthreads();
    for (int k = 0; k < 4; ++k) {
        const int a = blockIdx.x * kGroupBlock + k * 256 + threadIdx.x;
        const int s = sp[k];
        if (a >= n || s < 0 || s >= ns) {
            if (a < n) prow[a] = -1;
            continue;
        }
        int before = 0;
        const int me = k * 4 + w;
        for (int q = 0; q < me; ++q) before += wcnt[q][s];
        const int row = meta[8 + s] + boff[blockIdx.x * kMaxSpecies + s] + before + rank_in[k];
        prow[a] = row;
        row_atom[row] = a;
    }
}

// Small systems: the whole stable grouping in one block of 1024 threads
// (counts, padded offsets, ranks in ascending atom order).
constexpr int kSmallGroup = 16384;

__global__ __launch_bounds__(1024) void k_group_small(const int32_t* species, int n, int ns, int32_t* meta,
                                                     int32_t* prow, int32_t* row_atom, int rows_max,
                                                     unsigned* flags) {
    __shared__ int cnt[kMaxSpecies];
    __shared__ int off[kMaxSpecies];
    __shared__ int wcnt[16][kMaxSpecies];
    const int t = threadIdx.x, w = t / kWave;
    if (t < kMaxSpecies) cnt[t] = 0;
    for (int r = t; r < rows_max; r += 1024) row_atom[r] = -1;
    __syncthreads();
    for (int a = t; a < n; a += 1024) {
        const int s = species[a];
        if (s >= 0 && s < ns) atomicAdd(&cnt[s], 1);
        else set_flag(flags, NNP_FLAG_SPECIES);
    }
    __syncthreads();
    if (t == 0) {
        int o = 0;
        for (int q = 0; q < kMaxSpecies; ++q) {
            const int c = q < ns ? cnt[q] : 0;
            meta[q] = c;
            meta[8 + q] = o;
            off[q] = o;
            o += ((c + kTileM - 1) / kTileM) * kTileM;
        }
        meta[8 + kMaxSpecies] = o;
    }
    __syncthreads();
    for (int base = 0; base < n; base += 1024) {
        const int a = base + t;
        const int s = a < n ? species[a] : -1;
        int rank = 0;
        for (int q = 0; q < ns; ++q) {
            const unsigned long long m = ballot(s == q);
            if (s == q) rank = rank_below(m);
            if (lane_id() == 0) wcnt[w][q] = __popcll(m);
        }
        __syncthreads();
        if (a < n) {
            if (s >= 0 && s < ns) {
                int before = 0;
                for (int q = 0; q < w; ++q) before += wcnt[q][s];
                const int row = off[s] + before + rank;
                prow[a] = row;
                row_atom[row] = a;
            } else {
                prow[a] = -1;
            }
        }
        __syncthreads();
        if (t < ns) {
            int add = 0;
            for (int q = 0; q < 16; ++q) add += wcnt[q][t];
            off[t] += add;
        }
        __syncthreads();
    }
}

// zero AEV rows that no atom owns (padding of each species segment)
template <typename T>
__global__ void k_zero_pad_rows(const int32_t* row_atom, int rows, int stride, T* aev) {
    const int r = blockIdx.x;
    if (r >= rows || row_atom[r] >= 0) return;
    for (int c = threadIdx.x; c < stride; c += blockDim.x) aev[(size_t)r * stride + c] = (T)0;
}

// ---------------------------------------------------------------- GEMM tiles

// Species of 64-row tile t: last s with poff[s] <= 64 t.  Returns -1 past the end.
__device__ __forceinline__ int tile_species(const int32_t* meta, int ns, int row0) {
    if (row0 >= meta[8 + ns]) return -1;
    int s = 0;
    for (int q = 1; q < ns; ++q)
        if (meta[8 + q] <= row0) s = q;
    return s;
}

enum Epi { kEpiCelu = 0, kEpiCeluGrad = 1, kEpiPlain = 2 };

struct GemmArgs {
    const void* A;        // [rows][lda]  fp32 or bf16 (see AisBf16)
    int lda;
    const void* Bt[kMaxSpecies];   // [N][K] per species, fp32 or bf16
    const float* bias[kMaxSpecies];
    const float* Hprev;   // kEpiCeluGrad: activations whose CELU' multiplies (ldc layout)
    float* C;             // [rows][ldc]
    int ldc;
    int K, N;
    float alpha;
    const int32_t* meta;
    int ns;
};

__device__ __forceinline__ float epilogue(int epi, float acc, const GemmArgs& g, int s, int row, int col) {
    if (epi == kEpiCelu) {
        const float v = acc + g.bias[s][col];
        return v > 0.f ? v : g.alpha * (__expf(v / g.alpha) - 1.f);
    }
    if (epi == kEpiCeluGrad) {
        const float h = g.Hprev[(size_t)row * g.ldc + col];
        return h > 0.f ? acc : acc * (1.f + h / g.alpha);
    }
    return acc;
}

// FP32: 64x64 tile, K chunk 32, v_mfma_f32_16x16x4_f32
template <int kEpi>
__global__ __launch_bounds__(256) void k_gemm_f32(const GemmArgs g) {
    constexpr int BK = 32, LD = BK + 1;
    __shared__ float As[64 * LD];
    __shared__ float Bs[64 * LD];
    const int row0 = blockIdx.x * 64;
    const int s = tile_species(g.meta, g.ns, row0);
    if (s < 0) return;
    const int n0 = blockIdx.y * 64;
    const float* A = (const float*)g.A;
    const float* B = (const float*)g.Bt[s];
    const int t = threadIdx.x, w = t / kWave, l = lane_id();
    const int wm = w >> 1, wn = w & 1;
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = (f32x4){0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < g.K; k0 += BK) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int idx = t + 256 * q;
            const int r = idx >> 3, c4 = (idx & 7) * 4;
            const float4 va = *(const float4*)(A + (size_t)(row0 + r) * g.lda + k0 + c4);
            const float4 vb = *(const float4*)(B + (size_t)(n0 + r) * g.K + k0 + c4);
            As[r * LD + c4 + 0] = va.x; As[r * LD + c4 + 1] = va.y;
            As[r * LD + c4 + 2] = va.z; As[r * LD + c4 + 3] = va.w;
            Bs[r * LD + c4 + 0] = vb.x; Bs[r * LD + c4 + 1] = vb.y;
            Bs[r * LD + c4 + 2] = vb.z; Bs[r * LD + c4 + 3] = vb.w;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            float a[2], b[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) a[i] = As[(32 * wm + 16 * i + (l & 15)) * LD + kk + (l >> 4)];
#pragma unroll
            for (int j = 0; j < 2; ++j) b[j] = Bs[(32 * wn + 16 * j + (l & 15)) * LD + kk + (l >> 4)];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = row0 + 32 * wm + 16 * i + 4 * (l >> 4) + r;
                const int col = n0 + 32 * wn + 16 * j + (l & 15);
                g.C[(size_t)row * g.ldc + col] = epilogue(kEpi, acc[i][j][r], g, s, row, col);
            }
}

template <bool kAisBf16>
__device__ __forceinline__ void load_a8(const GemmArgs& g, int row, int k, uint16_t out[8]) {
    if (kAisBf16) {
        const u16x8 v = *(const u16x8*)((const uint16_t*)g.A + (size_t)row * g.lda + k);
#pragma unroll
        for (int q = 0; q < 8; ++q) out[q] = v[q];
    } else {
        const float* p = (const float*)g.A + (size_t)row * g.lda + k;
        const float4 x = *(const float4*)p, y = *(const float4*)(p + 4);
        out[0] = f32_to_bf16(x.x); out[1] = f32_to_bf16(x.y); out[2] = f32_to_bf16(x.z); out[3] = f32_to_bf16(x.w);
        out[4] = f32_to_bf16(y.x); out[5] = f32_to_bf16(y.y); out[6] = f32_to_bf16(y.z); out[7] = f32_to_bf16(y.w);
    }
}

// BF16: 64x64 tile, K chunk 64, v_mfma_f32_16x16x32_bf16
template <int kEpi, bool kAisBf16>
__global__ __launch_bounds__(256) void k_gemm_bf16(const GemmArgs g) {
    constexpr int BK = 64, LD = BK + 8;   // row stride 144 B
    __shared__ __attribute__((aligned(16))) uint16_t As[64 * LD];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[64 * LD];
    const int row0 = blockIdx.x * 64;
    const int s = tile_species(g.meta, g.ns, row0);
    if (s < 0) return;
    const int n0 = blockIdx.y * 64;
    const uint16_t* B = (const uint16_t*)g.Bt[s];
    const int t = threadIdx.x, w = t / kWave, l = lane_id();
    const int wm = w >> 1, wn = w & 1;
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = (f32x4){0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < g.K; k0 += BK) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int idx = t + 256 * q;          // 512 groups of 8 elements per 64x64 tile
            const int r = idx >> 3, c8 = (idx & 7) * 8;
            uint16_t av[8];
            load_a8<kAisBf16>(g, row0 + r, k0 + c8, av);
            u16x8 va, vb = *(const u16x8*)(B + (size_t)(n0 + r) * g.K + k0 + c8);
#pragma unroll
            for (int e = 0; e < 8; ++e) va[e] = av[e];
            *(u16x8*)(As + r * LD + c8) = va;
            *(u16x8*)(Bs + r * LD + c8) = vb;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < BK; kk += 32) {
            bf16x8 a[2], b[2];
#pragma unroll
            for (int i = 0; i < 2; ++i)
                a[i] = *(const bf16x8*)(As + (32 * wm + 16 * i + (l & 15)) * LD + kk + 8 * (l >> 4));
#pragma unroll
            for (int j = 0; j < 2; ++j)
                b[j] = *(const bf16x8*)(Bs + (32 * wn + 16 * j + (l & 15)) * LD + kk + 8 * (l >> 4));
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = row0 + 32 * wm + 16 * i + 4 * (l >> 4) + r;
                const int col = n0 + 32 * wn + 16 * j + (l & 15);
                g.C[(size_t)row * g.ldc + col] = epilogue(kEpi, acc[i][j][r], g, s, row, col);
            }
}

// ---------------------------------------------------------------- head, energies

// one wave per padded row: E = w . h + b; d = w * CELU'(h) in place
__global__ __launch_bounds__(256) void k_head(const int32_t* meta, int ns, const int32_t* row_atom, int rows_max,
                                             const MlpPtrs P, int K, int ld, float alpha, float* H, float* E_row,
                                             float* E_atomo) {
    const int r = blockIdx.x * 4 + threadIdx.x / kWave;
    const int l = lane_id();
    if (r >= rows_max || r >= meta[8 + ns]) return;
    const int s = tile_species(meta, ns, r);
    float* h = H + (size_t)r * ld;
    const float* wv = P.head_w[s];
    float acc = 0.f;
    for (int c = l; c < ld; c += kWave) {
        const float hv = c < K ? h[c] : 0.f;
        const float wc = c < K ? wv[c] : 0.f;
        acc += hv * wc;
        h[c] = row_atom[r] >= 0 ? (hv > 0.f ? wc : wc * (1.f + hv / alpha)) : 0.f;
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) acc += shfl_xor(acc, m);
    if (l == 0) {
        E_row[r] = acc + P.head_b[s];
        const int a = row_atom[r];
        if (a >= 0 && E_atomo) E_atomo[a] = acc + P.head_b[s];
    }
}

// float64 structure energies: per-thread partial sums in ascending atom
// order (energies already in atom order), then a fixed tree.  Self energies
// are added in float64 per atom.  Atoms without a network energy (invalid
// species, flagged) contribute zero.
template <int kThreads>
__global__ __launch_bounds__(kThreads) void k_energy(int n_mol, const int32_t* mstart, const int32_t* mend,
                                                    const int32_t* prow, const int32_t* species, const SelfE se,
                                                    const float* E_at, double* e_mol, float* e_atom) {
    __shared__ double part[kThreads];
    const int m = blockIdx.x;
    if (m >= n_mol) return;
    const int b = mstart[m], e = mend[m];
    double acc = 0.0;
    for (int a = b + threadIdx.x; a < e; a += kThreads) {
        const bool ok = prow[a] >= 0;
        const double v = ok ? (double)E_at[a] + se.e[species[a]] : 0.0;
        if (e_atom) e_atom[a] = (float)v;
        acc += v;
    }
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int st = kThreads / 2; st >= 1; st >>= 1) {
        if ((int)threadIdx.x < st) part[threadIdx.x] += part[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) e_mol[m] = part[0];
}

// Large single structure: fixed 4096-atom chunks summed per block, then the
// chunk sums in order by one block (deterministic, two fixed trees).
constexpr int kChunk = 4096;

__global__ __launch_bounds__(1024) void k_energy_chunks(int n, const int32_t* prow, const int32_t* species,
                                                       const SelfE se, const float* E_at, double* part,
                                                       float* e_atom) {
    __shared__ double red[1024];
    const int base = blockIdx.x * kChunk;
    double acc = 0.0;
    for (int q = 0; q < kChunk / 1024; ++q) {
        const int a = base + q * 1024 + threadIdx.x;
        if (a < n) {
            const bool ok = prow[a] >= 0;
            const double v = ok ? (double)E_at[a] + se.e[species[a]] : 0.0;
            if (e_atom) e_atom[a] = (float)v;
            acc += v;
        }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int st = 512; st >= 1; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_energy_final(int nparts, const double* part, double* e_mol) {
    __shared__ double red[256];
    double acc = 0.0;
    for (int q = threadIdx.x; q < nparts; q += 256) acc += part[q];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int st = 128; st >= 1; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) e_mol[0] = red[0];
}

__global__ __launch_bounds__(1024) void k_energy_single(int n, const int32_t* prow, const int32_t* species,
                                                       const SelfE se, const float* E_at, double* e_mol,
                                                       float* e_atom) {
    __shared__ double red[1024];
    double acc = 0.0;
    for (int a = threadIdx.x; a < n; a += 1024) {
        const bool ok = prow[a] >= 0;
        const double v = ok ? (double)E_at[a] + se.e[species[a]] : 0.0;
        if (e_atom) e_atom[a] = (float)v;
        acc += v;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int st = 512; st >= 1; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) e_mol[0] = red[0];
}

// the range of atom i's structure (contiguous structures; a structure
// without atoms keeps the zero range the caller filled in)
__device__ __forceinline__ void mol_range_at(const int32_t* mol, int n, int n_mol, int i, int32_t* start,
                                             int32_t* end, unsigned* flags) {
    const int m = mol ? mol[i] : 0;
    if (m < 0 || m >= n_mol) {
        set_flag(flags, NNP_FLAG_MOL);
        return;
    }
    const int prev = i > 0 ? (mol ? mol[i - 1] : 0) : -1;
    const int next = i + 1 < n ? (mol ? mol[i + 1] : 0) : -1;
    if (i > 0 && prev > m) set_flag(flags, NNP_FLAG_MOL);
    if (prev != m) start[m] = i;
    if (next != m) end[m] = i + 1;
}

__global__ void k_mol_ranges2(const int32_t* mol, int n, int n_mol, int32_t* start, int32_t* end, unsigned* flags) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) mol_range_at(mol, n, n_mol, i, start, end, flags);
}

// Small batches (serving): the zero fill and the ranges in one workgroup,
// one launch in place of three.
constexpr int kRangesSmall = 16384;
__global__ __launch_bounds__(1024) void k_mol_ranges_small(const int32_t* mol, int n, int n_mol, int32_t* start,
                                                          int32_t* end, unsigned* flags) {
    for (int m = threadIdx.x; m < n_mol; m += 1024) {
        start[m] = 0;
        end[m] = 0;
    }
    __syncthreads();   // the zeros before any range
    for (int i = threadIdx.x; i < n; i += 1024) mol_range_at(mol, n, n_mol, i, start, end, flags);
}

__global__ void k_atom_e(const int32_t* prow, int n, const int32_t* species, const SelfE se, const float* E_at,
                         float* e_atom) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= n) return;
    e_atom[a] = prow[a] >= 0 ? (float)((double)E_at[a] + se.e[species[a]]) : 0.f;
}

// scatter/gather of rows between atom order and grouped order
template <bool kToGrouped>
__global__ void k_permute_rows(const int32_t* prow, int n, int stride, const float* src, float* dst) {
    const int a = blockIdx.x;
    if (a >= n) return;
    const int r = prow[a];
    if (r < 0) return;
    const float* s = kToGrouped ? src + (size_t)a * stride : src + (size_t)r * stride;
    float* d = kToGrouped ? dst + (size_t)r * stride : dst + (size_t)a * stride;
    for (int c = threadIdx.x; c < stride; c += blockDim.x) d[c] = s[c];
}

__global__ void k_permute_rows_bf16(const int32_t* prow, int n, int stride, const float* src, uint16_t* dst) {
    const int a = blockIdx.x;
    if (a >= n) return;
    const int r = prow[a];
    if (r < 0) return;
    for (int c = threadIdx.x; c < stride; c += blockDim.x)
        dst[(size_t)r * stride + c] = f32_to_bf16(src[(size_t)a * stride + c]);
}

__global__ void k_gather_e(const int32_t* prow, int n, const int32_t* species, const SelfE se, const float* E_row,
                           float* e_atom) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= n) return;
    const int r = prow[a];
    e_atom[a] = r >= 0 ? (float)((double)E_row[r] + se.e[species[a]]) : 0.f;
}

}  // namespace

// ---------------------------------------------------------------- host side

hipError_t launch_species_group(const nnp_model* m, int n, const int32_t* species, const MlpWs& W, unsigned* flags,
                                hipStream_t s) {
    const int ns = m->aev.ns;
    if (n <= kSmallGroup) {
        k_group_small<<<1, 1024, 0, s>>>(species, n, ns, W.meta, W.prow, W.row_atom, W.rows_max, flags);
        return hipGetLastError();
    }
    const int nb = ceil_div(n > 0 ? n : 1, kGroupBlock);
    k_fill_i32<<<ceil_div(W.rows_max, 256), 256, 0, s>>>(W.row_atom, W.rows_max, -1);
    k_species_count<<<nb, 256, 0, s>>>(species, n, ns, W.bcount, flags);
    k_species_scan<<<1, 64, 0, s>>>(W.bcount, nb, ns, W.boff, W.meta);
    k_species_rank<<<nb, 256, 0, s>>>(species, n, ns, W.boff, W.meta, W.prow, W.row_atom);
    return hipGetLastError();
}

hipError_t launch_zero_pad_rows(const MlpWs& W, int stride, void* aev, bool bf16, hipStream_t s) {
    if (W.rows_max <= 0) return hipSuccess;
    if (bf16)
        k_zero_pad_rows<uint16_t><<<W.rows_max, 256, 0, s>>>(W.row_atom, W.rows_max, stride, (uint16_t*)aev);
    else
        k_zero_pad_rows<float><<<W.rows_max, 256, 0, s>>>(W.row_atom, W.rows_max, stride, (float*)aev);
    return hipGetLastError();
}

// MLP forward + adjoint on grouped rows.  aev: [rows_max][stride] (fp32 or
// bf16 for the BF16 form); h[l]: fp32 activation buffers [rows_max][wpad[l+1]];
// g_out: fp32 [rows_max][stride]; E_row: [rows_max].
hipError_t launch_mlp(const nnp_model* m, const MlpWs& W, const void* aev, bool aev_bf16, float* const* h,
                      float* g_out, float* E_row, float* E_atomo, hipStream_t s) {
    const int ns = m->aev.ns;
    const int L = m->n_layers;      // includes head
    const int tiles = ceil_div(W.rows_max, kTileM);
    const bool bf = m->precision == NNP_BF16_MLP;
    GemmArgs g;
    g.meta = W.meta;
    g.ns = ns;
    g.alpha = m->celu_alpha;
    g.Hprev = nullptr;
    // forward hidden layers 0..L-2
    for (int l = 0; l < L - 1; ++l) {
        g.A = l == 0 ? aev : (const void*)h[l - 1];
        g.lda = m->wpad[l];
        g.K = m->wpad[l];
        g.N = m->wpad[l + 1];
        g.C = h[l];
        g.ldc = m->wpad[l + 1];
        for (int q = 0; q < ns; ++q) {
            g.Bt[q] = bf ? (const void*)m->ptrs.Wb[q][l] : (const void*)m->ptrs.W[q][l];
            g.bias[q] = m->ptrs.b[q][l];
        }
        dim3 grid(tiles, g.N / 64);
        if (bf) {
            if (l == 0 && aev_bf16) k_gemm_bf16<kEpiCelu, true><<<grid, 256, 0, s>>>(g);
            else k_gemm_bf16<kEpiCelu, false><<<grid, 256, 0, s>>>(g);
        } else {
            k_gemm_f32<kEpiCelu><<<grid, 256, 0, s>>>(g);
        }
    }
    // head: energy and d_L (in place in h[L-2])
    k_head<<<ceil_div(W.rows_max, 4), 256, 0, s>>>(W.meta, ns, W.row_atom, W.rows_max, m->ptrs, m->widths[L - 1],
                                                  m->wpad[L - 1], m->celu_alpha, h[L - 2], E_row, E_atomo);
    if (!g_out) return hipGetLastError();
    // adjoint: d_{l-1} = (W_l^T d_l) * CELU'(h_{l-1}), l = L-2 .. 1; then g = W_0^T d_0
    for (int l = L - 2; l >= 0; --l) {
        g.A = h[l];
        g.lda = m->wpad[l + 1];
        g.K = m->wpad[l + 1];
        g.N = m->wpad[l];
        for (int q = 0; q < ns; ++q) g.Bt[q] = bf ? (const void*)m->ptrs.WTb[q][l] : (const void*)m->ptrs.WT[q][l];
        dim3 grid(tiles, g.N / 64);
        if (l > 0) {
            g.C = h[l - 1];
            g.ldc = m->wpad[l];
            g.Hprev = h[l - 1];
            if (bf) k_gemm_bf16<kEpiCeluGrad, false><<<grid, 256, 0, s>>>(g);
            else k_gemm_f32<kEpiCeluGrad><<<grid, 256, 0, s>>>(g);
        } else {
            g.C = g_out;
            g.ldc = m->aev.stride;
            g.Hprev = nullptr;
            if (bf) k_gemm_bf16<kEpiPlain, false><<<grid, 256, 0, s>>>(g);
            else k_gemm_f32<kEpiPlain><<<grid, 256, 0, s>>>(g);
        }
    }
    return hipGetLastError();
}

hipError_t launch_energy(int n, int n_mol, const int32_t* mol, const int32_t* species, const SelfE& se,
                         int32_t* mstart, int32_t* mend, bool ranges_ready, const MlpWs& W, const float* E_at,
                         double* e_mol, float* e_atom, unsigned* flags, hipStream_t s) {
    if (n_mol == 1 && !mol && n <= 2 * kChunk) {
        k_energy_single<<<1, 1024, 0, s>>>(n, W.prow, species, se, E_at, e_mol, e_atom);
        return hipGetLastError();
    }
    if (n_mol == 1 && n > 2 * kChunk) {
        // mol must still be validated: a single structure means every mol entry is 0
        if (mol && !ranges_ready) k_mol_ranges2<<<ceil_div(n, 256), 256, 0, s>>>(mol, n, n_mol, mstart, mend, flags);
        const int nparts = ceil_div(n, kChunk);
        double* part = (double*)W.bcount;   // >= nparts doubles: bcount holds 8 ints per 1024 atoms
        k_energy_chunks<<<nparts, 1024, 0, s>>>(n, W.prow, species, se, E_at, part, e_atom);
        k_energy_final<<<1, 256, 0, s>>>(nparts, part, e_mol);
        return hipGetLastError();
    }
    if (n_mol > 0) {
        if (ranges_ready) {
            // built and checked by the caller
        } else if (n <= kRangesSmall && n_mol <= kRangesSmall) {
            k_mol_ranges_small<<<1, 1024, 0, s>>>(mol, n, n_mol, mstart, mend, flags);
        } else {
            k_fill_i32<<<ceil_div(n_mol, 256), 256, 0, s>>>(mstart, n_mol, 0);
            k_fill_i32<<<ceil_div(n_mol, 256), 256, 0, s>>>(mend, n_mol, 0);
            if (n > 0) k_mol_ranges2<<<ceil_div(n, 256), 256, 0, s>>>(mol, n, n_mol, mstart, mend, flags);
        }
        if (n_mol == 1)
            k_energy<1024><<<1, 1024, 0, s>>>(n_mol, mstart, mend, W.prow, species, se, E_at, e_mol, e_atom);
        else
            k_energy<128><<<n_mol, 128, 0, s>>>(n_mol, mstart, mend, W.prow, species, se, E_at, e_mol, e_atom);
    } else if (e_atom && n > 0) {
        k_atom_e<<<ceil_div(n, 256), 256, 0, s>>>(W.prow, n, species, se, E_at, e_atom);
    }
    return hipGetLastError();
}

hipError_t launch_permute_rows(bool to_grouped, const int32_t* prow, int n, int stride, const float* src, float* dst,
                               hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (to_grouped) k_permute_rows<true><<<n, 256, 0, s>>>(prow, n, stride, src, dst);
    else k_permute_rows<false><<<n, 256, 0, s>>>(prow, n, stride, src, dst);
    return hipGetLastError();
}

hipError_t launch_permute_rows_bf16(const int32_t* prow, int n, int stride, const float* src, uint16_t* dst,
                                    hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_permute_rows_bf16<<<n, 256, 0, s>>>(prow, n, stride, src, dst);
    return hipGetLastError();
}

hipError_t launch_gather_e(const int32_t* prow, int n, const int32_t* species, const SelfE& se, const float* E_row,
                           float* e_atom, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_gather_e<<<ceil_div(n, 256), 256, 0, s>>>(prow, n, species, se, E_row, e_atom);
    return hipGetLastError();
}

}  // namespace nnp
