// Neighbour list (Sec. 2.1, "Preprocessing Modules"): directed pairs of atoms
// of the same structure closer than the list cutoff, minimum image in an
// orthorhombic box, rows sorted by neighbour index, plus the reverse index.
//
// Periodic systems use an integer cell list (cells at least r_list wide, a
// 27-cell stencil, or every cell along a dimension with fewer than 3 cells):
// without structure ids one block per cell stages the stencil's positions in
// LDS and builds the rows of the cell's atoms from there.  Systems with
// structure ids, and open systems (all atoms of the same structure), search
// per row from global memory.  Candidates of one row are streamed across the
// 64 lanes of a wave and compacted with ballots; the row is rank-sorted in
// LDS before it is written, so the output does not depend on the (atomic)
// order in which atoms were binned.
//
// The pair predicate is evaluated in float64 with every operation rounded
// (floating-point contraction is disabled in that function), so the pair set
// is reproducible bit for bit by any IEEE implementation.  A float32 screen
// decides every candidate outside a band around r_list^2 that covers its
// rounding; only the candidates inside the band reach the float64 predicate.
#include "md_internal.hpp"
#include "nnp_internal.hpp"

namespace nnp {
namespace {

constexpr int kRowsPerBlock = 4;              // one wave per row
constexpr int kRowLds = NNP_MAX_ROW;          // longest row the builder handles (staging stride)
constexpr int kMaxCellsPerDim = 128;

struct Grid {
    int periodic;
    int nc[3];          // cells per dimension
    int ns[3];          // stencil width per dimension (min(3, nc))
    double L[3];        // box sides (float32 widened)
    double inv_cs[3];   // nc / L
    float Lf[3];        // box sides
    float inv_Lf[3];    // 1 / L (float32, fast path only)
};

struct PairOut {
    bool keep;
    int packed_shift;
};

// Exact predicate.  No contraction: each +, -, *, / is rounded on its own.
__device__ __forceinline__ PairOut pair_predicate_exact(float3 xi, float3 xj, const Grid& g, double r2) {
#pragma clang fp contract(off)
    double d[3], n[3];
    const double a[3] = {(double)xi.x, (double)xi.y, (double)xi.z};
    const double b[3] = {(double)xj.x, (double)xj.y, (double)xj.z};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double d0 = b[k] - a[k];
        if (g.periodic) {
            n[k] = -rint(d0 / g.L[k]);
            double nl = n[k] * g.L[k];
            d[k] = d0 + nl;
        } else {
            n[k] = 0.0;
            d[k] = d0;
        }
    }
    double sx = d[0] * d[0];
    double sy = d[1] * d[1];
    double sz = d[2] * d[2];
    double d2 = (sx + sy) + sz;
    PairOut o;
    o.keep = d2 < r2;
    int ix = (int)n[0], iy = (int)n[1], iz = (int)n[2];
    o.packed_shift = (ix & 0xff) | ((iy & 0xff) << 8) | ((iz & 0xff) << 16);
    if (o.keep && (n[0] < -127.0 || n[0] > 127.0 || n[1] < -127.0 || n[1] > 127.0 || n[2] < -127.0 ||
                   n[2] > 127.0))
        o.packed_shift = -1;   // caller flags it
    return o;
}

// Same decision, float32 first.  With M the largest coordinate or box
// magnitude involved, every float32 component of d is within 4 ulp(M) of the
// float64 one, so |d2_f32 - d2_exact| < 2 r e + e^2 with e = 1e-5 M, which
// is 20x that bound.  Outside that band around r^2 the float32 decision (and,
// for kept pairs, the image shift, since then |d0/L + n| < 1/2 - 1e-6) equals
// the exact one; inside the band the exact float64 predicate decides.
__device__ __forceinline__ PairOut pair_predicate(float3 xi, float3 xj, const Grid& g, double r2, float rf) {
    float d[3], n[3];
    const float a[3] = {xi.x, xi.y, xi.z};
    const float b[3] = {xj.x, xj.y, xj.z};
    float M = 1.0f;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const float d0 = b[k] - a[k];
        M = fmaxf(M, fmaxf(fabsf(a[k]), fabsf(b[k])));
        if (g.periodic) {
            n[k] = -rintf(d0 * g.inv_Lf[k]);
            d[k] = d0 + n[k] * g.Lf[k];
            M = fmaxf(M, g.Lf[k]);
        } else {
            n[k] = 0.f;
            d[k] = d0;
        }
    }
    const float d2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    const float e = 1e-5f * M;
    const float band = e * (2.0f * rf + e);
    const float r2f = rf * rf;
    PairOut o;
    if (d2 > r2f + band) {
        o.keep = false;
        o.packed_shift = 0;
        return o;
    }
    if (d2 < r2f - band) {
        o.keep = true;
        if (fabsf(n[0]) > 127.f || fabsf(n[1]) > 127.f || fabsf(n[2]) > 127.f) {
            o.packed_shift = -1;
        } else {
            const int ix = (int)n[0], iy = (int)n[1], iz = (int)n[2];
            o.packed_shift = (ix & 0xff) | ((iy & 0xff) << 8) | ((iz & 0xff) << 16);
        }
        return o;
    }
    return pair_predicate_exact(xi, xj, g, r2);
}

__device__ __forceinline__ float3 load_pos(const float* pos, int i) {
    return make_float3(pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]);
}

__device__ __forceinline__ bool finite3(float3 p) {
    return isfinite(p.x) && isfinite(p.y) && isfinite(p.z);
}

__device__ __forceinline__ int cell_coord(float x, double L, double inv_cs, int nc) {
    // a coordinate already in [0, L) is its own image (floor(x / L) is 0
    // there), so only coordinates outside the box take the division
    double w = (double)x;
    if (w < 0.0 || w >= L) w -= L * floor(w / L);
    int c = (int)(w * inv_cs);
    return c < 0 ? 0 : (c >= nc ? nc - 1 : c);
}

// structure ranges for contiguous molecules; validates mol.  A structure
// without atoms keeps the zero range filled in before.
__device__ __forceinline__ void mol_range_of(const int32_t* mol, int n, int n_mol, int i, int32_t* start,
                                             int32_t* end, unsigned* flags) {
    const int m = mol[i];
    if (m < 0 || m >= n_mol) {
        set_flag(flags, NNP_FLAG_MOL);
        return;
    }
    const int prev = i > 0 ? mol[i - 1] : -1;
    const int next = i + 1 < n ? mol[i + 1] : -1;
    if (i > 0 && prev > m) set_flag(flags, NNP_FLAG_MOL);
    if (prev != m) start[m] = i;
    if (next != m) end[m] = i + 1;
}

__global__ void k_mol_ranges(const int32_t* mol, int n, int n_mol, int32_t* start, int32_t* end,
                             unsigned* flags, const int32_t* gate) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || (gate && *gate == 0)) return;
    mol_range_of(mol, n, n_mol, i, start, end, flags);
}

// Small batches (serving): the zero fill and the ranges in one workgroup,
// one launch in place of three; with pos (open systems) also k_finite's
// check of the coordinates.
constexpr int kMolSmall = 16384;
__global__ __launch_bounds__(1024) void k_mol_ranges_small(const int32_t* mol, int n, int n_mol, int32_t* start,
                                                          int32_t* end, unsigned* flags, const int32_t* gate,
                                                          const float* pos) {
    if (gate && *gate == 0) return;
    for (int m = threadIdx.x; m < n_mol; m += 1024) {
        start[m] = 0;
        end[m] = 0;
    }
    __syncthreads();   // the zeros before any range
    for (int i = threadIdx.x; i < n; i += 1024) {
        mol_range_of(mol, n, n_mol, i, start, end, flags);
        if (pos && !finite3(load_pos(pos, i))) set_flag(flags, NNP_FLAG_NONFINITE);
    }
}

__global__ void k_bin(const float* pos, int n, const Grid g, int32_t* cell_of, int32_t* cell_slot,
                      int32_t* cell_count, unsigned* flags, const int32_t* gate) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || (gate && *gate == 0)) return;
    const float3 p = load_pos(pos, i);
    if (!finite3(p)) {
        set_flag(flags, NNP_FLAG_NONFINITE);
        cell_of[i] = -1;
        return;
    }
    const int cx = cell_coord(p.x, g.L[0], g.inv_cs[0], g.nc[0]);
    const int cy = cell_coord(p.y, g.L[1], g.inv_cs[1], g.nc[1]);
    const int cz = cell_coord(p.z, g.L[2], g.inv_cs[2], g.nc[2]);
    const int c = (cx * g.nc[1] + cy) * g.nc[2] + cz;
    cell_of[i] = c;
    cell_slot[i] = atomicAdd(&cell_count[c], 1);
}

// Cell binning as k_bin, and by the block that finishes last (an integer
// ticket) the exclusive scan of the n_cells <= kBinScanCells counts into
// cell_start (n_cells + 1 entries, the total also to *total), after which it
// zeroes the counts and the ticket for the next build: a build on a
// workspace left by this kernel needs no zero fill.  The counts are read
// after the ticket with device-coherent loads.  kMd: the MD engine's
// rebuild decision and wrap come first (MdFront), in place of a gate word.
constexpr int kBinScanThreads = 1024, kBinScanItems = 8, kBinScanCells = kBinScanThreads * kBinScanItems;
__device__ __forceinline__ long long wave_inclusive_ll(long long v) {
    const int l = lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const long long u = __shfl_up(v, d, kWave);
        if (l >= d) v += u;
    }
    return v;
}
template <bool kMd>
__global__ __launch_bounds__(kBinScanThreads) void k_bin_scan(const float* pos, int n, const Grid g, int n_cells,
                                                              int32_t* cell_of, int32_t* cell_slot,
                                                              int32_t* cell_count, int32_t* cell_start,
                                                              int64_t* total, unsigned* ticket, unsigned* flags,
                                                              const int32_t* gate, const MdFront md) {
    __shared__ long long wsum[kBinScanThreads / kWave];
    __shared__ int s_last;
    const int t = threadIdx.x;
    const int i = blockIdx.x * kBinScanThreads + t;
    if (kMd) {
        // the same two largest displacements, in the same order, in every block
        __shared__ float s_m[kBinScanThreads / kWave][2];
        MdState cur{};
        if (t == 0) cur = *md.cur;
        float m1 = 0.f, m2 = 0.f;
        for (int q = t; q < md.n_parts; q += kBinScanThreads)
            top2_merge(m1, m2, md.d2_part[2 * q], md.d2_part[2 * q + 1]);
        top2_wave(m1, m2);
        if (lane_id() == 0) {
            s_m[t / kWave][0] = m1;
            s_m[t / kWave][1] = m2;
        }
        __syncthreads();
        __shared__ int s_gate;
        if (t == 0) {
            for (int q = 1; q < kBinScanThreads / kWave; ++q) top2_merge(m1, m2, s_m[q][0], s_m[q][1]);
            s_gate = md_decide(blockIdx.x == 0 ? md.nxt : nullptr, cur, m1, m2, md.rebuild_every, md.trig_len);
        }
        __syncthreads();
        if (!s_gate) return;
    } else if (gate && *gate == 0) {
        return;
    }
    if (i < n) {
        float3 p = load_pos(pos, i);
        if (kMd) {   // periodic boxes only: the kernel bins periodic boxes
            p.x = md_wrap_coord(p.x, g.Lf[0]);
            p.y = md_wrap_coord(p.y, g.Lf[1]);
            p.z = md_wrap_coord(p.z, g.Lf[2]);
            const float w[3] = {p.x, p.y, p.z};
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                md.pos[3 * (size_t)i + k] = w[k];
                md.ref[3 * (size_t)i + k] = w[k];
            }
        }
        if (!finite3(p)) {
            set_flag(flags, NNP_FLAG_NONFINITE);
            cell_of[i] = -1;
        } else {
            const int cx = cell_coord(p.x, g.L[0], g.inv_cs[0], g.nc[0]);
            const int cy = cell_coord(p.y, g.L[1], g.inv_cs[1], g.nc[1]);
            const int cz = cell_coord(p.z, g.L[2], g.inv_cs[2], g.nc[2]);
            const int c = (cx * g.nc[1] + cy) * g.nc[2] + cz;
            cell_of[i] = c;
            cell_slot[i] = atomicAdd(&cell_count[c], 1);
        }
    }
    __syncthreads();
    if (t == 0) {
        __threadfence();   // this block's counts before the ticket
        s_last = atomicAdd(ticket, 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (!s_last) return;
    __threadfence();   // every block's counts after the last ticket
    const int w = t / kWave, base = t * kBinScanItems;
    int32_t v[kBinScanItems];
    long long sum = 0;
#pragma unroll
    for (int k = 0; k < kBinScanItems; ++k) {
        v[k] = base + k < n_cells ? __hip_atomic_load(&cell_count[base + k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                  : 0;
        sum += v[k];
    }
    const long long inc = wave_inclusive_ll(sum);
    if (lane_id() == kWave - 1) wsum[w] = inc;
    __syncthreads();
    long long off = 0, all = 0;
    for (int q = 0; q < kBinScanThreads / kWave; ++q) {
        if (q < w) off += wsum[q];
        all += wsum[q];
    }
    long long ex = off + inc - sum;
#pragma unroll
    for (int k = 0; k < kBinScanItems; ++k) {
        if (base + k < n_cells) {
            cell_start[base + k] = (int32_t)ex;
            cell_count[base + k] = 0;
        }
        ex += v[k];
    }
    if (t == 0) {
        *total = all;
        cell_start[n_cells] = (int32_t)all;
        *ticket = 0u;
    }
}

__global__ void k_scatter(int n, const int32_t* cell_of, const int32_t* cell_slot, const int32_t* cell_start,
                          int32_t* cell_atoms, const int32_t* gate) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || (gate && *gate == 0)) return;
    const int c = cell_of[i];
    if (c >= 0) cell_atoms[cell_start[c] + cell_slot[i]] = i;
}

__global__ void k_finite(const float* pos, int n, unsigned* flags, const int32_t* gate) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || (gate && *gate == 0)) return;
    if (!finite3(load_pos(pos, i))) set_flag(flags, NNP_FLAG_NONFINITE);
}

// The stencil's source cells around cell ci (3 x 3 x 3, or every cell of a
// dimension with fewer than three), one per lane below the returned count
// n_src: beg[k] is source k's first slot in cell_atoms and off[k] the
// exclusive prefix of the sources' atom counts, off[n_src] their total.
// Wave-level.
__device__ __forceinline__ int stencil_sources(const Grid& g, int ci, const int32_t* cell_start, int* off,
                                               int* beg) {
    const int l = lane_id();
    const int cz = ci % g.nc[2];
    const int cy = (ci / g.nc[2]) % g.nc[1];
    const int cx = ci / (g.nc[2] * g.nc[1]);
    const int n_src = g.ns[0] * g.ns[1] * g.ns[2];
    int b0 = 0, cnt = 0;
    if (l < n_src) {
        int a, b, c;
        if (n_src == 27) {   // 3 x 3 x 3 stencil: constant divisors
            a = l / 9;
            b = (l / 3) % 3;
            c = l % 3;
        } else {
            a = l / (g.ns[1] * g.ns[2]);
            b = (l / g.ns[2]) % g.ns[1];
            c = l % g.ns[2];
        }
        // stencil: offsets -1..1 when nc >= 3 (wrapped periodically), else every cell of the dimension
        auto wrap = [](int x, int nc) { return x < 0 ? x + nc : (x >= nc ? x - nc : x); };
        const int ox = g.nc[0] >= 3 ? wrap(cx + a - 1, g.nc[0]) : a;
        const int oy = g.nc[1] >= 3 ? wrap(cy + b - 1, g.nc[1]) : b;
        const int oz = g.nc[2] >= 3 ? wrap(cz + c - 1, g.nc[2]) : c;
        const int cell = (ox * g.nc[1] + oy) * g.nc[2] + oz;
        b0 = cell_start[cell];
        cnt = cell_start[cell + 1] - b0;
    }
    // inclusive scan of counts over the first n_src lanes
    int inc = cnt;
    for (int d = 1; d < 32; d <<= 1) {
        int u = __shfl_up(inc, d, kWave);
        if (l >= d) inc += u;
    }
    if (l < n_src) {
        off[l] = inc - cnt;
        beg[l] = b0;
    }
    if (l == n_src - 1) off[n_src] = inc;
    return n_src;
}

// Slot in cell_atoms (or atom index without cells) of candidate t, and its
// source k: the last one with off[k] <= t (off[n_src] = total > t)
__device__ __forceinline__ int cand_slot(const int* off, const int* beg, int n_src, int t, int& k) {
    int lo = 0, hi = n_src;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= t) lo = mid; else hi = mid;
    }
    k = lo;
    return beg[lo] + (t - off[lo]);
}
__device__ __forceinline__ int cand_slot(const int* off, const int* beg, int n_src, int t) {
    int k;
    return cand_slot(off, beg, n_src, t, k);
}

// The kept pairs of row i, compacted in candidate order into the wave's LDS
// row (s_col, s_sh) with their count, are rank-sorted by neighbour index and
// written to the staging row i * kRowLds with the count; a row longer than
// kRowLds raises NNP_FLAG_ROW and is left empty.  Wave-level.
__device__ __forceinline__ void finish_row(int i, int count, int* s_col, int* s_sh, int32_t* row_count,
                                           int32_t* stage_col, int32_t* stage_sh, unsigned* flags) {
    const int l = lane_id();
    if (count > kRowLds) {
        if (l == 0) {
            set_flag(flags, NNP_FLAG_ROW);
            row_count[i] = 0;
        }
        wave_sync();
        return;
    }
    wave_sync();
    // rank sort (indices in a row are distinct); the row is read four entries
    // per 16-byte LDS load, several loads in flight
    int32_t* oc = stage_col + (size_t)i * kRowLds;
    int32_t* os = stage_sh + (size_t)i * kRowLds;
    for (int e = l; e < count; e += kWave) {
        const int je = s_col[e];
        int rank = 0, f = 0;
#pragma unroll 4
        for (; f + 4 <= count; f += 4) {
            const int4 q = *(const int4*)(s_col + f);
            rank += (q.x < je) + (q.y < je) + (q.z < je) + (q.w < je);
        }
        for (; f < count; ++f) rank += s_col[f] < je;
        oc[rank] = je;
        os[rank] = s_sh[e];
    }
    if (l == 0) row_count[i] = count;
    wave_sync();   // the LDS row is free for the wave's next row
}

// Compaction of one 64-candidate round: the kept lanes' (j, sh) appended to
// the LDS row in lane order.  Returns the new count (may exceed kRowLds: the
// entries past it are dropped and finish_row rejects the row).
__device__ __forceinline__ int append_kept(bool keep, int j, int sh, int count, int* s_col, int* s_sh) {
    const unsigned long long m = ballot(keep);
    if (keep) {
        const int p = count + rank_below(m);
        if (p < kRowLds) {
            s_col[p] = j;
            s_sh[p] = sh;
        }
    }
    return count + __popcll(m);
}

// The row of atom i (position xi) over candidates t = 0 .. total - 1:
// fetch(t, j, xj) gives candidate t's index j and returns whether it may be
// a neighbour, then with its position xj.  Wave-level.
template <class Fetch>
__device__ __forceinline__ void build_row(int i, float3 xi, int total, Fetch fetch, const Grid& g, double r2,
                                          float rf, int* s_col, int* s_sh, int32_t* row_count, int32_t* stage_col,
                                          int32_t* stage_sh, unsigned* flags) {
    int count = 0;
    for (int base = 0; base < total; base += kWave) {
        const int t = base + lane_id();
        bool keep = false;
        int j = -1, sh = 0;
        float3 xj;
        if (t < total && fetch(t, j, xj)) {
            PairOut o = pair_predicate(xi, xj, g, r2, rf);
            keep = o.keep;
            sh = o.packed_shift;
            if (keep && sh == -1) {
                set_flag(flags, NNP_FLAG_SHIFT);
                sh = 0;
            }
        }
        count = append_kept(keep, j, sh, count, s_col, s_sh);
    }
    finish_row(i, count, s_col, s_sh, row_count, stage_col, stage_sh, flags);
}

// The row of atom i of a periodic box over the block's staged candidates
// s_x[0 .. total) (position; the index in w of s_j).
// The float32 screen of pair_predicate without branches, with one magnitude
// bound for the block: lo / hi = r^2 -/+ the band of pair_predicate for M
// the largest coordinate magnitude or box side of any staged atom (at least
// each pair's own M, so the band is at least as wide as that pair's).  The
// rare lanes inside the band take the exact float64 predicate.  The same
// pairs as build_row.
__device__ __forceinline__ void build_row_staged(int i, float3 xi, int total, const float4* s_x, const float4* s_j,
                                                 const Grid& g, double r2, float lo, float hi, int* s_col, int* s_sh,
                                                 int32_t* row_count, int32_t* stage_col, int32_t* stage_sh,
                                                 unsigned* flags) {
    const int l = lane_id();
    int count = 0;
    bool bad_shift = false;
    for (int base = 0; base < total; base += kWave) {
        const int t = min(base + l, total - 1);
        const float4 q = s_x[t];
        const int j = __float_as_int(s_j[t].w);
        const float d0x = q.x - xi.x, d0y = q.y - xi.y, d0z = q.z - xi.z;
        const float nx = -rintf(d0x * g.inv_Lf[0]), ny = -rintf(d0y * g.inv_Lf[1]), nz = -rintf(d0z * g.inv_Lf[2]);
        const float dx = d0x + nx * g.Lf[0], dy = d0y + ny * g.Lf[1], dz = d0z + nz * g.Lf[2];
        const float d2 = dx * dx + dy * dy + dz * dz;
        const bool valid = base + l < total && j != i;
        bool keep = valid && d2 < lo;
        const bool undecided = valid && d2 >= lo && d2 <= hi;
        int sh = ((int)nx & 0xff) | (((int)ny & 0xff) << 8) | (((int)nz & 0xff) << 16);
        bool wide = fmaxf(fabsf(nx), fmaxf(fabsf(ny), fabsf(nz))) > 127.f;
        if (ballot(undecided)) {   // wave-uniform; rare
            if (undecided) {
                const PairOut o = pair_predicate_exact(xi, make_float3(q.x, q.y, q.z), g, r2);
                keep = o.keep;
                sh = o.packed_shift;
                wide = o.packed_shift == -1;
            }
        }
        if (keep && wide) {
            bad_shift = true;
            sh = 0;
        }
        count = append_kept(keep, j, sh, count, s_col, s_sh);
    }
    if (ballot(bad_shift) && l == 0) set_flag(flags, NNP_FLAG_SHIFT);
    finish_row(i, count, s_col, s_sh, row_count, stage_col, stage_sh, flags);
}

// The row of atom i of a periodic box with at least three cells along every
// dimension and every staged atom inside [0, L): each staged candidate also
// has its position with the image shift of its stencil cell applied (s_xs:
// x_j + n L, n in {-1, 0, 1}, index j in w; s_x: the unshifted position,
// the packed n in w), which for a pair within the cutoff is the minimum
// image (L > 2 r_list), so the float32 screen is a plain distance.  The
// shifted position is one rounding from the exact one, well inside the
// float32 error pair_predicate's band allows for; lanes inside the band take
// the exact predicate on the unshifted positions.  The same pairs as
// build_row.
__device__ __forceinline__ void build_row_shifted(int i, float3 xi, int total, const float4* s_x, const float4* s_xs,
                                                  const Grid& g, double r2, float lo, float hi, int* r_col,
                                                  int* r_sh, int32_t* row_count, int32_t* stage_col,
                                                  int32_t* stage_sh, unsigned* flags) {
    const int l = lane_id();
    int count = 0;
    bool bad_shift = false;
    for (int base = 0; base < total; base += kWave) {
        const int t = min(base + l, total - 1);
        const float4 q = s_xs[t];
        const int j = __float_as_int(q.w);
        const float dx = q.x - xi.x, dy = q.y - xi.y, dz = q.z - xi.z;
        const float d2 = dx * dx + dy * dy + dz * dz;
        const bool valid = base + l < total && j != i;
        bool keep = valid && d2 < lo;
        const bool undecided = valid && d2 >= lo && d2 <= hi;
        int sh = 0;
        if (keep) sh = __float_as_int(s_x[t].w);
        if (ballot(undecided)) {   // wave-uniform; rare
            if (undecided) {
                const float4 x = s_x[t];
                const PairOut o = pair_predicate_exact(xi, make_float3(x.x, x.y, x.z), g, r2);
                keep = o.keep;
                sh = o.packed_shift;
                if (keep && sh == -1) {
                    bad_shift = true;
                    sh = 0;
                }
            }
        }
        count = append_kept(keep, j, sh, count, r_col, r_sh);
    }
    if (ballot(bad_shift) && l == 0) set_flag(flags, NNP_FLAG_SHIFT);
    finish_row(i, count, r_col, r_sh, row_count, stage_col, stage_sh, flags);
}

// One wave per row: the row's pairs are found once, rank-sorted by
// neighbour index in LDS and written to a fixed-stride staging row
// (stage_col / stage_sh at i * kRowLds) with their count; k_compact then
// copies the rows to their CSR offsets.  A row longer than kRowLds raises
// NNP_FLAG_ROW and is left empty.  Candidates come from the atom's stencil
// cells (periodic) or its structure (free), each read from global memory.
__global__ __launch_bounds__(kRowsPerBlock* kWave) void k_rows(
    const float* pos, int n, const int32_t* mol, int n_mol, const Grid g, double r2, const int32_t* cell_of,
    const int32_t* cell_start, const int32_t* cell_atoms, const int32_t* mol_start, const int32_t* mol_end,
    int32_t* row_count, int32_t* stage_col, int32_t* stage_sh, unsigned* flags, const int32_t* gate) {
    if (gate && *gate == 0) return;
    __shared__ int s_off[kRowsPerBlock][28];
    __shared__ int s_beg[kRowsPerBlock][28];
    __shared__ __attribute__((aligned(16))) int s_col[kRowsPerBlock][kRowLds];
    __shared__ int s_sh[kRowsPerBlock][kRowLds];
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);   // wave-uniform: the row is a scalar
    const int l = lane_id();
    const int i = blockIdx.x * kRowsPerBlock + w;
    if (i >= n) return;
    const float3 xi = load_pos(pos, i);
    const int mi = mol ? mol[i] : 0;
    const float rf = (float)sqrt(r2);
    int n_src = 0;
    if (g.periodic) {
        const int ci = cell_of[i];
        if (ci < 0) {
            if (l == 0) row_count[i] = 0;
            return;
        }
        n_src = stencil_sources(g, ci, cell_start, s_off[w], s_beg[w]);
    } else {
        n_src = 1;
        if (l == 0) {
            int b = 0, e = n;
            if (mol) {
                if (mi >= 0 && mi < n_mol) {
                    b = mol_start[mi];
                    e = mol_end[mi];
                } else {
                    b = e = 0;
                }
            }
            s_off[w][0] = 0;
            s_beg[w][0] = b;
            s_off[w][1] = e > b ? e - b : 0;
        }
    }
    wave_sync();
    const int total = s_off[w][n_src];
    const int* off = s_off[w];
    const int* beg = s_beg[w];
    auto fetch = [&](int t, int& j, float3& xj) {
        const int idx = cand_slot(off, beg, n_src, t);
        j = g.periodic ? cell_atoms[idx] : idx;
        if (j == i || (mol && mol[j] != mi)) return false;
        xj = load_pos(pos, j);
        return true;
    };
    build_row(i, xi, total, fetch, g, r2, rf, s_col[w], s_sh[w], row_count, stage_col, stage_sh, flags);
}

// The same rows for a periodic system without structure ids, one block of
// W waves per cell: the block stages the positions of its stencil's atoms
// in LDS once, and its waves build the rows of the cell's atoms from there
// (each atom's position is read once per stencil it belongs to, not once
// per neighbour search that visits it).  A stencil of more than
// cell_cand(W) atoms is read from global memory per row instead.  Every
// block also empties the rows of its share of the atoms outside every cell
// (non-finite coordinates).  Large boxes take 8 waves per cell (about 20
// rows: 2-3 each), small ones 16, so that the launch still has many waves.
constexpr int kCellBlocksForW8 = 1024;
__host__ __device__ constexpr int cell_cand(int W) { return W == 16 ? 960 : 1024; }
template <int W>
__global__ __launch_bounds__(W* kWave) void k_rows_cells(
    const float* pos, int n, int n_cells, const Grid g, double r2, const int32_t* cell_of, const int32_t* cell_start,
    const int32_t* cell_atoms, int32_t* row_count, int32_t* stage_col, int32_t* stage_sh, unsigned* flags,
    const int32_t* gate) {
    if (gate && *gate == 0) return;
    constexpr int kCand = cell_cand(W);
    __shared__ int s_off[28];
    __shared__ int s_beg[28];
    __shared__ int s_mbits;
    __shared__ int s_outside;
    // staged atoms: position and index; with three or more cells along every
    // dimension the index moves to s_xs, beside the position shifted by the
    // stencil cell's image, and s_x holds that packed shift in its place
    __shared__ float4 s_x[kCand];
    __shared__ float4 s_xs[kCand];
    __shared__ __attribute__((aligned(16))) int s_col[W][kRowLds];
    __shared__ int s_sh[W][kRowLds];
    const int c = blockIdx.x;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    {
        const int per = (n + n_cells - 1) / n_cells;
        const int a1 = min(n, (c + 1) * per);
        for (int a = c * per + (int)threadIdx.x; a < a1; a += W * kWave)
            if (cell_of[a] < 0) row_count[a] = 0;
    }
    const int h0 = cell_start[c], h1 = cell_start[c + 1];
    if (h1 <= h0) return;
    int n_src = 0;
    if (w == 0) n_src = stencil_sources(g, c, cell_start, s_off, s_beg);
    if (threadIdx.x == 0) {
        s_mbits = 0;
        s_outside = 0;
    }
    __syncthreads();
    n_src = g.ns[0] * g.ns[1] * g.ns[2];
    const int total = s_off[n_src];
    const float rf = (float)sqrt(r2);
    if (total <= kCand) {
        // the staged atoms include the cell's own (its cell is in the stencil);
        // with three or more cells along every dimension each also gets the
        // image shift of its stencil cell: source k = 9 a + 3 b + c is cell
        // (cx + a - 1, cy + b - 1, cz + c - 1) wrapped, and an atom of a cell
        // wrapped up by the box (index -1 -> nc - 1) is shifted down by L
        const bool cells3 = g.nc[0] >= 3 && g.nc[1] >= 3 && g.nc[2] >= 3;
        const int ccz = c % g.nc[2], ccy = (c / g.nc[2]) % g.nc[1], ccx = c / (g.nc[2] * g.nc[1]);
        float mx = 0.f;
        bool outside = false;
        for (int t = threadIdx.x; t < total; t += W * kWave) {
            int k;
            const int j = cell_atoms[cand_slot(s_off, s_beg, n_src, t, k)];
            const float3 x = load_pos(pos, j);
            mx = fmaxf(mx, fmaxf(fabsf(x.x), fmaxf(fabsf(x.y), fabsf(x.z))));
            outside |= !(x.x >= 0.f && x.x < g.Lf[0] && x.y >= 0.f && x.y < g.Lf[1] && x.z >= 0.f && x.z < g.Lf[2]);
            if (!cells3) s_x[t] = make_float4(x.x, x.y, x.z, __int_as_float(j));
            if (cells3) {
                const int ox = ccx + k / 9 - 1, oy = ccy + (k / 3) % 3 - 1, oz = ccz + k % 3 - 1;
                const int nx = ox < 0 ? -1 : (ox >= g.nc[0] ? 1 : 0);
                const int ny = oy < 0 ? -1 : (oy >= g.nc[1] ? 1 : 0);
                const int nz = oz < 0 ? -1 : (oz >= g.nc[2] ? 1 : 0);
                const int sh = (nx & 0xff) | ((ny & 0xff) << 8) | ((nz & 0xff) << 16);
                s_x[t] = make_float4(x.x, x.y, x.z, __int_as_float(sh));
                s_xs[t] = make_float4(x.x + (float)nx * g.Lf[0], x.y + (float)ny * g.Lf[1], x.z + (float)nz * g.Lf[2],
                                      __int_as_float(j));
            }
        }
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) mx = fmaxf(mx, shfl_xor(mx, d));
        if (lane_id() == 0) atomicMax(&s_mbits, __float_as_int(mx));   // non-negative floats order as their bits
        if (ballot(outside) && lane_id() == 0) s_outside = 1;
        __syncthreads();
        float M = fmaxf(1.f, __int_as_float(s_mbits));
#pragma unroll
        for (int k = 0; k < 3; ++k) M = fmaxf(M, g.Lf[k]);
        const float e = 1e-5f * M, band = e * (2.0f * rf + e), r2f = rf * rf;
        // positions outside the box (not wrapped): the rows take the minimum
        // image pair by pair from the unshifted positions
        const bool shifted = cells3 && !s_outside;   // block-uniform
        for (int r = h0 + w; r < h1; r += W) {
            const int i = cell_atoms[r];
            const float3 xi = load_pos(pos, i);
            if (shifted)
                build_row_shifted(i, xi, total, s_x, s_xs, g, r2, r2f - band, r2f + band, s_col[w], s_sh[w],
                                  row_count, stage_col, stage_sh, flags);
            else
                build_row_staged(i, xi, total, s_x, cells3 ? s_xs : s_x, g, r2, r2f - band, r2f + band, s_col[w],
                                 s_sh[w], row_count, stage_col, stage_sh, flags);
        }
    } else {
        for (int r = h0 + w; r < h1; r += W) {
            const int i = cell_atoms[r];
            const float3 xi = load_pos(pos, i);
            auto fetch = [&](int t, int& j, float3& xj) {
                j = cell_atoms[cand_slot(s_off, s_beg, n_src, t)];
                if (j == i) return false;
                xj = load_pos(pos, j);
                return true;
            };
            build_row(i, xi, total, fetch, g, r2, rf, s_col[w], s_sh[w], row_count, stage_col, stage_sh, flags);
        }
    }
}

// Staging rows -> CSR at row_ptr (only the first row_ptr[i+1] - row_ptr[i]
// entries: a row cut short by a capacity clamp stays in bounds), and the
// reverse index: rev[p] of i -> j is the position of i in j's sorted staging
// row.  An absent reverse (only a clamped or truncated list can lack one)
// points the pair at itself and raises NNP_FLAG_REVERSE.
__global__ __launch_bounds__(kRowsPerBlock* kWave) void k_compact(
    int n, const int32_t* __restrict__ row_count, const int32_t* __restrict__ stage_col,
    const int32_t* __restrict__ stage_sh, const int32_t* __restrict__ row_ptr, int32_t* __restrict__ col,
    int8_t* __restrict__ shift, int32_t* __restrict__ rev, const int32_t* gate, unsigned* flags) {
    if (gate && *gate == 0) return;
    const int w = threadIdx.x / kWave;
    const int l = lane_id();
    const int i = blockIdx.x * kRowsPerBlock + w;
    if (i >= n) return;
    const int b = row_ptr[i];
    const int lim = row_ptr[i + 1] - b;
    const int cnt = min(row_count[i], lim);
    const int32_t* sc = stage_col + (size_t)i * kRowLds;
    const int32_t* ss = stage_sh + (size_t)i * kRowLds;
    for (int e = l; e < cnt; e += kWave) {
        const int j = sc[e];
        const int sh = ss[e];
        const int p = b + e;
        col[p] = j;
        shift[3 * p + 0] = (int8_t)(sh & 0xff);
        shift[3 * p + 1] = (int8_t)((sh >> 8) & 0xff);
        shift[3 * p + 2] = (int8_t)((sh >> 16) & 0xff);
        const int32_t* rj = stage_col + (size_t)j * kRowLds;
        const int bj = row_ptr[j];
        const int cj = min(row_count[j], row_ptr[j + 1] - bj);
        int lo = 0, hi = cj;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (rj[mid] < i) lo = mid + 1; else hi = mid;
        }
        const bool found = lo < cj && rj[lo] == i;
        rev[p] = found ? bj + lo : p;
        if (!found) set_flag(flags, NNP_FLAG_REVERSE);
    }
}

__global__ void k_fill_gated(int32_t* p, long n, int32_t v, const int32_t* gate) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || (gate && *gate == 0)) return;
    p[i] = v;
}

// ---------------------------------------------------------------- MD front (small systems)
//
// One workgroup does, for every atom: the first part of the MD step
// (md_first_atom), the two largest displacements since the last list build, the
// rebuild decision, and on rebuild steps the wrap into the box, the new
// reference positions and the cell binning (counts in LDS, a block scan for
// the cell starts, the scatter).  It replaces five to seven launches of the
// general path for systems up to kFrontAtoms atoms and kFrontCells cells.
constexpr int kFrontThreads = 1024;
constexpr int kFrontAtoms = 8192;
constexpr int kFrontCells = 4096;
constexpr int kFrontPer = kFrontAtoms / kFrontThreads;
constexpr int kFrontBatch = 4;
static_assert(kFrontPer % kFrontBatch == 0, "whole batches of atoms per thread");

template <bool kLangevin>
__global__ __launch_bounds__(kFrontThreads) void k_md_front(
    int n, float* __restrict__ pos, float* __restrict__ vel, const float* __restrict__ F,
    const float* __restrict__ inv_mass, const MdStepConst c, uint64_t step, float* __restrict__ ref,
    const MdState* cur_st, MdState* nxt, int rebuild_every, float trig_len, const Grid g, int n_cells,
    int32_t* __restrict__ cell_of,
    int32_t* __restrict__ cell_start, int32_t* __restrict__ cell_atoms, unsigned* flags) {
    __shared__ int s_cnt[kFrontCells + 1];
    __shared__ float s_max[kFrontThreads / kWave][2];
    __shared__ int s_wsum[kFrontThreads / kWave];
    __shared__ int s_gate;
    const int t = threadIdx.x, w = t / kWave, l = lane_id();
    MdState cur{};
    if (t == 0) cur = *cur_st;   // read now, used by the decision below
    float m1 = 0.f, m2 = 0.f;   // the two largest squared displacements
    float xs[kFrontPer][3];   // this thread's atoms after the half step (kept for the wrap and binning)
    // the atoms kFrontBatch at a time: every load of a batch before its first use
#pragma unroll
    for (int k0 = 0; k0 < kFrontPer; k0 += kFrontBatch) {
        MdAtomIn in[kFrontBatch];
#pragma unroll
        for (int u = 0; u < kFrontBatch; ++u) {
            const int a = t + (k0 + u) * kFrontThreads;
            if (a < n) in[u] = md_first_load(a, pos, vel, F, inv_mass, ref);
        }
#pragma unroll
        for (int u = 0; u < kFrontBatch; ++u) {
            const int a = t + (k0 + u) * kFrontThreads;
            if (a < n) top2_add(m1, m2, md_first_finish<kLangevin>(a, in[u], pos, vel, c, step, xs[k0 + u]));
        }
    }
    top2_wave(m1, m2);
    if (l == 0) {
        s_max[w][0] = m1;
        s_max[w][1] = m2;
    }
    __syncthreads();
    if (t == 0) {
        for (int q = 1; q < kFrontThreads / kWave; ++q) top2_merge(m1, m2, s_max[q][0], s_max[q][1]);
        s_gate = md_decide(nxt, cur, m1, m2, rebuild_every, trig_len);
    }
    __syncthreads();
    if (!s_gate) return;
    if (g.periodic)
        for (int q = t; q <= n_cells; q += kFrontThreads) s_cnt[q] = 0;
    __syncthreads();
    int my_cell[kFrontPer], my_slot[kFrontPer];
#pragma unroll
    for (int k = 0; k < kFrontPer; ++k) {
        const int a = t + k * kFrontThreads;
        my_cell[k] = -1;
        my_slot[k] = 0;
        if (a >= n) continue;
        float x[3];
        bool fin = true;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            float v = xs[k][d];
            fin = fin && isfinite(v);
            if (g.periodic && isfinite(v)) {
                const float L = g.Lf[d];
                if (v < 0.f || v >= L) {   // inside the box floor(v / L) is 0: v stays
                    v -= L * floorf(v / L);
                    if (v >= L) v -= L;
                    if (v < 0.f) v = 0.f;
                }
                pos[3 * a + d] = v;
            }
            ref[3 * a + d] = v;
            x[d] = v;
        }
        if (!fin) {
            set_flag(flags, NNP_FLAG_NONFINITE);
            if (g.periodic) cell_of[a] = -1;
            continue;
        }
        if (g.periodic) {
            const int cx = cell_coord(x[0], g.L[0], g.inv_cs[0], g.nc[0]);
            const int cy = cell_coord(x[1], g.L[1], g.inv_cs[1], g.nc[1]);
            const int cz = cell_coord(x[2], g.L[2], g.inv_cs[2], g.nc[2]);
            const int cc = (cx * g.nc[1] + cy) * g.nc[2] + cz;
            my_cell[k] = cc;
            my_slot[k] = atomicAdd(&s_cnt[cc], 1);
            cell_of[a] = cc;
        }
    }
    if (!g.periodic) return;
    __syncthreads();
    // exclusive scan of the cell counts: each thread owns a contiguous run of cells
    const int per = (n_cells + kFrontThreads - 1) / kFrontThreads;
    const int c0 = t * per, c1 = min(n_cells, c0 + per);
    int run = 0;
    for (int q = c0; q < c1; ++q) run += s_cnt[q];
    int inc = run;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const int u = __shfl_up(inc, d, kWave);
        if (l >= d) inc += u;
    }
    if (l == kWave - 1) s_wsum[w] = inc;
    __syncthreads();
    int off = 0;
    for (int q = 0; q < w; ++q) off += s_wsum[q];
    int ex = off + inc - run;
    __syncthreads();
    for (int q = c0; q < c1; ++q) {
        const int cnt = s_cnt[q];
        s_cnt[q] = ex;
        cell_start[q] = ex;
        ex += cnt;
    }
    if (t == kFrontThreads - 1) {
        int tot = 0;
        for (int q = 0; q < kFrontThreads / kWave; ++q) tot += s_wsum[q];
        cell_start[n_cells] = tot;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kFrontPer; ++k) {
        const int a = t + k * kFrontThreads;
        if (a < n && my_cell[k] >= 0) cell_atoms[s_cnt[my_cell[k]] + my_slot[k]] = a;
    }
}

struct WsLayout {
    size_t cell_count, cell_start, cell_of, cell_slot, cell_atoms, row_count, stage_col, stage_sh, mol_start,
        mol_end, scan_tmp, totals, end;
};

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

WsLayout ws_layout(int n, int n_mol, long n_cells) {
    WsLayout L;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o = align256(o + bytes); return r; };
    const int nn = n > 0 ? n : 1;
    L.cell_count = take(sizeof(int32_t) * (n_cells + 1));
    L.cell_start = take(sizeof(int32_t) * (n_cells + 1));
    L.cell_of = take(sizeof(int32_t) * nn);
    L.cell_slot = take(sizeof(int32_t) * nn);
    L.cell_atoms = take(sizeof(int32_t) * nn);
    L.row_count = take(sizeof(int32_t) * nn);
    L.stage_col = take(sizeof(int32_t) * (size_t)nn * kRowLds);
    L.stage_sh = take(sizeof(int32_t) * (size_t)nn * kRowLds);
    L.mol_start = take(sizeof(int32_t) * (n_mol > 0 ? n_mol : 1));
    L.mol_end = take(sizeof(int32_t) * (n_mol > 0 ? n_mol : 1));
    const long sn = n_cells > nn ? n_cells : nn;
    L.scan_tmp = take(sizeof(int64_t) * scan_tmp_elems((int)sn));
    L.totals = take(sizeof(int64_t) * 4);
    L.end = o;
    return L;
}

nnp_status make_grid(const float* box_host, float r_list, Grid* g) {
    g->periodic = box_host != nullptr;
    for (int k = 0; k < 3; ++k) {
        g->nc[k] = 1;
        g->ns[k] = 1;
        g->L[k] = 1.0;
        g->inv_cs[k] = 0.0;
        g->Lf[k] = 1.0f;
        g->inv_Lf[k] = 1.0f;
    }
    if (!box_host) return NNP_OK;
    const double r = (double)r_list;
    for (int k = 0; k < 3; ++k) {
        const double L = (double)box_host[k];
        if (!(L > 0.0) || !std::isfinite(L)) return NNP_E_ARG;
        if (L < 2.0 * r) return NNP_E_BOX;
        long nc = (long)std::floor(L / (r * (1.0 + 1e-9)));
        if (nc < 1) nc = 1;
        if (nc > kMaxCellsPerDim) nc = kMaxCellsPerDim;
        g->nc[k] = (int)nc;
        g->ns[k] = nc >= 3 ? 3 : (int)nc;
        g->L[k] = L;
        g->inv_cs[k] = (double)nc / L;
        g->Lf[k] = box_host[k];
        g->inv_Lf[k] = (float)(1.0 / L);
    }
    return NNP_OK;
}

}  // namespace

nnp_status neighbors_mol_ranges(void* ws, int32_t n, int32_t n_mol, const float* box_host, float r_list,
                                int32_t** start, int32_t** end) {
    Grid g;
    const nnp_status st = make_grid(box_host, r_list, &g);
    if (st != NNP_OK) return st;
    const long n_cells = g.periodic ? (long)g.nc[0] * g.nc[1] * g.nc[2] : 1;
    const WsLayout L = ws_layout(n, n_mol, n_cells);
    *start = (int32_t*)((char*)ws + L.mol_start);
    *end = (int32_t*)((char*)ws + L.mol_end);
    return NNP_OK;
}

bool md_front_fuses(int n, const float* box_host, float r_list) {
    Grid g;
    if (make_grid(box_host, r_list, &g) != NNP_OK) return false;
    return n > 0 && g.periodic && (long)g.nc[0] * g.nc[1] * g.nc[2] <= kBinScanCells;
}

bool md_front_fits(int n, const float* box_host, float r_list) {
    Grid g;
    if (make_grid(box_host, r_list, &g) != NNP_OK) return false;
    const long n_cells = g.periodic ? (long)g.nc[0] * g.nc[1] * g.nc[2] : 1;
    return n > 0 && n <= kFrontAtoms && n_cells <= kFrontCells;
}

nnp_status launch_md_front(int n, float* pos, float* vel, const float* F, const float* inv_mass, const MdStepConst& c,
                           uint64_t step, float* ref, const MdState* cur, MdState* nxt, int rebuild_every,
                           float trig_len, bool langevin, const float* box_host, float r_list, void* ws,
                           size_t ws_bytes, unsigned* flags, hipStream_t s) {
    Grid g;
    nnp_status stt = make_grid(box_host, r_list, &g);
    if (stt != NNP_OK) return stt;
    const long n_cells = g.periodic ? (long)g.nc[0] * g.nc[1] * g.nc[2] : 1;
    if (n <= 0 || n > kFrontAtoms || n_cells > kFrontCells) return NNP_E_ARG;
    const WsLayout L = ws_layout(n, 1, n_cells);
    if (!ws || ws_bytes < L.end) return NNP_E_ARG;
    char* base = (char*)ws;
    int32_t* cell_of = (int32_t*)(base + L.cell_of);
    int32_t* cell_start = (int32_t*)(base + L.cell_start);
    int32_t* cell_atoms = (int32_t*)(base + L.cell_atoms);
    if (langevin)
        k_md_front<true><<<1, kFrontThreads, 0, s>>>(n, pos, vel, F, inv_mass, c, step, ref, cur, nxt,
                                                     rebuild_every, trig_len, g, (int)n_cells, cell_of, cell_start,
                                                     cell_atoms, flags);
    else
        k_md_front<false><<<1, kFrontThreads, 0, s>>>(n, pos, vel, F, inv_mass, c, step, ref, cur, nxt,
                                                      rebuild_every, trig_len, g, (int)n_cells, cell_of, cell_start,
                                                      cell_atoms, flags);
    return hipGetLastError() == hipSuccess ? NNP_OK : NNP_E_HIP;
}

size_t neighbors_ws_bytes(int32_t n_atoms, int32_t n_mol, const float* box_host, float r_list) {
    Grid g;
    if (make_grid(box_host, r_list, &g) != NNP_OK) return 0;
    const long n_cells = g.periodic ? (long)g.nc[0] * g.nc[1] * g.nc[2] : 1;
    return ws_layout(n_atoms, n_mol, n_cells).end;
}

nnp_status read_and_clear_flags(nnp_model* m, hipStream_t s, uint32_t* out, int64_t* total_dev,
                                int64_t* total_host);

nnp_status build_neighbors(nnp_model* model, int32_t n, const float* pos, const int32_t* mol, int32_t n_mol,
                           const float* box_host, float r_list, nnp_nlist* nl, int64_t* n_pairs_host,
                           void* ws, size_t ws_bytes, hipStream_t s, bool sync, unsigned* flags_override,
                           const int32_t* gate, int64_t* need_pairs, bool cells_ready, RowsView* rows_out,
                           const MdFront* front) {
    Grid g;
    nnp_status st = make_grid(box_host, r_list, &g);
    if (st != NNP_OK) return st;
    const long n_cells = g.periodic ? (long)g.nc[0] * g.nc[1] * g.nc[2] : 1;
    // the MD front rides on the one-kernel binning of a gated build
    if (front && !(gate && g.periodic && !mol && !cells_ready && n > 0 && n_cells <= kBinScanCells))
        return NNP_E_ARG;
    const WsLayout L = ws_layout(n, n_mol, n_cells);
    if (!ws || ws_bytes < L.end) return NNP_E_ARG;
    char* base = (char*)ws;
    int32_t* cell_count = (int32_t*)(base + L.cell_count);
    int32_t* cell_start = (int32_t*)(base + L.cell_start);
    int32_t* cell_of = (int32_t*)(base + L.cell_of);
    int32_t* cell_slot = (int32_t*)(base + L.cell_slot);
    int32_t* cell_atoms = (int32_t*)(base + L.cell_atoms);
    int32_t* row_count = (int32_t*)(base + L.row_count);
    int32_t* stage_col = (int32_t*)(base + L.stage_col);
    int32_t* stage_sh = (int32_t*)(base + L.stage_sh);
    int32_t* mol_start = (int32_t*)(base + L.mol_start);
    int32_t* mol_end = (int32_t*)(base + L.mol_end);
    int64_t* scan_tmp = (int64_t*)(base + L.scan_tmp);
    int64_t* totals = (int64_t*)(base + L.totals);
    unsigned* flags = flags_override ? flags_override : model->flags;
    const double rl = (double)r_list;
    const double r2 = rl * rl;
    const int tb = 256;
    const int nb = ceil_div(n > 0 ? n : 1, tb);

    hipError_t he = hipSuccess;
    auto chk = [&](hipError_t x) { if (he == hipSuccess) he = x; };
    auto fill = [&](int32_t* p, long cnt) {
        if (cnt > 0) k_fill_gated<<<(int)((cnt + 255) / 256), 256, 0, s>>>(p, cnt, 0, gate);
    };
    prof_begin(model, NNP_STAGE_NEIGHBORS, s);
    if (n > 0) {
        // open systems check their coordinates here (periodic ones in the binning)
        bool finite_checked = false;
        if (mol) {
            if (n <= kMolSmall && n_mol <= kMolSmall) {
                finite_checked = !g.periodic && !cells_ready;
                k_mol_ranges_small<<<1, 1024, 0, s>>>(mol, n, n_mol, mol_start, mol_end, flags, gate,
                                                      finite_checked ? pos : nullptr);
            } else {
                fill(mol_start, n_mol);
                fill(mol_end, n_mol);
                k_mol_ranges<<<nb, tb, 0, s>>>(mol, n, n_mol, mol_start, mol_end, flags, gate);
            }
        }
        if (cells_ready) {
            // binned (and checked for finite coordinates) by the caller's front kernel
        } else if (g.periodic) {
            // up to kBinScanCells cells: binning and scan in one kernel, which
            // leaves the counts and its ticket zero, so that gated builds (the
            // MD engine's, always on the same workspace after an ungated
            // first build) skip the zero fill
            unsigned* ticket = (unsigned*)(totals + 2);
            const bool fused = n_cells <= kBinScanCells;
            if (!gate || !fused) fill(cell_count, n_cells + 1);
            if (fused) {
                if (!gate) fill((int32_t*)ticket, 1);
                if (front)
                    k_bin_scan<true><<<ceil_div(n, kBinScanThreads), kBinScanThreads, 0, s>>>(
                        pos, n, g, (int)n_cells, cell_of, cell_slot, cell_count, cell_start, totals + 1, ticket,
                        flags, gate, *front);
                else
                    k_bin_scan<false><<<ceil_div(n, kBinScanThreads), kBinScanThreads, 0, s>>>(
                        pos, n, g, (int)n_cells, cell_of, cell_slot, cell_count, cell_start, totals + 1, ticket,
                        flags, gate, MdFront{});
            } else {
                k_bin<<<nb, tb, 0, s>>>(pos, n, g, cell_of, cell_slot, cell_count, flags, gate);
                chk(launch_exclusive_scan_i32(cell_count, cell_start, totals + 1, (int)n_cells, scan_tmp, s, gate));
            }
            k_scatter<<<nb, tb, 0, s>>>(n, cell_of, cell_slot, cell_start, cell_atoms, gate);
        } else if (!finite_checked) {
            k_finite<<<nb, tb, 0, s>>>(pos, n, flags, gate);
        }
        if (g.periodic && !mol) {
            if (n_cells >= kCellBlocksForW8)
                k_rows_cells<8><<<(int)n_cells, 8 * kWave, 0, s>>>(pos, n, (int)n_cells, g, r2, cell_of, cell_start,
                                                                    cell_atoms, row_count, stage_col, stage_sh, flags,
                                                                    gate);
            else
                k_rows_cells<16><<<(int)n_cells, 16 * kWave, 0, s>>>(pos, n, (int)n_cells, g, r2, cell_of,
                                                                      cell_start, cell_atoms, row_count, stage_col,
                                                                      stage_sh, flags, gate);
        } else {
            k_rows<<<ceil_div(n, kRowsPerBlock), kRowsPerBlock * kWave, 0, s>>>(
                pos, n, mol, n_mol, g, r2, cell_of, cell_start, cell_atoms, mol_start, mol_end, row_count,
                stage_col, stage_sh, flags, gate);
        }
    }
    if (rows_out) {
        RowsView r{};
        r.count = row_count;
        r.col = stage_col;
        r.shift_packed = stage_sh;
        *rows_out = r;
        nl->n_atoms = n;
        nl->r_list = r_list;
        nl->n_pairs = -1;
        prof_end(model, NNP_STAGE_NEIGHBORS, s);
        chk(hipGetLastError());
        return he == hipSuccess ? NNP_OK : NNP_E_HIP;
    }
    // asynchronous builds: the row pointers are cut at the capacity if the list
    // is longer (every later read stays in bounds), and the overflow flagged
    const ScanClamp clamp{nl->capacity, need_pairs, flags};
    chk(launch_exclusive_scan_i32(row_count, nl->row_ptr, totals, n, scan_tmp, s, gate, sync ? nullptr : &clamp));
    chk(hipGetLastError());
    if (he != hipSuccess) {
        prof_end(model, NNP_STAGE_NEIGHBORS, s);
        return NNP_E_HIP;
    }
    int64_t total = 0;
    uint32_t fl = 0;
    if (!sync) {
        // the pair count is not read back: a list longer than the capacity is cut
        // short in bounds and flagged (NNP_FLAG_CAPACITY) for the caller to check
        nl->n_atoms = n;
        nl->r_list = r_list;
        nl->n_pairs = -1;
        if (n > 0)
            k_compact<<<ceil_div(n, kRowsPerBlock), kRowsPerBlock * kWave, 0, s>>>(
                n, row_count, stage_col, stage_sh, nl->row_ptr, nl->col, nl->shift, nl->rev, gate, flags);
        prof_end(model, NNP_STAGE_NEIGHBORS, s);
        return hipGetLastError() == hipSuccess ? NNP_OK : NNP_E_HIP;
    }
    st = read_and_clear_flags(model, s, &fl, totals, &total);
    if (st != NNP_OK) {
        prof_end(model, NNP_STAGE_NEIGHBORS, s);
        return st;
    }
    if (n_pairs_host) *n_pairs_host = total;
    nl->n_atoms = n;
    nl->r_list = r_list;
    nl->n_pairs = total;
    if (fl || total > nl->capacity || total > 0x7fffffffLL) prof_end(model, NNP_STAGE_NEIGHBORS, s);
    if (fl) {
        if (fl & NNP_FLAG_NONFINITE) return NNP_E_NONFINITE;
        if (fl & NNP_FLAG_ROW) return NNP_E_ROW;
        return NNP_E_ARG;
    }
    if (total > nl->capacity || total > 0x7fffffffLL) return NNP_E_CAPACITY;
    if (n > 0 && total > 0)
        k_compact<<<ceil_div(n, kRowsPerBlock), kRowsPerBlock * kWave, 0, s>>>(
            n, row_count, stage_col, stage_sh, nl->row_ptr, nl->col, nl->shift, nl->rev, nullptr, flags);
    prof_end(model, NNP_STAGE_NEIGHBORS, s);
    return hipGetLastError() == hipSuccess ? NNP_OK : NNP_E_HIP;
}

}  // namespace nnp
