// Fused species network: forward, head and adjoint of the
// 1008-256-192-160-1 CELU network (Sec. 2.2, "Neural Networks"; Sec. 2.4)
// for one tile of TM same-species atoms in a single kernel.
//
//   h1 = CELU(W1 a + b1), h2 = CELU(W2 h1 + b2), h3 = CELU(W3 h2 + b3)
//   E  = w4 . h3 + b4
//   d3 = w4 * CELU'(h3), d2 = (W3^T d3) * CELU'(h2), d1 = (W2^T d2) * CELU'(h1)
//   dE/da = W1^T d1
//
// Four waves split every layer's output columns (64 / 48 / 48 per wave; the
// 160-wide layer is padded to 192 with zero weights).  Each wave keeps its
// h1 and h2 columns in registers (MFMA accumulator layout) for the CELU'
// epilogues of the adjoint, which produces exactly the same columns.  The A
// operand of every GEMM is the previous layer's output, staged in one LDS
// tile (float32 for the FP32 form, bfloat16 for the BF16 form, where the
// GEMM inputs are bf16 by definition); the first layer streams the AEV tile
// through a double-buffered part of the same LDS.  B operands (weights) are
// pre-packed per species in MFMA fragment order, so a lane fetches its
// fragment with one 16-byte load; each wave reads only its own columns.
//   FP32 form: v_mfma_f32_16x16x4_f32   (a 16-byte B load covers 4 k-steps)
//   BF16 form: v_mfma_f32_16x16x32_bf16 (float32 accumulation)
// Only the AEV tile is read from and dE/dAEV written to HBM; activations
// never leave the CU.
#include <cstring>
#include <type_traits>

#include "nnp_internal.hpp"

namespace nnp {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
// Weight packs are read through global-address-space pointers: their
// addresses come from a table in memory, and as generic (flat) pointers the
// loads would also count against the LDS wait counter, so every wait for an
// LDS read would wait for the prefetched weights as well.
typedef __attribute__((address_space(1))) const f32x4 gfloat4;
typedef __attribute__((address_space(1))) const float gfloat;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef __attribute__((address_space(1))) const u16x8 gu16x8;

constexpr int K0 = 1024, N1 = 256, N2 = 192, N3 = 192;
constexpr int kThreads = 256;


template <bool BF>
struct Cfg;
template <>
struct Cfg<false> {                 // FP32
    typedef float act_t;
    static constexpr int kStep = 4;     // k per MFMA
    static constexpr int kLd = N1 + 4;  // act row stride (elements)
    static constexpr int kChunk = 64;   // layer-1 K chunk (32 for tiles above 16 rows)
    static constexpr int kPad = 4;      // chunk row padding
};
template <>
struct Cfg<true> {                  // BF16
    typedef uint16_t act_t;
    static constexpr int kStep = 32;
    static constexpr int kLd = N1 + 8;
    static constexpr int kChunk = 256;
    static constexpr int kPad = 8;
};

// CELU and its derivative from the output, h > 0 ? 1 : 1 + h / alpha (ia =
// 1 / alpha); both sides are evaluated and one selected, so the epilogues
// run without divergent branches
__device__ __forceinline__ float celu(float v, float alpha, float ia) {
    const float neg = alpha * (__expf(fminf(v, 0.f) * ia) - 1.f);
    return v > 0.f ? v : neg;
}
__device__ __forceinline__ float celu_grad_from_h(float h, float ia) { return h > 0.f ? 1.f : fmaf(h, ia, 1.f); }

// B fragments of one k-step (FP32: 16 k, four MFMA k-steps; BF16: 32 k)
template <bool BF>
struct Frag;
template <>
struct Frag<false> {
    typedef f32x4 reg_t;
    typedef gfloat4 mem_t;
    static constexpr int kK = 16;
};
template <>
struct Frag<true> {
    typedef u16x8 reg_t;
    typedef gu16x8 mem_t;
    static constexpr int kK = 32;
};

// A fragments of one k-step, one 16-byte LDS read per 16-row block: FP32,
// the four values a lane feeds the four 16x16x4 MFMAs of the step (features
// 16 kq + 4 (l / 16) .. + 3; the packed weights use the same order within the
// step); BF16, the eight values of one 16x16x32 MFMA.
template <bool BF>
struct AFrag;
template <>
struct AFrag<false> {
    typedef f32x4 type;
};
template <>
struct AFrag<true> {
    typedef bf16x8 type;
};

template <bool BF, int MB>
__device__ __forceinline__ void load_a(const typename Cfg<BF>::act_t* act, int ld, int kq,
                                       typename AFrag<BF>::type (&a)[MB]) {
    const int l = lane_id();
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
        if (!BF)
            a[mb] = *(const typename AFrag<BF>::type*)((const float*)act + (16 * mb + (l & 15)) * ld + 16 * kq +
                                                       4 * (l >> 4));
        else
            a[mb] = *(const typename AFrag<BF>::type*)((const uint16_t*)act + (16 * mb + (l & 15)) * ld + 32 * kq +
                                                       8 * (l >> 4));
    }
}

// The MFMAs of one k-step: acc[mb][nb] += A[16 mb.., step] B[step, nb] from
// the A fragments and B fragments given.
template <bool BF, int MB, int NCB>
__device__ __forceinline__ void mfma_kstep(const typename AFrag<BF>::type (&a)[MB],
                                           const typename Frag<BF>::reg_t (&b)[NCB], f32x4 (&acc)[MB][NCB]) {
    if (!BF) {
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) {
                const f32x4 av = __builtin_bit_cast(f32x4, a[mb]);
#pragma unroll
                for (int nb = 0; nb < NCB; ++nb) {
                    const f32x4 bq = __builtin_bit_cast(f32x4, b[nb]);
                    acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[j], bq[j], acc[mb][nb], 0, 0, 0);
                }
            }
    } else {
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int nb = 0; nb < NCB; ++nb)
                acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a[mb]),
                                                                      __builtin_bit_cast(bf16x8, b[nb]),
                                                                      acc[mb][nb], 0, 0, 0);
    }
}

// Ring of B-fragment registers for k-steps whose count is a multiple of the
// ring size: k-step t lives in slot t % RS and is loaded two k-steps ahead.
// The slots are indexed at compile time (the k loop is unrolled by RS), so
// no register moves tie a k-step to the completion of later loads.
template <int NK>
constexpr int ring_slots() { return NK % 3 == 0 ? 3 : 4; }

// The B-fragment ring of one product C[TM x (NCB*16 columns of this wave)] =
// A[TM x K] (LDS, stride ld) * B (packed, global); start() issues the loads
// of the first two k-steps, so that a caller can put them ahead of the
// epilogue and barrier that precede the product (the barrier waits only for
// LDS operations, not for these loads).
// FP32 pack: [nb][K/16][64 lanes][4]   BF16 pack: [nb][K/32][64 lanes][8]
// nbl (optional): the NCB output column blocks, in place of nb0 .. nb0 + NCB - 1
// (a negative entry reads block 0; its columns are discarded by the caller)
template <bool BF, int NCB, int K>
struct BPipe {
    typedef typename Frag<BF>::reg_t reg_t;
    typedef typename Frag<BF>::mem_t mem_t;
    static constexpr int NK = K / Frag<BF>::kK;
    static constexpr int RS = ring_slots<NK>();
    static_assert(NK % RS == 0 && NK >= 2, "k-steps must fill whole rings");
    reg_t rb[RS][NCB];
    int blk[NCB];
    const mem_t* B;
    __device__ __forceinline__ void start(const void* Bpack, int nb0, const int* nbl = nullptr) {
        const int l = lane_id();
        B = (const mem_t*)Bpack;
#pragma unroll
        for (int nb = 0; nb < NCB; ++nb) blk[nb] = nbl ? max(nbl[nb], 0) : nb0 + nb;
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int nb = 0; nb < NCB; ++nb) rb[t][nb] = B[((size_t)blk[nb] * NK + t) * 64 + l];
    }
};

// The product of a started ring: acc (+)= A * B over the K rows.
template <bool BF, int MB, int NCB, int K, bool kZero = true>
__device__ __forceinline__ void gemm_run(const typename Cfg<BF>::act_t* act, int ld, BPipe<BF, NCB, K>& p,
                                         f32x4 (&acc)[MB][NCB]) {
    constexpr int NK = BPipe<BF, NCB, K>::NK, RS = BPipe<BF, NCB, K>::RS;
    const int l = lane_id();
    if (kZero) {
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int nb = 0; nb < NCB; ++nb) acc[mb][nb] = (f32x4){0.f, 0.f, 0.f, 0.f};
    }
    // FP32 with up to two 16-row blocks: the A fragments one k-step ahead,
    // in a ring indexed like the B ring (slot indices known at compile time;
    // two slots live at a time).  BF16, and four row blocks, read theirs at
    // the step among its MFMAs: their ring would cost the registers of a
    // wave per SIMD (BF16, 32 rows: 180 against 168 VGPRs, two waves per
    // SIMD instead of three) or spill (64 rows)
    constexpr bool kAhead = !BF && MB <= 2;
    typename AFrag<BF>::type a[kAhead ? RS : 1][MB];
    if (kAhead) load_a<BF, MB>(act, ld, 0, a[0]);
    for (int k0 = 0; k0 < NK; k0 += RS) {
#pragma unroll
        for (int u = 0; u < RS; ++u) {
            const int kq = k0 + u;
            if (kq + 2 < NK) {
#pragma unroll
                for (int nb = 0; nb < NCB; ++nb)
                    p.rb[(u + 2) % RS][nb] = p.B[((size_t)p.blk[nb] * NK + kq + 2) * 64 + l];
            }
            if (kAhead && kq + 1 < NK) load_a<BF, MB>(act, ld, kq + 1, a[kAhead ? (u + 1) % RS : 0]);
            __builtin_amdgcn_sched_barrier(0);   // keep the prefetches ahead of this step's MFMAs
            if (!kAhead) load_a<BF, MB>(act, ld, kq, a[0]);
            mfma_kstep<BF, MB, NCB>(a[kAhead ? u : 0], p.rb[u], acc);
        }
    }
}

template <bool BF, int MB, int NCB, int K, bool kZero = true>
__device__ __forceinline__ void gemm_act(const typename Cfg<BF>::act_t* act, int ld, const void* Bpack, int nb0,
                                         f32x4 (&acc)[MB][NCB], const int* nbl = nullptr) {
    BPipe<BF, NCB, K> p;
    p.start(Bpack, nb0, nbl);
    gemm_run<BF, MB, NCB, K, kZero>(act, ld, p, acc);
}

template <bool BF>
__device__ __forceinline__ void put_act(typename Cfg<BF>::act_t* act, int idx, float v);
template <>
__device__ __forceinline__ void put_act<false>(float* act, int idx, float v) { act[idx] = v; }
template <>
__device__ __forceinline__ void put_act<true>(uint16_t* act, int idx, float v) { act[idx] = f32_to_bf16(v); }

}  // namespace

// One network's weights for every species (device table, one entry per network).
struct FusedNet {
    const void* Bf1[kMaxSpecies];   // forward packs
    const void* Bf2[kMaxSpecies];
    const void* Bf3[kMaxSpecies];
    const void* Ba3[kMaxSpecies];   // adjoint packs
    const void* Ba2[kMaxSpecies];
    const void* Ba1[kMaxSpecies];
    const float* b1[kMaxSpecies];
    const float* b2[kMaxSpecies];
    const float* b3[kMaxSpecies];
    const float* w4[kMaxSpecies];   // head weights, padded to N3
    float b4[kMaxSpecies];
};

namespace {

struct FusedArgs {
    const FusedNet* nets;            // [n_nets] (device)
    const int32_t* meta;
    const int32_t* row_atom;
    const void* aev;                 // [rows][K0] float32 or bf16
    float* g_out;                    // [rows][K0] float32 or null
    float* E_row;                    // [rows]
    float* E_atomo;                  // [n] atom order or null
    float alpha;
    int ns;
    // ensemble front (kEns): per network, d1 = dE/dh1 [n_nets][rows][N1] (act type) and E [n_nets][rows]
    void* d1_out;
    float* E_net;
    int rows;
    // per atom, the species present in its environment (bits 0-7 radial,
    // 8-15 angular); null: every feature block may be non-zero
    const uint32_t* amask;
};

constexpr int kXcds = 8;   // accelerator complex dies of one MI355X, each with its own L2

// The tile of this block.  A launch's blocks are dealt to the XCDs in turn
// (block b runs on XCD b mod 8); each XCD takes a contiguous range of tiles,
// so that tiles of one species, which stream the same weight packs, share
// an XCD's L2 instead of every L2 holding every species' packs.  The grid
// (x) is padded to a multiple of 8 blocks; the map is a bijection of the
// padded range, and a block past the last tile exits.
__device__ __forceinline__ int xcd_tile(int n_tiles) {
    const int per = (n_tiles + kXcds - 1) / kXcds;
    return (int)(blockIdx.x % kXcds) * per + (int)(blockIdx.x / kXcds);
}

// The 16-feature blocks (bit b: features 16 b .. 16 b + 15) that some atom of
// the tile rows row0 .. row0 + TM - 1 can have non-zero: a species' radial
// block when the species occurs within Rc_R of the atom, the two blocks of a
// species pair's angular bin when both occur within Rc_A.  Every block
// without a mask.  Wave-level: every lane of the calling wave returns it.
template <int TM>
__device__ __forceinline__ unsigned long long tile_blocks(const FusedArgs& A, int row0) {
    if (!A.amask) return ~0ull;
    const int l = lane_id();
    unsigned m = 0;
    for (int r = l; r < TM; r += kWave) {
        const int a = A.row_atom[row0 + r];
        if (a >= 0) m |= A.amask[a];
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) m |= (unsigned)shfl_xor((int)m, d);
    unsigned long long bm = 0;
    const int ns = A.ns;
    for (int q = 0; q < ns; ++q)
        if ((m >> q) & 1u) bm |= 1ull << q;
    int p = 0;
    for (int q = 0; q < ns; ++q)
        for (int u = q; u < ns; ++u, ++p)
            if ((m >> (8 + q)) & (m >> (8 + u)) & 1u) bm |= 3ull << (ns + 2 * p);
    return bm;
}

// The set blocks of bm in ascending order into list[0 .. n), then -1 up to
// the next multiple of gran (<= 64); returns that padded count.  Wave-level.
__device__ __forceinline__ int block_list(unsigned long long bm, int* list, int gran) {
    const int l = lane_id();
    const bool on = (bm >> l) & 1ull;
    const unsigned long long b = ballot(on);
    const int n = __popcll(b), n_pad = (n + gran - 1) / gran * gran;
    if (on) list[rank_below(b)] = l;
    if (l >= n && l < n_pad) list[l] = -1;
    return n_pad;
}

// dE/dAEV of the tile rows row0 .. for the output blocks b (16 columns
// each; a negative block is padding and is not stored)
template <int MB, int NCB>
__device__ __forceinline__ void store_g(float* g, int row0, const f32x4 (&acc)[MB][NCB], const int (&b)[NCB]) {
    const int l = lane_id();
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int nb = 0; nb < NCB; ++nb) {
            if (b[nb] < 0) continue;
            const int col = 16 * b[nb] + (l & 15);
#pragma unroll
            for (int r = 0; r < 4; ++r) g[(size_t)(row0 + 16 * mb + 4 * (l >> 4) + r) * K0 + col] = acc[mb][nb][r];
        }
}

// kEns: network blockIdx.y of an ensemble; stops after d1 (the adjoint of the
// first layer sums over networks, k_ens_adj1) and writes this network's
// energies to E_net.
template <bool BF, int TM, bool kEns>
__global__ __launch_bounds__(kThreads, 2) void k_mlp_fused(const FusedArgs A) {
    typedef typename Cfg<BF>::act_t act_t;
    constexpr int MB = TM / 16;
    constexpr int LD = Cfg<BF>::kLd;
    // layer-1 chunk: FP32 tiles above 16 rows take 32 k (the 64-k chunk makes them spill)
    constexpr int CH = (!BF && TM > 16) ? 32 : Cfg<BF>::kChunk, CLD = CH + Cfg<BF>::kPad;
    constexpr int kActBytes = TM * LD * (int)sizeof(act_t);
    constexpr int kStageBytes = 2 * TM * CLD * (int)sizeof(act_t);
    constexpr int kLdsBytes = kActBytes > kStageBytes ? kActBytes : kStageBytes;
    __shared__ __attribute__((aligned(16))) char smem[kLdsBytes];
    __shared__ float epart[TM][4];
    act_t* act = (act_t*)smem;
    const int tile = xcd_tile((A.rows + TM - 1) / TM);
    const int row0 = tile * TM;
    const int32_t* meta = A.meta;
    if (row0 >= A.rows || row0 >= meta[8 + A.ns]) return;
    int s = 0;
    for (int q = 1; q < A.ns; ++q)
        if (meta[8 + q] <= row0) s = q;
    // skip tiles that hold only segment padding
    if (row0 >= meta[8 + s] + meta[s]) return;
    const int t = threadIdx.x, w = t / kWave, l = lane_id();
    const float alpha = A.alpha, ia = 1.f / alpha;
    const int net = kEns ? blockIdx.y : 0;
    // this network's and species' pointers, loaded once (the table is read-only)
    const FusedNet* __restrict__ tab = A.nets + net;
    const void* const pBf1 = tab->Bf1[s];
    const void* const pBf2 = tab->Bf2[s];
    const void* const pBf3 = tab->Bf3[s];
    const void* const pBa3 = tab->Ba3[s];
    const void* const pBa2 = tab->Ba2[s];
    const void* const pBa1 = tab->Ba1[s];
    const float* const pb1 = tab->b1[s];
    const float* const pb2 = tab->b2[s];
    const float* const pb3 = tab->b3[s];
    const float* const pw4 = tab->w4[s];
    const float hb4 = tab->b4[s];

    // ---------------- active feature blocks of the tile
    // A 16-feature block of the AEV (a species' radial shells, or half of a
    // species pair's angular bin) is zero for an atom whose environment lacks
    // that species.  The first layer runs only over the k-steps that hold a
    // block some atom of the tile can have non-zero, and its adjoint only
    // over those output blocks: the skipped products are exact zeros, and
    // dE/dAEV is consumed only where the features are non-zero.  Without a
    // mask every block is active.
    constexpr int KS = Frag<BF>::kK;                          // features per k-step
    constexpr int NT = K0 / KS, TPC = CH / KS;
    constexpr int RS = 4, PD = 2, CPR = TPC >= RS ? 1 : RS / TPC;
    static_assert((TPC >= RS ? TPC % RS : RS % TPC) == 0 && (K0 / CH) % CPR == 0, "chunks hold whole ring turns");
    constexpr int kGran = TPC * CPR;                          // k-step list granularity
    __shared__ int s_kq[NT];                                  // active k-steps, then -1 (zero) padding
    __shared__ int s_ob[64];                                  // active adjoint output blocks, then -1
    __shared__ int s_n[2];
    if (t < kWave) {
        const unsigned long long bm = tile_blocks<TM>(A, row0);
        // k-steps: a 16-feature step is a block, a 32-feature step a block pair
        unsigned long long km = bm;
        if (KS == 32) {
            km = 0;
            for (int j = 0; j < NT; ++j)
                if ((bm >> (2 * j)) & 3ull) km |= 1ull << j;
        }
        const int nk_pad = block_list(km, s_kq, kGran);
        const int no_pad = block_list(bm, s_ob, 8);
        if (l == 0) {
            s_n[0] = nk_pad;
            s_n[1] = no_pad;
        }
    }
    __syncthreads();
    // This wave's bias and head-weight columns are read once, through
    // global-address-space pointers (as the weight packs), each ahead of the
    // product before its epilogue: the epilogues then hold no memory reads,
    // and their waits leave the next product's prefetched weights in flight.
    float cb1[4], cb2[3], cb3[3], cw4[3];
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) cb1[nb] = ((const gfloat*)pb1)[64 * w + 16 * nb + (l & 15)];
    // ---------------- layer 1: K0 -> N1 over the active k-steps, A streamed
    // from HBM through LDS (gathered by k-step)
    f32x4 h1[MB][4];
    {
        act_t* stage = act;
        const act_t* src = (const act_t*)A.aev + (size_t)row0 * K0;
        constexpr int kElems = TM * CH;                       // per chunk
        constexpr int kVec = 16 / sizeof(act_t);              // elements per 16-byte load (within one k-step)
        constexpr int kPer = kElems / kVec / kThreads > 0 ? kElems / kVec / kThreads : 1;
        typedef typename std::conditional<BF, u16x8, float4>::type vec_t;
        const int nk = s_n[0], nch = nk / TPC;
        vec_t pre[kPer];
        auto gload = [&](int c) {
#pragma unroll
            for (int q = 0; q < kPer; ++q) {
                const int idx = (t + kThreads * q) * kVec;
                if (idx < kElems) {
                    const int r = idx / CH, cc = idx % CH;
                    const int kq = s_kq[c * TPC + cc / KS];
                    if (kq >= 0) pre[q] = *(const vec_t*)(src + (size_t)r * K0 + kq * KS + cc % KS);
                    else pre[q] = vec_t{};
                }
            }
        };
        auto sstore = [&](int buf) {
#pragma unroll
            for (int q = 0; q < kPer; ++q) {
                const int idx = (t + kThreads * q) * kVec;
                if (idx < kElems) {
                    const int r = idx / CH, cc = idx % CH;
                    *(vec_t*)(stage + buf * TM * CLD + r * CLD + cc) = pre[q];
                }
            }
        };
        typedef typename Frag<BF>::reg_t reg_t;
        typedef typename Frag<BF>::mem_t mem_t;
        const mem_t* B1 = (const mem_t*)pBf1;
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int nb = 0; nb < 4; ++nb) h1[mb][nb] = (f32x4){0.f, 0.f, 0.f, 0.f};
        // B fragments of list entry e (k-step s_kq[e]; a zero-padding entry
        // reads k-step 0 against zero features) in ring slot e % 4, loaded two
        // entries ahead; a ring turn spans CPR chunks, so every slot index is
        // known at compile time
        reg_t rb[RS][4];
        auto loadB = [&](int e, reg_t (&d)[4]) {
            const int kq = max(s_kq[e], 0);
#pragma unroll
            for (int nb = 0; nb < 4; ++nb) d[nb] = B1[((size_t)(4 * w + nb) * NT + kq) * 64 + l];
        };
#pragma unroll
        for (int t0 = 0; t0 < PD; ++t0)
            if (t0 < nk) loadB(t0, rb[t0]);
        if (nch > 0) {   // a tile of atoms without neighbours has no active k-step (h1 = CELU(b1))
            gload(0);
            sstore(0);
        }
        __syncthreads();
        for (int c0 = 0; c0 < nch; c0 += CPR) {
#pragma unroll
            for (int cc = 0; cc < CPR; ++cc) {
                const int c = c0 + cc;
                if (c + 1 < nch) gload(c + 1);
                const act_t* cur = stage + (c & 1) * TM * CLD;
                // one k-step ahead within the chunk (as in gemm_run)
                constexpr bool kAhead = !BF && MB <= 2;
                typename AFrag<BF>::type a[2][MB];
                if (kAhead) load_a<BF, MB>(cur, CLD, 0, a[0]);
#pragma unroll
                for (int kq = 0; kq < TPC; ++kq) {
                    const int e = c * TPC + kq, slot = (cc * TPC + kq) % RS;
                    if (e + PD < nk) loadB(e + PD, rb[(slot + PD) % RS]);
                    if (kAhead && kq + 1 < TPC) load_a<BF, MB>(cur, CLD, kq + 1, a[(kq + 1) & 1]);
                    __builtin_amdgcn_sched_barrier(0);   // keep the prefetches ahead of this step's MFMAs
                    if (!kAhead) load_a<BF, MB>(cur, CLD, kq, a[kq & 1]);
                    mfma_kstep<BF, MB, 4>(a[kq & 1], rb[slot], h1);
                }
                if (c + 1 < nch) sstore((c + 1) & 1);
                __syncthreads();
            }
        }
    }
    // layer 2's first weight fragments, loaded while the epilogue runs
    BPipe<BF, 3, N1> p2;
    p2.start(pBf2, 3 * w);
#pragma unroll
    for (int nb = 0; nb < 3; ++nb) cb2[nb] = ((const gfloat*)pb2)[48 * w + 16 * nb + (l & 15)];
    // epilogue 1: h1 = CELU(z1 + b1) (kept), act = h1
    {
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int nb = 0; nb < 4; ++nb) {
                const int col = 64 * w + 16 * nb + (l & 15);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const float h = celu(h1[mb][nb][r] + cb1[nb], alpha, ia);
                    h1[mb][nb][r] = h;
                    put_act<BF>(act, (16 * mb + 4 * (l >> 4) + r) * LD + col, h);
                }
            }
    }
    __syncthreads();
    // ---------------- layer 2: N1 -> N2
    f32x4 h2[MB][3];
    gemm_run<BF, MB, 3, N1>(act, LD, p2, h2);
    BPipe<BF, 3, N2> p3;
    p3.start(pBf3, 3 * w);
#pragma unroll
    for (int nb = 0; nb < 3; ++nb) {
        cb3[nb] = ((const gfloat*)pb3)[48 * w + 16 * nb + (l & 15)];
        cw4[nb] = ((const gfloat*)pw4)[48 * w + 16 * nb + (l & 15)];
    }
    __syncthreads();
    {
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int nb = 0; nb < 3; ++nb) {
                const int col = 48 * w + 16 * nb + (l & 15);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const float h = celu(h2[mb][nb][r] + cb2[nb], alpha, ia);
                    h2[mb][nb][r] = h;
                    put_act<BF>(act, (16 * mb + 4 * (l >> 4) + r) * LD + col, h);
                }
            }
    }
    __syncthreads();
    // ---------------- layer 3: N2 -> N3 (160 padded to 192), head, d3
    BPipe<BF, 3, N3> pa3;
    {
        f32x4 z3[MB][3];
        gemm_run<BF, MB, 3, N2>(act, LD, p3, z3);
        if (A.g_out) pa3.start(pBa3, 3 * w);
        __syncthreads();
        float part[MB][4];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int r = 0; r < 4; ++r) part[mb][r] = 0.f;
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int nb = 0; nb < 3; ++nb) {
                const int col = 48 * w + 16 * nb + (l & 15);
                const float wc = cw4[nb];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const float h = celu(z3[mb][nb][r] + cb3[nb], alpha, ia);
                    part[mb][r] += h * wc;
                    put_act<BF>(act, (16 * mb + 4 * (l >> 4) + r) * LD + col, wc * celu_grad_from_h(h, ia));
                }
            }
        // reduce the 16 lanes sharing a row (columns), fixed butterfly
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                float v = part[mb][r];
#pragma unroll
                for (int m = 8; m >= 1; m >>= 1) v += shfl_xor(v, m);
                if ((l & 15) == 0) epart[16 * mb + 4 * (l >> 4) + r][w] = v;
            }
    }
    __syncthreads();
    if (t < TM) {
        const float e = ((epart[t][0] + epart[t][1]) + (epart[t][2] + epart[t][3])) + hb4;
        const int row = row0 + t;
        if (kEns) {
            A.E_net[(size_t)net * A.rows + row] = e;
        } else {
            A.E_row[row] = e;
            const int a = A.row_atom[row];
            if (a >= 0 && A.E_atomo) A.E_atomo[a] = e;
        }
    }
    if (!A.g_out) return;
    // ---------------- adjoint 3: d2 = (W3^T d3) * CELU'(h2)
    BPipe<BF, 4, N2> pa2;
    {
        f32x4 d[MB][3];
        gemm_run<BF, MB, 3, N3>(act, LD, pa3, d);
        pa2.start(pBa2, 4 * w);
        __syncthreads();
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int nb = 0; nb < 3; ++nb) {
                const int col = 48 * w + 16 * nb + (l & 15);
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    put_act<BF>(act, (16 * mb + 4 * (l >> 4) + r) * LD + col,
                                d[mb][nb][r] * celu_grad_from_h(h2[mb][nb][r], ia));
            }
    }
    __syncthreads();
    // ---------------- adjoint 2: d1 = (W2^T d2) * CELU'(h1)
    // adjoint 1 runs over the active output blocks (16 columns each, listed
    // in s_ob and padded with -1 to a multiple of eight): passes of four
    // blocks per wave, then one pass of two for a remainder of eight
    const int no = s_n[1], n16 = no / 16;
    BPipe<BF, 4, N1> pg4;
    BPipe<BF, 2, N1> pg2;
    {
        f32x4 d[MB][4];
        gemm_run<BF, MB, 4, N2>(act, LD, pa2, d);
        if (!kEns) {
            if (n16 > 0) pg4.start(pBa1, 0, s_ob + 4 * w);
            else if (no > 0) pg2.start(pBa1, 0, s_ob + 2 * w);
        }
        __syncthreads();
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int nb = 0; nb < 4; ++nb) {
                const int col = 64 * w + 16 * nb + (l & 15);
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    put_act<BF>(act, (16 * mb + 4 * (l >> 4) + r) * LD + col,
                                d[mb][nb][r] * celu_grad_from_h(h1[mb][nb][r], ia));
            }
    }
    __syncthreads();
    if (kEns) {
        // d1 tile out (this network's slice); the first layer's adjoint sums over networks
        act_t* dst = (act_t*)A.d1_out + ((size_t)net * A.rows + row0) * N1;
        for (int q = t; q < TM * N1; q += kThreads) dst[q] = act[(q / N1) * LD + (q % N1)];
        return;
    }
    // ---------------- adjoint 1: g = W1^T d1 over the active output blocks
    for (int pass = 0; pass < n16; ++pass) {
        const int* ob = s_ob + 16 * pass + 4 * w;
        int b[4];
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) b[nb] = ob[nb];
        f32x4 gacc[MB][4];
        gemm_run<BF, MB, 4, N1>(act, LD, pg4, gacc);
        if (pass + 1 < n16) pg4.start(pBa1, 0, ob + 16);
        else if (no > 16 * n16) pg2.start(pBa1, 0, s_ob + 16 * n16 + 2 * w);
        store_g<MB, 4>(A.g_out, row0, gacc, b);
    }
    if (no > 16 * n16) {
        const int* ob = s_ob + 16 * n16 + 2 * w;
        const int b[2] = {ob[0], ob[1]};
        f32x4 gacc[MB][2];
        gemm_run<BF, MB, 2, N1>(act, LD, pg2, gacc);
        store_g<MB, 2>(A.g_out, row0, gacc, b);
    }
}

// Ensemble, first layer's adjoint summed over networks:
//   g = (1 / n_nets) sum_net W1_net^T d1_net    (one GEMM with K = 256 n_nets)
// and the ensemble-mean energies.  Block (tile, pass): the tile's active
// output blocks 16 pass + 4 w .. + 3 (as in the single-network kernel).
template <bool BF, int TM>
__global__ __launch_bounds__(kThreads, 2) void k_ens_adj1(const FusedArgs A, int n_nets, float inv_nets,
                                                         float* E_atom_net, int n_atoms) {
    typedef typename Cfg<BF>::act_t act_t;
    constexpr int MB = TM / 16;
    constexpr int LD = Cfg<BF>::kLd;
    __shared__ __attribute__((aligned(16))) act_t act[TM * LD];
    const int row0 = xcd_tile((A.rows + TM - 1) / TM) * TM, pass = blockIdx.y;
    const int32_t* meta = A.meta;
    if (row0 >= meta[8 + A.ns]) return;
    int s = 0;
    for (int q = 1; q < A.ns; ++q)
        if (meta[8 + q] <= row0) s = q;
    if (row0 >= meta[8 + s] + meta[s]) return;
    const int t = threadIdx.x, w = t / kWave, l = lane_id();
    constexpr int kVec = 16 / (int)sizeof(act_t);
    typedef typename std::conditional<BF, u16x8, float4>::type vec_t;
    __shared__ int s_ob[64];
    __shared__ int s_no;
    if (t < kWave) {
        const int no = block_list(tile_blocks<TM>(A, row0), s_ob, 16);
        if (l == 0) s_no = no;
    }
    __syncthreads();
    const bool work = A.g_out && 16 * pass < s_no;   // block-uniform
    int blk[4], use[4];
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) {
        const int b = work ? s_ob[16 * pass + 4 * w + nb] : -1;
        use[nb] = b >= 0;
        blk[nb] = max(b, 0);
    }
    f32x4 acc[MB][4];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) acc[mb][nb] = (f32x4){0.f, 0.f, 0.f, 0.f};
    for (int net = 0; work && net < n_nets; ++net) {
        const act_t* src = (const act_t*)A.d1_out + ((size_t)net * A.rows + row0) * N1;
        for (int q = t * kVec; q < TM * N1; q += kThreads * kVec)
            *(vec_t*)(act + (q / N1) * LD + (q % N1)) = *(const vec_t*)(src + q);
        __syncthreads();
        gemm_act<BF, MB, 4, N1, false>(act, LD, A.nets[net].Ba1[s], 0, acc, blk);
        __syncthreads();
    }
    if (work) {
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int nb = 0; nb < 4; ++nb) {
                if (!use[nb]) continue;
                const int col = 16 * blk[nb] + (l & 15);
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    A.g_out[(size_t)(row0 + 16 * mb + 4 * (l >> 4) + r) * K0 + col] = acc[mb][nb][r] * inv_nets;
            }
    }
    if (pass == 0 && t < TM) {
        const int row = row0 + t;
        float e = 0.f;
        for (int net = 0; net < n_nets; ++net) e += A.E_net[(size_t)net * A.rows + row];
        e *= inv_nets;
        A.E_row[row] = e;
        const int a = A.row_atom[row];
        if (a >= 0) {
            if (A.E_atomo) A.E_atomo[a] = e;
            if (E_atom_net)
                for (int net = 0; net < n_nets; ++net)
                    E_atom_net[(size_t)net * n_atoms + a] = A.E_net[(size_t)net * A.rows + row];
        }
    }
}

}  // namespace

// ---------------------------------------------------------------- host side

bool fused_mlp_shape(const int* widths, int n_layers, int ns) {
    const int dim = ns * kNr + ns * (ns + 1) / 2 * kNa * kNz;
    return n_layers == 4 && dim <= K0 && dim > K0 - 64 && widths[1] == N1 && widths[2] == N2 &&
           widths[3] <= N3 && widths[3] > N3 - 64 && widths[4] == 1;
}

// Packs B[k][n] (k < K, n < N, accessor) into MFMA fragment order.
// FP32: out[((nb * K/16 + kq) * 64 + lane) * 4 + j] = B[16 kq + 4 j + lane/16][16 nb + lane%16]
// BF16: out[((nb * K/32 + ks) * 64 + lane) * 8 + e] = B[32 ks + 8 (lane/16) + e][16 nb + lane%16]
template <typename F>
static void pack_fp32(float* out, int K, int N, F B) {
    for (int nb = 0; nb < N / 16; ++nb)
        for (int kq = 0; kq < K / 16; ++kq)
            for (int lane = 0; lane < 64; ++lane)
                for (int j = 0; j < 4; ++j)
                    out[(((size_t)nb * (K / 16) + kq) * 64 + lane) * 4 + j] =
                        B(16 * kq + 4 * (lane / 16) + j, 16 * nb + lane % 16);
}

uint16_t host_bf16_bits(float f);

template <typename F>
static void pack_bf16(uint16_t* out, int K, int N, F B) {
    for (int nb = 0; nb < N / 16; ++nb)
        for (int ks = 0; ks < K / 32; ++ks)
            for (int lane = 0; lane < 64; ++lane)
                for (int e = 0; e < 8; ++e)
                    out[(((size_t)nb * (K / 32) + ks) * 64 + lane) * 8 + e] =
                        host_bf16_bits(B(32 * ks + 8 * (lane / 16) + e, 16 * nb + lane % 16));
}

// Builds the six packs of one species from row-major W_l [out][in] (host).
// Returns bytes used at dst (dst may be null to size).
size_t pack_fused_species(char* dst, bool bf16, const float* W1, const float* W2, const float* W3, int n_in,
                          int n3) {
    // logical padded matrices: W1p [N1][K0], W2p [N2][N1], W3p [N3][N2] (rows >= n3 zero)
    auto w1 = [&](int o, int i) { return i < n_in ? W1[(size_t)o * n_in + i] : 0.f; };
    auto w2 = [&](int o, int i) { return W2[(size_t)o * N1 + i]; };
    auto w3 = [&](int o, int i) { return o < n3 ? W3[(size_t)o * N2 + i] : 0.f; };
    struct L { int K, N; int kind; };
    const L layers[6] = {{K0, N1, 0}, {N1, N2, 1}, {N2, N3, 2}, {N3, N2, 3}, {N2, N1, 4}, {N1, K0, 5}};
    size_t off = 0;
    for (const L& q : layers) {
        const size_t bytes = (size_t)q.K * q.N * (bf16 ? 2 : 4);
        if (dst) {
            auto B = [&](int k, int n) -> float {
                switch (q.kind) {
                    case 0: return w1(n, k);     // forward: B[k][n] = W[n][k]
                    case 1: return w2(n, k);
                    case 2: return w3(n, k);
                    case 3: return w3(k, n);     // adjoint: B[k][n] = W[k][n]
                    case 4: return w2(k, n);
                    default: return w1(k, n);
                }
            };
            if (bf16) pack_bf16((uint16_t*)(dst + off), q.K, q.N, B);
            else pack_fp32((float*)(dst + off), q.K, q.N, B);
        }
        off += (bytes + 255) & ~(size_t)255;
    }
    return off;
}

size_t fused_net_bytes() { return sizeof(FusedNet); }

// Ensembles run as the two-kernel split (every network's forward and adjoint
// down to d1, then the first-layer adjoint summed over networks).  For one
// network the split measured within a few per cent of the fused kernel at
// 2,048-8,192 atoms (and slower in BF16), so a single network stays fused.
bool mlp_split(const nnp_model* m, int n_atoms) {
    (void)n_atoms;
    return m->fused && m->n_nets > 1;
}

// Fills the device-table entry of one network (host copy) from its packs and
// bias / head arrays.
void fused_net_entry(void* out, int ns, const char* const* packs, const float* const* b1, const float* const* b2,
                     const float* const* b3, const float* const* w4, const float* b4, bool bf16) {
    FusedNet& E = *(FusedNet*)out;
    std::memset(&E, 0, sizeof(E));
    const size_t unit = bf16 ? 2 : 4;
    const int KN[6][2] = {{K0, N1}, {N1, N2}, {N2, N3}, {N3, N2}, {N2, N1}, {N1, K0}};
    const void** dst[6] = {E.Bf1, E.Bf2, E.Bf3, E.Ba3, E.Ba2, E.Ba1};
    for (int q = 0; q < ns; ++q) {
        size_t off = 0;
        for (int k = 0; k < 6; ++k) {
            dst[k][q] = packs[q] + off;
            off += ((size_t)KN[k][0] * KN[k][1] * unit + 255) & ~(size_t)255;
        }
        E.b1[q] = b1[q];
        E.b2[q] = b2[q];
        E.b3[q] = b3[q];
        E.w4[q] = w4[q];
        E.b4[q] = b4[q];
    }
}

namespace {

// tile height: enough tiles to fill the chip twice over.  One network stops
// at 32 rows (the FP32 form's 64-row tile does not fit the register file, and
// the BF16 form's runs slower than two 32-row tiles); the BF16 ensemble takes
// 64 rows from 48 Ki atoms, where its first-layer adjoint over all networks
// gains from the taller tile.
int fused_tile_rows(int n_atoms, bool bf, bool ens) {
    int tm = n_atoms >= 48 * 1024 ? 64 : (n_atoms >= 12 * 1024 ? 32 : 16);
    if ((!bf || !ens) && tm > 32) tm = 32;
    return tm;
}

FusedArgs fused_args(const nnp_model* m, const MlpWs& W, const void* aev, float* g_out, float* E_row, float* E_atomo) {
    const bool bf = m->precision == NNP_BF16_MLP;
    FusedArgs A;
    std::memset(&A, 0, sizeof(A));
    A.nets = (const FusedNet*)(bf ? m->fused_tab_bf16 : m->fused_tab_fp32);
    A.meta = W.meta;
    A.row_atom = W.row_atom;
    A.aev = aev;
    A.g_out = g_out;
    A.E_row = E_row;
    A.E_atomo = E_atomo;
    A.alpha = m->celu_alpha;
    A.ns = m->aev.ns;
    A.rows = W.rows_max;
    A.amask = W.amask;
    return A;
}

}  // namespace

hipError_t launch_mlp_fused(const nnp_model* m, const MlpWs& W, const void* aev, float* g_out, float* E_row,
                            float* E_atomo, int n_atoms, hipStream_t s) {
    const bool bf = m->precision == NNP_BF16_MLP;
    const FusedArgs A = fused_args(m, W, aev, g_out, E_row, E_atomo);
    const int tm = fused_tile_rows(n_atoms, bf, false);
    const int grid = ceil_div(ceil_div(W.rows_max, tm), kXcds) * kXcds;   // whole rounds of the XCDs (xcd_tile)
    if (bf) {
        if (tm == 32) k_mlp_fused<true, 32, false><<<grid, kThreads, 0, s>>>(A);
        else k_mlp_fused<true, 16, false><<<grid, kThreads, 0, s>>>(A);
    } else {
        if (tm == 32) k_mlp_fused<false, 32, false><<<grid, kThreads, 0, s>>>(A);
        else k_mlp_fused<false, 16, false><<<grid, kThreads, 0, s>>>(A);
    }
    return hipGetLastError();
}

// Ensemble of m->n_nets networks on the shared features: every network's
// forward and adjoint down to d1 (grid.y = network), then the first layer's
// adjoint summed over networks and the mean energies.  d1_scratch:
// [n_nets][rows_max][256] (float32-sized), E_net: [n_nets][rows_max];
// E_atom_net: [n_nets][n_atoms] per-network atomic energies or null.
hipError_t launch_mlp_ensemble(const nnp_model* m, const MlpWs& W, const void* aev, float* g_out, float* E_row,
                               float* E_atomo, int n_atoms, void* d1_scratch, float* E_net, float* E_atom_net,
                               hipStream_t s) {
    const bool bf = m->precision == NNP_BF16_MLP;
    FusedArgs A = fused_args(m, W, aev, g_out, E_row, E_atomo);
    A.d1_out = d1_scratch;
    A.E_net = E_net;
    const int tm = fused_tile_rows(n_atoms, bf, true);
    const int gx = ceil_div(ceil_div(W.rows_max, tm), kXcds) * kXcds;   // whole rounds of the XCDs (xcd_tile)
    const dim3 g1(gx, m->n_nets), g2(gx, g_out ? 4 : 1);
    const float inv = 1.f / (float)m->n_nets;
    if (bf) {
        if (tm == 64) {
            k_mlp_fused<true, 64, true><<<g1, kThreads, 0, s>>>(A);
            k_ens_adj1<true, 64><<<g2, kThreads, 0, s>>>(A, m->n_nets, inv, E_atom_net, n_atoms);
        } else if (tm == 32) {
            k_mlp_fused<true, 32, true><<<g1, kThreads, 0, s>>>(A);
            k_ens_adj1<true, 32><<<g2, kThreads, 0, s>>>(A, m->n_nets, inv, E_atom_net, n_atoms);
        } else {
            k_mlp_fused<true, 16, true><<<g1, kThreads, 0, s>>>(A);
            k_ens_adj1<true, 16><<<g2, kThreads, 0, s>>>(A, m->n_nets, inv, E_atom_net, n_atoms);
        }
    } else {
        if (tm == 32) {
            k_mlp_fused<false, 32, true><<<g1, kThreads, 0, s>>>(A);
            k_ens_adj1<false, 32><<<g2, kThreads, 0, s>>>(A, m->n_nets, inv, E_atom_net, n_atoms);
        } else {
            k_mlp_fused<false, 16, true><<<g1, kThreads, 0, s>>>(A);
            k_ens_adj1<false, 16><<<g2, kThreads, 0, s>>>(A, m->n_nets, inv, E_atom_net, n_atoms);
        }
    }
    return hipGetLastError();
}

}  // namespace nnp
