// Device-wide exclusive prefix sum of int32 counts (three passes: block
// sums, scan of the block sums, block-local scan plus offset).  Used for
// cell starts and neighbour-row pointers.  Totals are carried in int64 so an
// overflowing pair count is detected rather than wrapped.
#include "nnp_internal.hpp"

namespace nnp {
namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 4;
constexpr int kScanBlock = kScanThreads * kScanItems;

// inclusive scan of v across the wave
__device__ __forceinline__ long long wave_inclusive(long long v) {
    const int l = lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        long long u = __shfl_up(v, d, kWave);
        if (l >= d) v += u;
    }
    return v;
}

// exclusive block scan of one value per thread; returns block total via *tot
__device__ long long block_exclusive(long long v, long long* tot) {
    __shared__ long long wsum[kScanThreads / kWave];
    const int w = threadIdx.x / kWave;
    long long inc = wave_inclusive(v);
    if (lane_id() == kWave - 1) wsum[w] = inc;
    __syncthreads();
    long long off = 0, all = 0;
    for (int i = 0; i < kScanThreads / kWave; ++i) {
        if (i < w) off += wsum[i];
        all += wsum[i];
    }
    __syncthreads();
    *tot = all;
    return off + inc - v;
}

__global__ __launch_bounds__(kScanThreads) void k_block_sums(const int32_t* in, int n, int64_t* bsum,
                                                             const int32_t* gate) {
    if (gate && *gate == 0) return;
    const int base = blockIdx.x * kScanBlock + threadIdx.x * kScanItems;
    long long s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k)
        if (base + k < n) s += in[base + k];
    long long tot;
    block_exclusive(s, &tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_sums(int64_t* bsum, int nb, int64_t* total,
                                                            int32_t* out_last, const int32_t* gate) {
    if (gate && *gate == 0) return;
    long long carry = 0;
    for (int c0 = 0; c0 < nb; c0 += kScanThreads) {
        const int i = c0 + threadIdx.x;
        long long v = i < nb ? bsum[i] : 0;
        long long tot;
        long long ex = block_exclusive(v, &tot);
        if (i < nb) bsum[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) {
        *total = carry;
        *out_last = carry > 0x7fffffffLL ? 0x7fffffff : (int32_t)carry;
    }
}

__global__ __launch_bounds__(kScanThreads) void k_block_scan(const int32_t* in, int n, const int64_t* boff,
                                                             int32_t* out, const int32_t* gate) {
    if (gate && *gate == 0) return;
    const int base = blockIdx.x * kScanBlock + threadIdx.x * kScanItems;
    int32_t v[kScanItems];
    long long s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = base + k < n ? in[base + k] : 0;
        s += v[k];
    }
    long long tot;
    long long ex = block_exclusive(s, &tot) + boff[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < n) out[base + k] = ex > 0x7fffffffLL ? 0x7fffffff : (int32_t)ex;
        ex += v[k];
    }
}

// Small inputs: one block of 1024 threads, 8 items per thread.
constexpr int kSmallThreads = 1024, kSmallItems = 8;

__global__ __launch_bounds__(kSmallThreads) void k_scan_small(const int32_t* in, int n, int32_t* out,
                                                              int64_t* total, const int32_t* gate, ScanClamp cl) {
    if (gate && *gate == 0) return;
    __shared__ long long wsum[kSmallThreads / kWave];
    const int t = threadIdx.x, w = t / kWave;
    const int base = t * kSmallItems;
    int32_t v[kSmallItems];
    long long s = 0;
#pragma unroll
    for (int k = 0; k < kSmallItems; ++k) {
        v[k] = base + k < n ? in[base + k] : 0;
        s += v[k];
    }
    long long inc = wave_inclusive(s);
    if (lane_id() == kWave - 1) wsum[w] = inc;
    __syncthreads();
    long long off = 0, all = 0;
    for (int q = 0; q < kSmallThreads / kWave; ++q) {
        if (q < w) off += wsum[q];
        all += wsum[q];
    }
    long long ex = off + inc - s;
    // with a clamp, outputs are cut at the capacity (a list longer than its
    // capacity is then read in bounds), the overflow flagged and its size kept
    const long long cap = cl.capacity >= 0 ? (long long)cl.capacity : 0x7fffffffLL;
#pragma unroll
    for (int k = 0; k < kSmallItems; ++k) {
        if (base + k < n) out[base + k] = (int32_t)(ex > cap ? cap : ex);
        ex += v[k];
    }
    if (t == 0) {
        *total = all;
        out[n] = (int32_t)(all > cap ? cap : all);
        if (cl.capacity >= 0 && all > cl.capacity) {
            set_flag(cl.flags, NNP_FLAG_CAPACITY);
            if (cl.need) atomicMax((unsigned long long*)cl.need, (unsigned long long)all);
        }
    }
}

__global__ void k_scan_clamp(int n, int32_t* out, const int64_t* total, ScanClamp cl, const int32_t* gate) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > n || (gate && *gate == 0)) return;
    const long long t = *total;
    if (t <= cl.capacity) return;
    if (i == 0) {
        set_flag(cl.flags, NNP_FLAG_CAPACITY);
        if (cl.need) atomicMax((unsigned long long*)cl.need, (unsigned long long)t);
    }
    if (out[i] > cl.capacity) out[i] = (int32_t)cl.capacity;
}

}  // namespace

size_t scan_tmp_elems(int n) { return (size_t)ceil_div(n > 0 ? n : 1, kScanBlock) + 1; }

// out has n + 1 entries; out[n] = total (saturated to int32); *total_out (device) = exact total.
// With a gate, every kernel does nothing while *gate == 0.
hipError_t launch_exclusive_scan_i32(const int32_t* in, int32_t* out, int64_t* total_out, int n,
                                     int64_t* block_tmp, hipStream_t s, const int32_t* gate, const ScanClamp* clamp) {
    ScanClamp cl{-1, nullptr, nullptr};
    if (clamp) cl = *clamp;
    if (n <= kSmallThreads * kSmallItems) {
        k_scan_small<<<1, kSmallThreads, 0, s>>>(in, n, out, total_out, gate, cl);
        return hipGetLastError();
    }
    const int nb = ceil_div(n > 0 ? n : 1, kScanBlock);
    k_block_sums<<<nb, kScanThreads, 0, s>>>(in, n, block_tmp, gate);
    k_scan_sums<<<1, kScanThreads, 0, s>>>(block_tmp, nb, total_out, out + n, gate);
    k_block_scan<<<nb, kScanThreads, 0, s>>>(in, n, block_tmp, out, gate);
    if (cl.capacity >= 0) k_scan_clamp<<<ceil_div(n + 1, 256), 256, 0, s>>>(n, out, total_out, cl, gate);
    return hipGetLastError();
}

}  // namespace nnp
