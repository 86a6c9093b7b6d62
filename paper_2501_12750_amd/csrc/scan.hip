// Device-wide exclusive prefix sum of 32-bit counts, in place, used by the
// surface extraction (triangle offsets per cube) and the scene build (radix
// sort offsets): block sums of 4096-element blocks, one workgroup scans those
// sums (and writes the total), then every block scans its elements from its
// start.
#include "vtx_internal.h"

namespace vtx {

namespace {

constexpr int kScanBlock = 256;
constexpr int kScanPer = 16;
constexpr int kScanSpan = kScanBlock * kScanPer;

// Exclusive scan of one value per thread over the workgroup; *total gets the
// workgroup's sum.
__device__ inline uint32_t block_excl_scan(uint32_t v, uint32_t* wsum, uint32_t* total) {
    const int lane = __lane_id(), wave = threadIdx.x >> 6;
    uint32_t incl = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t u = __shfl_up(incl, o);
        if (lane >= o) incl += u;
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    uint32_t before = 0, all = 0;
    for (int w = 0; w < kScanBlock / 64; ++w) {
        before += w < wave ? wsum[w] : 0u;
        all += wsum[w];
    }
    __syncthreads();
    *total = all;
    return before + incl - v;
}

// Thread t of block b sums elements b * kScanSpan + t * kScanPer + [0, kScanPer).
__global__ void __launch_bounds__(kScanBlock) k_scan_sums(const uint32_t* __restrict__ v, size_t n,
                                                          uint32_t* __restrict__ bsum) {
    __shared__ uint32_t wsum[kScanBlock / 64];
    const size_t base = (size_t)blockIdx.x * kScanSpan + (size_t)threadIdx.x * kScanPer;
    uint32_t s = 0;
    for (int i = 0; i < kScanPer; ++i)
        if (base + i < n) s += v[base + i];
    uint32_t total;
    (void)block_excl_scan(s, wsum, &total);
    if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

__global__ void __launch_bounds__(kScanBlock) k_scan_top(uint32_t* __restrict__ bsum, uint32_t nb,
                                                         unsigned long long* __restrict__ total_out) {
    __shared__ uint32_t wsum[kScanBlock / 64];
    uint32_t carry = 0;
    for (uint32_t b0 = 0; b0 < nb; b0 += kScanBlock) {
        const uint32_t b = b0 + threadIdx.x;
        const uint32_t x = b < nb ? bsum[b] : 0u;
        uint32_t total;
        const uint32_t ex = block_excl_scan(x, wsum, &total);
        if (b < nb) bsum[b] = carry + ex;
        carry += total;
    }
    if (threadIdx.x == 0 && total_out) *total_out = carry;
}

__global__ void __launch_bounds__(kScanBlock) k_scan_apply(uint32_t* __restrict__ v, size_t n,
                                                           const uint32_t* __restrict__ bsum) {
    __shared__ uint32_t wsum[kScanBlock / 64];
    const size_t base = (size_t)blockIdx.x * kScanSpan + (size_t)threadIdx.x * kScanPer;
    uint32_t x[kScanPer], s = 0;
#pragma unroll
    for (int i = 0; i < kScanPer; ++i) {
        x[i] = base + i < n ? v[base + i] : 0u;
        s += x[i];
    }
    uint32_t total;
    uint32_t run = bsum[blockIdx.x] + block_excl_scan(s, wsum, &total);
#pragma unroll
    for (int i = 0; i < kScanPer; ++i) {
        if (base + i < n) v[base + i] = run;
        run += x[i];
    }
}

}  // namespace

size_t scan_scratch_words(size_t n) { return (n + kScanSpan - 1) / kScanSpan + 1; }

hipError_t exclusive_scan(uint32_t* v, size_t n, uint32_t* bsum, unsigned long long* total, hipStream_t stream) {
    const size_t nb = (n + kScanSpan - 1) / kScanSpan;
    hipError_t e;
    if (nb && (e = dispatch(k_scan_sums, (unsigned)nb, kScanBlock, 0, stream, (const uint32_t*)v, n, bsum))) return e;
    if ((e = dispatch(k_scan_top, 1, kScanBlock, 0, stream, bsum, (uint32_t)nb, total))) return e;
    if (nb && (e = dispatch(k_scan_apply, (unsigned)nb, kScanBlock, 0, stream, v, n, (const uint32_t*)bsum))) return e;
    return hipSuccess;
}

}  // namespace vtx
