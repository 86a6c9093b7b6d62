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

// Sum of block b's elements (loads coalesced: element b * kScanSpan +
// r * kScanBlock + t for thread t, round r).
__global__ void __launch_bounds__(kScanBlock) k_scan_sums(const uint32_t* __restrict__ v, size_t n,
                                                          uint32_t* __restrict__ bsum) {
    __shared__ uint32_t wsum[kScanBlock / 64];
    const size_t base = (size_t)blockIdx.x * kScanSpan + threadIdx.x;
    uint32_t s = 0;
#pragma unroll
    for (int r = 0; r < kScanPer; ++r) {
        const size_t i = base + (size_t)r * kScanBlock;
        s += i < n ? v[i] : 0u;
    }
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

// Block b's elements, loaded and stored coalesced through LDS: thread t
// scans the kScanPer consecutive elements t * kScanPer + [0, kScanPer) of
// the block (the LDS index skips one word every 32 so those reads spread
// over the banks).
__device__ inline int scan_lds(int i) { return i + (i >> 5); }

__global__ void __launch_bounds__(kScanBlock) k_scan_apply(uint32_t* __restrict__ v, size_t n,
                                                           const uint32_t* __restrict__ bsum) {
    __shared__ uint32_t wsum[kScanBlock / 64];
    __shared__ uint32_t buf[kScanSpan + kScanSpan / 32];
    const size_t base = (size_t)blockIdx.x * kScanSpan;
    const int t = threadIdx.x;
#pragma unroll
    for (int r = 0; r < kScanPer; ++r) {
        const int i = r * kScanBlock + t;
        buf[scan_lds(i)] = base + i < n ? v[base + i] : 0u;
    }
    __syncthreads();
    uint32_t x[kScanPer], s = 0;
#pragma unroll
    for (int r = 0; r < kScanPer; ++r) {
        x[r] = buf[scan_lds(t * kScanPer + r)];
        s += x[r];
    }
    uint32_t total;
    uint32_t run = bsum[blockIdx.x] + block_excl_scan(s, wsum, &total);
#pragma unroll
    for (int r = 0; r < kScanPer; ++r) {
        buf[scan_lds(t * kScanPer + r)] = run;
        run += x[r];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kScanPer; ++r) {
        const int i = r * kScanBlock + t;
        if (base + i < n) v[base + i] = buf[scan_lds(i)];
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
