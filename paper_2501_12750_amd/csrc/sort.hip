// Stable least-significant-digit radix sort of (32-bit key, 32-bit value)
// pairs for the scene build (Morton order of the atoms, bonds by their first
// stored atom).  Each pass sorts by one 8-bit digit: every workgroup counts
// the digits of its tile of 4096 pairs; one exclusive scan over the counts,
// laid out digit-major (all tiles' counts of digit 0, then of digit 1, ...),
// gives each (digit, tile) the output position of its first pair; every
// workgroup then writes its pairs in index order, 256 at a time, each pair
// after the earlier pairs of its digit.  Passes keep the order of equal
// digits, so the whole sort keeps the order of equal keys.
#include "vtx_internal.h"

namespace vtx {

namespace {

constexpr int kSortBlock = 256;
constexpr int kSortRounds = 16;
constexpr size_t kSortTile = (size_t)kSortBlock * kSortRounds;
constexpr int kRadix = 256;

inline uint32_t sort_tiles(size_t n) { return (uint32_t)((n + kSortTile - 1) / kSortTile); }

// cnt[d * nt + t]: pairs of tile t whose digit is d.
__global__ void __launch_bounds__(kSortBlock) k_digit_count(const uint32_t* __restrict__ keys, size_t n, int shift,
                                                            uint32_t mask, uint32_t nt, uint32_t* __restrict__ cnt) {
    __shared__ uint32_t h[kRadix];
    h[threadIdx.x] = 0;
    __syncthreads();
    const size_t base = (size_t)blockIdx.x * kSortTile + threadIdx.x;
    for (int r = 0; r < kSortRounds; ++r) {
        const size_t i = base + (size_t)r * kSortBlock;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & mask], 1u);
    }
    __syncthreads();
    cnt[(size_t)threadIdx.x * nt + blockIdx.x] = h[threadIdx.x];
}

// Writes tile blockIdx.x's pairs at the positions off[d * nt + t] (the
// scanned counts) onward.  Within a round of 256 pairs a pair's place among
// its digit is its rank among the lanes of its wave with that digit, after
// the earlier waves' pairs of the digit.  kout may be null (values only).
__global__ void __launch_bounds__(kSortBlock) k_digit_scatter(const uint32_t* __restrict__ kin,
                                                              const uint32_t* __restrict__ vin, size_t n, int shift,
                                                              uint32_t mask, uint32_t nt,
                                                              const uint32_t* __restrict__ off,
                                                              uint32_t* __restrict__ kout,
                                                              uint32_t* __restrict__ vout) {
    constexpr int kWaves = kSortBlock / 64;
    __shared__ uint32_t next[kRadix];             // next output position of each digit
    __shared__ uint32_t wave_cnt[kWaves][kRadix]; // pairs of each digit in each wave this round
    const int tid = threadIdx.x, wave = tid >> 6;
    const int bits = 32 - __builtin_clz(mask);
    next[tid] = off[(size_t)tid * nt + blockIdx.x];
    const size_t base = (size_t)blockIdx.x * kSortTile + tid;
    for (int r = 0; r < kSortRounds; ++r) {
        // each thread clears and later adds up column tid only
        for (int w = 0; w < kWaves; ++w) wave_cnt[w][tid] = 0;
        const size_t i = base + (size_t)r * kSortBlock;
        const bool valid = i < n;
        const uint32_t k = valid ? kin[i] : 0u, v = valid ? vin[i] : 0u;
        const uint32_t d = (k >> shift) & mask;
        // lanes of this wave holding a pair with the same digit
        unsigned long long peers = __ballot(valid);
        for (int b = 0; b < bits; ++b) {
            const bool set = (d >> b) & 1u;
            const unsigned long long m = __ballot(set);
            peers &= set ? m : ~m;
        }
        const uint32_t rank = (uint32_t)__popcll(peers & __lanemask_lt());
        __syncthreads();
        if (valid && rank == 0) wave_cnt[wave][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t pos = next[d] + rank;
            for (int w = 0; w < wave; ++w) pos += wave_cnt[w][d];
            if (kout) kout[pos] = k;
            vout[pos] = v;
        }
        __syncthreads();
        uint32_t add = 0;
        for (int w = 0; w < kWaves; ++w) add += wave_cnt[w][tid];
        next[tid] += add;
    }
}

}  // namespace

size_t radix_sort_scratch_words(size_t n) {
    const size_t c = (size_t)kRadix * sort_tiles(n);
    return c + scan_scratch_words(c);
}

hipError_t radix_sort_pairs(uint32_t* keys, uint32_t* keys_alt, uint32_t* vals, uint32_t* vals_alt,
                            uint32_t* vals_out, size_t n, int end_bit, uint32_t* scratch, hipStream_t stream) {
    if (end_bit < 1 || end_bit > 32 || n >= ((size_t)1 << 32)) return hipErrorInvalidValue;
    const int passes = (end_bit + 7) / 8;
    // the last pass reads from keys/vals after an odd number of passes before
    // it, from the alternate buffers after an even number
    if (vals_out == ((passes - 1) % 2 ? vals_alt : vals)) return hipErrorInvalidValue;
    if (n == 0) return hipSuccess;
    const uint32_t nt = sort_tiles(n);
    uint32_t* cnt = scratch;
    uint32_t* bsum = scratch + (size_t)kRadix * nt;
    hipError_t e;
    for (int p = 0; p < passes; ++p) {
        const int shift = 8 * p;
        const int bits = end_bit - shift < 8 ? end_bit - shift : 8;
        const uint32_t mask = (1u << bits) - 1u;
        const uint32_t* ks = p % 2 ? keys_alt : keys;
        const uint32_t* vs = p % 2 ? vals_alt : vals;
        const bool last = p == passes - 1;
        uint32_t* kd = last ? nullptr : (p % 2 ? keys : keys_alt);
        uint32_t* vd = last ? vals_out : (p % 2 ? vals : vals_alt);
        if ((e = dispatch(k_digit_count, nt, kSortBlock, 0, stream, ks, n, shift, mask, nt, cnt))) return e;
        if ((e = exclusive_scan(cnt, (size_t)kRadix * nt, bsum, nullptr, stream))) return e;
        if ((e = dispatch(k_digit_scatter, nt, kSortBlock, 0, stream, ks, vs, n, shift, mask, nt,
                          (const uint32_t*)cnt, kd, vd)))
            return e;
    }
    return hipSuccess;
}

}  // namespace vtx
