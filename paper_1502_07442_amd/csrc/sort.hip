// Stable least-significant-digit radix sort of (uint64 key, uint32 value)
// pairs, 8 bits per pass. Every pass: a per-tile digit histogram, one
// exclusive scan over the digit-major histogram table, and a scatter in which
// each tile ranks its keys digit by digit in input order (wave-wide ballots
// find the lanes sharing a digit), which keeps the sort stable. The ranked
// tile is first laid out in LDS in digit order, then written out so that each
// digit's run of the tile goes to consecutive addresses.
#include "ngr_internal.hpp"

namespace ngr {
namespace {

constexpr int kThreads = 256;
constexpr int kRounds = 16;
constexpr int kTile = kThreads * kRounds;
constexpr int kDigits = 256;

__global__ __launch_bounds__(kThreads) void digit_histogram(const uint64_t* __restrict__ keys, uint64_t n,
                                                            int shift, uint32_t* __restrict__ hist,
                                                            uint32_t tiles)
{
    __shared__ uint32_t h[kDigits];
    h[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t base = (uint64_t)blockIdx.x * kTile;
    for (int r = 0; r < kRounds; ++r) {
        uint64_t i = base + (uint64_t)r * kThreads + threadIdx.x;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & 0xff], 1u);
    }
    __syncthreads();
    hist[(uint64_t)threadIdx.x * tiles + blockIdx.x] = h[threadIdx.x];
}

__global__ __launch_bounds__(kThreads) void digit_scatter(const uint64_t* __restrict__ kin,
                                                          const uint32_t* __restrict__ vin,
                                                          uint64_t* __restrict__ kout,
                                                          uint32_t* __restrict__ vout, uint64_t n, int shift,
                                                          const uint32_t* __restrict__ offsets,
                                                          const uint32_t* __restrict__ counts, uint32_t tiles)
{
    __shared__ uint32_t base[kDigits];      // running tile-local position of each digit
    __shared__ uint32_t first[kDigits];     // tile-local start of each digit's run
    __shared__ uint32_t wcount[kThreads / 64][kDigits];
    __shared__ uint64_t skey[kTile];
    __shared__ uint32_t sval[kTile];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // tile-local starts: exclusive scan of the tile's digit counts
    {
        const uint32_t c = counts[(uint64_t)tid * tiles + blockIdx.x];
        wcount[0][tid] = c;
        __syncthreads();
        for (int d = 1; d < kDigits; d <<= 1) {
            const uint32_t u = tid >= d ? wcount[0][tid - d] : 0u;
            __syncthreads();
            wcount[0][tid] += u;
            __syncthreads();
        }
        first[tid] = wcount[0][tid] - c;
        base[tid] = wcount[0][tid] - c;
        __syncthreads();
    }
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const uint64_t tile0 = (uint64_t)blockIdx.x * kTile;
    for (int r = 0; r < kRounds; ++r) {
        uint64_t i = tile0 + (uint64_t)r * kThreads + tid;
        bool valid = i < n;
        uint64_t key = valid ? kin[i] : 0;
        uint32_t val = valid ? vin[i] : 0;
        uint32_t digit = (uint32_t)((key >> shift) & 0xff);
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            uint64_t b = __ballot((digit >> bit) & 1u);
            peers &= ((digit >> bit) & 1u) ? b : ~b;
        }
        uint32_t rank = (uint32_t)__popcll(peers & lt);
        uint32_t cnt = (uint32_t)__popcll(peers);
#pragma unroll
        for (int w = 0; w < kThreads / 64; ++w) wcount[w][tid] = 0;
        __syncthreads();
        if (valid && rank == 0) wcount[wave][digit] = cnt;
        __syncthreads();
        {
            uint32_t run = base[tid];
#pragma unroll
            for (int w = 0; w < kThreads / 64; ++w) {
                uint32_t c = wcount[w][tid];
                wcount[w][tid] = run;
                run += c;
            }
            base[tid] = run;
        }
        __syncthreads();
        if (valid) {
            const uint32_t pos = wcount[wave][digit] + rank;   // tile-local, digit order
            skey[pos] = key;
            sval[pos] = val;
        }
        __syncthreads();
    }
    // write-out: consecutive threads take consecutive entries of the digit-ordered
    // tile, so each digit's run lands on consecutive global positions
    const uint32_t valid_n = (uint32_t)min<uint64_t>((uint64_t)kTile, n - tile0);
    for (uint32_t j = tid; j < valid_n; j += kThreads) {
        const uint64_t key = skey[j];
        const uint32_t digit = (uint32_t)((key >> shift) & 0xff);
        const uint64_t pos = (uint64_t)offsets[(uint64_t)digit * tiles + blockIdx.x] + (j - first[digit]);
        kout[pos] = key;
        vout[pos] = sval[j];
    }
}

}  // namespace

void radix_sort_pairs(Context& ctx, uint64_t* keys, uint32_t* vals, uint64_t* keys_tmp, uint32_t* vals_tmp,
                      uint64_t n, int bits)
{
    if (n <= 1) return;
    const uint32_t tiles = (uint32_t)((n + kTile - 1) / kTile);
    // per tile and digit: the counts, and their exclusive scan (digit-major)
    uint32_t* hist = static_cast<uint32_t*>(ctx.alloc((size_t)2 * kDigits * tiles * sizeof(uint32_t)));
    uint32_t* offs = hist + (size_t)kDigits * tiles;
    uint64_t* ka = keys;
    uint32_t* va = vals;
    uint64_t* kb = keys_tmp;
    uint32_t* vb = vals_tmp;
    int passes = (bits + 7) / 8;
    for (int p = 0; p < passes; ++p) {
        int shift = 8 * p;
        hipLaunchKernelGGL(digit_histogram, dim3(tiles), dim3(kThreads), 0, ctx.stream, ka, n, shift, hist, tiles);
        LAUNCH_CHECK("digit_histogram");
        scan_exclusive(ctx, hist, offs, (uint64_t)kDigits * tiles, nullptr);
        hipLaunchKernelGGL(digit_scatter, dim3(tiles), dim3(kThreads), 0, ctx.stream, ka, va, kb, vb, n, shift, offs, hist,
                           tiles);
        LAUNCH_CHECK("digit_scatter");
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    if (ka != keys) {
        HIP_CHECK(hipMemcpyAsync(keys, ka, n * sizeof(uint64_t), hipMemcpyDeviceToDevice, ctx.stream));
        HIP_CHECK(hipMemcpyAsync(vals, va, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, ctx.stream));
    }
    ctx.release(hist);
}

}  // namespace ngr
