// Stable least-significant-digit radix sort of (uint64 key, uint32 value)
// pairs, 8 bits per pass. Every pass: a per-tile digit histogram, one
// exclusive scan over the digit-major histogram table, and a scatter. In the
// scatter each wave loads its share of the tile at once and ranks it in input
// order (wave-wide ballots find the lanes sharing a digit), which keeps the
// sort stable; the waves' digit counts are then combined once. The ranked
// tile is laid out in LDS in digit order, then written out so that each
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
                                                          const uint32_t* __restrict__ offsets, uint32_t tiles)
{
    constexpr int kWaves = kThreads / 64;
    __shared__ uint32_t wcount[kWaves][kDigits];   // per wave: digit counts, then the wave's start per digit
    __shared__ uint32_t dest_base[kDigits];         // per digit: global start of its run minus the tile-local start
    __shared__ uint32_t wsum[kWaves];
    __shared__ uint64_t skey[kTile];
    __shared__ uint32_t sval[kTile];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
#pragma unroll
    for (int j = 0; j < kDigits / 64; ++j) wcount[wave][lane + 64 * j] = 0;
    const uint32_t gstart = offsets[(uint64_t)tid * tiles + blockIdx.x];   // digit tid's global start for this tile
    // a wave owns kRounds x 64 consecutive keys of the tile; all its loads are issued before the ranking
    const uint64_t tile0 = (uint64_t)blockIdx.x * kTile;
    const uint64_t w0 = tile0 + (uint64_t)wave * (kRounds * 64) + lane;
    uint64_t key[kRounds];
    uint32_t val[kRounds], rank[kRounds];
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
        const uint64_t i = w0 + (uint64_t)r * 64;
        key[r] = i < n ? kin[i] : 0ull;
        val[r] = i < n ? vin[i] : 0u;
    }
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    // wave-local ranking in input order: lanes sharing a digit are found with
    // ballots; the lowest of them advances the wave's count of that digit
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
        const bool valid = w0 + (uint64_t)r * 64 < n;
        const uint32_t digit = (uint32_t)((key[r] >> shift) & 0xff);
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const uint64_t b = __ballot((digit >> bit) & 1u);
            peers &= ((digit >> bit) & 1u) ? b : ~b;
        }
        const uint32_t pre = (uint32_t)__popcll(peers & lt);
        const uint32_t before = wcount[wave][digit];
        __builtin_amdgcn_wave_barrier();
        rank[r] = before + pre;
        if (valid && pre == 0) wcount[wave][digit] = before + (uint32_t)__popcll(peers);
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    // thread d: the tile's count of digit d, its tile-local start (a scan over
    // the digits: shuffles within a wave, wave totals through LDS) and the
    // start of each wave's run of d
    {
        uint32_t c[kWaves], tot = 0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) {
            c[w] = wcount[w][tid];
            tot += c[w];
        }
        uint32_t inc = tot;
#pragma unroll
        for (int s = 1; s < 64; s <<= 1) {
            const uint32_t u = __shfl_up(inc, s);
            if (lane >= s) inc += u;
        }
        if (lane == 63) wsum[wave] = inc;
        __syncthreads();
        uint32_t run = inc - tot;
        for (int w = 0; w < wave; ++w) run += wsum[w];
        dest_base[tid] = gstart - run;   // modulo 2^32; every position is below 2^32
#pragma unroll
        for (int w = 0; w < kWaves; ++w) {
            wcount[w][tid] = run;
            run += c[w];
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
        if (w0 + (uint64_t)r * 64 < n) {
            const uint32_t pos = wcount[wave][(uint32_t)((key[r] >> shift) & 0xff)] + rank[r];   // tile-local, digit order
            skey[pos] = key[r];
            sval[pos] = val[r];
        }
    }
    __syncthreads();
    // write-out: consecutive threads take consecutive entries of the digit-ordered
    // tile, so each digit's run lands on consecutive global positions
    const uint32_t valid_n = (uint32_t)min<uint64_t>((uint64_t)kTile, n - tile0);
#pragma unroll 4
    for (uint32_t j = tid; j < valid_n; j += kThreads) {
        const uint64_t k = skey[j];
        const uint64_t pos = dest_base[(uint32_t)((k >> shift) & 0xff)] + j;
        kout[pos] = k;
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
        hipLaunchKernelGGL(digit_scatter, dim3(tiles), dim3(kThreads), 0, ctx.stream, ka, va, kb, vb, n, shift, offs,
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
