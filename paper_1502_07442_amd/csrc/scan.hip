// Device-wide exclusive prefix sum of uint32 values (tiles of 2048, then a
// recursive scan of the tile sums). Used by the sort, the tree build and the
// group formation.
#include "ngr_internal.hpp"

namespace ngr {
namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

__device__ inline uint32_t wave_inclusive(uint32_t v, int lane)
{
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t u = __shfl_up(v, d, 64);
        if (lane >= d) v += u;
    }
    return v;
}

__global__ __launch_bounds__(kScanThreads) void scan_tiles(const uint32_t* in,
                                                           uint32_t* out, uint64_t n,
                                                           uint32_t* __restrict__ tile_sums)
{
    __shared__ uint32_t wsum[kScanThreads / 64];
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile + (uint64_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t acc = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        uint64_t i = base + k;
        v[k] = i < n ? in[i] : 0u;
        acc += v[k];
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t incl = wave_inclusive(acc, lane);
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    uint32_t wofs = 0, total = 0;
#pragma unroll
    for (int w = 0; w < kScanThreads / 64; ++w) {
        if (w < wave) wofs += wsum[w];
        total += wsum[w];
    }
    uint32_t run = wofs + incl - acc;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        uint64_t i = base + k;
        uint32_t x = v[k];
        if (i < n) out[i] = run;
        run += x;
    }
    if (tile_sums && threadIdx.x == 0) tile_sums[blockIdx.x] = total;
}

__global__ void add_tile_offsets(uint32_t* __restrict__ out, uint64_t n, const uint32_t* __restrict__ ofs)
{
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] += ofs[i / kScanTile];
}

}  // namespace

void scan_exclusive(Context& ctx, const uint32_t* in, uint32_t* out, uint64_t n, uint32_t* total)
{
    if (n == 0) {
        if (total) HIP_CHECK(hipMemsetAsync(total, 0, sizeof(uint32_t), ctx.stream));
        return;
    }
    uint64_t tiles = (n + kScanTile - 1) / kScanTile;
    if (tiles == 1) {
        hipLaunchKernelGGL(scan_tiles, dim3(1), dim3(kScanThreads), 0, ctx.stream, in, out, n, total);
        LAUNCH_CHECK("scan_tiles");
        return;
    }
    uint32_t* sums = static_cast<uint32_t*>(ctx.alloc(tiles * sizeof(uint32_t)));
    hipLaunchKernelGGL(scan_tiles, dim3((unsigned)tiles), dim3(kScanThreads), 0, ctx.stream, in, out, n, sums);
    LAUNCH_CHECK("scan_tiles");
    scan_exclusive(ctx, sums, sums, tiles, total);
    hipLaunchKernelGGL(add_tile_offsets, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, ctx.stream, out, n, sums);
    LAUNCH_CHECK("add_tile_offsets");
    ctx.release(sums);
}

}  // namespace ngr
