// Sink groups and the short-range group tree walk.
//
// Paper: Croker, ngravs (CPC). Eq. (1) and section 2.1: the pair force of a
// sink of species a and a source of species b is a per-pair law f_ab times
// the Newtonian force, with the active mass as a multiplier and the passive
// mass divided out. Section 2.2: one walk vectorised over the species'
// monopoles of each node; in the limit of one particle per monopole the walk
// reproduces the direct sum. Section 2.4.1: in TreePM mode the walk is
// restricted to short range and the force is modulated by a table of N_TAB
// samples of the short-range factor.
//
// Design (gfx950): one wavefront walks the tree for one species-pure group of
// at most 64 sinks (one sink per lane). The traversal is breadth-first in
// batches of 64 nodes, one node per lane, on a per-wave stack in device
// memory; nodes whose monopoles are accepted and leaves that are opened are
// buffered in LDS. Full buffers are expanded, one source species at a time,
// into LDS records {offset from the group centre (float64 x3), G_ab * mass}
// that every lane reads by broadcast while it evaluates the pair term for its
// own sink. The sink species' D force-factor tables sit in LDS as
// (value, slope) pairs and are read by a per-lane gather.
//
// Arithmetic per pair: offsets, r^2 and the accumulation in float64 (full
// rate on the vector ALU, like unpacked float32); the table interpolation and
// (r^2 + eps^2)^(-3/2), the cube of the hardware reciprocal square root, in
// float32.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "ngr_internal.hpp"

// Records evaluated per iteration of the pair loop (independent chains for
// the scheduler to interleave).
#ifndef NGR_EVAL_UNROLL
#define NGR_EVAL_UNROLL 4
#endif
#define NGR_STR2(x) #x
#define NGR_PRAGMA_UNROLL(n) _Pragma(NGR_STR2(unroll n))

namespace ngr {
namespace {

// Inclusive scans (sum or maximum) over the 64 lanes of a wave, all lanes
// active: DPP row shifts by 1, 2, 4 and 8 within each row of 16 lanes
// (lanes shifted in from outside the row read 0), then the last lane of
// rows 0 and 2 added into rows 1 and 3, and lane 31 into rows 2 and 3.
template <bool MAX>
__device__ inline uint32_t wave_scan(uint32_t v)
{
    auto join = [&](int u) { v = MAX ? max(v, (uint32_t)u) : v + (uint32_t)u; };
    join(__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, true));    // row_shr:1
    join(__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, true));    // row_shr:2
    join(__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, true));    // row_shr:4
    join(__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, true));    // row_shr:8
    join(__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false));   // row_bcast:15 into rows 1, 3
    join(__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false));   // row_bcast:31 into rows 2, 3
    return v;
}
__device__ inline uint32_t wave_incl(uint32_t v) { return wave_scan<false>(v); }
__device__ inline uint32_t lane63(uint32_t v) { return (uint32_t)__builtin_amdgcn_readlane((int)v, 63); }

// ------------------------------------------------------------- groups ----
// One thread per (node, species a). For a node holding more than Ng particles
// of species a (Ng of the node's box): a leaf is cut into chunks of Ng; an
// internal node groups runs of consecutive children whose species-a counts
// add up to at most Ng (children with more than Ng are handled by their own
// thread). A root forms one group when it holds at most Ng. Every group start
// is flagged.
__global__ void mark_group_starts(uint64_t nn, uint32_t D, const uint32_t* __restrict__ Ng_box,
                                  const uint32_t* __restrict__ node_box, const uint32_t* __restrict__ start,
                                  const uint32_t* __restrict__ count, const int32_t* __restrict__ parent,
                                  const int32_t* __restrict__ first_child, const uint8_t* __restrict__ n_child,
                                  uint32_t* __restrict__ flags)
{
    uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nn * D) return;
    uint64_t i = t / D;
    uint32_t a = (uint32_t)(t % D);
    uint32_t na = count[i * D + a];
    if (na == 0) return;
    const uint32_t Ng = Ng_box[node_box[i]];
    if (na <= Ng) {
        if (parent[i] < 0) flags[start[i * D + a]] = 1;
        return;
    }
    if (n_child[i] == 0) {
        uint32_t s0 = start[i * D + a];
        for (uint32_t k = 0; k < na; k += Ng) flags[s0 + k] = 1;
        return;
    }
    uint32_t run = 0;
    uint64_t c0 = (uint64_t)first_child[i], c1 = c0 + n_child[i];
    for (uint64_t c = c0; c < c1; ++c) {
        uint32_t nc = count[c * D + a];
        if (nc == 0) continue;
        if (nc > Ng) {
            run = 0;
            continue;
        }
        if (run + nc > Ng) run = 0;
        if (run == 0) flags[start[c * D + a]] = 1;
        run += nc;
    }
}

__global__ void scatter_group_starts(uint64_t n, const uint32_t* __restrict__ flags,
                                     const uint32_t* __restrict__ gidx, uint32_t* __restrict__ gstart)
{
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && flags[i]) gstart[gidx[i]] = (uint32_t)i;
}

// Count, integer bounding box (20-bit key lattice, hi exclusive) and box of
// each group; a group ends where the next one starts. One wave per group (at
// most 64 particles), one particle per lane.
__global__ void finish_groups(uint64_t ng, uint64_t n, uint32_t nbox, const uint64_t* __restrict__ boff,
                              const uint32_t* __restrict__ gstart, uint32_t* __restrict__ gcount,
                              uint32_t* __restrict__ glo, uint32_t* __restrict__ ghi, uint32_t* __restrict__ gbox,
                              const uint64_t* __restrict__ X, uint32_t* __restrict__ error_flag)
{
    const uint64_t g = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;   // the same for the whole wave
    const uint32_t lane = threadIdx.x & 63u;
    if (g >= ng) return;
    const uint64_t s = gstart[g], e = (g + 1 < ng) ? gstart[g + 1] : n;
    // box: the last k with boff[k] <= s
    uint32_t lo = 0, hi = nbox;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (boff[mid] <= s) lo = mid;
        else hi = mid;
    }
    if (e <= s || e - s > 64 || e > n || e > boff[lo + 1]) {   // groups hold 1..64 particles of one box
        if (lane == 0) {
            atomicOr(error_flag, 1u);
            gcount[g] = 0;
        }
        return;
    }
    // per axis, wave-wide maxima of k + 1 and of ~k (the complement of the
    // minimum); an empty lane holds 0 for both, which changes neither
    uint32_t nl[3] = {0u, 0u, 0u}, h[3] = {0u, 0u, 0u};
    if (s + lane < e) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const uint32_t k = (uint32_t)(X[a * n + s + lane] >> 44);
            nl[a] = ~k;
            h[a] = k + 1;
        }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        nl[a] = wave_scan<true>(nl[a]);
        h[a] = wave_scan<true>(h[a]);
    }
    if (lane == 63) {
        gcount[g] = (uint32_t)(e - s);
        gbox[g] = lo;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            glo[a * ng + g] = ~nl[a];
            ghi[a * ng + g] = h[a];
        }
    }
}

// First group of each segment: the group index at the segment's first sorted
// position (a position of n, past the end, gives ng).
__global__ void segment_firsts(uint32_t k, const uint64_t* __restrict__ pos, const uint32_t* __restrict__ gidx,
                               uint64_t n, uint32_t ng, uint32_t* __restrict__ out)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < k) out[t] = pos[t] < n ? gidx[pos[t]] : ng;
}

// ------------------------------------------------------- group order ----
// The walk hands out each segment's groups heaviest first. A group's cost is
// estimated as the number of particles within reach of its box times the
// share of a wave pass its sinks take: the particles are counted on a level-L
// grid of the group's simulation box (cells at least r_cut wide) over the
// cells that the group's bounding box covers, grown by one cell on every
// side; the share is 1/4, 1/2, 3/4 or 1 for groups of at most 16, 32, 48 or
// 64 sinks (the lane mappings of the walk). Cells of level L carry the total
// count of their node; particles of leaves above level L are counted one by
// one. The grid is then turned into a summed-volume table, so that any block
// of cells costs eight reads.

__global__ void density_grid(uint64_t nodes, uint32_t D, const uint32_t* __restrict__ Lbox,
                             const uint64_t* __restrict__ Hoff, const uint32_t* __restrict__ node_box,
                             const uint4* __restrict__ cell, const uint8_t* __restrict__ n_child,
                             const uint32_t* __restrict__ start, const uint32_t* __restrict__ count,
                             const uint64_t* __restrict__ X, uint64_t n, uint32_t* __restrict__ Hall)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nodes) return;
    const uint32_t box = node_box[i];
    const uint32_t L = Lbox[box];
    if (L == 0) return;
    uint32_t* H = Hall + Hoff[box];
    const uint4 c = cell[i];
    const uint32_t sh = (uint32_t)kLevels - L;
    if (c.w == L) {
        uint32_t tot = 0;
        for (uint32_t b = 0; b < D; ++b) tot += count[i * D + b];
        H[((uint64_t)(c.x >> sh) << (2 * L)) | ((uint64_t)(c.y >> sh) << L) | (c.z >> sh)] = tot;
    } else if (c.w < L && n_child[i] == 0) {
        for (uint32_t b = 0; b < D; ++b) {
            const uint64_t s = start[i * D + b], e = s + count[i * D + b];
            for (uint64_t j = s; j < e; ++j) {
                const uint64_t x = X[j] >> (64 - L), y = X[n + j] >> (64 - L), z = X[2 * n + j] >> (64 - L);
                atomicAdd(&H[(x << (2 * L)) | (y << L) | z], 1u);
            }
        }
    }
}

// A group's estimated work from its cost bucket b (half-octave steps):
// 2^(b/2), exact for even b and 1.5 times the lower power for odd b.
__device__ inline unsigned long long bucket_weight(uint32_t b)
{
    return (b & 1u) ? (3ull << (b >> 1)) >> 1 : 1ull << (b >> 1);
}

// Inclusive prefix sums of every box's grid along one axis (2: z, 1: y, 0: x);
// after all three the grid is a summed-volume table. One thread per line;
// Loff[k] is the first line of box k (boxes without a grid have none).
__global__ void density_prefix(uint64_t lines, uint32_t nbox, uint32_t axis, const uint32_t* __restrict__ Lbox,
                               const uint64_t* __restrict__ Hoff, const uint64_t* __restrict__ Loff,
                               uint32_t* __restrict__ Hall)
{
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= lines) return;
    uint32_t lo = 0, hi = nbox;   // the box: the last k with Loff[k] <= t
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (Loff[mid] <= t) lo = mid;
        else hi = mid;
    }
    const uint32_t L = Lbox[lo];
    const uint64_t li = t - Loff[lo], N = 1ull << L;
    const uint64_t u = li >> L, w = li & (N - 1);   // the line's two other coordinates
    uint64_t base, stride;
    if (axis == 2) {
        base = (u << (2 * L)) | (w << L);            // (x, y) = (u, w)
        stride = 1;
    } else if (axis == 1) {
        base = (u << (2 * L)) | w;                   // (x, z) = (u, w)
        stride = N;
    } else {
        base = (u << L) | w;                         // (y, z) = (u, w)
        stride = N * N;
    }
    uint32_t* H = Hall + Hoff[lo] + base;
    uint32_t sum = 0;
    for (uint64_t i = 0; i < N; ++i) {
        sum += H[i * stride];
        H[i * stride] = sum;
    }
}

// Sort key of every group: its segment, then the cost bucket descending
// (half-octave steps of the estimate above); value: the group index.
__global__ void group_order_keys(uint64_t ng, uint32_t D, const uint32_t* __restrict__ gstart,
                                 const uint32_t* __restrict__ gcount, const uint32_t* __restrict__ glo,
                                 const uint32_t* __restrict__ ghi, const uint32_t* __restrict__ gbox,
                                 const uint32_t* __restrict__ Lbox, const uint64_t* __restrict__ Hoff,
                                 const uint64_t* __restrict__ keys, const uint32_t* __restrict__ Hall,
                                 uint64_t* __restrict__ okey, uint32_t* __restrict__ oval,
                                 uint32_t* __restrict__ gbucket)
{
    const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ng) return;
    const uint32_t box = gbox[g];
    const uint32_t L = Lbox[box];
    uint64_t v = 1;
    if (L > 0) {
        const uint32_t* S = Hall + Hoff[box];
        const uint32_t sh = (uint32_t)kLevels - L;
        const int32_t N = 1 << L;
        // per axis, the grown block as one or two cell ranges (periodic wrap)
        int32_t r0[3][2], r1[3][2], nr[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int32_t c0 = (int32_t)(glo[a * ng + g] >> sh) - 1, c1 = (int32_t)((ghi[a * ng + g] - 1u) >> sh) + 1;
            r0[a][1] = r1[a][1] = 0;
            if (c1 - c0 + 1 >= N) {
                nr[a] = 1;
                r0[a][0] = 0;
                r1[a][0] = N - 1;
            } else {
                const int32_t a0 = (c0 + N) & (N - 1), a1 = c1 & (N - 1);
                if (a0 <= a1) {
                    nr[a] = 1;
                    r0[a][0] = a0;
                    r1[a][0] = a1;
                } else {
                    nr[a] = 2;
                    r0[a][0] = a0;
                    r1[a][0] = N - 1;
                    r0[a][1] = 0;
                    r1[a][1] = a1;
                }
            }
        }
        auto at = [&](int32_t x, int32_t y, int32_t z) -> uint64_t {
            return (x < 0 || y < 0 || z < 0) ? 0ull : (uint64_t)S[((uint64_t)x << (2 * L)) | ((uint64_t)y << L) | (uint64_t)z];
        };
        for (int i = 0; i < nr[0]; ++i)
            for (int j = 0; j < nr[1]; ++j)
                for (int k = 0; k < nr[2]; ++k) {
                    const int32_t x0 = r0[0][i] - 1, x1 = r1[0][i], y0 = r0[1][j] - 1, y1 = r1[1][j], z0 = r0[2][k] - 1,
                                  z1 = r1[2][k];
                    v += at(x1, y1, z1) - at(x0, y1, z1) - at(x1, y0, z1) - at(x1, y1, z0) + at(x0, y0, z1) +
                         at(x0, y1, z0) + at(x1, y0, z0) - at(x0, y0, z0);
                }
    }
    const uint32_t ns = gcount[g];
    v *= ns <= 16u ? 1u : ns <= 32u ? 2u : ns <= 48u ? 3u : 4u;
    const uint32_t msb = 63u - (uint32_t)__builtin_clzll(v);
    const uint32_t half = msb ? (uint32_t)(v >> (msb - 1)) & 1u : 0u;
    const uint32_t bucket = 2u * msb + half;            // < 128
    const uint64_t seg = (uint64_t)box * D + (keys[gstart[g]] >> kKeyBits);
    okey[g] = (seg << 8) | (255u - bucket);
    oval[g] = (uint32_t)g;
    gbucket[g] = bucket;
}

// Estimated work of every segment, the sum of its groups' weights: one
// workgroup per segment (a segment's groups are consecutive).
__global__ __launch_bounds__(256) void seg_work_init(const uint32_t* __restrict__ seg_first,
                                                     const uint32_t* __restrict__ gbucket,
                                                     unsigned long long* __restrict__ seg_work)
{
    __shared__ unsigned long long part[256];
    const uint32_t s = blockIdx.x;
    const uint32_t g0 = seg_first[s], g1 = seg_first[s + 1];
    unsigned long long sum = 0;
    for (uint32_t g = g0 + threadIdx.x; g < g1; g += blockDim.x) sum += bucket_weight(gbucket[g]);
    part[threadIdx.x] = sum;
    __syncthreads();
    for (uint32_t d = 128; d > 0; d >>= 1) {
        if (threadIdx.x < d) part[threadIdx.x] += part[threadIdx.x + d];
        __syncthreads();
    }
    if (threadIdx.x == 0) seg_work[s] = part[0];
}

// --------------------------------------------------------------- walk ----
constexpr uint32_t kPrune = 0, kAccept = 1, kOpen = 2;
constexpr int kBuf = 128;              // node / leaf buffer entries per wave
constexpr int kRec = 68;               // record slots per wave: 64 and up to 3 pads
constexpr int kWaveLds = kRec * 32 + kBuf * 4 * 2 + 68 * 4 + 64 * 4 + 8 * 4;   // bytes of LDS per wave
constexpr int kMaxWaves = 16;          // waves per workgroup
constexpr int kArenaWaves = 4;         // arena mode: waves per workgroup, one workgroup per CU
constexpr uint32_t kArenaStack = 21 * 512 + 512;   // arena mode: stack entries per wave
constexpr int kCtrlBytes = 1536;       // LDS control area ahead of the tables (next segment, per-wave counts)
// Accumulator laws: per wave, the core scale of each record (float64) after
// the other buffers; per workgroup, the core-factor table after the force
// tables (kCoreN intervals on u = r / (s + r) in [0, 1], PAIR layout, the
// last entry (1, 0)).
constexpr int kWaveLdsAcc = kWaveLds + kRec * 8;
constexpr int kCoreN = 2048;
constexpr int kCoreBytes = ((kCoreN + 1) * 8 + 255) & ~255;
// Table layouts in LDS. PAIR: per interval (value, slope to the next sample),
// with a (0, 0) entry that the clamped index reaches for r >= r_cut. VALUE:
// the samples only (plus one pad), the slope taken from the next sample and
// r >= r_cut zeroed by a compare; half the LDS for twice the tables.
enum TableMode { kPair = 0, kValue = 1 };

// Force-law and walk parameters of one box. The walk works in units of the
// box side: offsets, eps^2 and the table scales are in those units and the
// records carry G_ab m / box^2, so that the pair term's float32 kernel factor
// (r^2 + eps^2)^(-3/2) has the same range whatever the caller's length unit
// (box is 1 here; the accelerations come out in the caller's units).
struct BoxParams {
    double box, inv_box, eps2, R2, theta2;
    double G[NGR_MAX_SPECIES * NGR_MAX_SPECIES];   // G_ab, row a = sink species, D x D
    double* acc;               // 3 x n output, input order
    uint64_t in_off, n;        // first input index (over all boxes) and particles of the box
    const float2* pair;        // the box's tables, PAIR layout
    const float* value;        // the box's tables, VALUE layout
    float tscale, toff, tmax;
    uint32_t wrap_limit, D, ntab;
    double inv4pib;            // accumulator laws: 1 / (4 pi beta); 0 for a table law
    uint32_t cored, track;     // cored species mask (0 for a table law); N_perp tracking
    const double* old_acc;     // relative opening test: previous |a| of the box's particles (input order)
    double rel_k;              // relative opening test: alpha (box / 2^21)^2
    uint32_t relative;         // 1: the relative opening test, 0: the geometric one
    const double* corr;        // lattice corrections (pure-tree periodic mode): D x D tables, or NULL
    uint32_t corr_n;           // their intervals per axis
    double corr_scale;         // corr_n / (box / 2)
    double eps2_ab[NGR_MAX_SPECIES * NGR_MAX_SPECIES];   // per-pair eps^2, row a = sink species
    float toff_ab[NGR_MAX_SPECIES * NGR_MAX_SPECIES];    // r^2-grid table offset -eps_ab^2 / h of each pair
    double tie_rc2, tie_band;  // near ties: r_cut^2 and the band 1e-6 r_cut^2
};

// Per-lane-invariant values of the pair term, taken from the box.
struct PairParams {
    double box, inv_box, eps2;
    float tscale, toff, tmax;
};

struct WalkArgs {
    const uint4* cell;
    const int32_t* first_child;
    const uint8_t* n_child;
    const uint32_t* start;
    const uint32_t* count;
    const double4* mono;
    uint64_t nn;
    const uint64_t* X;
    const PRec* P;
    const double* mass;
    const uint32_t* perm;
    uint64_t n;
    const uint32_t* gstart;
    const uint32_t* gcount;
    const uint32_t* glo;
    const uint32_t* ghi;
    uint64_t ng;
    uint32_t D;                // species stride of the tree; segment s = box * D + species
    uint32_t nseg;
    const uint32_t* order;     // group indices: segment by segment, heaviest first
    const uint32_t* seg_first; // nseg + 1: groups of segment s are order[seg_first[s] .. seg_first[s + 1])
    uint32_t* queues;          // nseg: groups of each segment handed out so far
    unsigned long long* seg_work;   // nseg: estimated work of the groups not yet handed out
    const uint32_t* gbucket;   // per group: its cost bucket (the queue order's estimate)
    const uint32_t* sched;     // non-empty segments, most groups first
    uint32_t nsched;
    uint32_t* cursor;          // next entry of sched to start
    const BoxParams* boxes;
    unsigned long long* seg_counts;   // nseg x kSegCounts: pp, pn, near ties, pn by source species
    unsigned long long* gcounts;
    uint32_t* stacks;
    uint32_t stack_cap;
    uint32_t* error_flag;
    uint32_t max_steps;        // traversal batches per group never exceed the node count
    uint32_t tab_bytes;        // LDS bytes of the largest segment's tables
    BoxParams box0;            // the box of a one-box call (read from the arguments)
    const float2* core;        // accumulator laws: the core-factor table (kCoreN + 1 entries)
};

__device__ inline void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__device__ inline uint32_t uniform(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// Pair terms of this lane's sink with LDS records of one source species:
// records rec[0], rec[K], rec[2K], ... (iters of them; the caller offsets rec
// by the lane's replica).
// Lattice correction of one pair (pure-tree periodic mode, section 2.3):
// the table T holds, on n intervals per axis of [0, box/2]^3, the extra
// acceleration from every image of a unit source but the nearest; odd in
// each component's own axis, even in the others, so it is read trilinearly
// at |d| and each component takes the sign of its axis.
__device__ inline void lattice_correction(const double* __restrict__ T, uint32_t n, double scale, double dx,
                                          double dy, double dz, double& cx, double& cy, double& cz)
{
    const double u0 = fabs(dx) * scale, u1 = fabs(dy) * scale, u2 = fabs(dz) * scale;
    const uint32_t i0 = min((uint32_t)u0, n - 1u), i1 = min((uint32_t)u1, n - 1u), i2 = min((uint32_t)u2, n - 1u);
    const double f0 = u0 - i0, f1 = u1 - i1, f2 = u2 - i2;
    const uint64_t m = n + 1u;
    double sx = 0.0, sy = 0.0, sz = 0.0;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const uint32_t a = c >> 2, b = (c >> 1) & 1, d = c & 1;
        const double w = (a ? f0 : 1.0 - f0) * (b ? f1 : 1.0 - f1) * (d ? f2 : 1.0 - f2);
        const double* e = T + (((uint64_t)(i0 + a) * m + (i1 + b)) * m + (i2 + d)) * 3;
        sx = fma(w, e[0], sx);
        sy = fma(w, e[1], sy);
        sz = fma(w, e[2], sz);
    }
    cx = dx < 0.0 ? -sx : sx;
    cy = dy < 0.0 ? -sy : sy;
    cz = dz < 0.0 ? -sz : sz;
}

// Lattice corrections for the pair term (EW): table, intervals and scale.
struct LatticeCorr {
    const double* T;
    uint32_t n;
    double scale;
};

// Near-tie count (TIES): pair terms whose r^2 lies within `band` of rc2,
// the pairs a finite-precision cut-off test may keep or drop. Returned by
// the pair loop (0 without TIES).
struct TieBand {
    double rc2, band;
};

template <int GRID, int TAB, bool EPS0, bool WRAP, uint32_t K, bool EW = false, bool TIES = false>
__device__ inline uint32_t eval_records(const PairParams& A, double eps2, float toff, const double4* __restrict__ rec,
                                        uint32_t iters, const void* __restrict__ tbv, double ox, double oy, double oz,
                                        double& ax, double& ay, double& az,
                                        LatticeCorr lc = LatticeCorr{nullptr, 0u, 0.0}, TieBand tb = TieBand{0.0, -1.0})
{
    // a launch that holds unsoftened pairs evaluates its softened pairs exactly
    // as a launch without any (a box in a batch equals its single-box call)
    if (EPS0 && eps2 != 0.0)
        return eval_records<GRID, TAB, false, WRAP, K, EW, TIES>(A, eps2, toff, rec, iters, tbv, ox, oy, oz, ax, ay, az,
                                                                 lc, tb);
    uint32_t nties = 0;
    const float tscale = A.tscale, tmax = A.tmax;
    NGR_PRAGMA_UNROLL(NGR_EVAL_UNROLL)
    for (uint32_t it = 0; it < iters; ++it) {
        const double4 s = rec[it * K];
        double dx = s.x - ox, dy = s.y - oy, dz = s.z - oz;
        if (WRAP) {
            dx -= A.box * rint(dx * A.inv_box);
            dy -= A.box * rint(dy * A.inv_box);
            dz -= A.box * rint(dz * A.inv_box);
        }
        const double re2 = fma(dx, dx, fma(dy, dy, fma(dz, dz, eps2)));   // r^2 + eps^2
        if (TIES) {
            const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
            nties += fabs(r2 - tb.rc2) <= tb.band ? 1u : 0u;
        }
        const float sf = (float)re2;
        // (r^2+eps^2)^(-3/2) in float32 from the hardware rsqrt: a relative
        // error of a few 1e-7, the precision of the float32 table factor it
        // multiplies (finite for r^2+eps^2 above ~2e-26). Without softening
        // (EPS0, reached only for pairs with eps = 0) a pair can be closer
        // than that: there the cube is taken in float64 and refined (with
        // e = 1 - re2 z^2, z^3 (1 + 1.5 e) to ~1e-13).
        const float z = __builtin_amdgcn_rsqf(sf);
        float z3 = 0.0f;
        double z3d = 0.0;
        if (EPS0) {
            const double zd = (double)z, z2 = zd * zd;
            z3d = z2 * zd * fma(-1.5 * re2, z2, 2.5);
        } else {
            z3 = z * z * z;
        }
        float t;
        if (GRID == NGR_GRID_R2) t = fmaf(sf, tscale, toff);                 // r^2 / h, from r^2 + eps^2
        else t = __builtin_sqrtf((float)(re2 - eps2)) * tscale;             // r / h
        t = __builtin_amdgcn_fmed3f(t, 0.0f, tmax);
        const int k = (int)t;
        const float w = __builtin_amdgcn_fractf(t);
        float f;
        if (TAB == kPair) {
            const float2 T = static_cast<const float2*>(tbv)[k];
            f = fmaf(w, T.y, T.x);
        } else {
            const float* tv = static_cast<const float*>(tbv);
            const float t0 = tv[k], t1 = tv[k + 1];
            f = t < tmax ? fmaf(w, t1 - t0, t0) : 0.0f;
        }
        double coef = EPS0 ? (double)f * s.w * z3d : (double)(f * z3) * s.w;   // records carry G m
        if (EPS0) coef = re2 > 0.0 ? coef : 0.0;
        ax = fma(coef, dx, ax);
        ay = fma(coef, dy, ay);
        az = fma(coef, dz, az);
        if (EW) {
            double cx, cy, cz;
            lattice_correction(lc.T, lc.n, lc.scale, dx, dy, dz, cx, cy, cz);
            const double gm = s.w;
            ax = fma(gm, cx, ax);
            ay = fma(gm, cy, ay);
            az = fma(gm, cz, az);
        }
    }
    return nties;
}

// Pair terms of a cored pair of species (accumulator laws). With s the
// pair's core scale (record's core plus the sink's), the force of the
// Eq. (14) potential is (2/pi) [atan x - x / (1 + x^2)] / r^3, x = r / s.
// Written as C(u) / (s + r)^3 with u = r / (s + r), C is smooth and between
// 0.42 and 1.54 on [0, 1] and is read, linearly interpolated, from a table
// of kCoreN intervals (relative error below 3e-7); C(1) = 1 gives the
// Newtonian factor, so a pair without a core (s = 0) takes the softened law
// from r -> sqrt(r^2 + eps^2). r and 1 / (s + r) are the float32 hardware
// estimates (rsqrt times r^2, reciprocal), cubed in float64. The records
// carry G m / box^2 and rs[] the source's core scale (lengths in box units).
template <int GRID, int TAB, bool WRAP, uint32_t K>
__device__ inline void eval_cored(const PairParams& A, double eps2, const double4* __restrict__ rec,
                                  const double* __restrict__ rs, uint32_t iters, const void* __restrict__ tbv,
                                  const float2* __restrict__ core, double s_sink, double ox, double oy, double oz,
                                  double& ax, double& ay, double& az)
{
    const float tscale = A.tscale, tmax = A.tmax, eps2f = (float)eps2;
    NGR_PRAGMA_UNROLL(NGR_EVAL_UNROLL)
    for (uint32_t it = 0; it < iters; ++it) {
        const double4 s = rec[it * K];
        const double sc = rs[it * K] + s_sink;
        double dx = s.x - ox, dy = s.y - oy, dz = s.z - oz;
        if (WRAP) {
            dx -= A.box * rint(dx * A.inv_box);
            dy -= A.box * rint(dy * A.inv_box);
            dz -= A.box * rint(dz * A.inv_box);
        }
        const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
        // float32 from here: r and 1 / (s + r) from the hardware estimates,
        // a relative error of a few 1e-7, the precision of the float32 tables
        const float r2f = (float)r2, scf = (float)sc;
        const float re2 = scf > 0.0f ? r2f : r2f + eps2f;
        const float rr = re2 * __builtin_amdgcn_rsqf(re2);         // r (softened when s = 0)
        const float y = __builtin_amdgcn_rcpf(scf + rr);           // 1 / (s + r)
        float tu = rr * y * (float)kCoreN;
        tu = __builtin_amdgcn_fmed3f(tu, 0.0f, (float)kCoreN);
        // r = 0 makes tu NaN (its term is dropped below): the unsigned clamp
        // keeps the index inside the table whatever the conversion gives
        const uint32_t ku = min((uint32_t)(int)tu, (uint32_t)kCoreN);
        const float2 Cu = core[ku];
        const float c = fmaf(__builtin_amdgcn_fractf(tu), Cu.y, Cu.x);
        float t;
        if (GRID == NGR_GRID_R2) t = (float)r2 * tscale;
        else t = __builtin_sqrtf((float)r2) * tscale;
        t = __builtin_amdgcn_fmed3f(t, 0.0f, tmax);
        const int k = (int)t;
        const float w = __builtin_amdgcn_fractf(t);
        float f;
        if (TAB == kPair) {
            const float2 T = static_cast<const float2*>(tbv)[k];
            f = fmaf(w, T.y, T.x);
        } else {
            const float* tv = static_cast<const float*>(tbv);
            const float t0 = tv[k], t1 = tv[k + 1];
            f = t < tmax ? fmaf(w, t1 - t0, t0) : 0.0f;
        }
        // the cube in float64: a pair without core or softening (s = eps = 0)
        // may be closer than float32's cube allows (r below ~1e-13 box)
        const double yd = (double)y;
        double coef = (double)(f * c) * (yd * yd * yd) * s.w;
        coef = r2 > 0.0 ? coef : 0.0;
        ax = fma(coef, dx, ax);
        ay = fma(coef, dy, ay);
        az = fma(coef, dz, az);
    }
}

// Bytes of LDS the tables of one sink species take in a layout.
__host__ __device__ inline uint32_t table_bytes(int mode, uint32_t D, uint32_t ntab)
{
    const uint32_t raw = mode == kPair ? D * ntab * 8u : D * (ntab + 1u) * 4u;
    return (raw + 255u) & ~255u;
}

// Counters of one segment: pp, pn, near ties, then pn by source species.
constexpr int kSegCounts = 3 + NGR_MAX_SPECIES;

template <int GRID, int TAB, bool EPS0, bool ONE, bool ACC, bool EW = false, bool TIES = false>
__global__ __launch_bounds__(kMaxWaves * 64) void walk_kernel(WalkArgs A)
{
    constexpr int kBlocks = ACC || EW ? 1 : 3;   // sink blocks a lane can serve
    HIP_DYNAMIC_SHARED(unsigned char, smem);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
    const uint32_t D = A.D;                // species stride of the node arrays
    // LDS: control area (next segment; per-wave counts), the tables of one
    // segment, then per-wave buffers
    int32_t* ctrl = reinterpret_cast<int32_t*>(smem);
    unsigned long long* part = reinterpret_cast<unsigned long long*>(smem + 256);   // kSegCounts per wave
    unsigned char* tsm = smem + kCtrlBytes;
    constexpr int kWL = ACC ? kWaveLdsAcc : kWaveLds;
    unsigned char* wb = tsm + A.tab_bytes + wave * kWL;
    double4* rec = reinterpret_cast<double4*>(wb);
    double* recs = reinterpret_cast<double*>(wb + kWaveLds);            // ACC: core scale of each record
    float2* core_tab = reinterpret_cast<float2*>(tsm + A.tab_bytes - kCoreBytes);   // ACC
    uint32_t* pnb = reinterpret_cast<uint32_t*>(wb + kRec * 32);
    uint32_t* ppb = pnb + kBuf;
    uint32_t* scanb = ppb + kBuf;        // 68 entries
    uint32_t* pst = scanb + 68;          // 64 entries
    uint32_t* gpn = pst + 64;            // the group's particle-node records by source species (8 entries)
    unsigned long long* wcnt = part + kSegCounts * wave;   // this wave's counts of the segment
    uint32_t* stack = A.stacks + ((uint64_t)blockIdx.x * nwaves + wave) * A.stack_cap;
    const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    const uint64_t n = A.n;

    // One launch serves every segment (box, sink species). A workgroup holds
    // the tables of one segment at a time. Workgroups start on the segments
    // with the most groups (spread over them when there are fewer segments
    // than workgroups); when its segment's queue is empty, the whole
    // workgroup takes the next segment not yet started and, once every
    // segment has started, joins the one with the most groups left.
    uint32_t seg = A.sched[blockIdx.x % A.nsched];
    bool any_overflow = false;
    if (ACC)   // the core-factor table is the same for every segment; the first segment's barrier publishes it
        for (uint32_t k = threadIdx.x; k <= (uint32_t)kCoreN; k += blockDim.x) core_tab[k] = A.core[k];
    for (;;) {
        const uint32_t bxi = seg / D, a = seg % D;
        const BoxParams& P = ONE ? A.box0 : A.boxes[bxi];
        const uint32_t Dk = P.D, ntab = P.ntab;
        const uint32_t tstride = TAB == kPair ? ntab : ntab + 1;   // entries per table
        if (TAB == kPair) {
            float2* tab = reinterpret_cast<float2*>(tsm);
            const float2* src = P.pair + (uint64_t)a * Dk * ntab;
            for (uint32_t k = threadIdx.x; k < Dk * ntab; k += blockDim.x) tab[k] = src[k];
        } else {
            float* tab = reinterpret_cast<float*>(tsm);
            const float* src = P.value + (uint64_t)a * Dk * (ntab + 1);
            for (uint32_t k = threadIdx.x; k < Dk * (ntab + 1); k += blockDim.x) tab[k] = src[k];
        }
        __syncthreads();
        const PairParams pp{P.box, P.inv_box, P.eps2, P.tscale, P.toff, P.tmax};
        const double R2 = P.R2, theta2 = P.theta2, bx = P.box, scale = P.box * 0x1p-64;
        const uint32_t wrap_limit = P.wrap_limit;
        double* const acc = P.acc;
        const uint64_t in_off = P.in_off, nbx = P.n;
        const double* const Ga = P.G + a * Dk;
        const uint32_t g_begin = A.seg_first[seg], g_count = A.seg_first[seg + 1] - g_begin;
        const uint32_t cmask = ACC ? P.cored : 0u;          // cored species (accumulator laws)
        const bool core_a = (cmask >> a) & 1u;
        const double inv4pib = P.inv4pib;
        const bool track = P.track != 0u;
        uint32_t* const queue = A.queues + seg;
        const double tie_rc2 = P.tie_rc2, tie_band = P.tie_band;
        // the segment's counts accumulate in LDS (no registers held across groups)
        if ((uint32_t)lane < (uint32_t)kSegCounts) wcnt[lane] = 0ull;

    // Waves take groups from the segment's queue. Every lane executes the
    // atomic (lane 0 adds one, the others add zero), so no lane-dependent
    // branch surrounds it; lane 0 is the first active lane and its return
    // value is the wave's ticket. The loop exit then depends only on that
    // wave-uniform value and the lanes of a wave stay together (cross-lane
    // operations inside the loop need all of them).
    for (;;) {
        const uint32_t ticket = uniform(atomicAdd(queue, lane == 0 ? 1u : 0u));
        if (ticket >= g_count) break;
        const uint32_t g = A.order[g_begin + ticket];
        // the segment's work left drops by this group's weight; as for the
        // ticket, every lane executes the atomic (lane 0 subtracts)
        const unsigned long long wq = bucket_weight(uniform(A.gbucket[g]));
        atomicAdd(A.seg_work + seg, lane == 0 ? 0ull - wq : 0ull);
        const uint32_t s0 = A.gstart[g], ns = A.gcount[g];
        uint32_t lo[3], hi[3];
        bool wrap = false;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            lo[k] = A.glo[k * A.ng + g];
            hi[k] = A.ghi[k * A.ng + g];
            wrap |= (hi[k] - lo[k]) > wrap_limit;
        }
        wrap = wrap || EW;                // every pair needs its nearest image there
        // group centre: lattice units and box fraction
        const uint64_t C0 = (uint64_t)(lo[0] + hi[0]) << 43, C1 = (uint64_t)(lo[1] + hi[1]) << 43,
                       C2 = (uint64_t)(lo[2] + hi[2]) << 43;
        const double cf0 = (double)(lo[0] + hi[0]) * 0x1p-21, cf1 = (double)(lo[1] + hi[1]) * 0x1p-21,
                     cf2 = (double)(lo[2] + hi[2]) * 0x1p-21;
        // A group of at most 32 (16) sinks runs K = 2 (4) copies of itself,
        // one per 32 (16) lanes; copy q takes records q, q + K, q + 2K, ...
        // and the copies' sums are added at the end. Far away massless pads
        // after the last record give the copies equal trip counts. A group of
        // 33 to 48 sinks (table laws: a launch holds one law kind, and no
        // wrap) runs as three blocks of 16
        // sinks in K = 4 copies: lane l serves the sinks l mod 16 + 16 m,
        // m = 0, 1, 2, each over every fourth record, which costs three
        // quarters of one pass with a sink per lane. Groups that need the
        // periodic wrap run one copy.
        const bool blocks = !ACC && !wrap && ns > 32u && ns <= 48u;
        const uint32_t nblk = blocks ? 3u : 1u;
        const uint32_t lk = wrap ? 0u : (ns <= 16u || blocks) ? 2u : ns <= 32u ? 1u : 0u;
        const uint32_t K = 1u << lk;
        const uint32_t sink = (uint32_t)lane & ((64u >> lk) - 1u), replica = (uint32_t)lane >> (6u - lk);
        const double4* const rrec = rec + replica;
        // a million boxes away: past every cut-off (the table factor is 0), yet
        // r^2 stays finite in float32 for boxes below ~1e13
        const double4 pad = make_double4(1e6 * bx, 1e6 * bx, 1e6 * bx, 0.0);
        double ox[kBlocks], oy[kBlocks], oz[kBlocks], ax[kBlocks], ay[kBlocks], az[kBlocks];
#pragma unroll
        for (int m = 0; m < kBlocks; ++m) {
            ox[m] = oy[m] = oz[m] = ax[m] = ay[m] = az[m] = 0.0;
            const uint32_t sm = sink + 16u * (uint32_t)m;
            if ((uint32_t)m < nblk && sm < ns) {
                const uint64_t i = s0 + sm;
                ox[m] = (double)(int64_t)(A.X[i] - C0) * scale;
                oy[m] = (double)(int64_t)(A.X[n + i] - C1) * scale;
                oz[m] = (double)(int64_t)(A.X[2 * n + i] - C2) * scale;
            }
        }
        unsigned long long pn_src = 0, pp_src = 0, n_acc = 0, n_leaf = 0;
        const TieBand tband{tie_rc2, tie_band};
        if ((uint32_t)lane < (uint32_t)NGR_MAX_SPECIES) gpn[lane] = 0u;
        uint32_t nties = 0;                  // TIES: this lane's near ties
        // relative opening test: the smallest previous |a| of the group's sinks
        const bool rel = P.relative != 0u;
        double a_min = 0.0;
        if (rel) {
            double am = __builtin_inf();
            if ((uint32_t)lane < ns) am = P.old_acc[A.perm[s0 + lane] - in_off];
#pragma unroll
            for (int d = 32; d > 0; d >>= 1) am = fmin(am, __shfl_xor(am, d, 64));
            a_min = am;
        }
        // the sink's own core scale (accumulator laws, cored sink species)
        double s_sink = 0.0;
        if (ACC && core_a && sink < ns) s_sink = A.mass[s0 + sink] * inv4pib;
        // a pair of species (a, b) takes the cored law when either is cored
        auto cored_pair = [&](uint32_t b) { return ACC && (core_a || ((cmask >> b) & 1u)); };

        auto eval = [&](uint32_t b, uint32_t nrec) {
            const unsigned char* tb = tsm + (TAB == kPair ? 8u : 4u) * b * tstride;
            const uint32_t iters = (nrec + K - 1u) >> lk;
            // the pair's own softening (section 2: D^2 softenings); the pair
            // index is wave-uniform, so its address arithmetic stays scalar
            const uint32_t ab = uniform(a * Dk + b);
            const double e2 = P.eps2_ab[ab];
            const float to = P.toff_ab[ab];
            if (cored_pair(b)) {
                const double* rrs = recs + replica;
                double &x = ox[0], &y = oy[0], &z = oz[0], &gx = ax[0], &gy = ay[0], &gz = az[0];
                if (wrap) eval_cored<GRID, TAB, true, 1>(pp, e2, rec, recs, nrec, tb, core_tab, s_sink, x, y, z, gx, gy, gz);
                else if (lk == 0u) eval_cored<GRID, TAB, false, 1>(pp, e2, rec, recs, nrec, tb, core_tab, s_sink, x, y, z, gx, gy, gz);
                else if (lk == 1u) eval_cored<GRID, TAB, false, 2>(pp, e2, rrec, rrs, iters, tb, core_tab, s_sink, x, y, z, gx, gy, gz);
                else eval_cored<GRID, TAB, false, 4>(pp, e2, rrec, rrs, iters, tb, core_tab, s_sink, x, y, z, gx, gy, gz);
                return;
            }
            if (EW && P.corr) {
                const uint64_t m = P.corr_n + 1u;
                const LatticeCorr lc{P.corr + (uint64_t)(a * Dk + b) * m * m * m * 3u, P.corr_n, P.corr_scale};
                eval_records<GRID, TAB, EPS0, true, 1, true>(pp, e2, to, rec, nrec, tb, ox[0], oy[0], oz[0], ax[0], ay[0],
                                                             az[0], lc);
                return;
            }
            const LatticeCorr nolc{nullptr, 0u, 0.0};
            if (blocks) {
#pragma unroll
                for (int m = 0; m < kBlocks; ++m) {
                    const uint32_t t = eval_records<GRID, TAB, EPS0, false, 4, false, TIES>(
                        pp, e2, to, rrec, iters, tb, ox[m], oy[m], oz[m], ax[m], ay[m], az[m], nolc, tband);
                    if (TIES && sink + 16u * (uint32_t)m < ns) nties += t;
                }
                return;
            }
            double &x = ox[0], &y = oy[0], &z = oz[0], &gx = ax[0], &gy = ay[0], &gz = az[0];
            uint32_t t;
            if (wrap) t = eval_records<GRID, TAB, EPS0, true, 1, false, TIES>(pp, e2, to, rec, nrec, tb, x, y, z, gx, gy, gz, nolc, tband);
            else if (lk == 0u) t = eval_records<GRID, TAB, EPS0, false, 1, false, TIES>(pp, e2, to, rec, nrec, tb, x, y, z, gx, gy, gz, nolc, tband);
            else if (lk == 1u) t = eval_records<GRID, TAB, EPS0, false, 2, false, TIES>(pp, e2, to, rrec, iters, tb, x, y, z, gx, gy, gz, nolc, tband);
            else t = eval_records<GRID, TAB, EPS0, false, 4, false, TIES>(pp, e2, to, rrec, iters, tb, x, y, z, gx, gy, gz, nolc, tband);
            if (TIES && sink < ns) nties += t;
        };

        // Accepted nodes: one record per non-empty species monopole. The next
        // species' monopoles are loaded while this species is evaluated.
        auto flush_nodes = [&](uint32_t k) {
            const uint32_t node = (uint32_t)lane < k ? pnb[lane] : 0u;
            double4 r = make_double4(0.0, 0.0, 0.0, 0.0);
            if ((uint32_t)lane < k) r = A.mono[node];
            for (uint32_t b = 0; b < Dk; ++b) {
                const bool v = (uint32_t)lane < k && r.w > 0.0;
                const uint64_t m = __ballot(v);
                const uint32_t nrec = (uint32_t)__popcll(m);
                const bool cp = cored_pair(b);
                if (v) {
                    double d0 = r.x - cf0, d1 = r.y - cf1, d2 = r.z - cf2;
                    d0 -= rint(d0);
                    d1 -= rint(d1);
                    d2 -= rint(d2);
                    const uint32_t slot = (uint32_t)__popcll(m & lt);
                    rec[slot] = make_double4(d0 * bx, d1 * bx, d2 * bx, Ga[uniform(b)] * r.w);
                    if (cp) {
                        // a monopole of N_perp bodies: each of mass M / N_perp when tracked
                        double body = r.w;
                        if (track) body /= (double)A.count[(uint64_t)node * D + b];
                        recs[slot] = ((cmask >> b) & 1u) ? body * inv4pib : 0.0;
                    }
                }
                if (K > 1u && (uint32_t)lane < 3u) {
                    rec[nrec + lane] = pad;
                    if (cp) recs[nrec + lane] = 1.0;
                }
                wave_sync();
                if (b + 1 < Dk && (uint32_t)lane < k) r = A.mono[(uint64_t)(b + 1) * A.nn + node];
                if (nrec) eval(b, nrec);
                pn_src += nrec;
                if (lane == 0) gpn[b] += nrec;
                wave_sync();
            }
        };

        // Opened leaves: every particle, one source species at a time, in
        // chunks of up to 64 records. Each chunk's particle loads are issued
        // before the previous chunk is evaluated, so that their latency hides
        // behind the pair loop.
        auto flush_leaves = [&](uint32_t k) {
            const uint32_t leaf = (uint32_t)lane < k ? ppb[lane] : 0u;
            uint32_t cnt[NGR_MAX_SPECIES], stv[NGR_MAX_SPECIES];
#pragma unroll
            for (uint32_t q = 0; q < NGR_MAX_SPECIES; ++q) {
                cnt[q] = 0u;
                stv[q] = 0u;
                if ((uint32_t)lane < k && q < Dk) {
                    cnt[q] = A.count[(uint64_t)leaf * D + q];
                    stv[q] = A.start[(uint64_t)leaf * D + q];
                }
            }
            auto pick = [&](const uint32_t* arr, uint32_t b) {   // arr[b], b wave-uniform
                uint32_t v = 0u;
#pragma unroll
                for (uint32_t q = 0; q < NGR_MAX_SPECIES; ++q) v = q == b ? arr[q] : v;
                return v;
            };
            // species b's running counts into LDS; its particle total
            auto prep = [&](uint32_t b) -> uint32_t {
                const uint32_t incl = wave_incl(pick(cnt, b));
                const uint32_t T = lane63(incl);
                if (T) {
                    scanb[lane + 1] = incl;
                    scanb[0] = 0;              // every lane stores the same value
                    pst[lane] = pick(stv, b);
                    wave_sync();
                }
                return T;
            };
            PRec pr{};
            bool sv = false;
            // Loads of record base + lane of the current species. Leaf q holds
            // the records scanb[q] .. scanb[q + 1] - 1. In the window of 64
            // records from base, each leaf marks the position of its first
            // record there (position 0 for the leaf holding base); the running
            // maximum of the marks is each record's leaf. The second half of
            // the node buffer is free while leaves are flushed (fewer than 64
            // nodes are pending), and holds the marks.
            uint32_t* const mark = pnb + 64;
            auto stage = [&](uint32_t base, uint32_t T) {
                const uint32_t e = scanb[lane], f = scanb[lane + 1];
                mark[lane] = 0u;
                if ((uint32_t)lane < k && e < f && f > base && e < base + 64u) mark[max(e, base) - base] = (uint32_t)lane;
                wave_sync();
                const uint32_t q = wave_scan<true>(mark[lane]);
                const uint32_t r = base + lane;
                sv = r < T;
                if (sv) pr = A.P[pst[q] + (r - scanb[q])];
            };
            uint32_t b = 0, T = 0;
            for (; b < Dk; ++b) {
                T = prep(b);
                if (T) break;
            }
            if (b >= Dk) return;
            uint32_t base = 0;
            stage(base, T);
            for (;;) {
                const uint32_t nrec = min(64u, T - base);
                const bool cp = cored_pair(b);
                if (sv) {
                    // offsets from the group centre in box units (the box is 1):
                    // the high part's difference is exact, the low part rounds it once
                    double ex = pr.hx - cf0, ey = pr.hy - cf1, ez = pr.hz - cf2;
                    ex -= rint(ex);
                    ey -= rint(ey);
                    ez -= rint(ez);
                    rec[lane] = make_double4(ex + (double)pr.lx, ey + (double)pr.ly, ez + (double)pr.lz,
                                             Ga[uniform(b)] * pr.m);
                    if (cp) recs[lane] = ((cmask >> b) & 1u) ? pr.m * inv4pib : 0.0;
                }
                if (K > 1u && (uint32_t)lane < 3u) {
                    rec[nrec + lane] = pad;
                    if (cp) recs[nrec + lane] = 1.0;
                }
                wave_sync();
                // the next chunk: the rest of this species, else the next species with particles
                uint32_t nb = b, nbase = base + 64u, nT = T;
                if (nbase >= T) {
                    nbase = 0;
                    nT = 0;
                    for (nb = b + 1; nb < Dk; ++nb) {
                        nT = prep(nb);
                        if (nT) break;
                    }
                }
                if (nb < Dk) stage(nbase, nT);
                eval(b, nrec);
                pp_src += nrec;
                wave_sync();
                if (nb >= Dk) break;
                b = nb;
                base = nbase;
                T = nT;
            }
        };

        // breadth-first traversal in batches of 64 nodes
        uint32_t sp = 1, npn = 0, npp = 0;
        stack[0] = bxi;                    // the box's root; every lane stores the same value
        wave_sync();
        bool overflow = false;
        uint32_t steps = 0;
        while (sp > 0) {
            if (++steps > A.max_steps) {   // a node enters a group's stack at most once
                overflow = true;
                break;
            }
            const uint32_t take = min(sp, 64u);
            sp -= take;
            uint32_t node = 0, dec = kPrune, nc = 0;
            int32_t fc = 0;
            if ((uint32_t)lane < take) {
                node = stack[sp + lane];
                const uint4 cl = A.cell[node];
                const int32_t S = 1 << (kLevels - (int)cl.w);
                const uint32_t cc[3] = {cl.x, cl.y, cl.z};
                double D2 = 0.0, D2m = 0.0;
                bool inside = true;       // the group's box reaches into the node's cube grown to 1.2 sides
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    const int32_t w = (int32_t)(hi[k] - lo[k]);
                    int32_t d = (2 * (int32_t)cc[k] + S) - (int32_t)(lo[k] + hi[k]);
                    d = ((d + (1 << 20)) & ((1 << 21) - 1)) - (1 << 20);
                    const int32_t ad = d < 0 ? -d : d;
                    int32_t gp = 0;
                    if (S + w < (1 << 20)) gp = max(ad - (S + w), 0);
                    const int32_t gm = ad + S + w;
                    D2 += (double)gp * (double)gp;
                    D2m += (double)gm * (double)gm;
                    inside = inside && 5 * ad < 6 * S + 5 * w;
                }
                bool accept;
                if (rel) {
                    // M l^2 <= alpha a_min d^4 with M the node's mass over all
                    // species, l = 2 S and d^2 = D2 in half key units
                    double M = 0.0;
                    if (!inside && D2 < R2)
                        for (uint32_t b = 0; b < D; ++b) M += A.mono[(uint64_t)b * A.nn + node].w;
                    const double lhs = M * (double)(4ll * S * S);
                    const double rhs = (P.rel_k * a_min) * (D2 * D2);
                    accept = !inside && lhs <= rhs && D2m < R2;
                } else {
                    accept = (double)(4ll * S * S) < theta2 * D2 && D2m < R2;
                }
                if (D2 >= R2) dec = kPrune;
                else if (accept) dec = kAccept;
                else {
                    dec = kOpen;
                    nc = A.n_child[node];
                    fc = A.first_child[node];
                }
            }
            const uint64_t macc = __ballot(dec == kAccept);
            const uint64_t mleaf = __ballot(dec == kOpen && nc == 0);
            if (dec == kAccept) pnb[npn + __popcll(macc & lt)] = node;
            if (dec == kOpen && nc == 0) ppb[npp + __popcll(mleaf & lt)] = node;
            npn += (uint32_t)__popcll(macc);
            npp += (uint32_t)__popcll(mleaf);
            n_acc += (uint32_t)__popcll(macc);
            n_leaf += (uint32_t)__popcll(mleaf);
            const uint32_t myc = (dec == kOpen) ? nc : 0u;
            const uint32_t incl = wave_incl(myc);
            const uint32_t tot = lane63(incl);
            if (sp + tot > A.stack_cap) {
                overflow = true;
                break;
            }
            for (uint32_t k = 0; k < myc; ++k) stack[sp + incl - myc + k] = (uint32_t)fc + k;
            sp += tot;
            wave_sync();
            if (npn >= 64) {
                flush_nodes(64);
                uint32_t rest = npn - 64, v = 0;
                if ((uint32_t)lane < rest) v = pnb[64 + lane];
                wave_sync();
                if ((uint32_t)lane < rest) pnb[lane] = v;
                npn = rest;
                wave_sync();
            }
            if (npp >= 64) {
                flush_leaves(64);
                uint32_t rest = npp - 64, v = 0;
                if ((uint32_t)lane < rest) v = ppb[64 + lane];
                wave_sync();
                if ((uint32_t)lane < rest) ppb[lane] = v;
                npp = rest;
                wave_sync();
            }
        }
        any_overflow |= overflow;
        if (!overflow) {
            if (npn) flush_nodes(npn);
            if (npp) flush_leaves(npp);
        }
        // fold the copies' sums (fixed order); every copy then holds the
        // total, so lane l = c + 16 q of a blocked group keeps block q's sink
        // c + 16 q, i.e. sink l, like the other modes
#pragma unroll
        for (int m = 0; m < kBlocks; ++m) {
            if ((uint32_t)m >= nblk) break;
            if (K == 4u) {
                ax[m] += __shfl_xor(ax[m], 16, 64);
                ay[m] += __shfl_xor(ay[m], 16, 64);
                az[m] += __shfl_xor(az[m], 16, 64);
            }
            if (K >= 2u) {
                ax[m] += __shfl_xor(ax[m], 32, 64);
                ay[m] += __shfl_xor(ay[m], 32, 64);
                az[m] += __shfl_xor(az[m], 32, 64);
            }
        }
        double fx = ax[0], fy = ay[0], fz = az[0];
        if (kBlocks > 1 && blocks) {
            const uint32_t q = (uint32_t)lane >> 4;
#pragma unroll
            for (int m = 1; m < kBlocks; ++m)
                if (q == (uint32_t)m) {
                    fx = ax[m];
                    fy = ay[m];
                    fz = az[m];
                }
        }
        if ((uint32_t)lane < ns) {
            const uint64_t p = A.perm[s0 + lane] - in_off;
            acc[p] = fx;
            acc[nbx + p] = fy;
            acc[2 * nbx + p] = fz;
        }
        const unsigned long long pn = pn_src * ns, pp = pp_src * ns - ns;
        unsigned long long gties = 0;
        if (TIES) {
            uint32_t t = nties;
#pragma unroll
            for (int d = 32; d > 0; d >>= 1) t += (uint32_t)__shfl_xor((int)t, d, 64);
            gties = uniform(t);
        }
        wave_sync();                       // lane 0's gpn updates are visible
        if ((uint32_t)lane < (uint32_t)kSegCounts) {
            const unsigned long long v = lane == 0 ? pp : lane == 1 ? pn : lane == 2 ? gties
                                                                   : (unsigned long long)gpn[lane - 3] * ns;
            wcnt[lane] += v;
        }
        if (A.gcounts && (uint32_t)lane < 4u) {
            const unsigned long long v[4] = {n_acc, n_leaf, pn, pp};
            A.gcounts[4ull * g + lane] = v[lane];
        }
    }
        __syncthreads();                   // every wave is done with this segment's tables and counts
        if (wave == 0) {
            // next segment: the next one not started, else the one with the most
            // estimated work left (ranked at least 1 while a group is left)
            const uint32_t t = uniform(atomicAdd(A.cursor, lane == 0 ? 1u : 0u));
            uint32_t next = A.nseg;
            if (t < A.nsched) {
                next = A.sched[t];
            } else {
                uint32_t best = 0, best_s = A.nseg;
                for (uint32_t q = (uint32_t)lane; q < A.nseg; q += 64u) {
                    const uint32_t cnt = A.seg_first[q + 1] - A.seg_first[q];
                    const uint32_t h = __hip_atomic_load(A.queues + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    const uint32_t left = cnt - min(h, cnt);
                    const unsigned long long wl =
                        __hip_atomic_load(A.seg_work + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    const uint32_t rank = left ? (uint32_t)min((wl >> 12) + 1ull, 0xffffffffull) : 0u;
                    if (rank > best) {
                        best = rank;
                        best_s = q;
                    }
                }
                for (int d = 32; d > 0; d >>= 1) {
                    const uint32_t ob = (uint32_t)__shfl_xor((int)best, d, 64);
                    const uint32_t os = (uint32_t)__shfl_xor((int)best_s, d, 64);
                    if (ob > best || (ob == best && os < best_s)) {
                        best = ob;
                        best_s = os;
                    }
                }
                next = best ? best_s : A.nseg;
            }
            ctrl[0] = (int32_t)next;       // every lane stores the same value
        }
        __syncthreads();
        if (threadIdx.x < (unsigned)kSegCounts) {   // the segment's counts: one global atomic each per workgroup
            unsigned long long v = 0;
            for (int w = 0; w < nwaves; ++w) v += part[kSegCounts * w + threadIdx.x];
            if (v) atomicAdd(&A.seg_counts[(uint64_t)kSegCounts * seg + threadIdx.x], v);
        }
        seg = uniform((uint32_t)ctrl[0]);
        if (seg >= A.nseg) break;
    }
    if (lane == 0 && any_overflow) atomicOr(A.error_flag, 1u);
}

inline unsigned blocks_for(uint64_t work, unsigned threads) { return (unsigned)((work + threads - 1) / threads); }

// One box's table conversion: where its FP64 samples are and where its two
// layouts go.
struct TableJob {
    const double* src;           // the box's float64 samples (device): staged from the host, or the caller's
    uint64_t pair, value;        // first element in the PAIR and VALUE arrays
    uint32_t pairs, ntab;        // D * D tables of ntab samples
    uint32_t shared;             // 1: one table of ntab samples for every pair
    uint32_t box;
};

// Both layouts of every table of box blockIdx.y (grid-stride over the box's
// D * D * ntab entries): PAIR (value, slope to the next sample) with (0, 0)
// as the last entry; VALUE the samples and a zero pad. Each float is the FP64
// value (or difference) rounded once. A sample that is not finite lowers
// *bad_box to the box's index.
__global__ void convert_tables(const TableJob* __restrict__ jobs, float2* __restrict__ pair,
                               float* __restrict__ value, uint32_t* __restrict__ bad_box)
{
    const TableJob J = jobs[blockIdx.y];
    const uint64_t total = (uint64_t)J.pairs * J.ntab;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    // the trip count is the same for every lane (the bound test is inside)
    for (uint64_t base = (uint64_t)blockIdx.x * blockDim.x; base < total; base += stride) {
        const uint64_t e = base + threadIdx.x;
        if (e >= total) continue;
        const uint64_t ab = e / J.ntab, k = e % J.ntab;
        const double* src = J.src + (J.shared ? 0 : ab * J.ntab);
        if (!isfinite(src[k])) atomicMin(bad_box, J.box);
        pair[J.pair + e] = k + 1 < J.ntab ? make_float2((float)src[k], (float)(src[k + 1] - src[k]))
                                          : make_float2(0.0f, 0.0f);
        value[J.value + ab * (J.ntab + 1) + k] = (float)src[k];
        if (k + 1 == J.ntab) value[J.value + ab * (J.ntab + 1) + J.ntab] = 0.0f;
    }
}

}  // namespace

void Groups::free(Context& ctx)
{
    ctx.release(start);
    ctx.release(count);
    ctx.release(lo);
    ctx.release(hi);
    ctx.release(box);
    start = count = lo = hi = box = nullptr;
    ng = 0;
    nseg = 0;
    first.clear();
}

void make_groups(Context& ctx, const Tree& t, const std::vector<uint32_t>& group_size, Groups& g)
{
    const uint64_t n = t.n;
    const uint32_t D = t.D, nbox = t.nbox;
    g.ng = 0;
    g.nseg = nbox * D;
    g.first.assign(g.nseg + 1, 0);
    if (n == 0) return;
    ctx.stage("groups: mark");
    uint32_t* flags = static_cast<uint32_t*>(ctx.alloc(n * sizeof(uint32_t) * 2 + 64));
    uint32_t* gidx = flags + n;
    uint32_t* total = gidx + n;
    uint32_t* Ng_dev = static_cast<uint32_t*>(ctx.alloc(nbox * sizeof(uint32_t)));
    ctx.to_device(Ng_dev, group_size.data(), nbox * sizeof(uint32_t));
    HIP_CHECK(hipMemsetAsync(flags, 0, n * sizeof(uint32_t), ctx.stream));
    hipLaunchKernelGGL(mark_group_starts, dim3(blocks_for(t.nn * D, 256)), dim3(256), 0, ctx.stream, t.nn, D, Ng_dev,
                       t.node_box, t.start, t.count, t.parent, t.first_child, t.n_child, flags);
    LAUNCH_CHECK("mark_group_starts");
    scan_exclusive(ctx, flags, gidx, n, total);
    uint64_t w = 0;
    ctx.read_words(&w, total, 1);
    const uint32_t ngh = (uint32_t)(w & 0xffffffffu);
    if (ngh == 0 || ngh > n) fail(NGR_EDEVICE, "group formation produced an impossible group count");
    // first group of each segment: the group index at the segment's first particle
    std::vector<uint64_t> pos(g.nseg + 1);
    for (uint32_t k = 0; k < nbox; ++k)
        for (uint32_t a = 0; a < D; ++a) pos[(size_t)k * D + a] = t.bseg[(size_t)k * (NGR_MAX_SPECIES + 1) + a];
    pos[g.nseg] = n;
    uint64_t* pos_dev = static_cast<uint64_t*>(ctx.alloc(pos.size() * sizeof(uint64_t)));
    uint32_t* first_dev = static_cast<uint32_t*>(ctx.alloc(pos.size() * sizeof(uint32_t) + 64));
    uint32_t* errd = first_dev + pos.size();
    ctx.to_device(pos_dev, pos.data(), pos.size() * sizeof(uint64_t));
    HIP_CHECK(hipMemsetAsync(errd, 0, sizeof(uint32_t), ctx.stream));
    hipLaunchKernelGGL(segment_firsts, dim3(blocks_for(pos.size(), 256)), dim3(256), 0, ctx.stream, (uint32_t)pos.size(),
                       pos_dev, gidx, n, ngh, first_dev);
    LAUNCH_CHECK("segment_firsts");
    g.ng = ngh;
    g.start = static_cast<uint32_t*>(ctx.alloc((uint64_t)ngh * sizeof(uint32_t)));
    g.count = static_cast<uint32_t*>(ctx.alloc((uint64_t)ngh * sizeof(uint32_t)));
    g.lo = static_cast<uint32_t*>(ctx.alloc(3ull * ngh * sizeof(uint32_t)));
    g.hi = static_cast<uint32_t*>(ctx.alloc(3ull * ngh * sizeof(uint32_t)));
    g.box = static_cast<uint32_t*>(ctx.alloc((uint64_t)ngh * sizeof(uint32_t)));
    ctx.stage("groups: boxes");
    hipLaunchKernelGGL(scatter_group_starts, dim3(blocks_for(n, 256)), dim3(256), 0, ctx.stream, n, flags, gidx,
                       g.start);
    LAUNCH_CHECK("scatter_group_starts");
    hipLaunchKernelGGL(finish_groups, dim3(blocks_for((uint64_t)ngh * 64, 256)), dim3(256), 0, ctx.stream, (uint64_t)ngh,
                       n, nbox, t.boff_dev, g.start, g.count, g.lo, g.hi, g.box, t.X, errd);
    LAUNCH_CHECK("finish_groups");
    std::vector<uint32_t> fh(pos.size() + 1);
    ctx.to_host(fh.data(), first_dev, (pos.size() + 1) * sizeof(uint32_t));
    if (fh[pos.size()]) fail(NGR_EDEVICE, "group formation produced an inconsistent group");
    for (size_t k = 0; k < pos.size(); ++k) g.first[k] = fh[k];
    ctx.release(flags);
    ctx.release(Ng_dev);
    ctx.release(pos_dev);
    ctx.release(first_dev);
}

void make_law(const ngr_force_params& fp, uint32_t D, Law& law)
{
    law.D = D;
    law.ntab = fp.ntab;
    law.grid = fp.grid;
    law.r_cut = fp.r_cut;
    law.eps = fp.eps;
    law.theta = fp.theta;
    for (uint32_t k = 0; k < D * D; ++k) law.G[k] = fp.G[k];
    law.tables = fp.tables;
    law.tables_device = fp.tables && fp.tables_on_device;
    law.kind = fp.law;
    law.cored = fp.law == NGR_LAW_ACCUMULATOR ? fp.cored : 0u;
    law.beta = fp.beta;
    law.track = 1;
    law.corr = fp.lattice_corr;
    law.corr_n = fp.corr_n;
    law.opening = fp.opening;
    law.alpha = fp.alpha;
    law.old_acc = fp.old_acc;
    law.eps_ab.assign((size_t)D * D, fp.eps);
    if (fp.eps_ab)
        for (uint32_t k = 0; k < D * D; ++k) law.eps_ab[k] = fp.eps_ab[k];
    law.def.clear();
    if (!fp.tables) {
        const uint32_t ntab = fp.ntab;
        law.def.resize((size_t)ntab);
        for (uint32_t k = 0; k < ntab; ++k) {
            double r = fp.grid == NGR_GRID_R ? k * (fp.r_cut / (ntab - 1))
                                             : std::sqrt(k * (fp.r_cut * fp.r_cut / (ntab - 1)));
            double x = r / (2.0 * fp.r_s);
            law.def[k] = std::erfc(x) + r / (fp.r_s * std::sqrt(M_PI)) * std::exp(-x * x);
        }
    }
}

void* upload_tables(Context& ctx, const std::vector<Law>& laws, std::vector<LawTables>& out)
{
    const uint32_t nbox = (uint32_t)laws.size();
    std::vector<TableJob> jobs(nbox);
    std::vector<uint64_t> staged(nbox, 0);   // host samples: their place in the staging array
    uint64_t nraw = 0, np = 0, nv = 0;
    uint32_t max_entries = 0;
    bool any_device = false;
    for (uint32_t k = 0; k < nbox; ++k) {
        const Law& L = laws[k];
        TableJob& j = jobs[k];
        j.pairs = L.D * L.D;
        j.ntab = L.ntab;
        j.shared = L.tables ? 0u : 1u;
        j.box = k;
        j.pair = np;
        j.value = nv;
        if (L.tables_device) {
            any_device = true;
        } else {
            staged[k] = nraw;
            nraw += L.tables ? (uint64_t)j.pairs * L.ntab : L.ntab;
        }
        np += (uint64_t)j.pairs * L.ntab;
        nv += (uint64_t)j.pairs * (L.ntab + 1);
        max_entries = std::max(max_entries, j.pairs * L.ntab);
    }
    const size_t raw_bytes = ((nraw * sizeof(double)) + 255) & ~size_t(255), job_bytes = nbox * sizeof(TableJob);
    const size_t pair_bytes = ((np * sizeof(float2)) + 255) & ~size_t(255);
    const size_t value_bytes = ((nv * sizeof(float)) + 255) & ~size_t(255);
    unsigned char* block = static_cast<unsigned char*>(ctx.alloc(pair_bytes + value_bytes));
    float2* pair = reinterpret_cast<float2*>(block);
    float* value = reinterpret_cast<float*>(block + pair_bytes);
    unsigned char* stage = static_cast<unsigned char*>(ctx.alloc(raw_bytes + job_bytes + sizeof(uint64_t)));
    double* raw = reinterpret_cast<double*>(stage);
    TableJob* jobs_dev = reinterpret_cast<TableJob*>(stage + raw_bytes);
    uint32_t* bad_box = reinterpret_cast<uint32_t*>(stage + raw_bytes + job_bytes);   // 8 bytes, 8-aligned
    for (uint32_t k = 0; k < nbox; ++k) jobs[k].src = laws[k].tables_device ? laws[k].tables : raw + staged[k];
    ctx.sync();
    for (uint32_t k = 0; k < nbox; ++k) {
        const Law& L = laws[k];
        if (L.tables_device) continue;   // read in place by the conversion
        const double* src = L.tables ? L.tables : L.def.data();
        const size_t cnt = L.tables ? (size_t)jobs[k].pairs * L.ntab : L.ntab;
        HIP_CHECK(hipMemcpyAsync(raw + staged[k], src, cnt * sizeof(double), hipMemcpyHostToDevice, ctx.stream));
    }
    HIP_CHECK(hipMemcpyAsync(jobs_dev, jobs.data(), job_bytes, hipMemcpyHostToDevice, ctx.stream));
    HIP_CHECK(hipMemsetAsync(bad_box, 0xff, sizeof(uint64_t), ctx.stream));
    const unsigned gx = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(blocks_for(max_entries, 256), 64));
    hipLaunchKernelGGL(convert_tables, dim3(gx, nbox), dim3(256), 0, ctx.stream, jobs_dev, pair, value, bad_box);
    LAUNCH_CHECK("convert_tables");
    if (any_device) {
        // host tables were checked before the call; a device table is checked here
        uint64_t w = 0;
        ctx.read_words(&w, bad_box, 1);
        const uint32_t k = (uint32_t)(w & 0xffffffffu);
        if (k != 0xffffffffu) {
            ctx.release(stage);
            ctx.release(block);
            fail(NGR_EINVAL, (nbox > 1 ? "box " + std::to_string(k) + ": " : std::string()) +
                                 "a table entry is not finite");
        }
    }
    ctx.sync();                        // the caller's host tables are no longer read after this
    ctx.release(stage);
    out.resize(nbox);
    for (uint32_t k = 0; k < nbox; ++k) {
        out[k].pair = pair + jobs[k].pair;
        out[k].value = value + jobs[k].value;
    }
    return block;
}

// The core factor of the accumulator laws, C(u) = (2/pi) g(x) (1 + x)^3 with
// x = u / (1 - u) and g(x) = [atan x - x / (1 + x^2)] / x^3 (2/3 - 4x^2/5 +
// 6x^4/7 below x = 1e-2, where the difference cancels), at u = k / kCoreN,
// in the PAIR layout (value, slope to the next sample); C(1) = 1. Built in
// float64 on the host once per context.
static const float2* upload_core_table(Context& ctx)
{
    if (ctx.core.p) return static_cast<const float2*>(ctx.core.p);
    std::vector<double> c(kCoreN + 1);
    for (int k = 0; k < kCoreN; ++k) {
        const double u = (double)k / kCoreN, x = u / (1.0 - u);
        double v;
        if (x < 1e-2) {
            const double x2 = x * x;
            v = (2.0 / 3.0 - 0.8 * x2 + (6.0 / 7.0) * x2 * x2) * (1.0 + x) * (1.0 + x) * (1.0 + x);
        } else {
            const double q = 1.0 + 1.0 / x;
            v = (std::atan(x) - x / (1.0 + x * x)) * q * q * q;
        }
        c[k] = v * (2.0 / M_PI);
    }
    c[kCoreN] = 1.0;
    std::vector<float2> t(kCoreN + 1);
    for (int k = 0; k < kCoreN; ++k) t[k] = make_float2((float)c[k], (float)(c[k + 1] - c[k]));
    t[kCoreN] = make_float2(1.0f, 0.0f);
    if (ctx.arena) {                     // this call only: the context keeps nothing from the arena
        void* p = ctx.alloc(t.size() * sizeof(float2));
        ctx.to_device(p, t.data(), t.size() * sizeof(float2));
        return static_cast<const float2*>(p);
    }
    ctx.ensure(ctx.core, t.size() * sizeof(float2));
    ctx.to_device(ctx.core.p, t.data(), t.size() * sizeof(float2));
    return static_cast<const float2*>(ctx.core.p);
}

// Group indices segment by segment, each segment's groups in descending
// order of the density estimate (ties in tree order). Returns device memory
// of g.ng entries, to be released by the caller.
static uint32_t* order_groups(Context& ctx, const Tree& t, const Groups& g, const std::vector<Law>& laws,
                              uint32_t* gbucket)
{
    const uint64_t ng = g.ng;
    const uint32_t nbox = t.nbox;
    // per box: the finest level whose cells are at least r_cut wide, at most
    // 8, and no more cells in all than 2^26
    std::vector<uint32_t> L(nbox);
    std::vector<uint64_t> Hoff(nbox + 1, 0);
    uint32_t cap = 8;
    for (;;) {
        uint64_t cells = 0;
        for (uint32_t k = 0; k < nbox; ++k) {
            uint32_t l = 0;
            while (l < cap && std::ldexp(t.bbox[k], -(int)(l + 1)) >= laws[k].r_cut) ++l;
            L[k] = (t.boff[k + 1] > t.boff[k]) ? l : 0;
            Hoff[k] = cells;
            cells += L[k] ? (1ull << (3 * L[k])) : 0;
        }
        Hoff[nbox] = cells;
        if (cells <= (ctx.arena ? (1ull << 18) : (1ull << 26)) || cap == 0) break;
        --cap;
    }
    uint64_t* okey = static_cast<uint64_t*>(ctx.alloc(2 * ng * sizeof(uint64_t)));
    uint32_t* oval = static_cast<uint32_t*>(ctx.alloc(2 * ng * sizeof(uint32_t)));
    uint32_t* Ld = static_cast<uint32_t*>(ctx.alloc(nbox * sizeof(uint32_t)));
    uint64_t* Hoffd = static_cast<uint64_t*>(ctx.alloc((nbox + 1) * sizeof(uint64_t)));
    ctx.to_device(Ld, L.data(), nbox * sizeof(uint32_t));
    ctx.to_device(Hoffd, Hoff.data(), (nbox + 1) * sizeof(uint64_t));
    uint32_t* H = nullptr;
    if (Hoff[nbox]) {
        H = static_cast<uint32_t*>(ctx.alloc(Hoff[nbox] * sizeof(uint32_t)));
        HIP_CHECK(hipMemsetAsync(H, 0, Hoff[nbox] * sizeof(uint32_t), ctx.stream));
        uint32_t Lmax = 0;
        for (uint32_t k = 0; k < nbox; ++k) Lmax = std::max(Lmax, L[k]);
        const uint64_t nodes = t.level_start[std::min<uint32_t>(Lmax, t.depth) + 1];
        hipLaunchKernelGGL(density_grid, dim3(blocks_for(nodes, 256)), dim3(256), 0, ctx.stream, nodes, t.D, Ld, Hoffd,
                           t.node_box, t.cell, t.n_child, t.start, t.count, t.X, t.n, H);
        LAUNCH_CHECK("density_grid");
        // the summed-volume table: prefix sums along z, y and x
        std::vector<uint64_t> Loff(nbox + 1, 0);
        for (uint32_t k = 0; k < nbox; ++k) Loff[k + 1] = Loff[k] + (L[k] ? (1ull << (2 * L[k])) : 0);
        uint64_t* Loffd = static_cast<uint64_t*>(ctx.alloc((nbox + 1) * sizeof(uint64_t)));
        ctx.to_device(Loffd, Loff.data(), (nbox + 1) * sizeof(uint64_t));
        for (uint32_t axis = 3; axis-- > 0;) {
            hipLaunchKernelGGL(density_prefix, dim3(blocks_for(Loff[nbox], 256)), dim3(256), 0, ctx.stream, Loff[nbox],
                               nbox, axis, Ld, Hoffd, Loffd, H);
            LAUNCH_CHECK("density_prefix");
        }
        ctx.release(Loffd);
    }
    hipLaunchKernelGGL(group_order_keys, dim3(blocks_for(ng, 256)), dim3(256), 0, ctx.stream, ng, t.D, g.start,
                       g.count, g.lo, g.hi, g.box, Ld, Hoffd, t.keys, H, okey, oval, gbucket);
    LAUNCH_CHECK("group_order_keys");
    int bits = 8;
    while ((1ull << (bits - 8)) < g.nseg) bits += 8;
    radix_sort_pairs(ctx, okey, oval, okey + ng, oval + ng, ng, bits);
    if (H) ctx.release(H);
    ctx.release(okey);
    ctx.release(Ld);
    ctx.release(Hoffd);
    return oval;
}

// One launch over the boxes with part[k] set; adds their counts and times to
// out (the other boxes' segments are marked done before the launch).
static void walk_launch(Context& ctx, const Tree& t, const Groups& g, const std::vector<Law>& laws,
                        const std::vector<LawTables>& tables, const std::vector<double*>& accv,
                        uint64_t* group_counts_dev, WalkOut& out, bool count_ties, const std::vector<char>& part)
{
    const uint32_t nbox = t.nbox, D = t.D;
    bool any = false;
    for (uint32_t q = 0; q < g.nseg; ++q) any |= part[q / D] && g.first[q + 1] > g.first[q];
    if (!any) return;
    const uint32_t grid = laws[0].grid;
    bool eps0 = false, acc_law = false, ew = false;
    for (uint32_t k = 0; k < nbox; ++k) {
        if (!part[k]) continue;
        acc_law |= laws[k].kind == NGR_LAW_ACCUMULATOR;
        ew |= laws[k].corr != nullptr;
    }
    if (acc_law && ew) fail(NGR_EINVAL, "lattice corrections take the table laws only");
    const float2* core_table = acc_law ? upload_core_table(ctx) : nullptr;
    // lattice correction tables of every box that has them, one block
    std::vector<uint64_t> corr_off(nbox, 0);
    double* corr_dev = nullptr;
    if (ew) {
        uint64_t total = 0;
        for (uint32_t k = 0; k < nbox; ++k) {
            corr_off[k] = total;
            if (laws[k].corr) {
                const uint64_t m = laws[k].corr_n + 1ull;
                total += (uint64_t)laws[k].D * laws[k].D * m * m * m * 3ull;
            }
        }
        corr_dev = static_cast<double*>(ctx.alloc(total * sizeof(double)));
        std::vector<double> scaled;
        for (uint32_t k = 0; k < nbox; ++k)
            if (laws[k].corr) {
                const uint64_t m = laws[k].corr_n + 1ull, cnt = (uint64_t)laws[k].D * laws[k].D * m * m * m * 3ull;
                const double* src = laws[k].corr;
                const double b2 = t.bbox[k] * t.bbox[k];   // the records carry G m / box^2
                if (b2 != 1.0) {
                    scaled.assign(src, src + cnt);
                    for (double& v : scaled) v *= b2;
                    src = scaled.data();
                }
                ctx.to_device(corr_dev + corr_off[k], src, cnt * sizeof(double));
            }
    }
    uint32_t pair_max = 0, value_max = 0;
    for (uint32_t k = 0; k < nbox; ++k) {
        if (laws[k].grid != grid) fail(NGR_EINVAL, "the boxes of one call must share the table grid");
        if (!part[k]) continue;
        for (uint32_t ab = 0; ab < laws[k].D * laws[k].D; ++ab) eps0 |= laws[k].eps_ab[ab] == 0.0;
        pair_max = std::max(pair_max, table_bytes(kPair, laws[k].D, laws[k].ntab));
        value_max = std::max(value_max, table_bytes(kValue, laws[k].D, laws[k].ntab));
    }
    // layout and workgroup shape within the LDS of one workgroup: the
    // (value, slope) tables when at least 8 waves still fit beside them
    // (accumulator laws add the core-factor table and a core scale per record)
    const size_t lds_max = ctx.lds_per_block;
    const size_t wave_lds = acc_law ? kWaveLdsAcc : kWaveLds, extra = acc_law ? kCoreBytes : 0;
    int mode = kPair;
    size_t tab_bytes = pair_max + extra;
    if (kCtrlBytes + tab_bytes + 8 * wave_lds > lds_max) {
        mode = kValue;
        tab_bytes = value_max + extra;
    }
    if (kCtrlBytes + tab_bytes + wave_lds > lds_max) fail(NGR_EINVAL, "force tables do not fit in LDS");
    // In arena mode (no allocation) one workgroup of at most kArenaWaves
    // waves per CU, with stacks of 21 levels x 512 entries (the most a batch
    // walk can hold) plus a margin, all taken from the arena.
    const int waves = (int)std::min<size_t>(ctx.arena ? kArenaWaves : kMaxWaves,
                                            (lds_max - kCtrlBytes - tab_bytes) / wave_lds);
    const size_t lds = kCtrlBytes + tab_bytes + (size_t)waves * wave_lds;
    const size_t per_cu = std::max<size_t>(1, lds_max / lds);
    const int blocks = ctx.num_cu * (ctx.arena ? 1 : (int)std::min<size_t>(per_cu, 4));
    const uint32_t stack_cap = ctx.arena ? kArenaStack : 16384;
    uint32_t* stacks;
    if (ctx.arena) {
        stacks = static_cast<uint32_t*>(ctx.alloc((size_t)blocks * waves * stack_cap * sizeof(uint32_t)));
    } else {
        ctx.ensure(ctx.stacks, (size_t)blocks * waves * stack_cap * sizeof(uint32_t));
        stacks = static_cast<uint32_t*>(ctx.stacks.p);
    }

    // per-box parameters
    std::vector<BoxParams> bp(nbox);
    for (uint32_t k = 0; k < nbox; ++k) {
        const Law& law = laws[k];
        BoxParams& P = bp[k];
        std::memset(&P, 0, sizeof P);
        const double box = t.bbox[k];
        const double ib2 = 1.0 / (box * box);          // lengths squared in box units
        P.box = 1.0;
        P.inv_box = 1.0;
        P.eps2 = law.eps * law.eps * ib2;
        const double q = law.r_cut / box * 2097152.0;   // r_cut in half key units
        P.R2 = law.corr ? __builtin_inf() : q * q;      // with lattice corrections every pair interacts
        P.theta2 = law.theta * law.theta;
        const double wl = std::floor(1048576.0 * (1.0 - 2.0 * law.r_cut / box)) - 1.0;
        P.wrap_limit = wl < 0.0 ? 0u : (uint32_t)wl;
        const double rc2 = law.r_cut * law.r_cut;      // caller's units
        const double rc2u = rc2 * ib2, rcu = law.r_cut / box;
        if (law.grid == NGR_GRID_R2) {
            P.tscale = (float)((law.ntab - 1) / rc2u);
            P.toff = (float)(-(law.eps * law.eps) * ((law.ntab - 1) / rc2));   // -eps^2 / h, no unit
        } else {
            P.tscale = (float)((law.ntab - 1) / rcu);
            P.toff = 0.0f;
        }
        P.tmax = (float)(law.ntab - 1);
        P.tie_rc2 = rc2u;
        P.tie_band = 1e-6 * rc2u;
        for (uint32_t ab = 0; ab < law.D * law.D; ++ab) {
            const double e2 = law.eps_ab[ab] * law.eps_ab[ab];
            P.eps2_ab[ab] = e2 * ib2;
            P.toff_ab[ab] = law.grid == NGR_GRID_R2 ? (float)(-e2 * ((law.ntab - 1) / rc2)) : 0.0f;
        }
        for (uint32_t j = 0; j < law.D * law.D; ++j) P.G[j] = law.G[j] * ib2;
        P.acc = accv[k];
        P.in_off = t.boff[k];
        P.n = t.boff[k + 1] - t.boff[k];
        P.D = law.D;
        P.ntab = law.ntab;
        P.pair = tables[k].pair;
        P.value = tables[k].value;
        if (law.kind == NGR_LAW_ACCUMULATOR) {
            P.cored = law.cored;
            P.inv4pib = 1.0 / (4.0 * M_PI * law.beta * box);   // core scale in box units
        }
        P.track = law.track;
        if (law.corr) {
            P.corr = corr_dev + corr_off[k];
            P.corr_n = law.corr_n;
            P.corr_scale = (double)law.corr_n / 0.5;
        }
        if (law.opening == NGR_OPEN_RELATIVE) {
            const double u = box / 2097152.0;   // one half key unit
            P.relative = 1;
            P.rel_k = law.alpha * (u * u);
            P.old_acc = law.old_acc;
        }
    }
    BoxParams* boxes = static_cast<BoxParams*>(ctx.alloc(nbox * sizeof(BoxParams)));
    ctx.to_device(boxes, bp.data(), nbox * sizeof(BoxParams));

    // segments: first groups, queues, counts and the start schedule (most groups first)
    const uint32_t nseg = g.nseg;
    std::vector<uint32_t> sched;
    for (uint32_t q = 0; q < nseg; ++q)
        if (part[q / D] && g.first[q + 1] > g.first[q]) sched.push_back(q);
    std::stable_sort(sched.begin(), sched.end(), [&](uint32_t x, uint32_t y) {
        return g.first[x + 1] - g.first[x] > g.first[y + 1] - g.first[y];
    });
    const uint32_t nsched = (uint32_t)sched.size();
    // control block: seg_counts (kSegCounts x nseg u64) | queues (nseg) | cursor | error | seg_first (nseg+1) | sched
    const size_t cnt_bytes = (size_t)kSegCounts * nseg * sizeof(uint64_t);
    const size_t ctl_words = (size_t)nseg + 2 + (nseg + 1) + nsched;
    unsigned char* ctl = static_cast<unsigned char*>(ctx.alloc(cnt_bytes + ctl_words * sizeof(uint32_t)));
    unsigned long long* seg_counts = reinterpret_cast<unsigned long long*>(ctl);
    uint32_t* queues = reinterpret_cast<uint32_t*>(ctl + cnt_bytes);
    uint32_t* cursor = queues + nseg;
    uint32_t* err = cursor + 1;
    uint32_t* seg_first = err + 1;
    uint32_t* sched_dev = seg_first + nseg + 1;
    {
        std::vector<uint32_t> host((size_t)nseg + 2 + (nseg + 1) + nsched, 0);
        host[nseg] = std::min<uint32_t>((uint32_t)blocks, nsched);   // cursor: entries the first workgroups take
        for (uint32_t q = 0; q < nseg; ++q)   // another launch's segments start with their queue spent
            if (!part[q / D]) host[q] = g.first[q + 1] - g.first[q];
        for (uint32_t q = 0; q <= nseg; ++q) host[(size_t)nseg + 2 + q] = (uint32_t)g.first[q];
        for (uint32_t q = 0; q < nsched; ++q) host[(size_t)nseg + 2 + nseg + 1 + q] = sched[q];
        HIP_CHECK(hipMemsetAsync(seg_counts, 0, cnt_bytes, ctx.stream));
        ctx.to_device(queues, host.data(), host.size() * sizeof(uint32_t));
    }
    ctx.stage("walk: order");
    const bool timed = !ctx.arena;      // arena mode creates no events
    hipEvent_t e0 = nullptr, e1 = nullptr, e2 = nullptr;
    if (timed) {
        HIP_CHECK(hipEventCreate(&e0));
        HIP_CHECK(hipEventCreate(&e1));
        HIP_CHECK(hipEventCreate(&e2));
        HIP_CHECK(hipEventRecord(e0, ctx.stream));
    }
    uint32_t* gbucket = static_cast<uint32_t*>(ctx.alloc(std::max<uint64_t>(g.ng, 1) * sizeof(uint32_t)));
    uint32_t* order = order_groups(ctx, t, g, laws, gbucket);
    unsigned long long* seg_work =
        static_cast<unsigned long long*>(ctx.alloc(std::max<uint32_t>(nseg, 1) * sizeof(unsigned long long)));
    hipLaunchKernelGGL(seg_work_init, dim3(nseg), dim3(256), 0, ctx.stream, seg_first, gbucket, seg_work);
    LAUNCH_CHECK("seg_work_init");

    WalkArgs A{};
    A.cell = t.cell;
    A.first_child = t.first_child;
    A.n_child = t.n_child;
    A.start = t.start;
    A.count = t.count;
    A.mono = t.mono;
    A.nn = t.nn;
    A.X = t.X;
    A.mass = t.mass;
    A.P = t.P;
    A.perm = t.perm;
    A.n = t.n;
    A.gstart = g.start;
    A.gcount = g.count;
    A.glo = g.lo;
    A.ghi = g.hi;
    A.ng = g.ng;
    A.D = D;
    A.nseg = nseg;
    A.order = order;
    A.seg_first = seg_first;
    A.queues = queues;
    A.seg_work = seg_work;
    A.gbucket = gbucket;
    A.sched = sched_dev;
    A.nsched = nsched;
    A.cursor = cursor;
    A.boxes = boxes;
    A.seg_counts = seg_counts;
    A.gcounts = reinterpret_cast<unsigned long long*>(group_counts_dev);
    A.stacks = stacks;
    A.stack_cap = stack_cap;
    A.error_flag = err;
    A.max_steps = (uint32_t)std::min<uint64_t>(t.nn + 1, 0xffffffffull);
    A.tab_bytes = (uint32_t)tab_bytes;
    A.core = core_table;

    if (timed) HIP_CHECK(hipEventRecord(e1, ctx.stream));
    ctx.stage("walk: launch");
    A.box0 = bp[0];
    auto launch = [&](auto kernel) {
        hipLaunchKernelGGL(kernel, dim3(blocks), dim3(waves * 64), lds, ctx.stream, A);
        LAUNCH_CHECK("walk_kernel");
    };
    // a one-box call reads its box's parameters from the kernel arguments;
    // the accumulator laws read them from the table in device memory. The
    // near-tie count is an instantiation of the one-box table-law walk.
    const bool ties = count_ties && nbox == 1 && !acc_law && !ew;
    const int sel = (ties ? 32 : ew ? 24 : acc_law ? 16 : nbox == 1 ? 8 : 0) + (grid == NGR_GRID_R2 ? 4 : 0) +
                    (mode == kValue ? 2 : 0) + (eps0 ? 1 : 0);
    switch (sel) {
    case 32: launch(walk_kernel<NGR_GRID_R, kPair, false, true, false, false, true>); break;
    case 33: launch(walk_kernel<NGR_GRID_R, kPair, true, true, false, false, true>); break;
    case 34: launch(walk_kernel<NGR_GRID_R, kValue, false, true, false, false, true>); break;
    case 35: launch(walk_kernel<NGR_GRID_R, kValue, true, true, false, false, true>); break;
    case 36: launch(walk_kernel<NGR_GRID_R2, kPair, false, true, false, false, true>); break;
    case 37: launch(walk_kernel<NGR_GRID_R2, kPair, true, true, false, false, true>); break;
    case 38: launch(walk_kernel<NGR_GRID_R2, kValue, false, true, false, false, true>); break;
    case 39: launch(walk_kernel<NGR_GRID_R2, kValue, true, true, false, false, true>); break;
    case 24: launch(walk_kernel<NGR_GRID_R, kPair, false, false, false, true>); break;
    case 25: launch(walk_kernel<NGR_GRID_R, kPair, true, false, false, true>); break;
    case 26: launch(walk_kernel<NGR_GRID_R, kValue, false, false, false, true>); break;
    case 27: launch(walk_kernel<NGR_GRID_R, kValue, true, false, false, true>); break;
    case 28: launch(walk_kernel<NGR_GRID_R2, kPair, false, false, false, true>); break;
    case 29: launch(walk_kernel<NGR_GRID_R2, kPair, true, false, false, true>); break;
    case 30: launch(walk_kernel<NGR_GRID_R2, kValue, false, false, false, true>); break;
    case 31: launch(walk_kernel<NGR_GRID_R2, kValue, true, false, false, true>); break;
    case 0: launch(walk_kernel<NGR_GRID_R, kPair, false, false, false>); break;
    case 1: launch(walk_kernel<NGR_GRID_R, kPair, true, false, false>); break;
    case 2: launch(walk_kernel<NGR_GRID_R, kValue, false, false, false>); break;
    case 3: launch(walk_kernel<NGR_GRID_R, kValue, true, false, false>); break;
    case 4: launch(walk_kernel<NGR_GRID_R2, kPair, false, false, false>); break;
    case 5: launch(walk_kernel<NGR_GRID_R2, kPair, true, false, false>); break;
    case 6: launch(walk_kernel<NGR_GRID_R2, kValue, false, false, false>); break;
    case 7: launch(walk_kernel<NGR_GRID_R2, kValue, true, false, false>); break;
    case 8: launch(walk_kernel<NGR_GRID_R, kPair, false, true, false>); break;
    case 9: launch(walk_kernel<NGR_GRID_R, kPair, true, true, false>); break;
    case 10: launch(walk_kernel<NGR_GRID_R, kValue, false, true, false>); break;
    case 11: launch(walk_kernel<NGR_GRID_R, kValue, true, true, false>); break;
    case 12: launch(walk_kernel<NGR_GRID_R2, kPair, false, true, false>); break;
    case 13: launch(walk_kernel<NGR_GRID_R2, kPair, true, true, false>); break;
    case 14: launch(walk_kernel<NGR_GRID_R2, kValue, false, true, false>); break;
    case 15: launch(walk_kernel<NGR_GRID_R2, kValue, true, true, false>); break;
    case 16: launch(walk_kernel<NGR_GRID_R, kPair, false, false, true>); break;
    case 17: launch(walk_kernel<NGR_GRID_R, kPair, true, false, true>); break;
    case 18: launch(walk_kernel<NGR_GRID_R, kValue, false, false, true>); break;
    case 19: launch(walk_kernel<NGR_GRID_R, kValue, true, false, true>); break;
    case 20: launch(walk_kernel<NGR_GRID_R2, kPair, false, false, true>); break;
    case 21: launch(walk_kernel<NGR_GRID_R2, kPair, true, false, true>); break;
    case 22: launch(walk_kernel<NGR_GRID_R2, kValue, false, false, true>); break;
    default: launch(walk_kernel<NGR_GRID_R2, kValue, true, false, true>); break;
    }
    if (timed) HIP_CHECK(hipEventRecord(e2, ctx.stream));
    std::vector<uint64_t> counts((size_t)kSegCounts * nseg);
    uint32_t herr = 0;
    ctx.to_host(counts.data(), seg_counts, cnt_bytes);
    ctx.to_host(&herr, err, sizeof herr);
    ctx.stage("walk: done");
    ctx.release(order);
    ctx.release(seg_work);
    ctx.release(gbucket);
    ctx.release(ctl);
    ctx.release(boxes);
    if (corr_dev) ctx.release(corr_dev);
    float ms_order = 0.0f, ms = 0.0f;
    if (timed) {
        HIP_CHECK(hipEventElapsedTime(&ms_order, e0, e1));
        HIP_CHECK(hipEventElapsedTime(&ms, e1, e2));
        HIP_CHECK(hipEventDestroy(e0));
        HIP_CHECK(hipEventDestroy(e1));
        HIP_CHECK(hipEventDestroy(e2));
    }
    if (herr) fail(NGR_ENOMEM, "walk stack or step capacity exceeded");
    uint64_t nties = 0;
    for (uint32_t q = 0; q < nseg; ++q) {
        const uint64_t* c = &counts[(size_t)kSegCounts * q];
        out.box_pp[q / D] += c[0];
        out.box_pn[q / D] += c[1];
        nties += c[2];
        for (uint32_t b = 0; b < NGR_MAX_SPECIES; ++b) out.box_pnb[(size_t)(q / D) * NGR_MAX_SPECIES + b] += c[3 + b];
    }
    if (ties) out.ties = nties;
    out.ms_walk += ms;
    out.ms_order += ms_order;
}

void walk_force(Context& ctx, const Tree& t, const Groups& g, const std::vector<Law>& laws,
                const std::vector<LawTables>& tables, const std::vector<double*>& accv, uint64_t* group_counts_dev,
                WalkOut& out, bool count_ties)
{
    out = WalkOut{};
    const uint32_t nbox = t.nbox;
    out.box_pp.assign(nbox, 0);
    out.box_pn.assign(nbox, 0);
    out.box_pnb.assign((size_t)nbox * NGR_MAX_SPECIES, 0);
    if (t.n == 0 || g.ng == 0) {
        if (count_ties) out.ties = 0;
        return;
    }
    // A launch holds one law kind. A batch that mixes accumulator and table
    // laws walks each kind in a launch of its own, so every box runs the
    // kernel, and so the lane mapping, of its single-box call.
    bool acc = false, table = false;
    for (uint32_t k = 0; k < nbox; ++k) (laws[k].kind == NGR_LAW_ACCUMULATOR ? acc : table) = true;
    std::vector<char> part(nbox, 1);
    if (acc && table) {
        for (uint32_t k = 0; k < nbox; ++k) part[k] = laws[k].kind == NGR_LAW_ACCUMULATOR;
        walk_launch(ctx, t, g, laws, tables, accv, group_counts_dev, out, count_ties, part);
        for (uint32_t k = 0; k < nbox; ++k) part[k] = !part[k];
    }
    walk_launch(ctx, t, g, laws, tables, accv, group_counts_dev, out, count_ties, part);
    for (uint32_t k = 0; k < nbox; ++k) {
        out.pp += out.box_pp[k];
        out.pn += out.box_pn[k];
        for (uint32_t b = 0; b < NGR_MAX_SPECIES; ++b) out.pnb[b] += out.box_pnb[(size_t)k * NGR_MAX_SPECIES + b];
    }
}

}  // namespace ngr
