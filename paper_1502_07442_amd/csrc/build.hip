// Tree construction on the device: input checks, 64-bit lattice, keys,
// stable sort by (species, Morton key), gather, breadth-first octree with
// per-species ranges, and the bottom-up per-species monopoles.
//
// Paper: Croker, ngravs (CPC). Section 2: recursive halving of the volume;
// section 2.2: one tree over all species, whose nodes carry a mass and a
// centre of mass per species and optionally the per-species body count
// N_perp; section 2.4: one sort by gravitational type and then along the
// space-filling curve, with a single reordering of the particle data.
#include <algorithm>
#include <cmath>

#include "ngr_internal.hpp"

namespace ngr {
namespace {

enum : uint32_t { kBadSpecies = 1, kBadMass = 2, kBadPos = 4, kBadRegion = 8 };

// One box of a build as the device sees it.
struct BoxInDev {
    const double* pos;
    const uint64_t* lattice;
    const uint8_t* species;
    const double* mass;
    uint64_t n, off;          // particles and first index in the concatenated arrays
    double box;
    double region;            // non-periodic: positions must lie in [0, region); 0 for periodic
    uint32_t D, leaf, key_order;
};

// Spread the low 20 bits of v so that bit i lands on bit 3i.
__device__ inline uint64_t spread3(uint64_t v)
{
    v &= 0xfffffull;
    v = (v | (v << 32)) & 0x1f00000000ffffull;
    v = (v | (v << 16)) & 0x1f0000ff0000ffull;
    v = (v | (v << 8)) & 0x100f00f00f00f00full;
    v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
}

// Peano-Hilbert index of a point of the 20-bit key lattice (the curve of
// section 2.4), by J. Skilling's transpose method ("Programming the Hilbert
// curve", 2004): from the top bit down, the low bits are reflected (x) or
// exchanged with x (y, z) wherever the sub-cube of that bit requires; the
// result is Gray-coded and the three components interleaved like the Morton
// key (x's bit the highest of each 3-bit digit).
__device__ inline uint64_t hilbert60(uint32_t x, uint32_t y, uint32_t z)
{
    for (uint32_t q = 1u << (kLevels - 1); q > 1u; q >>= 1) {
        const uint32_t low = q - 1u;
        if (x & q) x ^= low;
        if (y & q) {
            x ^= low;
        } else {
            const uint32_t t = (x ^ y) & low;
            x ^= t;
            y ^= t;
        }
        if (z & q) {
            x ^= low;
        } else {
            const uint32_t t = (x ^ z) & low;
            x ^= t;
            z ^= t;
        }
    }
    y ^= x;
    z ^= y;
    uint32_t flip = 0;
    for (uint32_t q = 1u << (kLevels - 1); q > 1u; q >>= 1)
        if (z & q) flip ^= q - 1u;
    x ^= flip;
    y ^= flip;
    z ^= flip;
    return (spread3(x) << 2) | (spread3(y) << 1) | spread3(z);
}

// One thread per particle of box blockIdx.y (grid-stride over a bounded
// grid): checks the species id, mass and position; converts the position to
// the 64-bit lattice, X = floor(u * 2^64) with u = x / box taken modulo 1 (the
// box is periodic); forms the key species << 60 | curve index of the top 20
// bits of each axis (Morton: x the most significant bit of each 3-bit digit;
// or Peano-Hilbert); and counts each species of the box (the counts give its
// species segments).
// Per-box flags and counts take one global atomic per workgroup.
// One particle in input order between the ingest and the reordering: the
// lattice coordinates and the mass together, so that the reordering reads
// one 32-byte record per particle.
struct alignas(32) InRec {
    uint64_t x, y, z;
    double m;
};

__global__ void ingest(const BoxInDev* __restrict__ boxes, InRec* __restrict__ rin,
                       uint64_t* __restrict__ keys, uint32_t* __restrict__ idx,
                       uint16_t* __restrict__ boxid, uint32_t* __restrict__ flags,
                       unsigned long long* __restrict__ counts)
{
    __shared__ unsigned int local[NGR_MAX_SPECIES];
    __shared__ unsigned int local_bad;
    const uint32_t k = blockIdx.y;
    const BoxInDev B = boxes[k];
    if (threadIdx.x < NGR_MAX_SPECIES) local[threadIdx.x] = 0;
    if (threadIdx.x == 0) local_bad = 0;
    __syncthreads();
    uint32_t bad = 0;
    uint32_t mine[NGR_MAX_SPECIES] = {0, 0, 0, 0, 0, 0};
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < B.n; i += stride) {
        const uint32_t s = B.species[i];
        const double m = B.mass[i];
        if (s >= B.D) bad |= kBadSpecies;
#pragma unroll
        for (uint32_t b = 0; b < NGR_MAX_SPECIES; ++b) mine[b] += s == b ? 1u : 0u;
        if (!(m >= 0.0) || !isfinite(m)) bad |= kBadMass;
        uint64_t X[3];
        if (B.pos) {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const double x = B.pos[a * B.n + i];
                if (!isfinite(x)) bad |= kBadPos;
                if (B.region > 0.0 && !(x >= 0.0 && x < B.region)) bad |= kBadRegion;
                double u = x / B.box;
                u = u - floor(u);
                if (!(u < 1.0)) u = 0.0;
                X[a] = (uint64_t)(u * 18446744073709551616.0);
            }
        } else {
#pragma unroll
            for (int a = 0; a < 3; ++a) X[a] = B.lattice[a * B.n + i];
        }
        const uint64_t g = B.off + i;
        InRec r;
        r.x = X[0];
        r.y = X[1];
        r.z = X[2];
        r.m = m;
        rin[g] = r;
        const uint64_t mo = B.key_order == NGR_KEY_HILBERT
                                ? hilbert60((uint32_t)(X[0] >> 44), (uint32_t)(X[1] >> 44), (uint32_t)(X[2] >> 44))
                                : (spread3(X[0] >> 44) << 2) | (spread3(X[1] >> 44) << 1) | spread3(X[2] >> 44);
        keys[g] = ((uint64_t)(s & 0xfu) << kKeyBits) | mo;
        idx[g] = (uint32_t)g;
        if (boxid) boxid[g] = (uint16_t)k;
    }
    for (uint32_t b = 0; b < NGR_MAX_SPECIES; ++b)
        if (mine[b]) atomicAdd(&local[b], mine[b]);
    if (bad) atomicOr(&local_bad, bad);
    __syncthreads();
    if (threadIdx.x < NGR_MAX_SPECIES && local[threadIdx.x])
        atomicAdd(&counts[(uint64_t)k * NGR_MAX_SPECIES + threadIdx.x], (unsigned long long)local[threadIdx.x]);
    if (threadIdx.x == 0 && local_bad) atomicOr(&flags[k], local_bad);
}

// Checks of one box's inputs only (species id, mass, finite position); one
// global atomic per workgroup.
__global__ void check_box(uint64_t n, uint32_t D, const uint8_t* __restrict__ species, const double* __restrict__ mass,
                          const double* __restrict__ pos, uint32_t* __restrict__ flags)
{
    __shared__ unsigned int local_bad;
    if (threadIdx.x == 0) local_bad = 0;
    __syncthreads();
    uint32_t bad = 0;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        if (species[i] >= D) bad |= kBadSpecies;
        const double m = mass[i];
        if (!(m >= 0.0) || !isfinite(m)) bad |= kBadMass;
        if (pos && !(isfinite(pos[i]) && isfinite(pos[n + i]) && isfinite(pos[2 * n + i]))) bad |= kBadPos;
    }
    if (bad) atomicOr(&local_bad, bad);
    __syncthreads();
    if (threadIdx.x == 0 && local_bad) atomicOr(flags, local_bad);
}

// Sort key of the box pass: the box of each element, in the current order.
__global__ void box_keys(uint64_t n, const uint32_t* __restrict__ idx, const uint16_t* __restrict__ boxid,
                         uint64_t* __restrict__ kb)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) kb[i] = boxid[idx[i]];
}

__global__ void gather_keys(uint64_t n, const uint32_t* __restrict__ perm, const uint64_t* __restrict__ kin,
                            uint64_t* __restrict__ kout)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) kout[i] = kin[perm[i]];
}

// The single reordering of the particle data into sorted order: the
// lattice coordinates and masses, and the walk's split records.
__global__ void gather_particles(uint64_t n, const uint32_t* __restrict__ perm, const InRec* __restrict__ rin,
                                 uint64_t* __restrict__ Xout, double* __restrict__ mout, PRec* __restrict__ Pout)
{
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const InRec q = rin[perm[i]];
    const uint64_t x = q.x, y = q.y, z = q.z;
    const double m = q.m;
    Xout[i] = x;
    Xout[n + i] = y;
    Xout[2 * n + i] = z;
    mout[i] = m;
    PRec r;
    r.hx = (double)(x & ~kLowBits) * 0x1p-64;
    r.hy = (double)(y & ~kLowBits) * 0x1p-64;
    r.hz = (double)(z & ~kLowBits) * 0x1p-64;
    r.m = m;
    r.lx = (float)(uint32_t)(x & kLowBits) * 0x1p-64f;
    r.ly = (float)(uint32_t)(y & kLowBits) * 0x1p-64f;
    r.lz = (float)(uint32_t)(z & kLowBits) * 0x1p-64f;
    r.pad = 0.0f;
    Pout[i] = r;
}

// The roots: node k is box k's root, holding its species segments.
__global__ void init_roots(uint32_t nbox, uint32_t D, const uint64_t* __restrict__ bseg, uint8_t* level,
                           uint64_t* prefix, int32_t* parent, int32_t* first_child, uint8_t* n_child, uint4* cell,
                           uint32_t* start, uint32_t* count, uint32_t* node_box)
{
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nbox) return;
    level[k] = 0;
    prefix[k] = 0;
    parent[k] = -1;
    first_child[k] = -1;
    n_child[k] = 0;
    cell[k] = make_uint4(0, 0, 0, 0);
    node_box[k] = k;
    const uint64_t* sg = bseg + (uint64_t)k * (NGR_MAX_SPECIES + 1);
    for (uint32_t b = 0; b < D; ++b) {
        start[(uint64_t)k * D + b] = (uint32_t)sg[b];
        count[(uint64_t)k * D + b] = (uint32_t)(sg[b + 1] - sg[b]);
    }
}

__device__ inline uint64_t lower_bound(const uint64_t* __restrict__ keys, uint64_t lo, uint64_t hi, uint64_t key)
{
    while (lo < hi) {
        uint64_t mid = lo + ((hi - lo) >> 1);
        if (keys[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// One thread per (node of this level, octant): the start of the octant's
// particles of each species is found by binary search inside the node's
// species range (the range is sorted by key). The octant ends where the next
// one starts (the next thread, as a node's eight octants are consecutive lanes
// of one wave), the last at the end of the range, as every key of the range
// carries the node's prefix. Nodes holding more than B particles below level
// 20 split; a non-empty octant becomes a child.
__global__ void split_level(uint64_t level_begin, uint64_t n_level, uint32_t lvl, uint32_t D,
                            const uint32_t* __restrict__ leaf_size, const uint32_t* __restrict__ node_box,
                            const uint64_t* __restrict__ keys, const uint64_t* __restrict__ prefix,
                            const uint32_t* __restrict__ start, const uint32_t* __restrict__ count,
                            uint32_t* __restrict__ cstart, uint32_t* __restrict__ ccount,
                            uint32_t* __restrict__ flags)
{
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_level * 8) return;   // whole nodes: the block size is a multiple of 8
    const uint64_t p = level_begin + t / 8;
    const uint32_t o = (uint32_t)(t % 8);
    uint32_t total = 0;
    for (uint32_t b = 0; b < D; ++b) total += count[p * D + b];
    // a node's eight lanes leave together, so a lane's neighbour in the
    // exchange below (the next octant of the same node) is always active
    if (total <= leaf_size[node_box[p]] || lvl >= (uint32_t)kLevels) {
        flags[t] = 0;
        return;
    }
    const uint32_t sh = kKeyBits - 3 * (lvl + 1);
    const uint64_t klo = (prefix[p] * 8 + o) << sh;
    uint32_t tot = 0;
    for (uint32_t b = 0; b < D; ++b) {
        const uint32_t lo = start[p * D + b], hi = lo + count[p * D + b];
        const uint32_t a0 = (uint32_t)lower_bound(keys, lo, hi, ((uint64_t)b << kKeyBits) + klo);
        const uint32_t next = __shfl_down(a0, 1);
        const uint32_t a1 = o == 7 ? hi : next;
        cstart[t * D + b] = a0;
        ccount[t * D + b] = a1 - a0;
        tot += a1 - a0;
    }
    flags[t] = tot > 0;
}

// The same split for a level of few nodes, one wave per node: lane 8·o + b
// searches where octant o starts in the node's species-b range, so the
// searches of a node run side by side rather than one after another (at the
// top levels each search spans millions of keys). An octant ends where the
// next one starts, the last at the end of the range, as every key of the range
// carries the node's prefix. Same outputs as split_level.
__global__ __launch_bounds__(256) void split_level_wave(uint64_t level_begin, uint64_t n_level, uint32_t lvl,
                                                        uint32_t D, const uint32_t* __restrict__ leaf_size,
                                                        const uint32_t* __restrict__ node_box,
                                                        const uint64_t* __restrict__ keys,
                                                        const uint64_t* __restrict__ prefix,
                                                        const uint32_t* __restrict__ start,
                                                        const uint32_t* __restrict__ count,
                                                        uint32_t* __restrict__ cstart, uint32_t* __restrict__ ccount,
                                                        uint32_t* __restrict__ flags)
{
    const uint64_t w = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (w >= n_level) return;   // a whole wave leaves together
    const uint32_t lane = threadIdx.x & 63u, o = lane >> 3, b = lane & 7u;
    const uint64_t p = level_begin + w;
    const bool real = b < D;
    const uint32_t lo = real ? start[p * D + b] : 0u;
    const uint32_t cnt = real ? count[p * D + b] : 0u;
    // the node's particle count: each species' count once, from the lanes of octant 0
    uint32_t total = o == 0 ? cnt : 0u;
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) total += __shfl_xor(total, m);
    const uint64_t t = w * 8 + o;
    if (total <= leaf_size[node_box[p]] || lvl >= (uint32_t)kLevels) {   // uniform over the wave
        if (b == 0) flags[t] = 0;
        return;
    }
    const uint32_t sh = kKeyBits - 3 * (lvl + 1);
    const uint64_t klo = (prefix[p] * 8 + o) << sh;
    const uint32_t a0 = real ? (uint32_t)lower_bound(keys, lo, (uint64_t)lo + cnt, ((uint64_t)b << kKeyBits) + klo) : 0u;
    const uint32_t next = __shfl_down(a0, 8);
    const uint32_t a1 = o == 7 ? lo + cnt : next;
    if (real) {
        cstart[t * D + b] = a0;
        ccount[t * D + b] = a1 - a0;
    }
    uint32_t c = real ? a1 - a0 : 0u;
#pragma unroll
    for (int m = 1; m < 8; m <<= 1) c += __shfl_xor(c, m);
    if (b == 0) flags[t] = c > 0;
}

// Write the children found by split_level (in key order, after all
// children of earlier nodes of the level) and the parents' child links. A
// child's cell is read off its first particle: the top lvl + 1 bits of each
// lattice coordinate (whatever curve ordered the keys).
__global__ void emit_children(uint64_t level_begin, uint64_t n_level, uint64_t next_begin, uint32_t lvl,
                              uint32_t D, const uint32_t* __restrict__ flags, const uint32_t* __restrict__ offs,
                              const uint32_t* __restrict__ cstart, const uint32_t* __restrict__ ccount,
                              uint8_t* level, uint64_t* prefix, int32_t* parent, int32_t* first_child,
                              uint8_t* n_child, uint4* cell, uint32_t* start, uint32_t* count,
                              uint32_t* node_box, const PRec* __restrict__ P)
{
    uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_level * 8) return;
    uint64_t pl = t / 8;
    uint64_t p = level_begin + pl;
    uint32_t o = (uint32_t)(t % 8);
    if (o == 0) {
        uint32_t nc = 0;
        for (int k = 0; k < 8; ++k) nc += flags[pl * 8 + k];
        n_child[p] = (uint8_t)nc;
        first_child[p] = nc ? (int32_t)(next_begin + offs[pl * 8]) : -1;
    }
    if (!flags[t]) return;
    uint64_t c = next_begin + offs[t];
    level[c] = (uint8_t)(lvl + 1);
    prefix[c] = prefix[p] * 8 + o;
    parent[c] = (int32_t)p;
    node_box[c] = node_box[p];
    first_child[c] = -1;
    n_child[c] = 0;
    uint64_t j = 0;
    bool found = false;
    for (uint32_t b = 0; b < D; ++b) {
        start[c * D + b] = cstart[t * D + b];
        count[c * D + b] = ccount[t * D + b];
        if (!found && ccount[t * D + b]) {
            j = cstart[t * D + b];
            found = true;
        }
    }
    // the high part of a split record is the lattice word with its low bits
    // cleared, exactly, so it gives back the word's top lvl + 1 bits
    const PRec q = P[j];
    const uint32_t sh = 64u - (lvl + 1u), up = (uint32_t)kLevels - (lvl + 1u);
    cell[c] = make_uint4((uint32_t)((uint64_t)(q.hx * 0x1p64) >> sh) << up,
                         (uint32_t)((uint64_t)(q.hy * 0x1p64) >> sh) << up,
                         (uint32_t)((uint64_t)(q.hz * 0x1p64) >> sh) << up, lvl + 1);
}

// Number of leaves (nodes without children), over a bounded grid with one
// global atomic per workgroup.
__global__ void count_leaves(uint64_t nn, const uint8_t* __restrict__ n_child, unsigned long long* __restrict__ out)
{
    __shared__ unsigned long long part;
    if (threadIdx.x == 0) part = 0;
    __syncthreads();
    unsigned long long c = 0;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nn; i += stride) c += n_child[i] == 0;
    if (c) atomicAdd(&part, c);
    __syncthreads();
    if (threadIdx.x == 0 && part) atomicAdd(out, part);
}

// Nodes, leaves and deepest level of every box (for per-box statistics).
__global__ void node_counts(uint64_t nn, const uint32_t* __restrict__ node_box, const uint8_t* __restrict__ n_child,
                            const uint8_t* __restrict__ level, unsigned long long* __restrict__ nodes,
                            unsigned long long* __restrict__ leaves, uint32_t* __restrict__ depth)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nn) return;
    const uint32_t k = node_box[i];
    atomicAdd(&nodes[k], 1ull);
    if (n_child[i] == 0) atomicAdd(&leaves[k], 1ull);
    atomicMax(&depth[k], (uint32_t)level[i]);
}

// Monopoles of one level (section 2.2), one thread per (node, species b).
// A leaf sums its species-b particles directly, relative to the cell corner:
// from the split records, the high part minus the corner is exact and adding
// the low part rounds once, so each offset is the integer lattice difference
// converted to float64 (in units of the box). An internal node combines the
// monopoles of its children. Centres are kept as fractions of the box.
__global__ void monopole_level(uint64_t level_begin, uint64_t n_level, uint32_t D, uint64_t nn,
                               const uint4* __restrict__ cell, const int32_t* __restrict__ first_child,
                               const uint8_t* __restrict__ n_child, const uint32_t* __restrict__ start,
                               const uint32_t* __restrict__ count, const PRec* __restrict__ P,
                               double4* __restrict__ mono)
{
    uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_level * D) return;
    uint64_t i = level_begin + t / D;
    uint32_t b = (uint32_t)(t % D);
    double M = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
    double4 out;
    if (n_child[i] == 0) {
        const uint4 c = cell[i];
        const double cx = (double)c.x * 0x1p-20, cy = (double)c.y * 0x1p-20, cz = (double)c.z * 0x1p-20;
        uint64_t j0 = start[i * D + b], j1 = j0 + count[i * D + b];
#pragma unroll 4
        for (uint64_t j = j0; j < j1; ++j) {
            const PRec q = P[j];
            const double m = q.m;
            M += m;
            sx += m * ((q.hx - cx) + (double)q.lx);
            sy += m * ((q.hy - cy) + (double)q.ly);
            sz += m * ((q.hz - cz) + (double)q.lz);
        }
        out = M > 0.0 ? make_double4(cx + sx / M, cy + sy / M, cz + sz / M, M) : make_double4(0.0, 0.0, 0.0, 0.0);
    } else {
        // at most eight children: their records are loaded together, then
        // added in child order
        const uint64_t c0 = (uint64_t)first_child[i];
        const uint32_t nc = n_child[i];
        double4 r[8];
#pragma unroll
        for (uint32_t k = 0; k < 8; ++k) r[k] = k < nc ? mono[b * nn + c0 + k] : make_double4(0.0, 0.0, 0.0, 0.0);
#pragma unroll
        for (uint32_t k = 0; k < 8; ++k) {
            if (r[k].w > 0.0) {
                M += r[k].w;
                sx += r[k].w * r[k].x;
                sy += r[k].w * r[k].y;
                sz += r[k].w * r[k].z;
            }
        }
        out = M > 0.0 ? make_double4(sx / M, sy / M, sz / M, M) : make_double4(0.0, 0.0, 0.0, 0.0);
    }
    mono[b * nn + i] = out;
}

inline unsigned blocks_for(uint64_t work, unsigned threads) { return (unsigned)((work + threads - 1) / threads); }

// The top levels are split one wave per node, down to the first level of more
// than this many nodes (below it ranges are short and one thread per octant is
// faster).
constexpr uint64_t kWaveSplitNodes = 1u << 19;

template <class T>
void grow(Context& ctx, T*& p, uint64_t old_n, uint64_t new_n)
{
    T* q = static_cast<T*>(ctx.alloc(new_n * sizeof(T)));
    if (p && old_n) HIP_CHECK(hipMemcpyAsync(q, p, old_n * sizeof(T), hipMemcpyDeviceToDevice, ctx.stream));
    ctx.release(p);
    p = q;
}

void grow_nodes(Context& ctx, Tree& t, uint64_t need)
{
    if (need <= t.cap) return;
    uint64_t cap = std::max<uint64_t>(need, t.cap * 2);
    uint64_t used = t.nn;
    grow(ctx, t.level, used, cap);
    grow(ctx, t.prefix, used, cap);
    grow(ctx, t.parent, used, cap);
    grow(ctx, t.first_child, used, cap);
    grow(ctx, t.n_child, used, cap);
    grow(ctx, t.cell, used, cap);
    grow(ctx, t.start, used * t.D, cap * t.D);
    grow(ctx, t.count, used * t.D, cap * t.D);
    grow(ctx, t.node_box, used, cap);
    t.cap = cap;
}

}  // namespace

void validate_box(Context& ctx, const BoxIn& b, const std::string& where)
{
    if (!b.n) return;
    uint32_t* flags = static_cast<uint32_t*>(ctx.alloc(sizeof(uint32_t)));
    HIP_CHECK(hipMemsetAsync(flags, 0, sizeof(uint32_t), ctx.stream));
    const unsigned gx = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(blocks_for(b.n, 256), 4ull * ctx.num_cu));
    hipLaunchKernelGGL(check_box, dim3(gx), dim3(256), 0, ctx.stream, b.n, b.D, b.species, b.mass, b.pos, flags);
    LAUNCH_CHECK("check_box");
    uint32_t h = 0;
    ctx.to_host(&h, flags, sizeof h);
    ctx.release(flags);
    if (h & kBadSpecies) fail(NGR_EINVAL, where + "a species id is >= D");
    if (h & kBadMass) fail(NGR_EINVAL, where + "a mass is negative or not finite");
    if (h & kBadPos) fail(NGR_EINVAL, where + "a position is not finite");
}

void free_tree(Context& ctx, Tree& t)
{
    for (void* q : {(void*)t.X, (void*)t.mass, (void*)t.P, (void*)t.perm, (void*)t.keys, (void*)t.level, (void*)t.prefix,
                    (void*)t.parent, (void*)t.first_child, (void*)t.n_child, (void*)t.cell, (void*)t.start,
                    (void*)t.count, (void*)t.node_box, (void*)t.mono, (void*)t.boff_dev})
        ctx.release(q);
    t.X = nullptr;
    t.mass = nullptr;
    t.P = nullptr;
    t.perm = nullptr;
    t.keys = nullptr;
    t.level = nullptr;
    t.prefix = nullptr;
    t.parent = nullptr;
    t.first_child = nullptr;
    t.n_child = nullptr;
    t.cell = nullptr;
    t.start = nullptr;
    t.count = nullptr;
    t.node_box = nullptr;
    t.mono = nullptr;
    t.boff_dev = nullptr;
}

void build_forest(Context& ctx, const std::vector<BoxIn>& boxes, Tree& t, bool timed)
{
    auto mark = [&](int k) {
        if (timed) HIP_CHECK(hipEventRecord(ctx.event(k), ctx.stream));
    };
    const uint32_t nbox = (uint32_t)boxes.size();
    if (nbox == 0 || nbox > 65535) fail(NGR_EINVAL, "the number of boxes must be in 1..65535");
    uint32_t D = 0;
    uint64_t n = 0;
    t.nbox = nbox;
    t.boff.assign(nbox + 1, 0);
    t.bD.resize(nbox);
    t.bbox.resize(nbox);
    t.bleaf.resize(nbox);
    std::vector<BoxInDev> bin(nbox);
    for (uint32_t k = 0; k < nbox; ++k) {
        const BoxIn& b = boxes[k];
        D = std::max(D, b.D);
        t.boff[k] = n;
        t.bD[k] = b.D;
        t.bbox[k] = b.box;
        t.bleaf[k] = b.leaf_size;
        bin[k] = BoxInDev{b.pos, b.lattice, b.species, b.mass, b.n, n, b.box, b.region, b.D, b.leaf_size, b.key_order};
        n += b.n;
    }
    t.boff[nbox] = n;
    if (n >= (1ull << 32) - 1) fail(NGR_EINVAL, "the boxes hold 2^32 - 1 or more particles");
    t.n = n;
    t.D = D;
    t.box = t.bbox[0];
    t.region = boxes[0].region;
    t.leaf_size = t.bleaf[0];

    // ---- input checks, lattice, keys and species counts (one synchronisation)
    ctx.stage("build: input checks and keys");
    mark(0);
    const uint64_t n1 = std::max<uint64_t>(n, 1);
    t.X = static_cast<uint64_t*>(ctx.alloc(3 * n1 * sizeof(uint64_t)));
    t.mass = static_cast<double*>(ctx.alloc(n1 * sizeof(double)));
    t.P = static_cast<PRec*>(ctx.alloc(n1 * sizeof(PRec)));
    t.perm = static_cast<uint32_t*>(ctx.alloc(n1 * sizeof(uint32_t)));
    t.keys = static_cast<uint64_t*>(ctx.alloc(n1 * sizeof(uint64_t)));
    t.boff_dev = static_cast<uint64_t*>(ctx.alloc((nbox + 1) * sizeof(uint64_t)));
    ctx.to_device(t.boff_dev, t.boff.data(), (nbox + 1) * sizeof(uint64_t));
    std::vector<uint64_t> counts((size_t)nbox * NGR_MAX_SPECIES, 0);
    std::vector<uint32_t> flags(nbox, 0);
    InRec* rin = nullptr;
    uint16_t* boxid = nullptr;
    if (n) {
        rin = static_cast<InRec*>(ctx.alloc(n * sizeof(InRec)));
        if (nbox > 1) boxid = static_cast<uint16_t*>(ctx.alloc(n * sizeof(uint16_t)));
        BoxInDev* bin_dev = static_cast<BoxInDev*>(ctx.alloc(nbox * sizeof(BoxInDev)));
        uint32_t* flags_dev = static_cast<uint32_t*>(ctx.alloc(nbox * sizeof(uint32_t)));
        unsigned long long* counts_dev =
            static_cast<unsigned long long*>(ctx.alloc((size_t)nbox * NGR_MAX_SPECIES * sizeof(uint64_t)));
        ctx.to_device(bin_dev, bin.data(), nbox * sizeof(BoxInDev));
        HIP_CHECK(hipMemsetAsync(flags_dev, 0, nbox * sizeof(uint32_t), ctx.stream));
        HIP_CHECK(hipMemsetAsync(counts_dev, 0, (size_t)nbox * NGR_MAX_SPECIES * sizeof(uint64_t), ctx.stream));
        uint64_t nmax = 0;
        for (const BoxIn& b : boxes) nmax = std::max(nmax, b.n);
        // about four workgroups per CU over all boxes, at least one per box
        const uint64_t per_box = std::max<uint64_t>(1, (4ull * ctx.num_cu + nbox - 1) / nbox);
        const unsigned gx = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(blocks_for(nmax, 256), per_box));
        hipLaunchKernelGGL(ingest, dim3(gx, nbox), dim3(256), 0, ctx.stream, bin_dev, rin, t.keys, t.perm, boxid,
                           flags_dev, counts_dev);
        LAUNCH_CHECK("ingest");
        mark(1);
        ctx.to_host(flags.data(), flags_dev, nbox * sizeof(uint32_t));
        ctx.to_host(counts.data(), counts_dev, (size_t)nbox * NGR_MAX_SPECIES * sizeof(uint64_t));
        ctx.release(bin_dev);
        ctx.release(flags_dev);
        ctx.release(counts_dev);
    }
    for (uint32_t k = 0; k < nbox; ++k) {
        if (!flags[k]) continue;
        const std::string where = nbox > 1 ? "box " + std::to_string(k) + ": " : "";
        ctx.release(rin);
        ctx.release(boxid);
        if (flags[k] & kBadSpecies) fail(NGR_EINVAL, where + "a species id is >= D");
        if (flags[k] & kBadMass) fail(NGR_EINVAL, where + "a mass is negative or not finite");
        if (flags[k] & kBadPos) fail(NGR_EINVAL, where + "a position is not finite");
        fail(NGR_EINVAL, where + "a position lies outside the non-periodic box");
    }
    t.bseg.assign((size_t)nbox * (NGR_MAX_SPECIES + 1), 0);
    for (uint32_t k = 0; k < nbox; ++k) {
        uint64_t* sg = &t.bseg[(size_t)k * (NGR_MAX_SPECIES + 1)];
        sg[0] = t.boff[k];
        for (uint32_t b = 0; b < NGR_MAX_SPECIES; ++b)
            sg[b + 1] = sg[b] + (b < t.bD[k] ? counts[(size_t)k * NGR_MAX_SPECIES + b] : 0);
    }
    for (uint32_t b = 0; b <= NGR_MAX_SPECIES; ++b) t.seg[b] = t.bseg[b] - t.boff[0];

    // ---- sort by (box, species, key) and the one reordering
    ctx.stage("build: sort");
    if (!n) mark(1);
    mark(2);
    if (n) {
        uint64_t* ktmp = static_cast<uint64_t*>(ctx.alloc(n * sizeof(uint64_t)));
        uint32_t* vtmp = static_cast<uint32_t*>(ctx.alloc(n * sizeof(uint32_t)));
        uint64_t* keys0 = nullptr;
        if (nbox > 1) {
            keys0 = static_cast<uint64_t*>(ctx.alloc(n * sizeof(uint64_t)));
            HIP_CHECK(hipMemcpyAsync(keys0, t.keys, n * sizeof(uint64_t), hipMemcpyDeviceToDevice, ctx.stream));
        }
        radix_sort_pairs(ctx, t.keys, t.perm, ktmp, vtmp, n, 64);
        if (nbox > 1) {
            // stable by box last: within a box the key order (ties in input order) stays
            uint64_t* kb = static_cast<uint64_t*>(ctx.alloc(n * sizeof(uint64_t)));
            hipLaunchKernelGGL(box_keys, dim3(blocks_for(n, 256)), dim3(256), 0, ctx.stream, n, t.perm, boxid, kb);
            LAUNCH_CHECK("box_keys");
            const int bits = nbox <= 256 ? 8 : 16;
            radix_sort_pairs(ctx, kb, t.perm, ktmp, vtmp, n, bits);
            hipLaunchKernelGGL(gather_keys, dim3(blocks_for(n, 256)), dim3(256), 0, ctx.stream, n, t.perm, keys0, t.keys);
            LAUNCH_CHECK("gather_keys");
            ctx.release(kb);
            ctx.release(keys0);
        }
        hipLaunchKernelGGL(gather_particles, dim3(blocks_for(n, 256)), dim3(256), 0, ctx.stream, n, t.perm, rin, t.X,
                           t.mass, t.P);
        LAUNCH_CHECK("gather_particles");
        ctx.release(ktmp);
        ctx.release(vtmp);
        ctx.release(rin);
        ctx.release(boxid);
    }

    // ---- breadth-first octree over all boxes, level by level
    mark(3);
    ctx.stage("build: octree");
    t.nn = 0;
    t.cap = 0;
    grow_nodes(ctx, t, std::max<uint64_t>(1024 + nbox, n / 2 + nbox + 1));
    uint32_t* leaf_dev = static_cast<uint32_t*>(ctx.alloc(nbox * sizeof(uint32_t)));
    ctx.to_device(leaf_dev, t.bleaf.data(), nbox * sizeof(uint32_t));
    {
        uint64_t* bseg_dev = static_cast<uint64_t*>(ctx.alloc(t.bseg.size() * sizeof(uint64_t)));
        ctx.to_device(bseg_dev, t.bseg.data(), t.bseg.size() * sizeof(uint64_t));
        hipLaunchKernelGGL(init_roots, dim3(blocks_for(nbox, 64)), dim3(64), 0, ctx.stream, nbox, D, bseg_dev, t.level,
                           t.prefix, t.parent, t.first_child, t.n_child, t.cell, t.start, t.count, t.node_box);
        LAUNCH_CHECK("init_roots");
        ctx.release(bseg_dev);
    }
    t.nn = nbox;
    t.level_start.assign(1, 0);
    t.level_start.push_back(nbox);
    unsigned long long* leaves = static_cast<unsigned long long*>(ctx.alloc(2 * sizeof(unsigned long long)));
    uint32_t* total_dev = reinterpret_cast<uint32_t*>(leaves + 1);
    HIP_CHECK(hipMemsetAsync(leaves, 0, 2 * sizeof(unsigned long long), ctx.stream));
    uint32_t depth = 0;
    bool wave_split = true;   // the top levels, down to the first one of many nodes
    for (uint32_t lvl = 0; lvl <= (uint32_t)kLevels; ++lvl) {
        uint64_t lb = t.level_start[lvl], nl = t.level_start[lvl + 1] - lb;
        if (nl == 0) break;
        depth = lvl;
        uint64_t slots = nl * 8;
        uint32_t* fl = static_cast<uint32_t*>(ctx.alloc(slots * sizeof(uint32_t) * 2));
        uint32_t* offs = fl + slots;
        uint32_t* cst = static_cast<uint32_t*>(ctx.alloc(slots * D * sizeof(uint32_t) * 2));
        uint32_t* ccn = cst + slots * D;
        wave_split = wave_split && nl <= kWaveSplitNodes;
        if (wave_split) {
            hipLaunchKernelGGL(split_level_wave, dim3(blocks_for(nl * 64, 256)), dim3(256), 0, ctx.stream, lb, nl, lvl, D,
                               leaf_dev, t.node_box, t.keys, t.prefix, t.start, t.count, cst, ccn, fl);
            LAUNCH_CHECK("split_level_wave");
        } else {
            hipLaunchKernelGGL(split_level, dim3(blocks_for(slots, 256)), dim3(256), 0, ctx.stream, lb, nl, lvl, D,
                               leaf_dev, t.node_box, t.keys, t.prefix, t.start, t.count, cst, ccn, fl);
            LAUNCH_CHECK("split_level");
        }
        scan_exclusive(ctx, fl, offs, slots, total_dev);
        uint64_t next_word = 0;
        ctx.read_words(&next_word, total_dev, 1);
        const uint32_t next = (uint32_t)(next_word & 0xffffffffu);
        uint64_t nb = t.level_start[lvl + 1];
        grow_nodes(ctx, t, nb + next);
        hipLaunchKernelGGL(emit_children, dim3(blocks_for(slots, 256)), dim3(256), 0, ctx.stream, lb, nl, nb, lvl, D, fl,
                           offs, cst, ccn, t.level, t.prefix, t.parent, t.first_child, t.n_child, t.cell, t.start,
                           t.count, t.node_box, t.P);
        LAUNCH_CHECK("emit_children");
        ctx.release(fl);
        ctx.release(cst);
        t.nn = nb + next;
        t.level_start.push_back(nb + next);
    }
    t.depth = depth;
    hipLaunchKernelGGL(count_leaves, dim3((unsigned)std::min<uint64_t>(blocks_for(t.nn, 256), 4u * ctx.num_cu)), dim3(256),
                       0, ctx.stream, t.nn, t.n_child, leaves);
    LAUNCH_CHECK("count_leaves");
    mark(4);
    ctx.stage("build: done");
    uint64_t nleaves = 0;
    ctx.read_words(&nleaves, leaves, 1);
    if (timed) {
        t.ms_ingest = ctx.elapsed(0, 1);
        t.ms_sort = ctx.elapsed(2, 3);
        t.ms_octree = ctx.elapsed(3, 4);
    }
    ctx.release(leaves);
    ctx.release(leaf_dev);
    t.n_leaves = nleaves;
}

void box_node_counts(Context& ctx, const Tree& t, std::vector<uint64_t>& nodes, std::vector<uint64_t>& leaves,
                     std::vector<uint32_t>& depth)
{
    const uint32_t nbox = t.nbox;
    nodes.assign(nbox, 0);
    leaves.assign(nbox, 0);
    depth.assign(nbox, 0);
    unsigned char* buf = static_cast<unsigned char*>(ctx.alloc(nbox * (2 * sizeof(uint64_t) + sizeof(uint32_t))));
    unsigned long long* nd = reinterpret_cast<unsigned long long*>(buf);
    unsigned long long* lf = nd + nbox;
    uint32_t* dp = reinterpret_cast<uint32_t*>(lf + nbox);
    HIP_CHECK(hipMemsetAsync(buf, 0, nbox * (2 * sizeof(uint64_t) + sizeof(uint32_t)), ctx.stream));
    if (t.nn) {
        hipLaunchKernelGGL(node_counts, dim3(blocks_for(t.nn, 256)), dim3(256), 0, ctx.stream, t.nn, t.node_box, t.n_child,
                           t.level, nd, lf, dp);
        LAUNCH_CHECK("node_counts");
    }
    ctx.to_host(nodes.data(), nd, nbox * sizeof(uint64_t));
    ctx.to_host(leaves.data(), lf, nbox * sizeof(uint64_t));
    ctx.to_host(depth.data(), dp, nbox * sizeof(uint32_t));
    ctx.release(buf);
}

void compute_monopoles(Context& ctx, Tree& t)
{
    const uint32_t D = t.D;
    ctx.stage("monopoles");
    ctx.release(t.mono);
    t.mono = static_cast<double4*>(ctx.alloc(std::max<uint64_t>(t.nn * D, 1) * sizeof(double4)));
    for (int lvl = (int)t.depth; lvl >= 0; --lvl) {
        uint64_t lb = t.level_start[lvl], nl = t.level_start[lvl + 1] - lb;
        if (!nl) continue;
        hipLaunchKernelGGL(monopole_level, dim3(blocks_for(nl * D, 256)), dim3(256), 0, ctx.stream, lb, nl, D, t.nn,
                           t.cell, t.first_child, t.n_child, t.start, t.count, t.P, t.mono);
        LAUNCH_CHECK("monopole_level");
    }
    t.has_monopoles = true;
}

}  // namespace ngr
