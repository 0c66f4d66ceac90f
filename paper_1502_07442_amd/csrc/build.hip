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

enum : uint32_t { kBadSpecies = 1, kBadMass = 2, kBadPos = 4 };

// One thread per particle: flags bad species ids, masses and positions, and
// counts each species (the counts give the species segments of the sort).
__global__ void check_inputs(uint64_t n, uint32_t D, const uint8_t* __restrict__ species,
                             const double* __restrict__ mass, const double* __restrict__ pos,
                             uint32_t* __restrict__ flags, unsigned long long* __restrict__ counts)
{
    // grid-stride over a bounded grid: one global atomic per workgroup and
    // species (same-address atomics from the whole chip are slow)
    __shared__ unsigned int local[NGR_MAX_SPECIES];
    __shared__ unsigned int local_bad;
    if (threadIdx.x < NGR_MAX_SPECIES) local[threadIdx.x] = 0;
    if (threadIdx.x == 0) local_bad = 0;
    __syncthreads();
    uint32_t bad = 0;
    uint32_t mine[NGR_MAX_SPECIES] = {0, 0, 0, 0, 0, 0};
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint32_t s = species[i];
        const double m = mass[i];
        if (s >= D) bad |= kBadSpecies;
#pragma unroll
        for (uint32_t b = 0; b < NGR_MAX_SPECIES; ++b) mine[b] += s == b ? 1u : 0u;
        if (!(m >= 0.0) || !isfinite(m)) bad |= kBadMass;
        if (pos && !(isfinite(pos[i]) && isfinite(pos[n + i]) && isfinite(pos[2 * n + i]))) bad |= kBadPos;
    }
    for (uint32_t b = 0; b < D; ++b)
        if (mine[b]) atomicAdd(&local[b], mine[b]);
    if (bad) atomicOr(&local_bad, bad);
    __syncthreads();
    if (threadIdx.x < D && local[threadIdx.x]) atomicAdd(&counts[threadIdx.x], (unsigned long long)local[threadIdx.x]);
    if (threadIdx.x == 0 && local_bad) atomicOr(flags, local_bad);
}

// Positions to 64-bit lattice coordinates, X = floor(u * 2^64) with
// u = x / box taken modulo 1 (the box is periodic).
__global__ void to_lattice(uint64_t n3, const double* __restrict__ x, double box, uint64_t* __restrict__ X)
{
    uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n3) return;
    double u = x[k] / box;
    u = u - floor(u);
    if (u >= 1.0) u = 0.0;
    X[k] = (uint64_t)(u * 18446744073709551616.0);
}

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

// Key = species << 60 | Morton interleave of the top 20 bits of each axis,
// x the most significant bit of each 3-bit digit; value = input index.
__global__ void make_keys(uint64_t n, const uint64_t* __restrict__ X, const uint8_t* __restrict__ species,
                          uint64_t* __restrict__ keys, uint32_t* __restrict__ idx)
{
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint64_t m = (spread3(X[i] >> 44) << 2) | (spread3(X[n + i] >> 44) << 1) | spread3(X[2 * n + i] >> 44);
    keys[i] = ((uint64_t)species[i] << kKeyBits) | m;
    idx[i] = (uint32_t)i;
}

// The single reordering of the particle data into sorted order.
__global__ void gather_particles(uint64_t n, const uint32_t* __restrict__ perm, const uint64_t* __restrict__ Xin,
                                 const double* __restrict__ min, uint64_t* __restrict__ Xout,
                                 double* __restrict__ mout)
{
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t p = perm[i];
    Xout[i] = Xin[p];
    Xout[n + i] = Xin[n + p];
    Xout[2 * n + i] = Xin[2 * n + p];
    mout[i] = min[p];
}

__global__ void init_root(uint32_t D, const uint64_t* __restrict__ seg_dev, uint8_t* level, uint64_t* prefix,
                          int32_t* parent, int32_t* first_child, uint8_t* n_child, uint4* cell,
                          uint32_t* start, uint32_t* count)
{
    if (threadIdx.x != 0) return;
    level[0] = 0;
    prefix[0] = 0;
    parent[0] = -1;
    first_child[0] = -1;
    n_child[0] = 0;
    cell[0] = make_uint4(0, 0, 0, 0);
    for (uint32_t b = 0; b < D; ++b) {
        start[b] = (uint32_t)seg_dev[b];
        count[b] = (uint32_t)(seg_dev[b + 1] - seg_dev[b]);
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

// One thread per (node of this level, octant): the octant's particles of each
// species are found by binary search inside the node's species range (the
// range is sorted by key). Nodes holding more than B particles below level 20
// split; a non-empty octant becomes a child.
__global__ void split_level(uint64_t level_begin, uint64_t n_level, uint32_t lvl, uint32_t D, uint32_t B,
                            const uint64_t* __restrict__ keys, const uint64_t* __restrict__ prefix,
                            const uint32_t* __restrict__ start, const uint32_t* __restrict__ count,
                            uint32_t* __restrict__ cstart, uint32_t* __restrict__ ccount,
                            uint32_t* __restrict__ flags)
{
    uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_level * 8) return;
    uint64_t p = level_begin + t / 8;
    uint32_t o = (uint32_t)(t % 8);
    uint64_t total = 0;
    for (uint32_t b = 0; b < D; ++b) total += count[p * D + b];
    if (total <= B || lvl >= (uint32_t)kLevels) {
        flags[t] = 0;
        return;
    }
    const uint32_t sh = kKeyBits - 3 * (lvl + 1);
    const uint64_t cp = prefix[p] * 8 + o;
    const uint64_t klo = cp << sh, khi = (cp + 1) << sh;
    uint64_t tot = 0;
    for (uint32_t b = 0; b < D; ++b) {
        uint64_t lo = start[p * D + b], hi = lo + count[p * D + b];
        uint64_t sb = (uint64_t)b << kKeyBits;
        uint64_t a0 = lower_bound(keys, lo, hi, sb + klo);
        uint64_t a1 = lower_bound(keys, a0, hi, sb + khi);
        cstart[t * D + b] = (uint32_t)a0;
        ccount[t * D + b] = (uint32_t)(a1 - a0);
        tot += a1 - a0;
    }
    flags[t] = tot > 0;
}

// Write the children found by split_level (in octant order, after all
// children of earlier nodes of the level) and the parents' child links.
__global__ void emit_children(uint64_t level_begin, uint64_t n_level, uint64_t next_begin, uint32_t lvl,
                              uint32_t D, const uint32_t* __restrict__ flags, const uint32_t* __restrict__ offs,
                              const uint32_t* __restrict__ cstart, const uint32_t* __restrict__ ccount,
                              uint8_t* level, uint64_t* prefix, int32_t* parent, int32_t* first_child,
                              uint8_t* n_child, uint4* cell, uint32_t* start, uint32_t* count)
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
    first_child[c] = -1;
    n_child[c] = 0;
    uint4 pc = cell[p];
    uint32_t half = 1u << (kLevels - lvl - 1);
    cell[c] = make_uint4(pc.x + ((o >> 2) & 1u) * half, pc.y + ((o >> 1) & 1u) * half, pc.z + (o & 1u) * half,
                         lvl + 1);
    for (uint32_t b = 0; b < D; ++b) {
        start[c * D + b] = cstart[t * D + b];
        count[c * D + b] = ccount[t * D + b];
    }
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

// Monopoles of one level (section 2.2), one thread per (node, species b).
// A leaf sums its species-b particles directly, relative to the cell corner
// so that the differences are exact integers; an internal node combines the
// monopoles of its children. Centres are kept as fractions of the box.
__global__ void monopole_level(uint64_t level_begin, uint64_t n_level, uint32_t D, uint64_t nn, uint64_t n,
                               const uint4* __restrict__ cell, const int32_t* __restrict__ first_child,
                               const uint8_t* __restrict__ n_child, const uint32_t* __restrict__ start,
                               const uint32_t* __restrict__ count, const uint64_t* __restrict__ X,
                               const double* __restrict__ mass, double4* __restrict__ mono)
{
    uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_level * D) return;
    uint64_t i = level_begin + t / D;
    uint32_t b = (uint32_t)(t % D);
    double M = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
    double4 out;
    if (n_child[i] == 0) {
        uint4 c = cell[i];
        uint64_t cx = (uint64_t)c.x << 44, cy = (uint64_t)c.y << 44, cz = (uint64_t)c.z << 44;
        uint64_t j0 = start[i * D + b], j1 = j0 + count[i * D + b];
        for (uint64_t j = j0; j < j1; ++j) {
            double m = mass[j];
            M += m;
            sx += m * (double)(X[j] - cx);
            sy += m * (double)(X[n + j] - cy);
            sz += m * (double)(X[2 * n + j] - cz);
        }
        const double s64 = 0x1p-64;
        out = M > 0.0 ? make_double4(((double)cx + sx / M) * s64, ((double)cy + sy / M) * s64,
                                     ((double)cz + sz / M) * s64, M)
                      : make_double4(0.0, 0.0, 0.0, 0.0);
    } else {
        uint64_t c0 = (uint64_t)first_child[i], c1 = c0 + n_child[i];
        for (uint64_t c = c0; c < c1; ++c) {
            double4 r = mono[b * nn + c];
            if (r.w > 0.0) {
                M += r.w;
                sx += r.w * r.x;
                sy += r.w * r.y;
                sz += r.w * r.z;
            }
        }
        out = M > 0.0 ? make_double4(sx / M, sy / M, sz / M, M) : make_double4(0.0, 0.0, 0.0, 0.0);
    }
    mono[b * nn + i] = out;
}

inline unsigned blocks_for(uint64_t work, unsigned threads) { return (unsigned)((work + threads - 1) / threads); }

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
    t.cap = cap;
}

}  // namespace

void build_tree(Context& ctx, const ngr_particles& p, uint32_t leaf_size, Tree& t)
{
    const uint64_t n = p.n;
    const uint32_t D = p.D;
    t.n = n;
    t.D = D;
    t.box = p.box;
    t.leaf_size = leaf_size;

    // ---- input checks and species counts (the one synchronisation before the build)
    ctx.stage("build: input checks");
    uint32_t* flags = static_cast<uint32_t*>(ctx.alloc((1 + NGR_MAX_SPECIES) * sizeof(uint64_t)));
    unsigned long long* counts = reinterpret_cast<unsigned long long*>(flags + 2);
    HIP_CHECK(hipMemsetAsync(flags, 0, (1 + NGR_MAX_SPECIES) * sizeof(uint64_t), ctx.stream));
    if (n) {
        hipLaunchKernelGGL(check_inputs, dim3((unsigned)std::min<uint64_t>(blocks_for(n, 256), 4u * ctx.num_cu)), dim3(256), 0,
                           ctx.stream, n, D, p.species, p.mass, p.pos, flags, counts);
        LAUNCH_CHECK("check_inputs");
    }
    uint64_t host[1 + NGR_MAX_SPECIES];
    ctx.read_words(host, flags, 1 + NGR_MAX_SPECIES);
    ctx.release(flags);
    uint32_t bad = (uint32_t)(host[0] & 0xffffffffu);
    if (bad & kBadSpecies) fail(NGR_EINVAL, "a species id is >= D");
    if (bad & kBadMass) fail(NGR_EINVAL, "a mass is negative or not finite");
    if (bad & kBadPos) fail(NGR_EINVAL, "a position is not finite");
    t.seg[0] = 0;
    for (uint32_t b = 0; b < D; ++b) t.seg[b + 1] = t.seg[b] + host[1 + b];
    for (uint32_t b = D; b < NGR_MAX_SPECIES; ++b) t.seg[b + 1] = t.seg[D];

    // ---- lattice, keys, sort, gather
    ctx.stage("build: keys and sort");
    t.X = static_cast<uint64_t*>(ctx.alloc(3 * std::max<uint64_t>(n, 1) * sizeof(uint64_t)));
    t.mass = static_cast<double*>(ctx.alloc(std::max<uint64_t>(n, 1) * sizeof(double)));
    t.perm = static_cast<uint32_t*>(ctx.alloc(std::max<uint64_t>(n, 1) * sizeof(uint32_t)));
    t.keys = static_cast<uint64_t*>(ctx.alloc(std::max<uint64_t>(n, 1) * sizeof(uint64_t)));
    if (n) {
        uint64_t* Xin = static_cast<uint64_t*>(ctx.alloc(3 * n * sizeof(uint64_t)));
        if (p.pos) {
            hipLaunchKernelGGL(to_lattice, dim3(blocks_for(3 * n, 256)), dim3(256), 0, ctx.stream, 3 * n, p.pos, p.box, Xin);
            LAUNCH_CHECK("to_lattice");
        } else {
            HIP_CHECK(hipMemcpyAsync(Xin, p.lattice, 3 * n * sizeof(uint64_t), hipMemcpyDeviceToDevice, ctx.stream));
        }
        uint64_t* ktmp = static_cast<uint64_t*>(ctx.alloc(n * sizeof(uint64_t)));
        uint32_t* vtmp = static_cast<uint32_t*>(ctx.alloc(n * sizeof(uint32_t)));
        hipLaunchKernelGGL(make_keys, dim3(blocks_for(n, 256)), dim3(256), 0, ctx.stream, n, Xin, p.species, t.keys, t.perm);
        LAUNCH_CHECK("make_keys");
        radix_sort_pairs(ctx, t.keys, t.perm, ktmp, vtmp, n, 64);
        hipLaunchKernelGGL(gather_particles, dim3(blocks_for(n, 256)), dim3(256), 0, ctx.stream, n, t.perm, Xin, p.mass, t.X, t.mass);
        LAUNCH_CHECK("gather_particles");
        ctx.release(ktmp);
        ctx.release(vtmp);
        ctx.release(Xin);
    }

    // ---- breadth-first octree
    ctx.stage("build: octree");
    t.nn = 0;
    t.cap = 0;
    grow_nodes(ctx, t, std::max<uint64_t>(1024, n / 2 + 1));
    {
        uint64_t* seg_dev = static_cast<uint64_t*>(ctx.alloc((NGR_MAX_SPECIES + 1) * sizeof(uint64_t)));
        ctx.write_words(seg_dev, t.seg, NGR_MAX_SPECIES + 1);
        hipLaunchKernelGGL(init_root, dim3(1), dim3(64), 0, ctx.stream, D, seg_dev, t.level, t.prefix, t.parent, t.first_child, t.n_child,
                                          t.cell, t.start, t.count);
        LAUNCH_CHECK("init_root");
        ctx.release(seg_dev);
    }
    t.nn = 1;
    t.level_start.assign(1, 0);
    t.level_start.push_back(1);
    unsigned long long* leaves = static_cast<unsigned long long*>(ctx.alloc(2 * sizeof(unsigned long long)));
    uint32_t* total_dev = reinterpret_cast<uint32_t*>(leaves + 1);
    HIP_CHECK(hipMemsetAsync(leaves, 0, 2 * sizeof(unsigned long long), ctx.stream));
    uint32_t depth = 0;
    for (uint32_t lvl = 0; lvl <= (uint32_t)kLevels; ++lvl) {
        uint64_t lb = t.level_start[lvl], nl = t.level_start[lvl + 1] - lb;
        if (nl == 0) break;
        depth = lvl;
        uint64_t slots = nl * 8;
        uint32_t* fl = static_cast<uint32_t*>(ctx.alloc(slots * sizeof(uint32_t) * 2));
        uint32_t* offs = fl + slots;
        uint32_t* cst = static_cast<uint32_t*>(ctx.alloc(slots * D * sizeof(uint32_t) * 2));
        uint32_t* ccn = cst + slots * D;
        hipLaunchKernelGGL(split_level, dim3(blocks_for(slots, 256)), dim3(256), 0, ctx.stream, lb, nl, lvl, D, leaf_size, t.keys, t.prefix,
                                                                    t.start, t.count, cst, ccn, fl);
        LAUNCH_CHECK("split_level");
        scan_exclusive(ctx, fl, offs, slots, total_dev);
        uint64_t next_word = 0;
        ctx.read_words(&next_word, total_dev, 1);
        const uint32_t next = (uint32_t)(next_word & 0xffffffffu);
        uint64_t nb = t.level_start[lvl + 1];
        grow_nodes(ctx, t, nb + next);
        hipLaunchKernelGGL(emit_children, dim3(blocks_for(slots, 256)), dim3(256), 0, ctx.stream, lb, nl, nb, lvl, D, fl, offs, cst, ccn, t.level, t.prefix, t.parent, t.first_child, t.n_child,
            t.cell, t.start, t.count);
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
    ctx.stage("build: done");
    uint64_t nleaves = 0;
    ctx.read_words(&nleaves, leaves, 1);
    ctx.release(leaves);
    t.n_leaves = nleaves;
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
        hipLaunchKernelGGL(monopole_level, dim3(blocks_for(nl * D, 256)), dim3(256), 0, ctx.stream, lb, nl, D, t.nn, t.n, t.cell,
                                                                         t.first_child, t.n_child, t.start,
                                                                         t.count, t.X, t.mass, t.mono);
        LAUNCH_CHECK("monopole_level");
    }
    t.has_monopoles = true;
}

}  // namespace ngr
