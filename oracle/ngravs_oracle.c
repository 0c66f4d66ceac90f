/*
 * FP64 CPU oracle for the periodic short-range multi-species tree force.
 *
 * TEST INFRASTRUCTURE ONLY (see ngravs_oracle.h): plain, slow, obviously
 * correct. Each function names the part of the paper it follows:
 * K. A. S. Croker, "ngravs: Distinct gravitational interactions in GADGET-2"
 * (Computer Physics Communications).
 *
 * Readings taken where the paper is silent are listed next to the code that
 * takes them; the library under test implements the same readings.
 */
#include "ngravs_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>

#define ORC_PI 3.14159265358979323846
#endif

#define KEY_BITS 60u
#define KEY_MASK ((1ull << KEY_BITS) - 1ull)
#define TWO_M64 0x1p-64

struct orc_tree {
    uint64_t n;
    uint32_t D, B;
    uint32_t key_order;   /* ORC_KEY_MORTON or ORC_KEY_HILBERT */
    double box;
    /* particle data in sorted order */
    uint32_t* perm;       /* sorted position -> input index */
    uint64_t* K;          /* full keys (species << 60 | morton) */
    uint64_t* X[3];
    uint8_t* s;
    double* m;
    uint64_t seg[ORC_MAX_SPECIES + 1];
    /* nodes, breadth first */
    uint64_t nn, cap;
    uint8_t* level;
    uint64_t* prefix;
    int32_t* parent;
    int32_t* first_child;
    uint8_t* n_child;
    uint32_t* start[ORC_MAX_SPECIES];
    uint32_t* count[ORC_MAX_SPECIES];
    /* monopoles */
    double* M[ORC_MAX_SPECIES];
    double* com[ORC_MAX_SPECIES][3];
    /* groups */
    uint64_t ng, gcap;
    uint8_t* gs;
    uint32_t* gstart;
    uint32_t* gcount;
    uint32_t* glo[3];
    uint32_t* ghi[3];
};

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------- lattice --
 * Positions become 64-bit lattice coordinates so that the periodic wrap of a
 * difference is exact integer arithmetic: X = floor(u * 2^64) with u = x/box
 * taken modulo 1 (the box is periodic, section 2.4.1 TreePM mode). */
void orc_lattice(uint64_t n, const double* x, double box, uint64_t* X)
{
    for (uint64_t k = 0; k < 3 * n; ++k) {
        double u = x[k] / box;
        u = u - floor(u);
        if (u >= 1.0) u = 0.0;
        X[k] = (uint64_t)(u * 18446744073709551616.0);
    }
}

/* ---------------------------------------------------------------- keys --
 * Spatial keys (section 2.4: particles are sorted by gravitational type and
 * then along a space-filling curve). Reading: a Morton curve on the top 20
 * bits of each axis, x the most significant bit of every 3-bit digit. */
uint64_t orc_morton(uint32_t kx, uint32_t ky, uint32_t kz)
{
    uint64_t m = 0;
    for (unsigned b = 0; b < ORC_LEVELS; ++b) {
        m |= (uint64_t)((kx >> b) & 1u) << (3 * b + 2);
        m |= (uint64_t)((ky >> b) & 1u) << (3 * b + 1);
        m |= (uint64_t)((kz >> b) & 1u) << (3 * b);
    }
    return m;
}

/*
 * The Peano-Hilbert curve the paper's code sorts by (section 2.4), on the
 * same 20-bit lattice, by the transpose method of J. Skilling, "Programming
 * the Hilbert curve" (AIP Conf. Proc. 707, 2004). The three coordinates are
 * turned into the curve's transposed form (bit j of component i is bit
 * 3j + 2 - i of the index) by undoing, from the top bit down, the reflections
 * and axis exchanges of each sub-cube and then Gray-coding; the index is the
 * interleave of the transposed components, x's component the most
 * significant of every 3-bit digit (as in the Morton layout). Every aligned
 * cube of side 2^(20-l) is one contiguous index range of 3(20-l) low bits.
 */
static void hilbert_axes_to_transpose(uint32_t x[3])
{
    const uint32_t top = 1u << (ORC_LEVELS - 1);
    for (uint32_t q = top; q > 1; q >>= 1) {
        const uint32_t low = q - 1;
        for (unsigned i = 0; i < 3; ++i) {
            if (x[i] & q) {
                x[0] ^= low;                        /* reflect the low bits of x */
            } else {
                const uint32_t t = (x[0] ^ x[i]) & low;   /* exchange the low bits of x and axis i */
                x[0] ^= t;
                x[i] ^= t;
            }
        }
    }
    x[1] ^= x[0];                                   /* Gray code */
    x[2] ^= x[1];
    uint32_t t = 0;
    for (uint32_t q = top; q > 1; q >>= 1)
        if (x[2] & q) t ^= q - 1;
    for (unsigned i = 0; i < 3; ++i) x[i] ^= t;
}

static void hilbert_transpose_to_axes(uint32_t x[3])
{
    const uint32_t t0 = x[2] >> 1;                  /* Gray decode */
    x[2] ^= x[1];
    x[1] ^= x[0];
    x[0] ^= t0;
    for (uint32_t q = 2; q != (1u << ORC_LEVELS); q <<= 1) {   /* redo the exchanges and reflections */
        const uint32_t low = q - 1;
        for (int i = 2; i >= 0; --i) {
            if (x[i] & q) {
                x[0] ^= low;
            } else {
                const uint32_t t = (x[0] ^ x[i]) & low;
                x[0] ^= t;
                x[i] ^= t;
            }
        }
    }
}

uint64_t orc_hilbert(uint32_t kx, uint32_t ky, uint32_t kz)
{
    uint32_t x[3] = {kx, ky, kz};
    hilbert_axes_to_transpose(x);
    uint64_t h = 0;
    for (unsigned b = 0; b < ORC_LEVELS; ++b)
        for (unsigned i = 0; i < 3; ++i)
            h |= (uint64_t)((x[i] >> b) & 1u) << (3 * b + 2 - i);
    return h;
}

void orc_hilbert_decode(uint64_t h, uint32_t k[3])
{
    uint32_t x[3] = {0, 0, 0};
    for (unsigned b = 0; b < ORC_LEVELS; ++b)
        for (unsigned i = 0; i < 3; ++i)
            x[i] |= (uint32_t)((h >> (3 * b + 2 - i)) & 1u) << b;
    hilbert_transpose_to_axes(x);
    for (unsigned i = 0; i < 3; ++i) k[i] = x[i];
}

void orc_keys_order(uint64_t n, const uint64_t* X, const uint8_t* species, uint32_t key_order, uint64_t* K)
{
    for (uint64_t i = 0; i < n; ++i) {
        uint32_t kx = (uint32_t)(X[i] >> 44);
        uint32_t ky = (uint32_t)(X[n + i] >> 44);
        uint32_t kz = (uint32_t)(X[2 * n + i] >> 44);
        uint64_t c = key_order == ORC_KEY_HILBERT ? orc_hilbert(kx, ky, kz) : orc_morton(kx, ky, kz);
        K[i] = ((uint64_t)species[i] << KEY_BITS) | c;
    }
}

void orc_keys(uint64_t n, const uint64_t* X, const uint8_t* species, uint64_t* K)
{
    orc_keys_order(n, X, species, ORC_KEY_MORTON, K);
}

/* ---------------------------------------------------------------- sort --
 * One stable sort by (species, key), so that particle data are grouped by
 * type and each type is in curve order (section 2.4). Ties keep input order. */
static const uint64_t* g_sort_keys;
static int cmp_key_index(const void* a, const void* b)
{
    uint32_t i = *(const uint32_t*)a, j = *(const uint32_t*)b;
    if (g_sort_keys[i] < g_sort_keys[j]) return -1;
    if (g_sort_keys[i] > g_sort_keys[j]) return 1;
    return (i > j) - (i < j);
}

void orc_sort(uint64_t n, const uint64_t* K, uint32_t* perm)
{
    for (uint64_t i = 0; i < n; ++i) perm[i] = (uint32_t)i;
    g_sort_keys = K;
    qsort(perm, n, sizeof(uint32_t), cmp_key_index);
}

/* ---------------------------------------------------------------- tree -- */
static uint32_t deinterleave(uint64_t prefix, unsigned level, unsigned axis_shift)
{
    /* axis_shift: 2 for x, 1 for y, 0 for z */
    uint32_t c = 0;
    for (unsigned d = 0; d < level; ++d)
        c |= (uint32_t)((prefix >> (3 * d + axis_shift)) & 1u) << d;
    return c;
}

/* Cell of a node in 20-bit key units: [c, c + 2^(20-level)) per axis. With
 * the Hilbert order the prefix is decoded (the point at the start of the
 * node's index range lies in its cell) and cut to the level. */
static void node_cell(const orc_tree* t, uint64_t i, uint32_t c[3], uint32_t* S)
{
    unsigned l = t->level[i];
    if (t->key_order == ORC_KEY_HILBERT) {
        uint32_t k[3];
        orc_hilbert_decode(l ? t->prefix[i] << (KEY_BITS - 3 * l) : 0u, k);
        for (unsigned a = 0; a < 3; ++a) c[a] = l ? (k[a] >> (ORC_LEVELS - l)) << (ORC_LEVELS - l) : 0u;
    } else {
        for (unsigned a = 0; a < 3; ++a)
            c[a] = l ? deinterleave(t->prefix[i], l, 2 - a) << (ORC_LEVELS - l) : 0u;
    }
    *S = 1u << (ORC_LEVELS - l);
}

static uint64_t lower_bound_key(const orc_tree* t, uint64_t lo, uint64_t hi, uint64_t key)
{
    /* first sorted index in [lo, hi) whose Morton part is >= key */
    while (lo < hi) {
        uint64_t mid = lo + (hi - lo) / 2;
        if ((t->K[mid] & KEY_MASK) < key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

static void grow_nodes(orc_tree* t)
{
    uint64_t c = t->cap ? 2 * t->cap : 1024;
    t->level = realloc(t->level, c * sizeof(uint8_t));
    t->prefix = realloc(t->prefix, c * sizeof(uint64_t));
    t->parent = realloc(t->parent, c * sizeof(int32_t));
    t->first_child = realloc(t->first_child, c * sizeof(int32_t));
    t->n_child = realloc(t->n_child, c * sizeof(uint8_t));
    for (uint32_t b = 0; b < t->D; ++b) {
        t->start[b] = realloc(t->start[b], c * sizeof(uint32_t));
        t->count[b] = realloc(t->count[b], c * sizeof(uint32_t));
    }
    t->cap = c;
}

/*
 * The octree (section 2: the volume is halved recursively until particles
 * sit in their own leaves; the tree holds every species, section 2.2).
 * Reading: a node is a leaf once it holds at most B particles of all species
 * together, or at the deepest key level (20). Children are the non-empty
 * octants. For every node and species b the node records where its
 * species-b particles start in sorted order and how many there are (N_perp,
 * section 2.2). Nodes are appended breadth first, which orders them by level
 * and then by prefix.
 */
orc_tree* orc_tree_build_order(uint64_t n, uint32_t D, double box, const uint64_t* X,
                               const uint8_t* species, const double* mass, uint32_t leaf_size,
                               uint32_t key_order)
{
    orc_tree* t = calloc(1, sizeof(orc_tree));
    t->n = n;
    t->D = D;
    t->B = leaf_size;
    t->key_order = key_order;
    t->box = box;
    uint64_t* Kin = malloc((n ? n : 1) * sizeof(uint64_t));
    orc_keys_order(n, X, species, key_order, Kin);
    t->perm = malloc((n ? n : 1) * sizeof(uint32_t));
    orc_sort(n, Kin, t->perm);
    t->K = malloc((n ? n : 1) * sizeof(uint64_t));
    for (unsigned a = 0; a < 3; ++a) t->X[a] = malloc((n ? n : 1) * sizeof(uint64_t));
    t->s = malloc((n ? n : 1));
    t->m = malloc((n ? n : 1) * sizeof(double));
    for (uint64_t i = 0; i < n; ++i) {
        uint32_t p = t->perm[i];
        t->K[i] = Kin[p];
        for (unsigned a = 0; a < 3; ++a) t->X[a][i] = X[a * n + p];
        t->s[i] = species[p];
        t->m[i] = mass[p];
    }
    free(Kin);
    for (uint32_t b = 0; b <= D; ++b) t->seg[b] = 0;
    for (uint64_t i = 0; i < n; ++i) t->seg[t->s[i] + 1]++;
    for (uint32_t b = 0; b < D; ++b) t->seg[b + 1] += t->seg[b];

    grow_nodes(t);
    t->nn = 1;
    t->level[0] = 0;
    t->prefix[0] = 0;
    t->parent[0] = -1;
    for (uint32_t b = 0; b < D; ++b) {
        t->start[b][0] = (uint32_t)t->seg[b];
        t->count[b][0] = (uint32_t)(t->seg[b + 1] - t->seg[b]);
    }
    for (uint64_t i = 0; i < t->nn; ++i) {
        uint64_t total = 0;
        for (uint32_t b = 0; b < D; ++b) total += t->count[b][i];
        unsigned l = t->level[i];
        t->first_child[i] = -1;
        t->n_child[i] = 0;
        if (total <= leaf_size || l == ORC_LEVELS) continue;
        unsigned sh = KEY_BITS - 3 * (l + 1);
        for (unsigned o = 0; o < 8; ++o) {
            uint64_t cp = t->prefix[i] * 8 + o;
            uint64_t klo = cp << sh, khi = (cp + 1) << sh;
            uint32_t cs[ORC_MAX_SPECIES], cc[ORC_MAX_SPECIES];
            uint64_t tot = 0;
            for (uint32_t b = 0; b < D; ++b) {
                uint64_t lo = t->start[b][i], hi = lo + t->count[b][i];
                uint64_t a0 = lower_bound_key(t, lo, hi, klo);
                uint64_t a1 = lower_bound_key(t, lo, hi, khi);
                cs[b] = (uint32_t)a0;
                cc[b] = (uint32_t)(a1 - a0);
                tot += cc[b];
            }
            if (!tot) continue;
            if (t->nn == t->cap) grow_nodes(t);
            uint64_t c = t->nn++;
            t->level[c] = (uint8_t)(l + 1);
            t->prefix[c] = cp;
            t->parent[c] = (int32_t)i;
            t->first_child[c] = -1;
            t->n_child[c] = 0;
            for (uint32_t b = 0; b < D; ++b) {
                t->start[b][c] = cs[b];
                t->count[b][c] = cc[b];
            }
            if (t->n_child[i] == 0) t->first_child[i] = (int32_t)c;
            t->n_child[i]++;
        }
    }
    return t;
}

orc_tree* orc_tree_build(uint64_t n, uint32_t D, double box, const uint64_t* X,
                         const uint8_t* species, const double* mass, uint32_t leaf_size)
{
    return orc_tree_build_order(n, D, box, X, species, mass, leaf_size, ORC_KEY_MORTON);
}

void orc_tree_free(orc_tree* t)
{
    if (!t) return;
    free(t->perm); free(t->K); free(t->s); free(t->m);
    for (unsigned a = 0; a < 3; ++a) { free(t->X[a]); free(t->glo[a]); free(t->ghi[a]); }
    free(t->level); free(t->prefix); free(t->parent); free(t->first_child); free(t->n_child);
    for (uint32_t b = 0; b < ORC_MAX_SPECIES; ++b) {
        free(t->start[b]); free(t->count[b]); free(t->M[b]);
        for (unsigned a = 0; a < 3; ++a) free(t->com[b][a]);
    }
    free(t->gs); free(t->gstart); free(t->gcount);
    free(t);
}

uint64_t orc_tree_n_nodes(const orc_tree* t) { return t->nn; }

void orc_tree_export(const orc_tree* t, uint32_t* perm, uint64_t* keys,
                     uint8_t* level, uint64_t* prefix, int32_t* parent,
                     int32_t* first_child, uint8_t* n_child,
                     uint32_t* start, uint32_t* count)
{
    uint64_t n = t->n, nn = t->nn;
    if (perm) memcpy(perm, t->perm, n * sizeof(uint32_t));
    if (keys) memcpy(keys, t->K, n * sizeof(uint64_t));
    if (level) memcpy(level, t->level, nn);
    if (prefix) memcpy(prefix, t->prefix, nn * sizeof(uint64_t));
    if (parent) memcpy(parent, t->parent, nn * sizeof(int32_t));
    if (first_child) memcpy(first_child, t->first_child, nn * sizeof(int32_t));
    if (n_child) memcpy(n_child, t->n_child, nn);
    for (uint32_t b = 0; b < t->D; ++b) {
        if (start) memcpy(start + b * nn, t->start[b], nn * sizeof(uint32_t));
        if (count) memcpy(count + b * nn, t->count[b], nn * sizeof(uint32_t));
    }
}

/* ----------------------------------------------------------- monopoles --
 * One monopole per species in every node (section 2.2: the walk vectorises
 * over each species' monopole mass and centre). Direct sums over the node's
 * particles of that species: M_b = sum m, and the centre of mass taken
 * relative to the cell corner so that the differences are exact integers. */
void orc_monopoles(orc_tree* t)
{
    uint64_t nn = t->nn;
    for (uint32_t b = 0; b < t->D; ++b) {
        free(t->M[b]);
        t->M[b] = malloc(nn * sizeof(double));
        for (unsigned a = 0; a < 3; ++a) {
            free(t->com[b][a]);
            t->com[b][a] = malloc(nn * sizeof(double));
        }
    }
    const double scale = t->box * TWO_M64;
    for (uint64_t i = 0; i < nn; ++i) {
        uint32_t c[3], S;
        node_cell(t, i, c, &S);
        uint64_t corner[3];
        for (unsigned a = 0; a < 3; ++a) corner[a] = (uint64_t)c[a] << 44;
        for (uint32_t b = 0; b < t->D; ++b) {
            double M = 0.0, off[3] = {0.0, 0.0, 0.0};
            uint64_t j0 = t->start[b][i], j1 = j0 + t->count[b][i];
            for (uint64_t j = j0; j < j1; ++j) {
                M += t->m[j];
                for (unsigned a = 0; a < 3; ++a)
                    off[a] += t->m[j] * (double)(t->X[a][j] - corner[a]);
            }
            t->M[b][i] = M;
            for (unsigned a = 0; a < 3; ++a)
                t->com[b][a][i] = M > 0.0 ? ((double)corner[a] + off[a] / M) * scale : 0.0;
        }
    }
}

void orc_monopoles_export(const orc_tree* t, double* M, double* com)
{
    uint64_t nn = t->nn;
    for (uint32_t b = 0; b < t->D; ++b) {
        if (M) memcpy(M + b * nn, t->M[b], nn * sizeof(double));
        if (com)
            for (unsigned a = 0; a < 3; ++a)
                memcpy(com + (b * 3 + a) * nn, t->com[b][a], nn * sizeof(double));
    }
}

/* -------------------------------------------------------------- groups --
 * Reading (the paper walks the tree once per particle): sinks share a walk
 * in species-pure groups of at most Ng particles, a group being one node's
 * species-a particles or a run of consecutive sibling nodes whose species-a
 * counts add up to at most Ng. A leaf with more than Ng particles of the
 * species is cut into consecutive chunks of Ng. The group's box is the
 * integer bounding box of its particles on the 20-bit key lattice. */
static void emit_group(orc_tree* t, uint8_t a, uint64_t start, uint64_t count)
{
    if (t->ng == t->gcap) {
        uint64_t c = t->gcap ? 2 * t->gcap : 256;
        t->gs = realloc(t->gs, c);
        t->gstart = realloc(t->gstart, c * sizeof(uint32_t));
        t->gcount = realloc(t->gcount, c * sizeof(uint32_t));
        for (unsigned ax = 0; ax < 3; ++ax) {
            t->glo[ax] = realloc(t->glo[ax], c * sizeof(uint32_t));
            t->ghi[ax] = realloc(t->ghi[ax], c * sizeof(uint32_t));
        }
        t->gcap = c;
    }
    uint64_t g = t->ng++;
    t->gs[g] = a;
    t->gstart[g] = (uint32_t)start;
    t->gcount[g] = (uint32_t)count;
    for (unsigned ax = 0; ax < 3; ++ax) {
        uint32_t lo = 0xffffffffu, hi = 0;
        for (uint64_t j = start; j < start + count; ++j) {
            uint32_t k = (uint32_t)(t->X[ax][j] >> 44);
            if (k < lo) lo = k;
            if (k + 1 > hi) hi = k + 1;
        }
        t->glo[ax][g] = lo;
        t->ghi[ax][g] = hi;
    }
}

static void group_visit(orc_tree* t, uint64_t i, uint8_t a, uint32_t Ng)
{
    if (t->n_child[i] == 0) {
        uint64_t s0 = t->start[a][i], c = t->count[a][i];
        for (uint64_t k = 0; k < c; k += Ng)
            emit_group(t, a, s0 + k, c - k < Ng ? c - k : Ng);
        return;
    }
    uint64_t run_start = 0, run_count = 0;
    for (uint64_t c = (uint64_t)t->first_child[i]; c < (uint64_t)t->first_child[i] + t->n_child[i]; ++c) {
        uint32_t na = t->count[a][c];
        if (na == 0) continue;
        if (na > Ng) {
            if (run_count) emit_group(t, a, run_start, run_count);
            run_count = 0;
            group_visit(t, c, a, Ng);
            continue;
        }
        if (run_count + na > Ng) {
            emit_group(t, a, run_start, run_count);
            run_count = 0;
        }
        if (run_count == 0) run_start = t->start[a][c];
        run_count += na;
    }
    if (run_count) emit_group(t, a, run_start, run_count);
}

uint64_t orc_groups(orc_tree* t, uint32_t group_size)
{
    t->ng = 0;
    for (uint32_t a = 0; a < t->D; ++a) {
        uint32_t na = t->count[a][0];
        if (na == 0) continue;
        if (na <= group_size) emit_group(t, (uint8_t)a, t->start[a][0], na);
        else group_visit(t, 0, (uint8_t)a, group_size);
    }
    return t->ng;
}

void orc_groups_export(const orc_tree* t, uint8_t* species, uint32_t* start,
                       uint32_t* count, uint32_t* lo, uint32_t* hi)
{
    uint64_t ng = t->ng;
    if (species) memcpy(species, t->gs, ng);
    if (start) memcpy(start, t->gstart, ng * sizeof(uint32_t));
    if (count) memcpy(count, t->gcount, ng * sizeof(uint32_t));
    for (unsigned a = 0; a < 3; ++a) {
        if (lo) memcpy(lo + a * ng, t->glo[a], ng * sizeof(uint32_t));
        if (hi) memcpy(hi + a * ng, t->ghi[a], ng * sizeof(uint32_t));
    }
}

/* ----------------------------------------------------------------- MAC --
 * Opening test (section 2: the walk stops where the monopole of the deeper
 * branches is accurate enough; section 2.4.1: in TreePM mode the walk is
 * restricted to short range). Reading: geometric Barnes-Hut on the exact
 * integer key lattice. d_min is the smallest periodic distance between the
 * node's cell and the group's box and d_max an upper bound on the largest.
 * The node is pruned when d_min >= r_cut. It is accepted as a monopole when
 * its side S < theta * d_min and d_max < r_cut, i.e. only when all of it
 * lies inside the cut-off sphere of every sink: a monopole of a node cut by
 * that sphere would count particles the short-range sum excludes. Otherwise
 * it is opened. Lengths are in half key units so every quantity is an exact
 * integer; R2 and theta2 are the squared cut-off (same units) and theta^2. */
int orc_mac(const orc_tree* t, uint64_t node, const uint32_t lo[3],
            const uint32_t hi[3], double R2, double theta2)
{
    uint32_t c[3], S;
    node_cell(t, node, c, &S);
    const int64_t half = 1ll << ORC_LEVELS;       /* half the period, half units */
    int64_t D2 = 0, D2max = 0;
    for (unsigned a = 0; a < 3; ++a) {
        int64_t w = (int64_t)hi[a] - (int64_t)lo[a];
        int64_t d = (2 * (int64_t)c[a] + (int64_t)S) - ((int64_t)lo[a] + (int64_t)hi[a]);
        d = ((d + half) % (2 * half) + 2 * half) % (2 * half) - half;
        int64_t ad = d < 0 ? -d : d;
        int64_t g = 0;
        if ((int64_t)S + w < half) {
            g = ad - ((int64_t)S + w);
            if (g < 0) g = 0;
        }
        int64_t gmax = ad + (int64_t)S + w;
        D2 += g * g;
        D2max += gmax * gmax;
    }
    if ((double)D2 >= R2) return ORC_PRUNE;
    double S4 = (double)(4 * (int64_t)S * (int64_t)S);
    if (S4 < theta2 * (double)D2 && (double)D2max < R2) return ORC_ACCEPT;
    return ORC_OPEN;
}

/*
 * The relative opening test (section 2.2: the walk keeps the stock code's
 * criterion, which compares the previously computed acceleration with a
 * Newtonian estimate of the node's contribution). Reading, per group: with
 * M the node's mass over all species, l its side and d_min as above, the
 * node is accepted when M l^2 / d_min^4 <= alpha a_min, a_min the smallest
 * previous |a| of the group's sinks, and when d_max < r_cut (the short-range
 * clause above); it is opened when the group's box reaches into the node's
 * cube grown to 1.2 times its side (the stock code's guard against accepting
 * a node that holds the sink), and pruned when d_min >= r_cut. In half key
 * units l = 2 S and lengths scale by u = box / 2^21, so the test is
 * M (4 S^2) <= (alpha u^2 a_min) D2^2, evaluated in float64 in that order;
 * rel_k = alpha u^2.
 */
int orc_mac_relative(const orc_tree* t, uint64_t node, const uint32_t lo[3],
                     const uint32_t hi[3], double R2, double rel_k, double a_min)
{
    uint32_t c[3], S;
    node_cell(t, node, c, &S);
    const int64_t half = 1ll << ORC_LEVELS;
    int64_t D2 = 0, D2max = 0;
    int inside = 1;
    for (unsigned a = 0; a < 3; ++a) {
        int64_t w = (int64_t)hi[a] - (int64_t)lo[a];
        int64_t d = (2 * (int64_t)c[a] + (int64_t)S) - ((int64_t)lo[a] + (int64_t)hi[a]);
        d = ((d + half) % (2 * half) + 2 * half) % (2 * half) - half;
        int64_t ad = d < 0 ? -d : d;
        int64_t g = 0;
        if ((int64_t)S + w < half) {
            g = ad - ((int64_t)S + w);
            if (g < 0) g = 0;
        }
        int64_t gmax = ad + (int64_t)S + w;
        D2 += g * g;
        D2max += gmax * gmax;
        /* group box within the grown cube on this axis: |d| < 1.2 S + w */
        if (!(5 * ad < 6 * (int64_t)S + 5 * w)) inside = 0;
    }
    if ((double)D2 >= R2) return ORC_PRUNE;
    if (inside) return ORC_OPEN;
    double M = 0.0;
    for (uint32_t b = 0; b < t->D; ++b) M += t->M[b][node];
    const double lhs = M * (double)(4 * (int64_t)S * (int64_t)S);
    const double rhs = (rel_k * a_min) * ((double)D2 * (double)D2);
    if (lhs <= rhs && (double)D2max < R2) return ORC_ACCEPT;
    return ORC_OPEN;
}

static void mac_constants(const orc_tree* t, const orc_law* law, double* R2, double* theta2)
{
    double q = law->r_cut / t->box * 2097152.0;   /* r_cut in half key units */
    *R2 = law->corr ? INFINITY : q * q;    /* with lattice corrections every pair interacts */
    *theta2 = law->theta * law->theta;
}

/* Depth-first walk from the root with children in octant order. */
typedef struct { uint64_t* e; uint64_t n, cap; } list_t;

static void list_push(list_t* L, uint64_t v)
{
    if (L->n == L->cap) {
        L->cap = L->cap ? 2 * L->cap : 1024;
        L->e = realloc(L->e, L->cap * sizeof(uint64_t));
    }
    L->e[L->n++] = v;
}

/* rel: 0 for the geometric test, else the relative one with rel_k, a_min */
typedef struct { int rel; double R2, theta2, rel_k, a_min; } mac_args;

static void walk(const orc_tree* t, uint64_t i, const uint32_t lo[3], const uint32_t hi[3],
                 const mac_args* m, list_t* L)
{
    int d = m->rel ? orc_mac_relative(t, i, lo, hi, m->R2, m->rel_k, m->a_min)
                   : orc_mac(t, i, lo, hi, m->R2, m->theta2);
    if (d == ORC_PRUNE) return;
    if (d == ORC_ACCEPT) { list_push(L, i | (1ull << 32)); return; }
    if (t->n_child[i] == 0) { list_push(L, i | (2ull << 32)); return; }
    for (uint64_t c = (uint64_t)t->first_child[i]; c < (uint64_t)t->first_child[i] + t->n_child[i]; ++c)
        walk(t, c, lo, hi, m, L);
}

static void group_list(const orc_tree* t, const orc_law* law, uint64_t g, list_t* L)
{
    mac_args m = {0, 0.0, 0.0, 0.0, 0.0};
    mac_constants(t, law, &m.R2, &m.theta2);
    if (law->opening == ORC_OPEN_RELATIVE) {
        const double u = t->box / 2097152.0;    /* one half key unit */
        m.rel = 1;
        m.rel_k = law->alpha * (u * u);
        m.a_min = INFINITY;
        for (uint64_t i = t->gstart[g]; i < t->gstart[g] + t->gcount[g]; ++i) {
            double a = law->old_acc[t->perm[i]];
            if (a < m.a_min) m.a_min = a;
        }
    }
    uint32_t lo[3], hi[3];
    for (unsigned a = 0; a < 3; ++a) { lo[a] = t->glo[a][g]; hi[a] = t->ghi[a][g]; }
    L->n = 0;
    walk(t, 0, lo, hi, &m, L);
}

uint64_t orc_group_list(const orc_tree* t, const orc_law* law, uint64_t g,
                        uint64_t* entries, uint64_t cap)
{
    list_t L = {0, 0, 0};
    group_list(t, law, g, &L);
    for (uint64_t k = 0; k < L.n && k < cap; ++k) entries[k] = L.e[k];
    uint64_t n = L.n;
    free(L.e);
    return n;
}

/* -------------------------------------------------------------- forces --
 * Tabulated short-range force factor (section 2.4.1: the factor is sampled
 * at N_TAB points before the run and applied during the walk). Reading: the
 * samples are uniform in r (grid R) or in r^2 (grid R2) on [0, r_cut] with
 * both ends included, and the value between samples is the straight line
 * through the two neighbours. */
double orc_factor(const double* T, uint32_t ntab, uint32_t grid, double r2, double r_cut)
{
    double t = grid == ORC_GRID_R ? sqrt(r2) * ((double)(ntab - 1) / r_cut)
                                  : r2 * ((double)(ntab - 1) / (r_cut * r_cut));
    if (t > (double)(ntab - 1)) t = (double)(ntab - 1);
    double kf = floor(t);
    if (kf > (double)(ntab - 2)) kf = (double)(ntab - 2);
    uint32_t k = (uint32_t)kf;
    double w = t - kf;
    return T[k] + w * (T[k + 1] - T[k]);
}

/*
 * The accumulator ("Mahalo") laws of section 3.3. A cored object of mass M
 * has the density of Eq. (15); two objects whose cores are M_1 and m_1 (0 for
 * a point-like one) have the mutual potential of Eq. (14),
 *     Phi(r) = -(2 M m / (pi r)) atan(r / s),  s = (M_1 + m_1) / (4 pi beta),
 * which is Newton's potential for s = 0. The acceleration of the passive
 * object is -(1/m) dPhi/dr toward the source:
 *     (2 M / pi) [atan(r/s) - r s / (r^2 + s^2)] / r^3  =  M * orc_cored_radial(r, s).
 * Readings: the printed core radius of Eq. (15), M / (2 beta pi), makes the
 * density integrate to M / 2; M / (4 beta pi) integrates to M and, since the
 * mutual potential of two such densities has the sum of their core radii as
 * its scale, reproduces the scale (M_1 + m_1) / (4 pi beta) of Eq. (14). In
 * Phi_10, Eq. (16) (cored sink, point-like sources) the source carries no core, so
 * its body count N_perp cannot enter the scale: s = m_1 / (4 pi beta) (the
 * printed form agrees for N_perp = 1). A monopole of N_perp bodies of a cored
 * species weighs M / N_perp per body (section 2.2's optional N_perp tracking);
 * without tracking it counts as one body of mass M.
 * For r / s below 1e-2 the bracket is taken from its series,
 *     atan x - x / (1 + x^2) = (2/3) x^3 - (4/5) x^5 + (6/7) x^7 - ...,
 * which avoids the cancellation of the two terms.
 */
double orc_cored_radial(double r, double s)
{
    if (!(s > 0.0)) return 1.0 / (r * r * r);
    const double x = r / s;
    double h;   /* [atan x - x / (1 + x^2)] / x^3 */
    if (x < 1e-2) {
        const double x2 = x * x;
        h = 2.0 / 3.0 - 0.8 * x2 + (6.0 / 7.0) * x2 * x2;
    } else {
        h = (atan(x) - x / (1.0 + x * x)) / (x * x * x);
    }
    return (2.0 / ORC_PI) * h / (s * s * s);
}

/*
 * One pair term (Eq. (1) with the active mass as a multiplier and the
 * passive mass divided out, section 2.1): the acceleration of a sink of
 * species a due to a source of species b and active mass mu at offset d
 * (source minus sink, minimum image) is
 *     G_ab * mu * f_ab(r) * d / (r^2 + eps^2)^(3/2)      for r < r_cut,
 * with the tabulated law; with the accumulator laws the Plummer factor of a
 * pair with a core (s > 0) is replaced by orc_cored_radial(r, s), where
 * s = (mu_body [b cored] + m_sink [a cored]) / (4 pi beta) and mu_body is
 * the mass of one source body.
 * Readings: a single Plummer softening; f evaluated at the unsoftened r;
 * G_ab * f > 0 attracts.
 * Pairs within 1e-6 r_cut^2 of the cut-off add their magnitude to the
 * sink's tie slack: a finite-precision evaluation may keep or drop them.
 */
typedef struct {
    const double* G; const double* tab; uint32_t ntab, grid, D;
    double rc, rc2, eps2, band;
    const double* eps_ab;      /* per-pair softening (section 2: D^2 softenings), or NULL */
    uint32_t kind, cored;
    double inv4pib;
    const double* corr;        /* lattice correction tables, or NULL */
    uint32_t corr_n;
    double corr_scale;         /* corr_n / (box / 2) */
} pair_ctx;

/*
 * Lattice correction (section 2.3: tabulated corrections from the infinite
 * image lattice, interpolated to the particle offsets as the stock code
 * does). A table T holds, on the grid d in [0, box/2]^3 of n intervals per
 * axis, the extra acceleration of a sink from all images of a unit source at
 * offset d other than the nearest; it is odd in each component's own axis
 * and even in the others, so the value at d is the trilinear interpolation
 * at |d| with each component's sign set by its axis.
 */
static void lattice_correction(const double* T, uint32_t n, double scale, const double d[3], double out[3])
{
    uint32_t i[3];
    double f[3];
    for (unsigned x = 0; x < 3; ++x) {
        double u = fabs(d[x]) * scale;
        uint32_t k = (uint32_t)u;
        if (k > n - 1) k = n - 1;
        i[x] = k;
        f[x] = u - (double)k;
        out[x] = 0.0;
    }
    const uint64_t m = n + 1;
    for (unsigned c = 0; c < 8; ++c) {
        unsigned cx = c >> 2, cy = (c >> 1) & 1, cz = c & 1;
        double w = (cx ? f[0] : 1.0 - f[0]) * (cy ? f[1] : 1.0 - f[1]) * (cz ? f[2] : 1.0 - f[2]);
        const double* e = T + (((uint64_t)(i[0] + cx) * m + (i[1] + cy)) * m + (i[2] + cz)) * 3;
        for (unsigned x = 0; x < 3; ++x) out[x] += w * e[x];
    }
    for (unsigned x = 0; x < 3; ++x)
        if (d[x] < 0.0) out[x] = -out[x];
}

static int pair_term(const pair_ctx* P, uint32_t a, uint32_t b, double mu, double mu_body,
                     double m_sink, const double d[3], double acc[3], double* slack)
{
    double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    if (r2 == 0.0) return 0;         /* coincident: no direction, no force */
    int inside = r2 < P->rc2;
    int tie = fabs(r2 - P->rc2) <= P->band;
    if (!inside && !tie) return 0;
    const double* T = P->tab + ((uint64_t)a * P->D + b) * P->ntab;
    double f = orc_factor(T, P->ntab, P->grid, r2, P->rc);
    double radial;
    double s = 0.0;
    if (P->kind == ORC_LAW_ACCUMULATOR)
        s = (((P->cored >> b) & 1u) ? mu_body : 0.0) * P->inv4pib +
            (((P->cored >> a) & 1u) ? m_sink : 0.0) * P->inv4pib;
    if (s > 0.0) {
        radial = orc_cored_radial(sqrt(r2), s);
    } else {
        double re2 = r2 + (P->eps_ab ? P->eps_ab[a * P->D + b] * P->eps_ab[a * P->D + b] : P->eps2);
        radial = 1.0 / (re2 * sqrt(re2));
    }
    double k = P->G[a * P->D + b] * mu * f * radial;
    if (inside)
        for (unsigned x = 0; x < 3; ++x) acc[x] += k * d[x];
    if (inside && P->corr) {
        const uint64_t m = P->corr_n + 1;
        double cr[3];
        lattice_correction(P->corr + ((uint64_t)a * P->D + b) * m * m * m * 3, P->corr_n, P->corr_scale, d, cr);
        const double gm = P->G[a * P->D + b] * mu;
        for (unsigned x = 0; x < 3; ++x) acc[x] += gm * cr[x];
    }
    if (tie) *slack += fabs(k) * sqrt(r2);
    return tie;
}

static void make_pair_ctx(pair_ctx* P, const orc_law* law, uint32_t D, double box)
{
    P->corr = law->corr;
    P->corr_n = law->corr_n;
    P->corr_scale = law->corr ? (double)law->corr_n / (0.5 * box) : 0.0;
    P->G = law->G; P->tab = law->tables; P->ntab = law->ntab; P->grid = law->grid; P->D = D;
    P->rc = law->r_cut; P->rc2 = law->r_cut * law->r_cut; P->eps2 = law->eps * law->eps;
    P->eps_ab = law->eps_ab;
    P->band = 1e-6 * P->rc2;
    P->kind = law->kind;
    P->cored = law->cored;
    P->inv4pib = law->kind == ORC_LAW_ACCUMULATOR ? 1.0 / (4.0 * ORC_PI * law->beta) : 0.0;
}

static double wrap_periodic(double d, double box)
{
    if (d >= 0.5 * box) d -= box;
    else if (d < -0.5 * box) d += box;
    return d;
}

/*
 * Tree force for every sink of the listed groups (all groups when
 * groups == NULL). The walk runs once per group and its list is used for
 * every sink of the group; each accepted node contributes one monopole per
 * non-empty species (section 2.2), each opened leaf its particles. Output is
 * in input order; counts (3 + ORC_MAX_SPECIES entries) = {particle-particle,
 * particle-node interactions, near ties, particle-node interactions of each
 * source species}, an interaction being one evaluation of the pair term on a
 * list entry and a near tie one whose r^2 lies within 1e-6 r_cut^2 of r_cut^2.
 * group_counts (4 per group, optional) = {accepted nodes, opened leaves, pn,
 * pp}.
 */
int orc_tree_force(const orc_tree* t, const orc_law* law,
                   const uint32_t* groups, uint64_t n_sub,
                   double* acc, double* slack, uint64_t* counts,
                   uint64_t* group_counts)
{
    if (!t->M[0] && t->D) return -1;
    uint64_t ng = groups ? n_sub : t->ng;
    pair_ctx P;
    make_pair_ctx(&P, law, t->D, t->box);
    const double scale = t->box * TWO_M64;
    const uint64_t n = t->n;
    uint64_t pp = 0, pn = 0, ties = 0;
    uint64_t pnb[ORC_MAX_SPECIES] = {0};
#pragma omp parallel reduction(+ : pp, pn, ties, pnb[:ORC_MAX_SPECIES])
    {
        list_t L = {0, 0, 0};
#pragma omp for schedule(dynamic, 1)
        for (uint64_t q = 0; q < ng; ++q) {
            uint64_t g = groups ? groups[q] : q;
            group_list(t, law, g, &L);
            uint32_t a = t->gs[g];
            uint64_t s0 = t->gstart[g], ns = t->gcount[g];
            uint64_t n_acc = 0, n_leaf = 0, g_pn = 0, g_pp = 0;
            for (uint64_t k = 0; k < L.n; ++k) {
                uint64_t node = L.e[k] & 0xffffffffull;
                if ((L.e[k] >> 32) == 1) {
                    n_acc++;
                    for (uint32_t b = 0; b < t->D; ++b) {
                        g_pn += t->M[b][node] > 0.0;
                        pnb[b] += (t->M[b][node] > 0.0) * ns;
                    }
                } else {
                    n_leaf++;
                    for (uint32_t b = 0; b < t->D; ++b) g_pp += t->count[b][node];
                }
            }
            g_pn *= ns;
            g_pp = g_pp * ns - ns;   /* every sink meets itself once */
            pn += g_pn;
            pp += g_pp;
            if (group_counts) {
                group_counts[4 * q + 0] = n_acc;
                group_counts[4 * q + 1] = n_leaf;
                group_counts[4 * q + 2] = g_pn;
                group_counts[4 * q + 3] = g_pp;
            }
            for (uint64_t i = s0; i < s0 + ns; ++i) {
                double ai[3] = {0.0, 0.0, 0.0}, sl = 0.0;
                double xi[3];
                for (unsigned x = 0; x < 3; ++x) xi[x] = (double)t->X[x][i] * scale;
                for (uint64_t k = 0; k < L.n; ++k) {
                    uint64_t node = L.e[k] & 0xffffffffull;
                    if ((L.e[k] >> 32) == 1) {
                        for (uint32_t b = 0; b < t->D; ++b) {
                            double Mb = t->M[b][node];
                            if (!(Mb > 0.0)) continue;
                            double d[3];
                            for (unsigned x = 0; x < 3; ++x)
                                d[x] = wrap_periodic(t->com[b][x][node] - xi[x], t->box);
                            double body = Mb;
                            if (law->track_counts && t->count[b][node]) body = Mb / (double)t->count[b][node];
                            ties += pair_term(&P, a, b, Mb, body, t->m[i], d, ai, &sl);
                        }
                    } else {
                        for (uint32_t b = 0; b < t->D; ++b) {
                            uint64_t j0 = t->start[b][node], j1 = j0 + t->count[b][node];
                            for (uint64_t j = j0; j < j1; ++j) {
                                if (j == i) continue;
                                double d[3];
                                for (unsigned x = 0; x < 3; ++x)
                                    d[x] = (double)(int64_t)(t->X[x][j] - t->X[x][i]) * scale;
                                ties += pair_term(&P, a, b, t->m[j], t->m[j], t->m[i], d, ai, &sl);
                            }
                        }
                    }
                }
                uint32_t p = t->perm[i];
                for (unsigned x = 0; x < 3; ++x) acc[x * n + p] = ai[x];
                if (slack) slack[p] = sl;
            }
        }
        free(L.e);
    }
    if (counts) {
        counts[0] = pp;
        counts[1] = pn;
        counts[2] = ties;
        for (uint32_t b = 0; b < ORC_MAX_SPECIES; ++b) counts[3 + b] = pnb[b];
    }
    return 0;
}

/*
 * The plain definition the tree approximates: the minimum-image direct sum
 * over every other particle within the cut-off (in the limit where every
 * particle is its own monopole the walk reproduces it exactly, section 2.2).
 * For the listed sinks (input indices); acc is 3 x n_sinks. A cell list with
 * cells no smaller than r_cut visits exactly the same pairs as the double
 * loop; the double loop is used when fewer than 3 cells fit per axis.
 */
int orc_direct(uint64_t n, uint32_t D, double box, const uint64_t* X,
               const uint8_t* species, const double* mass, const orc_law* law,
               const uint32_t* sinks, uint64_t n_sinks, double* acc, double* slack)
{
    pair_ctx P;
    make_pair_ctx(&P, law, D, box);
    const double scale = box * TWO_M64;
    int64_t nc = (int64_t)floor(box / (law->r_cut * (1.0 + 1e-9)));
    if (nc > 1024) nc = 1024;
    uint32_t* cell_of = NULL;
    uint64_t* cell_start = NULL;
    uint32_t* cell_items = NULL;
    if (nc >= 3) {
        uint64_t ncell = (uint64_t)nc * nc * nc;
        cell_of = malloc((n ? n : 1) * sizeof(uint32_t));
        cell_start = calloc(ncell + 1, sizeof(uint64_t));
        cell_items = malloc((n ? n : 1) * sizeof(uint32_t));
        for (uint64_t j = 0; j < n; ++j) {
            int64_t c[3];
            for (unsigned x = 0; x < 3; ++x) {
                c[x] = (int64_t)((double)X[x * n + j] * TWO_M64 * (double)nc);
                if (c[x] > nc - 1) c[x] = nc - 1;
            }
            cell_of[j] = (uint32_t)((c[0] * nc + c[1]) * nc + c[2]);
            cell_start[cell_of[j] + 1]++;
        }
        for (uint64_t c = 0; c < ncell; ++c) cell_start[c + 1] += cell_start[c];
        uint64_t* fill = malloc((ncell + 1) * sizeof(uint64_t));
        memcpy(fill, cell_start, (ncell + 1) * sizeof(uint64_t));
        for (uint64_t j = 0; j < n; ++j) cell_items[fill[cell_of[j]]++] = (uint32_t)j;
        free(fill);
    }
#pragma omp parallel for schedule(dynamic, 16)
    for (uint64_t q = 0; q < n_sinks; ++q) {
        uint64_t i = sinks[q];
        uint32_t a = species[i];
        double ai[3] = {0.0, 0.0, 0.0}, sl = 0.0;
        if (nc >= 3) {
            int64_t ci = cell_of[i];
            int64_t cz = ci % nc, cy = (ci / nc) % nc, cx = ci / (nc * nc);
            for (int64_t ox = -1; ox <= 1; ++ox)
                for (int64_t oy = -1; oy <= 1; ++oy)
                    for (int64_t oz = -1; oz <= 1; ++oz) {
                        int64_t c = (((cx + ox + nc) % nc) * nc + (cy + oy + nc) % nc) * nc + (cz + oz + nc) % nc;
                        for (uint64_t k = cell_start[c]; k < cell_start[c + 1]; ++k) {
                            uint64_t j = cell_items[k];
                            if (j == i) continue;
                            double d[3];
                            for (unsigned x = 0; x < 3; ++x)
                                d[x] = (double)(int64_t)(X[x * n + j] - X[x * n + i]) * scale;
                            pair_term(&P, a, species[j], mass[j], mass[j], mass[i], d, ai, &sl);
                        }
                    }
        } else {
            for (uint64_t j = 0; j < n; ++j) {
                if (j == i) continue;
                double d[3];
                for (unsigned x = 0; x < 3; ++x)
                    d[x] = (double)(int64_t)(X[x * n + j] - X[x * n + i]) * scale;
                pair_term(&P, a, species[j], mass[j], mass[j], mass[i], d, ai, &sl);
            }
        }
        for (unsigned x = 0; x < 3; ++x) acc[x * n_sinks + q] = ai[x];
        if (slack) slack[q] = sl;
    }
    free(cell_of); free(cell_start); free(cell_items);
    return 0;
}
