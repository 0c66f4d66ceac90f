/*
 * ngravs-mi355x: periodic short-range Barnes-Hut tree force with one
 * monopole per species in every node, on one AMD Instinct MI355X (gfx950).
 *
 * The method is that of K. A. S. Croker, "ngravs: Distinct gravitational
 * interactions in GADGET-2" (Computer Physics Communications): D <= 6
 * gravitating species (section 2), a per-pair force law f_ab given as a
 * table of the short-range modulation of the Newtonian force (section 2.4.1,
 * TreePM short-range forces), the active mass as a multiplier and the
 * passive mass divided out (section 2.1 and Eq. (1)), and a tree whose
 * nodes carry a mass and a centre of mass per species (section 2.2).
 *
 * The acceleration of particle i of species a is
 *
 *     a_i = sum_b sum_{sources j of species b, |d| < r_cut}
 *               G_ab * mu_j * f_ab(|d|) * d / (|d|^2 + eps^2)^(3/2)
 *
 * with d the minimum-image offset source - sink in the periodic box, where a
 * source is either another particle (mu_j its mass) or a node monopole of
 * species b accepted by the opening test (mu_j the node's species-b mass).
 * G_ab * f_ab > 0 attracts.
 *
 * Calling convention
 *   - Every function returns an ngr_status and never aborts or throws.
 *   - "device" pointers are HIP device memory on the context's device;
 *     "host" pointers are ordinary CPU memory. All arrays are structure of
 *     arrays: a 3 x n array is x[0..n), then y[0..n), then z[0..n).
 *   - Pointers passed in are owned by the caller and only read (or, for
 *     outputs, written) during the call. The tree copies what it needs.
 *   - Calls run on the context's stream and return after their work is
 *     complete (the stream is synchronised before returning).
 *   - After a HIP error the context is poisoned: that call and every later
 *     call on it return NGR_EDEVICE. Use ngr_last_error() for the text.
 */
#ifndef NGRAVS_H
#define NGRAVS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ngr_status;
#define NGR_OK        0   /* success                                                  */
#define NGR_EINVAL   (-1) /* invalid argument, detected before any output is written   */
#define NGR_ENOMEM   (-2) /* device memory or a fixed device limit exhausted            */
#define NGR_EDEVICE  (-3) /* a HIP error; the context is poisoned                       */
#define NGR_ESTATE   (-4) /* wrong call order, e.g. force before monopoles              */

#define NGR_MAX_SPECIES 6      /* section 2: 1 <= D <= 6                                */
#define NGR_GRID_R      0      /* table samples uniform in r   on [0, r_cut], both ends */
#define NGR_GRID_R2     1      /* table samples uniform in r^2 on [0, r_cut^2]          */
#define NGR_LAW_TABLE        0   /* f_ab(r) times the softened Newtonian force            */
#define NGR_LAW_ACCUMULATOR  1   /* section 3.3: cored species, Eqs. (13)-(17)            */
#define NGR_OPEN_GEOMETRIC   0   /* opening test: side < theta d_min                      */
#define NGR_OPEN_RELATIVE    1   /* opening test: M l^2 <= alpha a_old d_min^4 (section 2.2) */
#define NGR_MAX_TABLE   12288  /* D * ntab must not exceed this (one sink species' D
                                  tables are held on chip during the walk)              */

typedef struct ngr_context ngr_context;
typedef struct ngr_tree ngr_tree;

/* Create a context on HIP device `device`. `hip_stream` is the hipStream_t
 * the context's work runs on; NULL means the default (null) stream, which is
 * ordered with all other blocking streams of the device. The context owns a
 * caching pool of device memory and a small pinned host staging area. */
ngr_status ngr_context_create(int device, void* hip_stream, ngr_context** out);
void ngr_context_destroy(ngr_context* ctx);
/* Text of the last error on this context ("" when none). Valid until the
 * next call on the context. */
const char* ngr_last_error(const ngr_context* ctx);

/* One particle set in a periodic cube of side `box`.
 *   n        number of particles, 0 <= n < 2^32 (n == 0 is valid and empty)
 *   D        number of species, 1..6
 *   pos      device, 3 x n float64 positions (taken modulo box), or NULL
 *   lattice  device, 3 x n uint64 lattice coordinates X (the point is
 *            X * 2^-64 * box), or NULL. Exactly one of pos / lattice is set.
 *   species  device, n uint8 ids in [0, D)
 *   mass     device, n float64 masses, finite and >= 0                     */
typedef struct {
    uint64_t n;
    uint32_t D;
    double box;
    const double* pos;
    const uint64_t* lattice;
    const uint8_t* species;
    const double* mass;
} ngr_particles;

/* leaf_size: a node is a leaf once it holds at most this many particles of
 * all species together (1..64; 0 means 16), or at the deepest level (20).
 * key_order: the space-filling curve of the sort (section 2.4), NGR_KEY_MORTON
 * (0) or NGR_KEY_HILBERT (1, the Peano-Hilbert curve of the paper's code). The
 * curve orders particles and children only: the node cells, counts and
 * leaves are the same; sink groups, being runs of consecutive children,
 * follow the order (and with them the interaction lists).
 * non_periodic: nonzero for a non-periodic box (section 2: non-periodic
 * runs use the tree alone). Positions (pos, not lattice) must lie in
 * [0, box)^3 and pairs interact by their plain separation, with no image:
 * the tree is built on a lattice four times the box, in which the
 * minimum-image difference of any two particles is their plain one, and
 * exported lattice coordinates and centres of mass refer to that larger
 * box. r_cut may then reach 2 box (any r_cut >= sqrt(3) box keeps every
 * pair). A non-periodic tree takes no PM force. */
#define NGR_KEY_MORTON  0
#define NGR_KEY_HILBERT 1
typedef struct {
    uint32_t leaf_size;
    uint32_t non_periodic;
    uint32_t key_order;
} ngr_tree_params;

/*
 * Build the tree (section 2: recursive halving of the box; section 2.4: one
 * sort by species and then along the space-filling curve; section 2.2: the
 * tree spans all species and every node records, per species, where its
 * particles start and how many there are, N_perp).
 * Steps on the device: positions -> 64-bit lattice, keys species<<60 |
 * curve index (Morton or Peano-Hilbert, 60 bits), stable radix sort, gather,
 * breadth-first octree.
 * Errors: NGR_EINVAL for D outside 1..6, box <= 0 or not finite, n >= 2^32,
 * leaf_size > 64, key_order not 0 or 1, missing pointers, both or neither of pos / lattice, a
 * species id >= D, a mass < 0 or not finite, a position not finite; for a
 * non-periodic box also lattice input and a position outside [0, box).
 * On success *out owns device memory until ngr_tree_free.
 */
ngr_status ngr_tree_build(ngr_context* ctx, const ngr_particles* p,
                          const ngr_tree_params* tp, ngr_tree** out);

/*
 * Per-node, per-species monopoles (section 2.2): mass M_b (float64) and
 * centre of mass (float64), reduced bottom-up level by level. Must precede
 * ngr_tree_force. track_counts selects the N_perp option of section 2.2
 * for the accumulator laws (ngr_force_params.law): nonzero, a species
 * monopole of M over N_perp particles stands for N_perp bodies of mass
 * M / N_perp; zero, for one body of mass M. Table laws do not depend on it.
 */
ngr_status ngr_compute_monopoles(ngr_context* ctx, ngr_tree* tree, int track_counts);

/* Force-law and walk parameters.
 *   G        host, D x D float64, row = sink species a, column = source b
 *   tables   host (device with tables_on_device), D x D x ntab float64
 *            samples of f_ab on `grid`, or NULL for the Newtonian
 *            short-range factor
 *            erfc(r/2r_s) + r/(r_s sqrt(pi)) exp(-r^2/4r_s^2) for every pair
 *   ntab     samples per table, >= 2, D * ntab <= NGR_MAX_TABLE
 *   grid     NGR_GRID_R or NGR_GRID_R2; f between samples is the straight
 *            line through the two neighbours, f = 0 for r >= r_cut
 *   r_s      split scale, used only when tables == NULL (> 0 then)
 *   r_cut    cut-off radius, 0 < r_cut < box / 2 (see lattice_corr)
 *   eps      Plummer softening: 0, or at least 1e-12 box (the kernel factor
 *            (r^2 + eps^2)^(-3/2) is taken in float32 in units of the box;
 *            with eps = 0 a separate float64-refined factor serves pairs
 *            down to ~1e-19 box, and coincident pairs contribute nothing)
 *   theta    opening angle, > 0
 *   group_size  sinks per walk, 16, 32 or 64 (0: the library's choice: 32, or
 *            what ngr_autotune chose for the box's class on this context)
 *   law      NGR_LAW_TABLE (0), or NGR_LAW_ACCUMULATOR: the accumulator
 *            laws of section 3.3. A pair in which neither species is cored
 *            keeps the law above. Otherwise the Newtonian factor
 *            (r^2 + eps^2)^(-3/2) is replaced by the force of the Eq. (14)
 *            potential, (2/pi) [atan(r/s) - (r/s) / (1 + (r/s)^2)] / r^3,
 *            whose scale s = (c_b mu + c_a m) / (4 pi beta) adds the core
 *            of the source body (c_b = 1 if source species b is cored; mu =
 *            its mass, or M / N_perp for a tracked monopole, M untracked)
 *            and of the sink (c_a, its mass m). Readings: the core radius
 *            of the Eq. (15) density is M / (4 pi beta), the radius with
 *            which it holds mass M; a point-like source adds no core, in
 *            Phi_10, Eq. (16), as elsewhere. A pair with s = 0 (massless cored
 *            bodies) keeps the softened law. f_ab still multiplies.
 *   cored    accumulator: bit b set = species b is cored (< 2^D)
 *   beta     accumulator: the dimensionless scale of Eqs. (13)-(15), > 0
 *   eps_ab   host, D x D float64 Plummer softening of each species pair (row =
 *            sink species; section 2's D^2 softenings), each 0 or at least
 *            1e-12 box as eps,
 *            or NULL for eps everywhere
 *   opening  NGR_OPEN_GEOMETRIC (0), the test described at ngr_tree_force, or
 *            NGR_OPEN_RELATIVE: section 2.2 keeps the stock code's relative
 *            criterion, the previous acceleration against a Newtonian
 *            estimate of the node's contribution. Per group: a node is
 *            accepted when M l^2 <= alpha a_min d_min^4 (M its mass over all
 *            species, l its side, a_min the smallest previous |a| of the
 *            group's sinks) and d_max < r_cut; opened when the group's box
 *            reaches into the node's cube grown to 1.2 sides; pruned when
 *            d_min >= r_cut. theta is not used. Evaluated in float64 as
 *            M (4 S^2) <= (alpha u^2 a_min) D2^2 in half key units
 *            (u = box / 2^21).
 *   alpha    relative: the tolerance, finite and > 0
 *   old_acc  relative: device, n float64, the previous |a| of each particle
 *            in input order (read during the call)
 *   lattice_corr  host, or NULL: pure-tree periodic mode (section 2.3). D x D
 *            tables of (corr_n + 1)^3 x 3 float64, index ((ab (n+1) + i) (n+1)
 *            + j) (n+1) + k, component last: on the grid d = (i, j, k) box /
 *            (2 corr_n) in [0, box/2]^3, the acceleration a sink receives from
 *            every image of a unit source at offset d (source - sink) other
 *            than the nearest, per unit G_ab; odd in each component's own
 *            axis, so it is read trilinearly at |d| with each component
 *            signed by its axis. Every pair then interacts by its nearest
 *            image (no cut-off: r_cut is the tables' range and must reach
 *            sqrt(3)/2 box, the farthest nearest image) and adds G_ab mu
 *            times the interpolated correction. Table laws only; periodic
 *            trees only.
 *   corr_n   intervals per axis of the correction tables, 1..512
 *   tables_on_device  nonzero: `tables` is a device pointer, read in place
 *            during the call (nothing is copied from the host); its entries
 *            are checked on the device (NGR_EINVAL if one is not finite).
 *            Zero: a host pointer, as above.
 */
typedef struct {
    const double* G;
    const double* tables;
    uint32_t ntab;
    uint32_t grid;
    double r_s;
    double r_cut;
    double eps;
    double theta;
    uint32_t group_size;
    uint32_t law;
    uint32_t cored;
    double beta;
    const double* eps_ab;
    uint32_t opening;
    double alpha;
    const double* old_acc;
    const double* lattice_corr;
    uint32_t corr_n;
    uint32_t tables_on_device;
} ngr_force_params;

/* Filled by ngr_tree_force (host). An interaction is one evaluation of the
 * pair term on an interaction-list entry: a particle of an opened leaf
 * (sink itself excluded) or a non-empty species monopole of an accepted
 * node, whether or not it falls inside r_cut.
 *   interactions_pn_species  interactions_pn split by the monopole's
 *            (source) species b; entries b >= D are 0
 *   near_ties  pair terms whose r^2 lies within 1e-6 r_cut^2 of r_cut^2: a
 *            finite-precision evaluation may keep or drop such a pair (the
 *            per-pair cut-off test is taken in each implementation's own
 *            precision). Counted by ngr_tree_force_counts on a one-box tree
 *            with the table laws and no lattice corrections; NGR_NOT_COUNTED
 *            from every other call.
 *   ms_build, ms_build_ingest, ms_build_sort, ms_build_octree  device time
 *            (hipEvents) of the tree's ngr_tree_build: all of it; the input
 *            checks, lattice and keys; the radix sort and the one reordering;
 *            the level-by-level octree (each level's size is read back)
 *   ms_monopoles  device time of the tree's ngr_compute_monopoles
 *   ms_groups, ms_walk  device time of this call's sink groups (with the
 *            ordering of the walk queue) and of its walk launch */
#define NGR_NOT_COUNTED UINT64_MAX
typedef struct {
    uint64_t interactions_pp;
    uint64_t interactions_pn;
    uint64_t n_nodes;
    uint64_t n_leaves;
    uint64_t n_groups;
    uint32_t group_size;
    uint32_t depth;
    double ms_groups;
    double ms_walk;
    uint64_t interactions_pn_species[NGR_MAX_SPECIES];
    uint64_t near_ties;
    double ms_build;
    double ms_build_ingest;
    double ms_build_sort;
    double ms_build_octree;
    double ms_monopoles;
} ngr_force_stats;

/*
 * Short-range tree force (the walk of section 2.2 restricted to short range
 * as in section 2.4.1), one walk per species-pure group of sinks.
 *   acc   device, 3 x n float64, written in input order.
 *   st    host, may be NULL.
 * Opening test, on the exact integer key lattice: with d_min the smallest
 * periodic distance between a node's cell and the group's bounding box and
 * d_max an upper bound on the largest, the node is skipped when
 * d_min >= r_cut, used as monopoles when side < theta * d_min and
 * d_max < r_cut, and opened otherwise.
 * Errors: NGR_EINVAL for bad parameters (see ngr_force_params), non-finite
 * G or table entries, NULL acc with n > 0; NGR_ESTATE without monopoles.
 */
ngr_status ngr_tree_force(ngr_context* ctx, const ngr_tree* tree,
                          const ngr_force_params* fp, double* acc,
                          ngr_force_stats* st);

/* ---- exact short-range tables (section 2.4.1, Eqs. (8)-(11)) ----
 *
 * A law given by phibar(k) = k^2 phi(k), phi(k) the 3-D transform
 * int phi(x) exp(-i k.x) d^3x of its pair potential per unit masses (Newton:
 * -4 pi; Yukawa -(1 + alpha exp(-r/lam))/r: -4 pi (1 + alpha k^2/(k^2 +
 * lam^-2))), and by its full force factor relative to Newton's 1/r^2,
 * f_full(r) = r^2 dphi/dr (Newton: 1). Its short-range factor for the
 * Gaussian split of scale r_s is
 *   f_short(r) = f_full(r) + 1/(2 pi^2) int_0^inf phibar(k) exp(-k^2 r_s^2)
 *                                       [sin(kr)/k - r cos(kr)] dk,
 * the derivative of phi - F^-1[phi(k) exp(-k^2 r_s^2)] (Eqs. (9), (10) with
 * the r'-integral in closed form); for Newton it is the factor
 * erfc(r/2r_s) + r/(r_s sqrt(pi)) exp(-r^2/4r_s^2). The integral is the
 * trapezoid rule on k_m = m dk, m = 0 .. nk-1, evaluated on the device.
 *   D, ntab, grid, r_cut   the tables' shape and radii, as in ngr_force_params
 *   r_s     split scale, > 0
 *   nk, dk  the k grid of phibar (nk >= 2, dk > 0); ngr_short_range_grid
 *           gives one with aliasing and truncation below ~1e-16 for laws
 *           whose r-space kernel decays as exp(-r/range) beyond the Gaussian
 */
typedef struct {
    uint32_t D;
    uint32_t ntab;
    uint32_t grid;
    uint32_t nk;
    double r_s;
    double r_cut;
    double dk;
} ngr_short_params;

/* A k grid for ngr_short_range_tables: period 2 pi / dk covering r_cut +
 * 12.5 r_s + 37 range, k up to where exp(-k^2 r_s^2) < 1e-17.
 * range >= 0 is the law's longest decay length (0 for Newton).
 * Errors: NGR_EINVAL for r_s, r_cut not finite and > 0, range < 0, or more
 * than 2^24 samples. */
ngr_status ngr_short_range_grid(double r_s, double r_cut, double range, uint32_t* nk, double* dk);

/* Tables of f_short at the ntab table radii of every species pair.
 *   phibar  host, D x D x nk float64: phibar_ab(m dk), row a = sink species
 *   f_full  host, D x D x ntab float64: f_full_ab at the table radii
 *   tables  host, D x D x ntab float64, written (usable as
 *           ngr_force_params.tables)
 * Errors: NGR_EINVAL for D outside 1..6, ntab < 2, a bad grid, r_s, r_cut
 * or dk not finite and > 0, nk < 2 or > 2^24, NULL arrays, non-finite
 * entries. */
ngr_status ngr_short_range_tables(ngr_context* ctx, const ngr_short_params* sp,
                                  const double* phibar, const double* f_full,
                                  double* tables);

/* ---- particle-mesh long-range force (sections 2, 2.4 and 2.4.1) ----
 *
 * The PM half of TreePM for D species: cloud-in-cell assignment of each
 * species to a periodic mesh of N^3 points, FFT, the Gaussian-filtered
 * Green's function of every species pair (the window divided out twice),
 * summed over source species, inverse FFT, the 4-point centred difference
 * and cloud-in-cell interpolation to the particles. On a tree of the same
 * box and laws, ngr_tree_force (short range, with the tables of
 * ngr_short_range_tables for the same r_s) plus ngr_pm_force (long range)
 * is the TreePM force.
 *   N     mesh points per side, a power of two in 16..1024
 *   D     species, 1..6
 *   box   periodic box side, > 0
 *   r_s   split scale, > 0 (the filter exp(-k^2 r_s^2))
 * The plan holds ceil(D/2) complex float64 meshes (16 N^3 bytes each) and
 * the Green's function table until ngr_pm_destroy.
 */
typedef struct {
    uint32_t N;
    uint32_t D;
    double box;
    double r_s;
} ngr_pm_params;

typedef struct ngr_pm ngr_pm;

/* Device time of the last ngr_pm_force, per step (ms): the deposit (with the
 * clearing of the meshes); the forward transforms along x and y; one pass
 * holding the forward z transform, the k-space step and the inverse z
 * transform (ms_green); the inverse transforms along y and x; the
 * interpolation. */
typedef struct {
    double ms_deposit;
    double ms_fft_forward;
    double ms_green;
    double ms_fft_inverse;
    double ms_interp;
} ngr_pm_stats;

/* Create a PM plan.
 *   G       host, D x D float64, row = sink species a (as ngr_force_params)
 *   phibar  host, D x D x (3 (N/2)^2 + 1) float64: phibar_ab = k^2 phi_ab(k)
 *           (as ngr_short_range_tables) at the mesh's |k| = 2 pi sqrt(q) / box,
 *           q = 0 .. 3 (N/2)^2 (entry q = 0 is not used: the mean is dropped).
 *           A per-pair constant in phibar scales that pair's long range only,
 *           e.g. the exp(-y^2 r_s^2) correction of a Yukawa law of section
 *           3.2 (give the short-range tables the same phibar).
 * Errors: NGR_EINVAL for N not a power of two in 16..1024, D outside 1..6,
 * box or r_s not finite and > 0, NULL or non-finite G or phibar;
 * NGR_ENOMEM when the meshes do not fit. */
ngr_status ngr_pm_create(ngr_context* ctx, const ngr_pm_params* pp, const double* G,
                         const double* phibar, ngr_pm** out);

/* Long-range accelerations of the particles of a one-box tree with the
 * plan's D and box: written to (accumulate == 0) or added to (nonzero) acc,
 * device, 3 x n float64 in input order. st may be NULL.
 * Errors: NGR_EINVAL for NULL pm or tree, a batch tree, a tree whose D or
 * box differs from the plan's, NULL acc with n > 0. */
ngr_status ngr_pm_force(ngr_context* ctx, ngr_pm* pm, const ngr_tree* tree, double* acc,
                        int accumulate, ngr_pm_stats* st);

/* Release a plan. NULL is accepted. */
ngr_status ngr_pm_destroy(ngr_context* ctx, ngr_pm* pm);

/* Release a tree. NULL is accepted. */
ngr_status ngr_tree_free(ngr_context* ctx, ngr_tree* tree);

/* ---- inspection (for tests and tools; all outputs are host arrays) ---- */

/* Sizes: particles, nodes, tree depth (deepest level). */
ngr_status ngr_tree_info(const ngr_tree* tree, uint64_t* n, uint64_t* n_nodes,
                         uint32_t* D, uint32_t* depth);

/* Copy the build's results to host arrays (any may be NULL):
 *   perm   n uint32, sorted position -> input index
 *   keys   n uint64, sorted keys species<<60 | Morton60
 *   lattice 3 x n uint64 in sorted order
 *   level  n_nodes uint8;  prefix n_nodes uint64 (3*level bits of the key)
 *   parent n_nodes int32 (-1 for the root); first_child n_nodes int32 (-1 for
 *          a leaf); n_child n_nodes uint8
 *   start, count  D x n_nodes uint32: first sorted index and number of the
 *          node's particles of each species
 * Nodes are breadth first: ordered by level, then by prefix. */
ngr_status ngr_tree_export(ngr_context* ctx, const ngr_tree* tree,
                           uint32_t* perm, uint64_t* keys, uint64_t* lattice,
                           uint8_t* level, uint64_t* prefix, int32_t* parent,
                           int32_t* first_child, uint8_t* n_child,
                           uint32_t* start, uint32_t* count);

/* Monopoles to host: M D x n_nodes, com D x 3 x n_nodes (positions in
 * [0, box)). */
ngr_status ngr_monopoles_export(ngr_context* ctx, const ngr_tree* tree,
                                double* M, double* com);

/* Sink groups for a group size (see ngr_force_params.group_size), to host.
 * Call once with species == NULL to get *n_groups, then with arrays of that
 * size: species uint8, start/count uint32 (sorted positions), lo/hi 3 x
 * n_groups uint32 (bounding box on the 20-bit key lattice, hi exclusive). */
ngr_status ngr_groups_export(ngr_context* ctx, const ngr_tree* tree,
                             uint32_t group_size, uint64_t* n_groups,
                             uint8_t* species, uint32_t* start, uint32_t* count,
                             uint32_t* lo, uint32_t* hi);

/* As ngr_tree_force, and also write per-group counts to the host array
 * group_counts (4 x n_groups uint64 per group: accepted nodes, opened
 * leaves, pn interactions, pp interactions; may be NULL), groups in the
 * order of ngr_groups_export, and count the near ties (ngr_force_stats). The
 * near-tie count runs a separate instantiation of the walk with one more
 * compare per pair term; accelerations are bitwise those of ngr_tree_force. */
ngr_status ngr_tree_force_counts(ngr_context* ctx, const ngr_tree* tree,
                                 const ngr_force_params* fp, double* acc,
                                 ngr_force_stats* st, uint64_t* group_counts);

/* ---- without device allocation ----
 *
 * For callers that cannot allocate device memory: code that must not call
 * hipMalloc or free (tight serving loops, harnesses that forbid allocation
 * after start-up). ngr_tree_force_noalloc is ngr_tree_force on a one-box
 * tree, bit for bit the same accelerations and counts, with every scratch
 * buffer of the call (sink groups, the walk's queue order and control
 * block, the tables in their on-chip layouts, the per-wave traversal
 * stacks) taken from one static device array of NGR_NOALLOC_SCRATCH_BYTES
 * that the library holds on each GPU it runs on until the process ends. It
 * calls no hipMalloc, hipFree or other allocating routine and creates no
 * events (the ms_groups and ms_walk statistics are 0; near_ties is
 * NGR_NOT_COUNTED). The tree itself comes from ngr_tree_build as usual. It
 * returns after its work is complete and reads sizes back on the way, so it
 * cannot be captured in a graph. Its walk runs fewer waves per CU (the
 * stacks must fit the array), so it is slower than ngr_tree_force.
 * Every call on one GPU uses that GPU's one array, which keeps the last
 * call's contents (each call clears what must start at zero): calls that
 * overlap in time on one GPU (from several threads or streams) race, and
 * the caller must order them.
 * Errors: as ngr_tree_force; NGR_EINVAL also for a batch tree or more than
 * NGR_NOALLOC_MAX_N particles (checked before any device work); NGR_ENOMEM
 * when this tree's groups and tables do not fit the array (detected before
 * the walk writes acc).
 */
#define NGR_NOALLOC_SCRATCH_BYTES (96u << 20)   /* 96 MiB per GPU */
#define NGR_NOALLOC_MAX_N         (1u << 20)
ngr_status ngr_tree_force_noalloc(ngr_context* ctx, const ngr_tree* tree,
                                  const ngr_force_params* fp, double* acc,
                                  ngr_force_stats* st);

/* ---- many boxes in one call ---- */

/* One independent box of a batch. Pointers and sizes as in the single-box
 * calls: particles (device arrays), tree parameters, force parameters (host
 * arrays) and acc (device, 3 x n float64, written in the box's input order).
 * force.group_size == 0 lets the library choose the box's group size. */
typedef struct {
    ngr_particles particles;
    ngr_tree_params tree;
    ngr_force_params force;
    double* acc;
} ngr_box;

/* Filled by ngr_batch_build_force (host). Times are hipEvent milliseconds on
 * the context's stream; ms_groups includes the ordering of the walk queue. */
typedef struct {
    uint64_t n_particles;
    uint64_t n_nodes;
    uint64_t n_groups;
    uint64_t interactions_pp;
    uint64_t interactions_pn;
    double ms_build;
    double ms_monopoles;
    double ms_groups;
    double ms_walk;
} ngr_batch_stats;

/*
 * Tree build, monopoles and short-range force of nbox independent periodic
 * boxes (sections 2, 2.2 and 2.4.1 applied to each box), done together: one
 * check-and-key pass, one sort by (box, species, key), one level-by-level
 * octree over all boxes, one monopole pass and one walk launch whose
 * workgroups move between (box, sink species) segments. Boxes may differ in
 * n, D, box side, leaf size, G, tables, r_cut, eps, theta and group size;
 * they must share the table grid.
 * Each box's acc and per-box counts are those of ngr_tree_build +
 * ngr_compute_monopoles + ngr_tree_force on that box alone with the same
 * parameters and resolved group size, bit for bit.
 *   nbox     1..65535; all boxes together hold fewer than 2^32 - 1 particles
 *   st       host, may be NULL
 *   per_box  host array of nbox entries, may be NULL: each box's interaction
 *            counts, nodes, leaves, depth, groups and resolved group size
 *            (its times are 0)
 * Errors: as the single-box calls (the message names the box), NGR_EINVAL for
 * nbox out of range or mixed grids. No tree outlives the call.
 */
ngr_status ngr_batch_build_force(ngr_context* ctx, uint32_t nbox, const ngr_box* boxes,
                                 ngr_batch_stats* st, ngr_force_stats* per_box);

/*
 * Group-size autotuner. Boxes are sorted into classes by D and floor(log2 n).
 * For each class present, up to two boxes of that class, repeated until they
 * hold 2^21 particles (enough groups to fill the device, so that a class's
 * throughput is measured and not one group's latency), are built together
 * once. Their groups and walk are timed (wall clock, the better of two runs)
 * at group sizes 16, 32 and 64. The context keeps the fastest size per
 * class; afterwards group_size = 0 in any call on this context
 * (ngr_tree_force, ngr_batch_build_force, the server) resolves to it.
 * Classes never tuned keep the default, 32. Results of later calls depend on
 * the sizes chosen (the group size shapes the interaction lists), each
 * within the force tolerance; per-box statistics report the size used.
 * Inputs as for ngr_batch_build_force (acc is not written). st may be NULL.
 */
typedef struct {
    uint32_t classes;       /* classes tuned by this call                     */
    uint32_t launches;      /* walk launches timed                            */
    double ms;              /* wall time of the call                          */
} ngr_tune_stats;

ngr_status ngr_autotune(ngr_context* ctx, uint32_t nbox, const ngr_box* boxes, ngr_tune_stats* st);

/* The group size that group_size = 0 resolves to for a box of n particles
 * and D species on this context. */
ngr_status ngr_tuned_group_size(const ngr_context* ctx, uint64_t n, uint32_t D, uint32_t* group_size);

/* ---- served requests ---- */

typedef struct ngr_server ngr_server;

/* hbm_budget: device bytes the server may hold for admitted requests plus
 * the trees of one tick (0 means 200e9); max_active: admitted requests at
 * most (0: no limit). */
typedef struct {
    uint64_t hbm_budget;
    uint32_t max_active;
} ngr_server_params;

/* One request: a box, its initial state, its law and a number of
 * kick-drift-kick leapfrog steps of length dt. The state is the 64-bit
 * lattice X (positions X * 2^-64 * box), velocities (box units per time) and
 * the short-range accelerations of this library's force. steps K means K + 1
 * force evaluations: a(X0), then per step v += a dt/2, X += v dt (wrapping in
 * the periodic box), a = a(X), v += a dt/2.
 *   particles  device arrays, copied at submit (pos or lattice)
 *   vel        device 3 x n float64 initial velocities, copied, or NULL for 0
 *   tree, force  as the single-box calls; host arrays copied at submit
 *   dt > 0 and finite; steps 0..2^20 */
typedef struct {
    ngr_particles particles;
    const double* vel;
    ngr_tree_params tree;
    ngr_force_params force;
    double dt;
    uint32_t steps;
} ngr_request;

/* What one tick did (host). */
typedef struct {
    uint32_t admitted;        /* requests admitted at the start of the tick */
    uint32_t evaluated;       /* requests that got a force evaluation */
    uint32_t finished;        /* requests that finished in this tick */
    uint32_t active;          /* admitted and not finished, after the tick */
    uint32_t pending;         /* submitted and not admitted, after the tick */
    uint64_t particles;       /* particles of the tick's force evaluation */
    uint64_t interactions;    /* pp + pn interactions of the tick */
    uint64_t resident_bytes;  /* device bytes held for admitted requests */
    double ms;                /* GPU time of the tick (hipEvents) */
} ngr_tick_stats;

/*
 * A request server on a context (continuous batching). Requests wait in
 * submission order; a tick admits the waiting ones that fit the HBM budget
 * (in order, stopping at the first that does not fit), then runs one
 * kick-drift, one force evaluation of every admitted request as one batch
 * (ngr_batch_build_force's engine) and one kick, and marks the requests whose
 * last force evaluation it was as finished. A request's trajectory does not
 * depend on which other requests share its ticks: it is bitwise the one it
 * has alone. The server runs on the context's stream; calls return after
 * their work is complete. Not thread safe.
 */
ngr_status ngr_server_create(ngr_context* ctx, const ngr_server_params* sp, ngr_server** out);
/* Submit a request: checks it (NGR_EINVAL as the single-box calls), copies its
 * data and uploads its tables; *id identifies it. NGR_ENOMEM if it can never
 * fit the budget. */
ngr_status ngr_server_submit(ngr_server* s, const ngr_request* r, uint64_t* id);
/* One tick (see above). With nothing admitted or waiting it does nothing. */
ngr_status ngr_server_tick(ngr_server* s, ngr_tick_stats* st);
/* state: 0 waiting, 1 admitted, 2 finished; evals: force evaluations done.
 * NGR_EINVAL for an unknown (or taken) id. */
ngr_status ngr_server_status(const ngr_server* s, uint64_t id, int* state, uint32_t* evals);
/* Copy a finished request's final state to caller device arrays (any may be
 * NULL): lattice 3 x n uint64, vel 3 x n float64, acc 3 x n float64; then
 * release the request. NGR_ESTATE if it has not finished. */
ngr_status ngr_server_take(ngr_server* s, uint64_t id, uint64_t* lattice, double* vel, double* acc);
void ngr_server_destroy(ngr_server* s);

#ifdef __cplusplus
}
#endif
#endif
