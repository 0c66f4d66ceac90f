/*
 * FP64 CPU oracle for the periodic short-range multi-species tree force of
 * ngravs (Croker, "ngravs: Distinct gravitational interactions in GADGET-2").
 *
 * TEST INFRASTRUCTURE ONLY. This code exists to check the GPU library. Only
 * the tests, the smoke check and the benchmark's CPU-baseline leg may load
 * it; the product path never does. It shares no code with the GPU library.
 *
 * Everything is plain, slow and in double precision: a stable library sort,
 * recursive halving of the box, direct per-node sums, a depth-first walk per
 * sink group, and a scalar force loop.
 *
 * Conventions (all arrays are structure-of-arrays):
 *   - positions are 64-bit lattice coordinates X in [0, 2^64)^3; the point is
 *     X * 2^-64 * box;
 *   - "sorted order" is the order of the stable sort by (species, curve key),
 *     the curve Morton or Peano-Hilbert;
 *   - nodes are stored breadth first: by level, then by curve prefix;
 *   - per-species node arrays are laid out [species][node].
 */
#ifndef NGRAVS_ORACLE_H
#define NGRAVS_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_GRID_R = 0, ORC_GRID_R2 = 1 };
enum { ORC_MAX_SPECIES = 6, ORC_LEVELS = 20 };
enum { ORC_PRUNE = 0, ORC_ACCEPT = 1, ORC_OPEN = 2 };

typedef struct orc_tree orc_tree;

typedef struct {
    const double* G;       /* D*D, row = sink species, column = source species */
    const double* tables;  /* D*D*ntab force-factor samples                    */
    uint32_t ntab;         /* >= 2                                              */
    uint32_t grid;         /* ORC_GRID_R or ORC_GRID_R2                         */
    double r_cut;          /* cut-off radius, 0 < r_cut < box/2                 */
    double eps;            /* Plummer softening, >= 0                           */
    double theta;          /* opening angle, > 0                                */
    uint32_t kind;         /* ORC_LAW_TABLE or ORC_LAW_ACCUMULATOR              */
    uint32_t cored;        /* accumulator: bit b set = species b is cored       */
    double beta;           /* accumulator: dimensionless scale, > 0             */
    uint32_t track_counts; /* accumulator: 1 = monopole bodies weigh M/N_perp,
                              0 = a monopole counts as one body of mass M        */
    const double* eps_ab;  /* D x D Plummer softening per species pair (row = sink
                              species), or NULL: eps for every pair               */
    uint32_t opening;      /* ORC_OPEN_GEOMETRIC or ORC_OPEN_RELATIVE             */
    double alpha;          /* relative: the force-error tolerance, > 0            */
    const double* old_acc; /* relative: n previous |a| in input order             */
    const double* corr;    /* lattice corrections (section 2.3), or NULL: D x D
                              tables of (corr_n + 1)^3 x 3 on [0, box/2]^3; with
                              them every pair interacts (no cut-off)              */
    uint32_t corr_n;       /* intervals per axis of the correction tables        */
} orc_law;

enum { ORC_LAW_TABLE = 0, ORC_LAW_ACCUMULATOR = 1 };
enum { ORC_OPEN_GEOMETRIC = 0, ORC_OPEN_RELATIVE = 1 };

int      orc_num_threads(void);

/* lattice, keys, sort */
void     orc_lattice(uint64_t n, const double* x, double box, uint64_t* X);
uint64_t orc_morton(uint32_t kx, uint32_t ky, uint32_t kz);
void     orc_keys(uint64_t n, const uint64_t* X, const uint8_t* species, uint64_t* K);
/* Peano-Hilbert index (60 bits) of a point of the 20-bit lattice, its
 * inverse, and keys species << 60 | curve index in either order. */
enum { ORC_KEY_MORTON = 0, ORC_KEY_HILBERT = 1 };
uint64_t orc_hilbert(uint32_t kx, uint32_t ky, uint32_t kz);
void     orc_hilbert_decode(uint64_t h, uint32_t k[3]);
void     orc_keys_order(uint64_t n, const uint64_t* X, const uint8_t* species, uint32_t key_order, uint64_t* K);
void     orc_sort(uint64_t n, const uint64_t* K, uint32_t* perm);

/* tree */
orc_tree* orc_tree_build(uint64_t n, uint32_t D, double box, const uint64_t* X,
                         const uint8_t* species, const double* mass, uint32_t leaf_size);
/* As orc_tree_build with the particles sorted along the given curve
 * (ORC_KEY_MORTON or ORC_KEY_HILBERT); prefixes are then curve prefixes. */
orc_tree* orc_tree_build_order(uint64_t n, uint32_t D, double box, const uint64_t* X,
                               const uint8_t* species, const double* mass, uint32_t leaf_size,
                               uint32_t key_order);
void     orc_tree_free(orc_tree* t);
uint64_t orc_tree_n_nodes(const orc_tree* t);
void     orc_tree_export(const orc_tree* t, uint32_t* perm, uint64_t* keys,
                         uint8_t* level, uint64_t* prefix, int32_t* parent,
                         int32_t* first_child, uint8_t* n_child,
                         uint32_t* start, uint32_t* count);

/* monopoles */
void     orc_monopoles(orc_tree* t);
void     orc_monopoles_export(const orc_tree* t, double* M, double* com);

/* sink groups */
uint64_t orc_groups(orc_tree* t, uint32_t group_size);
void     orc_groups_export(const orc_tree* t, uint8_t* species, uint32_t* start,
                           uint32_t* count, uint32_t* lo, uint32_t* hi);

/* interaction list of one group: entries are node | kind << 32 */
int      orc_mac_relative(const orc_tree* t, uint64_t node, const uint32_t lo[3],
                          const uint32_t hi[3], double R2, double rel_k, double a_min);
int      orc_mac(const orc_tree* t, uint64_t node, const uint32_t lo[3],
                 const uint32_t hi[3], double R2, double theta2);
uint64_t orc_group_list(const orc_tree* t, const orc_law* law, uint64_t g,
                        uint64_t* entries, uint64_t cap);

/* forces */
int      orc_tree_force(const orc_tree* t, const orc_law* law,
                        const uint32_t* groups, uint64_t n_groups_subset,
                        double* acc, double* slack, uint64_t* counts,
                        uint64_t* group_counts);
int      orc_direct(uint64_t n, uint32_t D, double box, const uint64_t* X,
                    const uint8_t* species, const double* mass, const orc_law* law,
                    const uint32_t* sinks, uint64_t n_sinks, double* acc, double* slack);
double   orc_factor(const double* T, uint32_t ntab, uint32_t grid, double r2, double r_cut);
double   orc_cored_radial(double r, double s);

#ifdef __cplusplus
}
#endif
#endif
