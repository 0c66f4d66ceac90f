// Internal declarations of the ngravs-mi355x library (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "../../include/ngravs.h"

namespace ngr {

constexpr int kLevels = 20;           // key levels: 20 bits per axis, 60-bit Morton key
constexpr int kKeyBits = 60;
constexpr uint64_t kKeyMask = (1ull << kKeyBits) - 1ull;
constexpr int kWave = 64;

// Thrown inside the library only; converted to a status at the C-ABI.
struct Error {
    ngr_status status;
    std::string msg;
};

[[noreturn]] void fail(ngr_status s, const std::string& msg);
void hip_check(hipError_t e, const char* what, const char* file, int line);
#define HIP_CHECK(x) ::ngr::hip_check((x), #x, __FILE__, __LINE__)
#define LAUNCH_CHECK(what) ::ngr::hip_check(hipGetLastError(), what, __FILE__, __LINE__)

struct DevMem {
    void* p = nullptr;
    size_t bytes = 0;
};

// Device memory comes from a caching pool owned by the context: blocks are
// obtained with hipMalloc, returned to the pool by release() and handed out
// again to later requests. All work of a context runs on its one stream, so
// a block released after the launches that use it can only be reused by
// launches enqueued after them. Memory goes back to the device when the
// context is destroyed.
struct Context {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    bool poisoned = false;
    int num_cu = 0;
    size_t lds_per_block = 0;
    bool trace = false;
    std::chrono::steady_clock::time_point t_created = std::chrono::steady_clock::now();
    std::string err;
    std::multimap<size_t, void*> free_blocks;     // size class -> block
    std::map<void*, size_t> live_blocks;          // block -> size class
    // persistent scratch reused across calls
    DevMem stacks;          // per-wave traversal stacks of the walk
    DevMem counters;        // small device counters (queues, statistics, flags)
    DevMem core;            // core-factor table of the accumulator laws (built on first use)
    std::map<uint64_t, uint32_t> tuned;           // group size per class (D << 8 | floor(log2 n))
    uint64_t* pinned = nullptr;                   // pinned host staging, kPinnedWords
    static constexpr size_t kPinnedWords = 64;
    hipEvent_t ev[8] = {};                        // timing events, created on first use
    hipEvent_t event(int k);
    float elapsed(int k0, int k1);                // ms between two recorded events (synchronises)
    // Arena mode (the no-allocation entry point): while `arena` is set,
    // alloc() hands out consecutive 256-byte aligned pieces of the caller's
    // device buffer and fails with NGR_ENOMEM when it is used up; release()
    // of such a piece does nothing; no events are created and the
    // context's persistent buffers are neither grown nor kept.
    unsigned char* arena = nullptr;
    size_t arena_size = 0, arena_used = 0;
    bool in_arena(const void* p) const
    {
        return arena && p >= arena && static_cast<const unsigned char*>(p) < arena + arena_size;
    }

    void* alloc(size_t bytes);
    void release(void* p);
    void ensure(DevMem& m, size_t bytes);
    void sync();
    void free_all();
    void stage(const char* what);                 // progress trace (NGR_TRACE=1)
    // copy `words` uint64 values device -> host / host -> device through
    // pinned memory (synchronises the stream)
    void read_words(uint64_t* host, const void* dev, size_t words);
    void write_words(void* dev, const uint64_t* host, size_t words);
    // blocking copies of larger arrays (synchronise the stream first)
    void to_host(void* host, const void* dev, size_t bytes);
    void to_device(void* dev, const void* host, size_t bytes);
};

// One box to build: caller-owned device arrays of one periodic box.
struct BoxIn {
    uint64_t n = 0;
    uint32_t D = 1;
    double box = 1.0;
    uint32_t leaf_size = 16;
    uint32_t key_order = NGR_KEY_MORTON; // space-filling curve of the keys
    const double* pos = nullptr;         // 3 x n, or NULL
    const uint64_t* lattice = nullptr;   // 3 x n, or NULL
    const uint8_t* species = nullptr;
    const double* mass = nullptr;
    double region = 0.0;                 // non-periodic: the user's box (box is 4 region), else 0
};

// The tree of one or more independent boxes built together. Particles of all
// boxes are kept in one sorted array, box after box; nodes are breadth first
// over all boxes (level by level, box after box within a level); the roots
// are nodes 0 .. nbox-1. Per-node arrays of species use the largest D of the
// boxes as stride (species a box does not have are empty).
// A particle as the walk reads it for its leaf records: the position as a
// fraction of the box, split into a high part (the lattice coordinate with
// its low 11 bits cleared, exact in float64) and a low part (those 11 bits,
// exact in float32), and the mass. The high part minus a group centre is
// exact, so adding the low part rounds once, exactly as converting the
// integer lattice difference would.
struct alignas(16) PRec {
    double hx, hy, hz, m;
    float lx, ly, lz, pad;
};
constexpr uint64_t kLowBits = 0x7ffull;

struct Tree {
    uint64_t n = 0;                // particles of all boxes
    uint32_t D = 0;                // species stride: the largest D of the boxes
    uint32_t nbox = 0;
    // per box (host)
    std::vector<uint64_t> boff;    // nbox + 1: first sorted particle (= first input index) of each box
    std::vector<uint32_t> bD;      // species of each box
    std::vector<double> bbox;      // box side
    std::vector<uint32_t> bleaf;   // leaf size
    std::vector<uint64_t> bseg;    // nbox x (NGR_MAX_SPECIES + 1): species segments, sorted positions
    uint64_t* boff_dev = nullptr;  // device copy of boff
    // one-box conveniences (box 0)
    double box = 0.0;
    double region = 0.0;           // non-periodic box 0: the user's box (box = 4 region), else 0
    uint32_t leaf_size = 16;
    uint64_t seg[NGR_MAX_SPECIES + 1] = {0};
    // particles in sorted order (box, species, Morton key)
    uint64_t* X = nullptr;         // 3 x n lattice coordinates
    double* mass = nullptr;        // n
    PRec* P = nullptr;             // n, the same particles split for the walk's leaf records
    uint32_t* perm = nullptr;      // n, sorted position -> input index (over all boxes)
    uint64_t* keys = nullptr;      // n sorted keys (species << 60 | Morton), per box
    // nodes, breadth first; capacity cap
    uint64_t nn = 0, cap = 0;
    uint32_t depth = 0;
    std::vector<uint64_t> level_start;  // host: first node of each level, size depth+2
    uint8_t* level = nullptr;
    uint64_t* prefix = nullptr;
    int32_t* parent = nullptr;
    int32_t* first_child = nullptr;
    uint8_t* n_child = nullptr;
    uint4* cell = nullptr;         // corner (20-bit key units) x, y, z and level
    uint32_t* start = nullptr;     // nn x D, [node * D + b]
    uint32_t* count = nullptr;     // nn x D
    uint32_t* node_box = nullptr;  // nn, the box of each node
    uint64_t n_leaves = 0;
    // monopoles: D x nn records {com_x, com_y, com_z (box fraction), M}
    double4* mono = nullptr;
    bool has_monopoles = false;
    bool track_counts = true;      // N_perp option of the monopoles (accumulator laws)
    // device time of the build's phases and of the monopoles (single-box calls)
    float ms_ingest = 0.0f, ms_sort = 0.0f, ms_octree = 0.0f, ms_monopoles = 0.0f;
};
void free_tree(Context& ctx, Tree& t);

// ---- argument checks (api.hip) ----
bool finite_pos(double v);
// Check one box's particles and tree parameters; fill b. `where` prefixes messages.
void check_particles(const ngr_particles* p, const ngr_tree_params* tp, const std::string& where, BoxIn& b);
// Check one box's force parameters; returns group_size (0: caller's choice).
uint32_t check_force_params(uint32_t D, double box, const ngr_force_params* fp, const std::string& where);
// The group size used when the caller passes 0.
uint32_t chosen_group_size(const Context& ctx, uint64_t n, uint32_t D);
uint64_t size_class(uint64_t n, uint32_t D);

// ---- device scan (scan.hip) ----
// Exclusive prefix sum of n uint32 values; out may alias in. If total is
// non-null the sum of all values is written to *total (device).
void scan_exclusive(Context& ctx, const uint32_t* in, uint32_t* out, uint64_t n, uint32_t* total);

// ---- radix sort (sort.hip) ----
// Stable sort of n (key, value) pairs by the key bits [0, bits), LSD, 8 bits
// per pass. Results in keys/vals; scratch buffers of the same size given.
void radix_sort_pairs(Context& ctx, uint64_t* keys, uint32_t* vals, uint64_t* keys_tmp,
                      uint32_t* vals_tmp, uint64_t n, int bits);

// ---- build steps (build.hip) ----
// Check, key, sort and build the tree of every box in one pass. Boxes with an
// invalid species id, mass or position fail with NGR_EINVAL naming the box.
// timed: record the phases' device times in t (events on the context's stream).
void build_forest(Context& ctx, const std::vector<BoxIn>& boxes, Tree& t, bool timed = false);
// The device checks of one box's inputs alone (NGR_EINVAL as build_forest).
void validate_box(Context& ctx, const BoxIn& b, const std::string& where);
void compute_monopoles(Context& ctx, Tree& t);
// Nodes, leaves and deepest level of each box of a tree (host vectors).
void box_node_counts(Context& ctx, const Tree& t, std::vector<uint64_t>& nodes, std::vector<uint64_t>& leaves,
                     std::vector<uint32_t>& depth);

// ---- groups and walk (walk.hip) ----
// Groups of sinks, ordered like the particles (box, species, key). A segment
// is one (box, species) pair: segment s = box * D + species (D = tree stride);
// its groups are first[s] .. first[s + 1).
struct Groups {
    uint64_t ng = 0;
    uint32_t nseg = 0;
    uint32_t* start = nullptr;     // ng
    uint32_t* count = nullptr;     // ng
    uint32_t* lo = nullptr;        // 3 x ng
    uint32_t* hi = nullptr;        // 3 x ng
    uint32_t* box = nullptr;       // ng, box of each group
    std::vector<uint64_t> first;   // host, nseg + 1
    void free(Context& ctx);
};
// group_size: per box, 16, 32 or 64
void make_groups(Context& ctx, const Tree& t, const std::vector<uint32_t>& group_size, Groups& g);

// Force law and walk parameters of one box. The tables stay where the
// caller keeps them (host) until upload_tables.
struct Law {
    uint32_t D = 0, ntab = 0, grid = 0;
    double G[NGR_MAX_SPECIES * NGR_MAX_SPECIES];
    double r_cut = 0, eps = 0, theta = 0;
    const double* tables = nullptr;   // D x D x ntab samples (host, or device with tables_device), or NULL: def for every pair
    bool tables_device = false;
    std::vector<double> def;          // host, ntab samples of the Newtonian short-range factor
    uint32_t kind = NGR_LAW_TABLE;    // accumulator laws: cored species mask, beta, N_perp tracking
    uint32_t cored = 0;
    uint32_t track = 1;
    double beta = 0;
    std::vector<double> eps_ab;       // D x D Plummer softening per pair (eps everywhere unless given)
    uint32_t opening = NGR_OPEN_GEOMETRIC;
    double alpha = 0;
    const double* old_acc = nullptr;  // device, previous |a| of the box's particles (relative test)
    const double* corr = nullptr;     // host, lattice correction tables (pure-tree periodic mode), or NULL
    uint32_t corr_n = 0;
};
void make_law(const ngr_force_params& fp, uint32_t D, Law& law);

// A box's tables on the device in both LDS layouts (see the walk): PAIR,
// D x D x ntab (value, slope to the next sample) with a (0, 0) last entry;
// VALUE, D x D x (ntab + 1) samples and a zero pad.
struct LawTables {
    const float2* pair = nullptr;
    const float* value = nullptr;
};
// Upload and convert the tables of every law (one conversion launch). The
// returned memory block holds all of them; release it after the last walk
// that uses them.
void* upload_tables(Context& ctx, const std::vector<Law>& laws, std::vector<LawTables>& out);

struct WalkOut {
    uint64_t pp = 0, pn = 0;
    uint64_t pnb[NGR_MAX_SPECIES] = {0, 0, 0, 0, 0, 0};   // pn by source species
    uint64_t ties = NGR_NOT_COUNTED;        // near ties (counted on request, one-box table laws)
    std::vector<uint64_t> box_pp, box_pn;   // per box
    std::vector<uint64_t> box_pnb;          // per box, NGR_MAX_SPECIES each
    double ms_walk = 0.0, ms_order = 0.0;
};
// laws and acc: one per box of the tree; acc[k] is box k's 3 x n_k output.
// Particle-mesh long-range force (pm.hip).
struct PmPlan {
    uint32_t N = 0, D = 0, p = 0, nq = 0;
    double box = 0.0, r_s = 0.0;
    uint32_t U = 0;            // unique law tables
    double* gq = nullptr;      // nq x U: phibar_t exp(-k^2 r_s^2) / (k^2 N^3)
    double mix_coef[NGR_MAX_SPECIES * NGR_MAX_SPECIES] = {};    // G_ab times the pair's factor
    uint32_t mix_table[NGR_MAX_SPECIES * NGR_MAX_SPECIES] = {}; // the pair's unique table
    double* s2 = nullptr;      // N: sinc^2(pi n / N) of each grid index
    double2* tw = nullptr;     // N / 2 twiddles exp(-2 pi i m / N)
    double2* mesh = nullptr;   // ceil(D/2) complex meshes of N^3 points
    ~PmPlan();
};
struct PmTimes {
    float deposit = 0, fft_forward = 0, green = 0, fft_inverse = 0, interp = 0;
};
void pm_create(Context& ctx, const ngr_pm_params& pp, const double* G, const double* phibar, PmPlan& pl);
void pm_force(Context& ctx, PmPlan& pl, const Tree& t, double* acc, int accumulate, PmTimes* times);
void pm_destroy(Context& ctx, PmPlan& pl);
// Exact short-range tables (short.hip).
void short_range_grid(double r_s, double r_cut, double range, uint32_t* nk, double* dk);
void short_range_tables(Context& ctx, const ngr_short_params& sp, const double* phibar, const double* f_full,
                        double* tables);
void walk_force(Context& ctx, const Tree& t, const Groups& g, const std::vector<Law>& laws,
                const std::vector<LawTables>& tables, const std::vector<double*>& acc, uint64_t* group_counts_dev,
                WalkOut& out, bool count_ties = false);

// ---- served requests (serve.hip) ----
struct Server;
Server* server_create(Context& ctx, const ngr_server_params* sp);
void server_destroy(Server* s);
uint64_t server_submit(Server& s, const ngr_request* r);
void server_tick(Server& s, ngr_tick_stats* st);
void server_status(const Server& s, uint64_t id, int* state, uint32_t* evals);
void server_take(Server& s, uint64_t id, uint64_t* lattice, double* vel, double* acc);

}  // namespace ngr
