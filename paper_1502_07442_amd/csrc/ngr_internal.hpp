// Internal declarations of the ngravs-mi355x library (gfx950).
#pragma once

#include <hip/hip_runtime.h>

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
    std::string err;
    std::multimap<size_t, void*> free_blocks;     // size class -> block
    std::map<void*, size_t> live_blocks;          // block -> size class
    // persistent scratch reused across calls
    DevMem stacks;          // per-wave traversal stacks of the walk
    DevMem counters;        // small device counters (queues, statistics, flags)
    uint64_t* pinned = nullptr;                   // pinned host staging, kPinnedWords
    static constexpr size_t kPinnedWords = 64;

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

struct Tree {
    uint64_t n = 0;
    uint32_t D = 0;
    double box = 0.0;
    uint32_t leaf_size = 16;
    // particles in sorted order (species, then Morton key)
    uint64_t* X = nullptr;         // 3 x n lattice coordinates
    double* mass = nullptr;        // n
    uint32_t* perm = nullptr;      // n, sorted position -> input index
    uint64_t* keys = nullptr;      // n sorted keys
    uint64_t seg[NGR_MAX_SPECIES + 1] = {0};   // species segments (host copy)
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
    uint64_t n_leaves = 0;
    // monopoles: D x nn records {com_x, com_y, com_z (box fraction), M}
    double4* mono = nullptr;
    bool has_monopoles = false;
};

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
void build_tree(Context& ctx, const ngr_particles& p, uint32_t leaf_size, Tree& t);
void compute_monopoles(Context& ctx, Tree& t);

// ---- groups and walk (walk.hip) ----
struct Groups {
    uint64_t ng = 0;
    uint32_t size = 64;
    uint32_t* start = nullptr;     // ng
    uint32_t* count = nullptr;     // ng
    uint32_t* lo = nullptr;        // 3 x ng
    uint32_t* hi = nullptr;        // 3 x ng
    uint64_t first[NGR_MAX_SPECIES + 1] = {0};   // first group of each species (host)
    void free(Context& ctx);
};
void make_groups(Context& ctx, const Tree& t, uint32_t group_size, Groups& g);

struct Law {
    uint32_t D = 0, ntab = 0, grid = 0;
    double G[NGR_MAX_SPECIES * NGR_MAX_SPECIES];
    double r_cut = 0, eps = 0, theta = 0;
    float2* table = nullptr;       // device, D x D x ntab (value, slope to next), last = (0, 0)
    float* table_v = nullptr;      // device, D x D x (ntab + 1) samples plus a zero pad (same block)
};
void upload_law(Context& ctx, const ngr_force_params& fp, uint32_t D, Law& law);

struct WalkOut {
    uint64_t pp = 0, pn = 0;
    double ms_walk = 0.0;
};
void walk_force(Context& ctx, const Tree& t, const Groups& g, const Law& law, double* acc,
                uint64_t* group_counts_dev, WalkOut& out);

}  // namespace ngr
