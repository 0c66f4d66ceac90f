// The short-range tree force for callers that cannot allocate device memory.
//
// Every scratch buffer of one ngr_tree_force call (sink groups, the walk's
// queue order and control block, the tables in their on-chip layouts, the
// per-wave traversal stacks) is carved from one file-scope device array,
// `scratch`, through the context's arena mode. Each GPU holds its own copy
// of the array from the library's load until the process ends. Host code
// never uses the array's name as an address: the address on each device is
// looked up once with hipGetSymbolAddress (with that device current) and
// kept per device.
#include <cstring>
#include <mutex>

#include "ngr_internal.hpp"

#define NGR_API extern "C" __attribute__((visibility("default")))

struct ngr_context : ngr::Context {};
struct ngr_tree : ngr::Tree {};

namespace {

static __device__ __align__(256) unsigned char scratch[NGR_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_lock;
void* g_scratch[kMaxDevices] = {};

// The array's address on `device` (the current device), looked up on the
// first call for that device.
void* scratch_on(int device)
{
    if (device < 0 || device >= kMaxDevices) ngr::fail(NGR_EINVAL, "device index out of range for the static scratch");
    std::lock_guard<std::mutex> hold(g_lock);
    if (!g_scratch[device]) {
        void* p = nullptr;
        ngr::hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)", __FILE__,
                       __LINE__);
        if (!p) ngr::fail(NGR_EDEVICE, "hipGetSymbolAddress returned no address for the static scratch");
        g_scratch[device] = p;
    }
    return g_scratch[device];
}

// Leaves arena mode whatever happens inside the call.
struct ArenaScope {
    ngr::Context& c;
    ArenaScope(ngr::Context& ctx, void* base, size_t bytes) : c(ctx)
    {
        c.arena = static_cast<unsigned char*>(base);
        c.arena_size = bytes;
        c.arena_used = 0;
    }
    ~ArenaScope()
    {
        c.arena = nullptr;
        c.arena_size = c.arena_used = 0;
    }
};

}  // namespace

NGR_API ngr_status ngr_tree_force_noalloc(ngr_context* ctx, const ngr_tree* tree, const ngr_force_params* fp,
                                          double* acc, ngr_force_stats* st)
{
    if (!ctx) return NGR_EINVAL;
    if (ctx->poisoned) return NGR_EDEVICE;
    try {
        using ngr::fail;
        ngr::hip_check(hipSetDevice(ctx->device), "hipSetDevice", __FILE__, __LINE__);
        if (!tree) fail(NGR_EINVAL, "tree is NULL");
        if (tree->nbox != 1) fail(NGR_EINVAL, "the tree must hold one box");
        if (tree->n > NGR_NOALLOC_MAX_N)
            fail(NGR_EINVAL, "the no-allocation force takes at most NGR_NOALLOC_MAX_N (2^20) particles, the tree "
                             "holds " + std::to_string(tree->n));
        if (!tree->has_monopoles) fail(NGR_ESTATE, "ngr_compute_monopoles must precede the force");
        if (fp && fp->lattice_corr && tree->region > 0.0) fail(NGR_EINVAL, "lattice corrections need a periodic tree");
        uint32_t gs = ngr::check_force_params(tree->D, tree->box, fp, "");
        if (!gs) gs = ngr::chosen_group_size(*ctx, tree->n, tree->D);
        if (!acc && tree->n) fail(NGR_EINVAL, "acc is NULL");
        void* base = scratch_on(ctx->device);
        ngr::Context& c = *ctx;
        ngr::Groups g;
        std::vector<ngr::Law> laws(1);
        std::vector<ngr::LawTables> tabs;
        ngr::WalkOut wo;
        {
            ArenaScope arena(c, base, NGR_NOALLOC_SCRATCH_BYTES);
            ngr::make_groups(c, *tree, std::vector<uint32_t>{gs}, g);
            ngr::make_law(*fp, tree->D, laws[0]);
            laws[0].track = tree->track_counts ? 1u : 0u;
            if (tree->n) ngr::upload_tables(c, laws, tabs);
            ngr::walk_force(c, *tree, g, laws, tabs, std::vector<double*>{acc}, nullptr, wo, false);
            c.sync();
        }
        if (st) {
            std::memset(st, 0, sizeof *st);
            st->interactions_pp = wo.pp;
            st->interactions_pn = wo.pn;
            st->n_nodes = tree->nn;
            st->n_leaves = tree->n_leaves;
            st->n_groups = g.ng;
            st->group_size = gs;
            st->depth = tree->depth;
            for (int b = 0; b < NGR_MAX_SPECIES; ++b) st->interactions_pn_species[b] = wo.pnb[b];
            st->near_ties = NGR_NOT_COUNTED;
            st->ms_build_ingest = tree->ms_ingest;
            st->ms_build_sort = tree->ms_sort;
            st->ms_build_octree = tree->ms_octree;
            st->ms_build = (double)tree->ms_ingest + tree->ms_sort + tree->ms_octree;
            st->ms_monopoles = tree->ms_monopoles;
        }
        ctx->err.clear();
        return NGR_OK;
    } catch (const ngr::Error& e) {
        ctx->err = e.msg;
        if (e.status == NGR_EDEVICE) ctx->poisoned = true;
        return e.status;
    } catch (const std::bad_alloc&) {
        ctx->err = "host memory exhausted";
        return NGR_ENOMEM;
    }
}
