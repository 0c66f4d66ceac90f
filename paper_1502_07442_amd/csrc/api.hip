// The C-ABI of libngravs: argument checks on the host before any device
// work, error statuses, and the context's stream and memory.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>

#include "ngr_internal.hpp"

#define NGR_API extern "C" __attribute__((visibility("default")))

struct ngr_context : ngr::Context {};
struct ngr_tree : ngr::Tree {};
struct ngr_server {
    ngr_context* ctx;
    ngr::Server* impl;
};
struct ngr_pm : ngr::PmPlan {};

namespace ngr {

void fail(ngr_status s, const std::string& msg) { throw Error{s, msg}; }

void hip_check(hipError_t e, const char* what, const char* file, int line)
{
    if (e == hipSuccess) return;
    char buf[512];
    std::snprintf(buf, sizeof buf, "%s failed: %s (%s:%d)", what, hipGetErrorString(e), file, line);
    fail(e == hipErrorOutOfMemory ? NGR_ENOMEM : NGR_EDEVICE, buf);
}

void* Context::alloc(size_t bytes)
{
    if (arena) {
        const size_t need = (std::max<size_t>(bytes, 1) + 255) & ~size_t(255);
        if (need > arena_size - arena_used) {
            char buf[200];
            std::snprintf(buf, sizeof buf, "the static scratch of %zu MiB is too small for this call (%zu bytes "
                                           "more needed)", arena_size >> 20, need - (arena_size - arena_used));
            fail(NGR_ENOMEM, buf);
        }
        void* p = arena + arena_used;
        arena_used += need;
        return p;
    }
    size_t cls = 256;
    while (cls < bytes) cls += cls < (1u << 20) ? cls : (cls >> 2);   // 256 B doubling, then 25 % steps
    auto it = free_blocks.lower_bound(cls);
    if (it != free_blocks.end() && it->first <= cls + (cls >> 1)) {
        void* p = it->second;
        live_blocks[p] = it->first;
        free_blocks.erase(it);
        return p;
    }
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, cls);
    if (e == hipErrorOutOfMemory) {
        (void)hipGetLastError();
        // give cached blocks back and try once more
        sync();
        for (auto& kv : free_blocks) (void)hipFree(kv.second);
        free_blocks.clear();
        e = hipMalloc(&p, cls);
        if (e == hipErrorOutOfMemory) {
            (void)hipGetLastError();
            fail(NGR_ENOMEM, "device memory exhausted");
        }
    }
    hip_check(e, "hipMalloc", __FILE__, __LINE__);
    live_blocks[p] = cls;
    return p;
}

void Context::release(void* p)
{
    if (!p || in_arena(p)) return;
    auto it = live_blocks.find(p);
    if (it == live_blocks.end()) fail(NGR_EDEVICE, "release of a block the pool does not own");
    free_blocks.emplace(it->second, p);
    live_blocks.erase(it);
}

void Context::free_all()
{
    for (auto& kv : free_blocks) (void)hipFree(kv.second);
    for (auto& kv : live_blocks) (void)hipFree(kv.first);
    free_blocks.clear();
    live_blocks.clear();
}

void Context::ensure(DevMem& m, size_t bytes)
{
    if (m.bytes >= bytes) return;
    if (arena) fail(NGR_EDEVICE, "a persistent buffer would grow in arena mode");
    release(m.p);
    m.p = alloc(bytes);
    m.bytes = bytes;
}

void Context::stage(const char* what)
{
    if (trace) {
        const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_created).count();
        std::fprintf(stderr, "[ngravs %10.3f ms] %s\n", ms, what);
        std::fflush(stderr);
    }
}

void Context::read_words(uint64_t* host, const void* dev, size_t words)
{
    if (words > kPinnedWords) fail(NGR_EINVAL, "read_words: too many words");
    hip_check(hipMemcpyAsync(pinned, dev, words * sizeof(uint64_t), hipMemcpyDeviceToHost, stream),
              "hipMemcpyAsync", __FILE__, __LINE__);
    sync();
    std::memcpy(host, pinned, words * sizeof(uint64_t));
}

void Context::write_words(void* dev, const uint64_t* host, size_t words)
{
    if (words > kPinnedWords) fail(NGR_EINVAL, "write_words: too many words");
    sync();
    std::memcpy(pinned, host, words * sizeof(uint64_t));
    hip_check(hipMemcpyAsync(dev, pinned, words * sizeof(uint64_t), hipMemcpyHostToDevice, stream),
              "hipMemcpyAsync", __FILE__, __LINE__);
    sync();
}

void Context::to_host(void* host, const void* dev, size_t bytes)
{
    if (!bytes) return;
    sync();
    hip_check(hipMemcpy(host, dev, bytes, hipMemcpyDeviceToHost), "hipMemcpy", __FILE__, __LINE__);
}

void Context::to_device(void* dev, const void* host, size_t bytes)
{
    if (!bytes) return;
    sync();
    hip_check(hipMemcpy(dev, host, bytes, hipMemcpyHostToDevice), "hipMemcpy", __FILE__, __LINE__);
}

void Context::sync() { hip_check(hipStreamSynchronize(stream), "hipStreamSynchronize", __FILE__, __LINE__); }

hipEvent_t Context::event(int k)
{
    if (!ev[k]) hip_check(hipEventCreate(&ev[k]), "hipEventCreate", __FILE__, __LINE__);
    return ev[k];
}

float Context::elapsed(int k0, int k1)
{
    hip_check(hipEventSynchronize(ev[k1]), "hipEventSynchronize", __FILE__, __LINE__);
    float ms = 0.0f;
    hip_check(hipEventElapsedTime(&ms, ev[k0], ev[k1]), "hipEventElapsedTime", __FILE__, __LINE__);
    return ms;
}

}  // namespace ngr

namespace ngr {

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }


// Checks of one box's force parameters (D species, box side); returns the
// group size (0 resolved by the caller's rule).
uint32_t check_force_params(uint32_t D, double box, const ngr_force_params* fp, const std::string& where)
{
    using ngr::fail;
    if (!fp) fail(NGR_EINVAL, where + "force params are NULL");
    if (!fp->G) fail(NGR_EINVAL, where + "G is NULL");
    if (fp->ntab < 2) fail(NGR_EINVAL, where + "ntab must be >= 2");
    if ((uint64_t)D * fp->ntab > NGR_MAX_TABLE) fail(NGR_EINVAL, where + "D * ntab exceeds NGR_MAX_TABLE");
    if (fp->grid != NGR_GRID_R && fp->grid != NGR_GRID_R2) fail(NGR_EINVAL, where + "grid must be NGR_GRID_R or NGR_GRID_R2");
    if (!ngr::finite_pos(fp->r_cut)) fail(NGR_EINVAL, where + "r_cut must be finite and > 0");
    if (fp->lattice_corr) {
        if (!(fp->r_cut >= 0.8660254037844387 * box)) fail(NGR_EINVAL, where + "with lattice corrections r_cut must reach sqrt(3)/2 box");
        if (fp->corr_n < 1 || fp->corr_n > 512) fail(NGR_EINVAL, where + "corr_n must be in 1..512");
        if (fp->law != NGR_LAW_TABLE) fail(NGR_EINVAL, where + "lattice corrections take the table laws only");
        const uint64_t m = fp->corr_n + 1ull, cnt = (uint64_t)D * D * m * m * m * 3ull;
        for (uint64_t k = 0; k < cnt; ++k)
            if (!std::isfinite(fp->lattice_corr[k])) fail(NGR_EINVAL, where + "a lattice correction is not finite");
    } else if (!(fp->r_cut < 0.5 * box)) {
        fail(NGR_EINVAL, where + "r_cut must be < box / 2");
    }
    if (!(std::isfinite(fp->eps) && fp->eps >= 0.0)) fail(NGR_EINVAL, where + "eps must be finite and >= 0");
    // the pair factor (r^2 + eps^2)^(-3/2) is taken in float32 in units of the box
    if (fp->eps > 0.0 && fp->eps < 1e-12 * box) fail(NGR_EINVAL, where + "eps must be 0 or at least 1e-12 box");
    if (!ngr::finite_pos(fp->theta)) fail(NGR_EINVAL, where + "theta must be finite and > 0");
    if (!fp->tables && !ngr::finite_pos(fp->r_s)) fail(NGR_EINVAL, where + "r_s must be finite and > 0 when tables is NULL");
    const uint32_t gs = fp->group_size;
    if (gs != 0 && gs != 16 && gs != 32 && gs != 64) fail(NGR_EINVAL, where + "group_size must be 16, 32 or 64 (or 0)");
    if (fp->law != NGR_LAW_TABLE && fp->law != NGR_LAW_ACCUMULATOR)
        fail(NGR_EINVAL, where + "law must be NGR_LAW_TABLE or NGR_LAW_ACCUMULATOR");
    if (fp->law == NGR_LAW_ACCUMULATOR) {
        if (fp->cored >> D) fail(NGR_EINVAL, where + "cored names a species >= D");
        if (!ngr::finite_pos(fp->beta)) fail(NGR_EINVAL, where + "beta must be finite and > 0");
    }
    for (uint32_t k = 0; k < D * D; ++k)
        if (!std::isfinite(fp->G[k])) fail(NGR_EINVAL, where + "G has a non-finite entry");
    if (fp->opening != NGR_OPEN_GEOMETRIC && fp->opening != NGR_OPEN_RELATIVE)
        fail(NGR_EINVAL, where + "opening must be NGR_OPEN_GEOMETRIC or NGR_OPEN_RELATIVE");
    if (fp->opening == NGR_OPEN_RELATIVE) {
        if (!ngr::finite_pos(fp->alpha)) fail(NGR_EINVAL, where + "alpha must be finite and > 0");
        if (!fp->old_acc) fail(NGR_EINVAL, where + "old_acc is NULL");
    }
    if (fp->eps_ab)
        for (uint32_t k = 0; k < D * D; ++k)
            if (!(std::isfinite(fp->eps_ab[k]) && fp->eps_ab[k] >= 0.0) ||
                (fp->eps_ab[k] > 0.0 && fp->eps_ab[k] < 1e-12 * box))
                fail(NGR_EINVAL, where + "eps_ab entries must be finite and 0 or at least 1e-12 box");
    if (fp->tables && !fp->tables_on_device)   // device tables are checked on the device
        for (uint64_t k = 0; k < (uint64_t)D * D * fp->ntab; ++k)
            if (!std::isfinite(fp->tables[k])) fail(NGR_EINVAL, where + "a table entry is not finite");
    return gs;
}

// The autotuner's class of a box: its D and floor(log2 n).
uint64_t size_class(uint64_t n, uint32_t D)
{
    uint32_t l = 0;
    while (l < 63 && (2ull << l) <= n) ++l;
    return ((uint64_t)D << 8) | l;
}

// Group size of a box when the caller leaves it to the library (0): what
// ngr_autotune measured fastest for the box's class on this context, else
// 32. With groups of at most 32 (16) sinks evaluating 2 (4) records per lane
// slot, 32 gave the shortest walk on the many-box workload (256 clustered
// boxes of 2^12..2^18 particles, D 1..4: walk 41 ms at 32 against 45 ms at
// 16 and 64).
uint32_t chosen_group_size(const Context& ctx, uint64_t n, uint32_t D)
{
    auto it = ctx.tuned.find(size_class(n, D));
    return it == ctx.tuned.end() ? 32u : it->second;
}

void check_particles(const ngr_particles* p, const ngr_tree_params* tp, const std::string& where, ngr::BoxIn& b)
{
    using ngr::fail;
    if (!p) fail(NGR_EINVAL, where + "particles are NULL");
    if (p->D < 1 || p->D > NGR_MAX_SPECIES) fail(NGR_EINVAL, where + "D must be in 1..6");
    if (!ngr::finite_pos(p->box)) fail(NGR_EINVAL, where + "box must be finite and > 0");
    if (p->n >= (1ull << 32) - 1) fail(NGR_EINVAL, where + "n must be < 2^32 - 1");
    const uint32_t B = tp && tp->leaf_size ? tp->leaf_size : 16;
    if (B > 64) fail(NGR_EINVAL, where + "leaf_size must be in 1..64");
    const uint32_t order = tp ? tp->key_order : NGR_KEY_MORTON;
    if (order != NGR_KEY_MORTON && order != NGR_KEY_HILBERT)
        fail(NGR_EINVAL, where + "key_order must be NGR_KEY_MORTON or NGR_KEY_HILBERT");
    if (p->n) {
        if (!p->species || !p->mass) fail(NGR_EINVAL, where + "species or mass is NULL");
        if ((p->pos == nullptr) == (p->lattice == nullptr)) fail(NGR_EINVAL, where + "exactly one of pos and lattice must be set");
    }
    b.n = p->n;
    b.D = p->D;
    b.box = p->box;
    b.region = 0.0;
    if (tp && tp->non_periodic) {
        // a non-periodic box sits in the first quarter of a lattice four
        // times its size: every difference is then below half that lattice
        if (p->n && !p->pos) fail(NGR_EINVAL, where + "a non-periodic box takes positions, not lattice coordinates");
        b.region = p->box;
        b.box = 4.0 * p->box;
    }
    b.leaf_size = B;
    b.key_order = order;
    b.pos = p->pos;
    b.lattice = p->lattice;
    b.species = p->species;
    b.mass = p->mass;
}

}  // namespace ngr

namespace {

void free_tree_memory(ngr::Context& c, ngr::Tree& t) { ngr::free_tree(c, t); }

template <class F>
ngr_status guarded(ngr_context* ctx, F&& f)
{
    if (!ctx) return NGR_EINVAL;
    if (ctx->poisoned) return NGR_EDEVICE;
    try {
        ngr::hip_check(hipSetDevice(ctx->device), "hipSetDevice", __FILE__, __LINE__);
        f();
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

ngr_status force_impl(ngr_context* ctx, const ngr_tree* tree, const ngr_force_params* fp, double* acc,
                      ngr_force_stats* st, uint64_t* group_counts_host, bool count_ties)
{
    return guarded(ctx, [&] {
        using ngr::fail;
        if (!tree) fail(NGR_EINVAL, "tree is NULL");
        if (!tree->has_monopoles) fail(NGR_ESTATE, "ngr_compute_monopoles must precede ngr_tree_force");
        if (fp && fp->lattice_corr && tree->region > 0.0) fail(NGR_EINVAL, "lattice corrections need a periodic tree");
        uint32_t gs = ngr::check_force_params(tree->D, tree->box, fp, "");
        if (!gs) gs = ngr::chosen_group_size(*ctx, tree->n, tree->D);
        if (!acc && tree->n) fail(NGR_EINVAL, "acc is NULL");
        ngr::Context& c = *ctx;
        ngr::Groups g;
        std::vector<ngr::Law> laws(1);
        std::vector<ngr::LawTables> tabs;
        void* tab_block = nullptr;
        ngr::WalkOut wo;
        uint64_t* gc = nullptr;
        hipEvent_t e0, e1;
        ngr::hip_check(hipEventCreate(&e0), "hipEventCreate", __FILE__, __LINE__);
        ngr::hip_check(hipEventCreate(&e1), "hipEventCreate", __FILE__, __LINE__);
        try {
            ngr::hip_check(hipEventRecord(e0, c.stream), "hipEventRecord", __FILE__, __LINE__);
            ngr::make_groups(c, *tree, std::vector<uint32_t>{gs}, g);
            ngr::hip_check(hipEventRecord(e1, c.stream), "hipEventRecord", __FILE__, __LINE__);
            ngr::make_law(*fp, tree->D, laws[0]);
            laws[0].track = tree->track_counts ? 1u : 0u;
            if (tree->n) tab_block = ngr::upload_tables(c, laws, tabs);
            if (group_counts_host && g.ng) gc = static_cast<uint64_t*>(c.alloc(g.ng * 4 * sizeof(uint64_t)));
            ngr::walk_force(c, *tree, g, laws, tabs, std::vector<double*>{acc}, gc, wo, count_ties);
            if (gc) c.to_host(group_counts_host, gc, g.ng * 4 * sizeof(uint64_t));
            c.sync();
        } catch (...) {
            c.release(gc);
            c.release(tab_block);
            g.free(c);
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            throw;
        }
        float ms_groups = 0.0f;
        ngr::hip_check(hipEventElapsedTime(&ms_groups, e0, e1), "hipEventElapsedTime", __FILE__, __LINE__);
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (st) {
            std::memset(st, 0, sizeof *st);
            st->interactions_pp = wo.pp;
            st->interactions_pn = wo.pn;
            st->n_nodes = tree->nn;
            st->n_leaves = tree->n_leaves;
            st->n_groups = g.ng;
            st->group_size = gs;
            st->depth = tree->depth;
            st->ms_groups = ms_groups + wo.ms_order;
            st->ms_walk = wo.ms_walk;
            for (int b = 0; b < NGR_MAX_SPECIES; ++b) st->interactions_pn_species[b] = wo.pnb[b];
            st->near_ties = wo.ties;
            st->ms_build_ingest = tree->ms_ingest;
            st->ms_build_sort = tree->ms_sort;
            st->ms_build_octree = tree->ms_octree;
            st->ms_build = (double)tree->ms_ingest + tree->ms_sort + tree->ms_octree;
            st->ms_monopoles = tree->ms_monopoles;
        }
        c.release(gc);
        c.release(tab_block);
        g.free(c);
    });
}

}  // namespace

NGR_API ngr_status ngr_context_create(int device, void* hip_stream, ngr_context** out)
{
    if (!out) return NGR_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return device < 0 ? NGR_EINVAL : NGR_EDEVICE;
    ngr_context* c = new (std::nothrow) ngr_context();
    if (!c) return NGR_ENOMEM;
    c->device = device;
    try {
        ngr::hip_check(hipSetDevice(device), "hipSetDevice", __FILE__, __LINE__);
        hipDeviceProp_t prop;
        ngr::hip_check(hipGetDeviceProperties(&prop, device), "hipGetDeviceProperties", __FILE__, __LINE__);
        c->num_cu = prop.multiProcessorCount;
        c->stream = static_cast<hipStream_t>(hip_stream);   // NULL: the default stream
        c->own_stream = false;
        ngr::hip_check(hipHostMalloc(reinterpret_cast<void**>(&c->pinned), ngr::Context::kPinnedWords * sizeof(uint64_t),
                                     hipHostMallocDefault),
                       "hipHostMalloc", __FILE__, __LINE__);
        const char* tr = std::getenv("NGR_TRACE");
        c->trace = tr && tr[0] && tr[0] != '0';
        c->lds_per_block = prop.sharedMemPerBlock;
    } catch (const ngr::Error& e) {
        delete c;
        return e.status;
    }
    *out = c;
    return NGR_OK;
}

NGR_API void ngr_context_destroy(ngr_context* ctx)
{
    if (!ctx) return;
    if (!ctx->poisoned) (void)hipStreamSynchronize(ctx->stream);
    for (hipEvent_t& e : ctx->ev)
        if (e) (void)hipEventDestroy(e);
    ctx->free_all();
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
}

NGR_API const char* ngr_last_error(const ngr_context* ctx) { return ctx ? ctx->err.c_str() : "no context"; }

NGR_API ngr_status ngr_tree_build(ngr_context* ctx, const ngr_particles* p, const ngr_tree_params* tp, ngr_tree** out)
{
    if (out) *out = nullptr;
    return guarded(ctx, [&] {
        using ngr::fail;
        if (!p || !out) fail(NGR_EINVAL, "particles or out is NULL");
        std::vector<ngr::BoxIn> boxes(1);
        ngr::check_particles(p, tp, "", boxes[0]);
        ngr_tree* t = new ngr_tree();
        try {
            ngr::build_forest(*ctx, boxes, *t, true);
            ctx->sync();
        } catch (...) {
            try {
                free_tree_memory(*ctx, *t);
            } catch (...) {
            }
            delete t;
            throw;
        }
        *out = t;
    });
}

NGR_API ngr_status ngr_compute_monopoles(ngr_context* ctx, ngr_tree* tree, int track_counts)
{
    return guarded(ctx, [&] {
        if (!tree) ngr::fail(NGR_EINVAL, "tree is NULL");
        ngr::hip_check(hipEventRecord(ctx->event(4), ctx->stream), "hipEventRecord", __FILE__, __LINE__);
        ngr::compute_monopoles(*ctx, *tree);
        ngr::hip_check(hipEventRecord(ctx->event(5), ctx->stream), "hipEventRecord", __FILE__, __LINE__);
        tree->track_counts = track_counts != 0;
        ctx->sync();
        tree->ms_monopoles = ctx->elapsed(4, 5);
    });
}

NGR_API ngr_status ngr_tree_force(ngr_context* ctx, const ngr_tree* tree, const ngr_force_params* fp, double* acc,
                                  ngr_force_stats* st)
{
    return force_impl(ctx, tree, fp, acc, st, nullptr, false);
}

NGR_API ngr_status ngr_tree_force_counts(ngr_context* ctx, const ngr_tree* tree, const ngr_force_params* fp,
                                         double* acc, ngr_force_stats* st, uint64_t* group_counts)
{
    return force_impl(ctx, tree, fp, acc, st, group_counts, true);
}

NGR_API ngr_status ngr_tree_free(ngr_context* ctx, ngr_tree* tree)
{
    if (!tree) return NGR_OK;
    if (!ctx) return NGR_EINVAL;
    ngr_status s = guarded(ctx, [&] {
        free_tree_memory(*ctx, *tree);
        ctx->sync();
    });
    delete tree;
    return s;
}

NGR_API ngr_status ngr_tree_info(const ngr_tree* tree, uint64_t* n, uint64_t* n_nodes, uint32_t* D, uint32_t* depth)
{
    if (!tree) return NGR_EINVAL;
    if (n) *n = tree->n;
    if (n_nodes) *n_nodes = tree->nn;
    if (D) *D = tree->D;
    if (depth) *depth = tree->depth;
    return NGR_OK;
}

namespace {
template <class T>
void copy_out(ngr::Context& c, T* host, const T* dev, uint64_t count)
{
    if (host && count) c.to_host(host, dev, count * sizeof(T));
}
}  // namespace

NGR_API ngr_status ngr_tree_export(ngr_context* ctx, const ngr_tree* tree, uint32_t* perm, uint64_t* keys,
                                   uint64_t* lattice, uint8_t* level, uint64_t* prefix, int32_t* parent,
                                   int32_t* first_child, uint8_t* n_child, uint32_t* start, uint32_t* count)
{
    return guarded(ctx, [&] {
        if (!tree) ngr::fail(NGR_EINVAL, "tree is NULL");
        const uint64_t n = tree->n, nn = tree->nn, D = tree->D;
        copy_out(*ctx, perm, tree->perm, n);
        copy_out(*ctx, keys, tree->keys, n);
        copy_out(*ctx, lattice, tree->X, 3 * n);
        copy_out(*ctx, level, tree->level, nn);
        copy_out(*ctx, prefix, tree->prefix, nn);
        copy_out(*ctx, parent, tree->parent, nn);
        copy_out(*ctx, first_child, tree->first_child, nn);
        copy_out(*ctx, n_child, tree->n_child, nn);
        std::vector<uint32_t> tmp;
        for (int which = 0; which < 2; ++which) {
            uint32_t* dst = which ? count : start;
            if (!dst || !nn) continue;
            tmp.resize(nn * D);
            copy_out(*ctx, tmp.data(), which ? tree->count : tree->start, nn * D);
            ctx->sync();
            for (uint64_t i = 0; i < nn; ++i)
                for (uint64_t b = 0; b < D; ++b) dst[b * nn + i] = tmp[i * D + b];
        }
        ctx->sync();
    });
}

NGR_API ngr_status ngr_monopoles_export(ngr_context* ctx, const ngr_tree* tree, double* M, double* com)
{
    return guarded(ctx, [&] {
        if (!tree) ngr::fail(NGR_EINVAL, "tree is NULL");
        if (!tree->has_monopoles) ngr::fail(NGR_ESTATE, "no monopoles");
        const uint64_t nn = tree->nn, D = tree->D;
        std::vector<double4> h(nn * D);
        copy_out(*ctx, h.data(), tree->mono, nn * D);
        ctx->sync();
        for (uint64_t b = 0; b < D; ++b)
            for (uint64_t i = 0; i < nn; ++i) {
                const double4 r = h[b * nn + i];
                if (M) M[b * nn + i] = r.w;
                if (com) {
                    com[(b * 3 + 0) * nn + i] = r.x * tree->box;
                    com[(b * 3 + 1) * nn + i] = r.y * tree->box;
                    com[(b * 3 + 2) * nn + i] = r.z * tree->box;
                }
            }
    });
}

NGR_API ngr_status ngr_groups_export(ngr_context* ctx, const ngr_tree* tree, uint32_t group_size, uint64_t* n_groups,
                                     uint8_t* species, uint32_t* start, uint32_t* count, uint32_t* lo, uint32_t* hi)
{
    return guarded(ctx, [&] {
        if (!tree || !n_groups) ngr::fail(NGR_EINVAL, "tree or n_groups is NULL");
        uint32_t gs = group_size ? group_size : ngr::chosen_group_size(*ctx, tree->n, tree->D);
        if (gs != 16 && gs != 32 && gs != 64) ngr::fail(NGR_EINVAL, "group_size must be 16, 32 or 64 (or 0)");
        ngr::Groups g;
        try {
            ngr::make_groups(*ctx, *tree, std::vector<uint32_t>{gs}, g);
            *n_groups = g.ng;
            if (species) {
                for (uint32_t a = 0; a < tree->D; ++a)
                    for (uint64_t k = g.first[a]; k < g.first[a + 1]; ++k) species[k] = (uint8_t)a;
                copy_out(*ctx, start, g.start, g.ng);
                copy_out(*ctx, count, g.count, g.ng);
                copy_out(*ctx, lo, g.lo, 3 * g.ng);
                copy_out(*ctx, hi, g.hi, 3 * g.ng);
            }
            ctx->sync();
        } catch (...) {
            g.free(*ctx);
            throw;
        }
        g.free(*ctx);
        ctx->sync();
    });
}

NGR_API ngr_status ngr_batch_build_force(ngr_context* ctx, uint32_t nbox, const ngr_box* boxes, ngr_batch_stats* st,
                                         ngr_force_stats* per_box)
{
    return guarded(ctx, [&] {
        using ngr::fail;
        if (!boxes) fail(NGR_EINVAL, "boxes is NULL");
        if (nbox == 0 || nbox > 65535) fail(NGR_EINVAL, "nbox must be in 1..65535");
        std::vector<ngr::BoxIn> in(nbox);
        std::vector<uint32_t> gs(nbox);
        std::vector<ngr::Law> laws(nbox);
        std::vector<double*> acc(nbox);
        for (uint32_t k = 0; k < nbox; ++k) {
            const std::string where = "box " + std::to_string(k) + ": ";
            ngr::check_particles(&boxes[k].particles, &boxes[k].tree, where, in[k]);
            if (boxes[k].force.lattice_corr && in[k].region > 0.0)
                ngr::fail(NGR_EINVAL, where + "lattice corrections need a periodic box");
            gs[k] = ngr::check_force_params(in[k].D, in[k].box, &boxes[k].force, where);
            if (!gs[k]) gs[k] = ngr::chosen_group_size(*ctx, in[k].n, in[k].D);
            if (!boxes[k].acc && in[k].n) fail(NGR_EINVAL, where + "acc is NULL");
            if (boxes[k].force.grid != boxes[0].force.grid) fail(NGR_EINVAL, where + "the boxes must share the table grid");
            acc[k] = boxes[k].acc;
        }
        for (uint32_t k = 0; k < nbox; ++k) ngr::make_law(boxes[k].force, in[k].D, laws[k]);
        ngr::Context& c = *ctx;
        ngr::Tree t;
        ngr::Groups g;
        ngr::WalkOut wo;
        std::vector<ngr::LawTables> tabs;
        void* tab_block = nullptr;
        std::vector<uint64_t> bnodes, bleaves;
        std::vector<uint32_t> bdepth;
        hipEvent_t ev[4];
        for (auto& e : ev) ngr::hip_check(hipEventCreate(&e), "hipEventCreate", __FILE__, __LINE__);
        auto destroy = [&] {
            for (auto& e : ev) (void)hipEventDestroy(e);
        };
        try {
            ngr::hip_check(hipEventRecord(ev[0], c.stream), "hipEventRecord", __FILE__, __LINE__);
            ngr::build_forest(c, in, t);
            ngr::hip_check(hipEventRecord(ev[1], c.stream), "hipEventRecord", __FILE__, __LINE__);
            ngr::compute_monopoles(c, t);
            ngr::hip_check(hipEventRecord(ev[2], c.stream), "hipEventRecord", __FILE__, __LINE__);
            ngr::make_groups(c, t, gs, g);
            ngr::hip_check(hipEventRecord(ev[3], c.stream), "hipEventRecord", __FILE__, __LINE__);
            tab_block = ngr::upload_tables(c, laws, tabs);
            ngr::walk_force(c, t, g, laws, tabs, acc, nullptr, wo);
            if (per_box) ngr::box_node_counts(c, t, bnodes, bleaves, bdepth);
            c.sync();
        } catch (...) {
            try {
                ngr::free_tree(c, t);
                g.free(c);
                c.release(tab_block);
            } catch (...) {
            }
            destroy();
            throw;
        }
        float ms[3] = {0, 0, 0};
        for (int i = 0; i < 3; ++i)
            ngr::hip_check(hipEventElapsedTime(&ms[i], ev[i], ev[i + 1]), "hipEventElapsedTime", __FILE__, __LINE__);
        destroy();
        if (st) {
            std::memset(st, 0, sizeof *st);
            st->n_particles = t.n;
            st->n_nodes = t.nn;
            st->n_groups = g.ng;
            st->interactions_pp = wo.pp;
            st->interactions_pn = wo.pn;
            st->ms_build = ms[0];
            st->ms_monopoles = ms[1];
            st->ms_groups = ms[2] + wo.ms_order;
            st->ms_walk = wo.ms_walk;
        }
        if (per_box) {
            const uint32_t D = t.D;
            for (uint32_t k = 0; k < nbox; ++k) {
                ngr_force_stats& b = per_box[k];
                std::memset(&b, 0, sizeof b);
                b.interactions_pp = wo.box_pp[k];
                b.interactions_pn = wo.box_pn[k];
                b.n_nodes = bnodes[k];
                b.n_leaves = bleaves[k];
                b.n_groups = g.first.empty() ? 0 : g.first[(size_t)(k + 1) * D] - g.first[(size_t)k * D];
                b.group_size = gs[k];
                b.depth = bdepth[k];
                for (int q = 0; q < NGR_MAX_SPECIES; ++q) b.interactions_pn_species[q] = wo.box_pnb[(size_t)k * NGR_MAX_SPECIES + q];
                b.near_ties = NGR_NOT_COUNTED;
            }
        }
        ngr::free_tree(c, t);
        g.free(c);
        c.release(tab_block);
    });
}

NGR_API ngr_status ngr_short_range_grid(double r_s, double r_cut, double range, uint32_t* nk, double* dk)
{
    if (!nk || !dk || !ngr::finite_pos(r_s) || !ngr::finite_pos(r_cut) || !(std::isfinite(range) && range >= 0.0))
        return NGR_EINVAL;
    const double period = r_cut + 12.5 * r_s + 37.0 * range;
    if (std::sqrt(17.0 * std::log(10.0)) / r_s / (2.0 * M_PI / period) > (double)(1u << 24)) return NGR_EINVAL;
    ngr::short_range_grid(r_s, r_cut, range, nk, dk);
    return NGR_OK;
}

NGR_API ngr_status ngr_short_range_tables(ngr_context* ctx, const ngr_short_params* sp, const double* phibar,
                                          const double* f_full, double* tables)
{
    return guarded(ctx, [&] {
        using ngr::fail;
        if (!sp) fail(NGR_EINVAL, "short-range params are NULL");
        if (sp->D < 1 || sp->D > NGR_MAX_SPECIES) fail(NGR_EINVAL, "D must be in 1..6");
        if (sp->ntab < 2) fail(NGR_EINVAL, "ntab must be >= 2");
        if (sp->grid != NGR_GRID_R && sp->grid != NGR_GRID_R2) fail(NGR_EINVAL, "grid must be NGR_GRID_R or NGR_GRID_R2");
        if (!ngr::finite_pos(sp->r_s)) fail(NGR_EINVAL, "r_s must be finite and > 0");
        if (!ngr::finite_pos(sp->r_cut)) fail(NGR_EINVAL, "r_cut must be finite and > 0");
        if (!ngr::finite_pos(sp->dk)) fail(NGR_EINVAL, "dk must be finite and > 0");
        if (sp->nk < 2 || sp->nk > (1u << 24)) fail(NGR_EINVAL, "nk must be in 2..2^24");
        if (!phibar || !f_full || !tables) fail(NGR_EINVAL, "phibar, f_full and tables must not be NULL");
        const uint64_t pairs = (uint64_t)sp->D * sp->D;
        for (uint64_t k = 0; k < pairs * sp->nk; ++k)
            if (!std::isfinite(phibar[k])) fail(NGR_EINVAL, "phibar has a non-finite entry");
        for (uint64_t k = 0; k < pairs * sp->ntab; ++k)
            if (!std::isfinite(f_full[k])) fail(NGR_EINVAL, "f_full has a non-finite entry");
        ngr::short_range_tables(*ctx, *sp, phibar, f_full, tables);
    });
}

NGR_API ngr_status ngr_autotune(ngr_context* ctx, uint32_t nbox, const ngr_box* boxes, ngr_tune_stats* st)
{
    return guarded(ctx, [&] {
        using ngr::fail;
        const auto t0 = std::chrono::steady_clock::now();
        if (!boxes) fail(NGR_EINVAL, "boxes is NULL");
        if (nbox == 0 || nbox > 65535) fail(NGR_EINVAL, "nbox must be in 1..65535");
        std::vector<ngr::BoxIn> in(nbox);
        for (uint32_t k = 0; k < nbox; ++k) {
            const std::string where = "box " + std::to_string(k) + ": ";
            ngr::check_particles(&boxes[k].particles, &boxes[k].tree, where, in[k]);
            if (boxes[k].force.lattice_corr && in[k].region > 0.0)
                fail(NGR_EINVAL, where + "lattice corrections need a periodic box");
            (void)ngr::check_force_params(in[k].D, in[k].box, &boxes[k].force, where);
            if (boxes[k].force.grid != boxes[0].force.grid) fail(NGR_EINVAL, where + "the boxes must share the table grid");
        }
        // up to two boxes of each class (D, floor(log2 n)), in input order
        std::map<uint64_t, std::vector<uint32_t>> cls;
        for (uint32_t k = 0; k < nbox; ++k) {
            if (in[k].n == 0) continue;
            auto& v = cls[ngr::size_class(in[k].n, in[k].D)];
            if (v.size() < 2) v.push_back(k);
        }
        ngr::Context& c = *ctx;
        uint32_t launches = 0;
        const uint32_t cand[3] = {16, 32, 64};
        for (auto& kv : cls) {
            // the class's samples, repeated until they hold 2^21 particles:
            // enough groups to fill the device, so that the time measured is
            // the class's throughput in a batch and not one group's latency
            std::vector<ngr::BoxIn> sub;
            std::vector<ngr::Law> laws;
            std::vector<double*> accs;
            std::vector<double*> scratch;
            uint64_t held = 0;
            while (held < (1ull << 21) && sub.size() < 4096)
                for (uint32_t k : kv.second) {
                    sub.push_back(in[k]);
                    laws.emplace_back();
                    ngr::make_law(boxes[k].force, in[k].D, laws.back());
                    double* a = static_cast<double*>(c.alloc(3 * in[k].n * sizeof(double)));
                    scratch.push_back(a);
                    accs.push_back(a);
                    held += in[k].n;
                }
            ngr::Tree t;
            std::vector<ngr::LawTables> tabs;
            void* tab_block = nullptr;
            double best = 0.0;
            uint32_t best_gs = 32;
            try {
                ngr::build_forest(c, sub, t);
                ngr::compute_monopoles(c, t);
                tab_block = ngr::upload_tables(c, laws, tabs);
                for (uint32_t gi = 0; gi < 3; ++gi) {
                    // the groups and the walk (both grow with the group count), the better of two runs
                    double ms = 0.0;
                    for (int rep = 0; rep < 2; ++rep) {
                        c.sync();
                        const auto w0 = std::chrono::steady_clock::now();
                        ngr::Groups g;
                        ngr::WalkOut wo;
                        ngr::make_groups(c, t, std::vector<uint32_t>(sub.size(), cand[gi]), g);
                        ngr::walk_force(c, t, g, laws, tabs, accs, nullptr, wo);
                        c.sync();
                        const double e = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - w0).count();
                        g.free(c);
                        ms = rep == 0 ? e : std::min(ms, e);
                        ++launches;
                    }
                    if (gi == 0 || ms < best) {
                        best = ms;
                        best_gs = cand[gi];
                    }
                }
            } catch (...) {
                try {
                    ngr::free_tree(c, t);
                    c.release(tab_block);
                    for (double* a : scratch) c.release(a);
                } catch (...) {
                }
                throw;
            }
            ngr::free_tree(c, t);
            c.release(tab_block);
            for (double* a : scratch) c.release(a);
            c.tuned[kv.first] = best_gs;
        }
        if (st) {
            st->classes = (uint32_t)cls.size();
            st->launches = launches;
            st->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        }
    });
}

NGR_API ngr_status ngr_tuned_group_size(const ngr_context* ctx, uint64_t n, uint32_t D, uint32_t* group_size)
{
    if (!ctx || !group_size || D < 1 || D > NGR_MAX_SPECIES) return NGR_EINVAL;
    *group_size = ngr::chosen_group_size(*ctx, n, D);
    return NGR_OK;
}

NGR_API ngr_status ngr_pm_create(ngr_context* ctx, const ngr_pm_params* pp, const double* G, const double* phibar,
                                 ngr_pm** out)
{
    return guarded(ctx, [&] {
        using ngr::fail;
        if (!out) fail(NGR_EINVAL, "out is NULL");
        *out = nullptr;
        if (!pp) fail(NGR_EINVAL, "PM params are NULL");
        if (pp->N < 16 || pp->N > 1024 || (pp->N & (pp->N - 1))) fail(NGR_EINVAL, "N must be a power of two in 16..1024");
        if (pp->D < 1 || pp->D > NGR_MAX_SPECIES) fail(NGR_EINVAL, "D must be in 1..6");
        if (!ngr::finite_pos(pp->box)) fail(NGR_EINVAL, "box must be finite and > 0");
        if (!ngr::finite_pos(pp->r_s)) fail(NGR_EINVAL, "r_s must be finite and > 0");
        if (!G || !phibar) fail(NGR_EINVAL, "G and phibar must not be NULL");
        const uint64_t pairs = (uint64_t)pp->D * pp->D, nq = 3ull * (pp->N / 2) * (pp->N / 2) + 1;
        for (uint64_t k = 0; k < pairs; ++k)
            if (!std::isfinite(G[k])) fail(NGR_EINVAL, "G has a non-finite entry");
        for (uint64_t k = 0; k < pairs * nq; ++k)
            if (!std::isfinite(phibar[k])) fail(NGR_EINVAL, "phibar has a non-finite entry");
        ngr_pm* pm = new ngr_pm();
        try {
            ngr::pm_create(*ctx, *pp, G, phibar, *pm);
        } catch (...) {
            try {
                ngr::pm_destroy(*ctx, *pm);
            } catch (...) {
            }
            delete pm;
            throw;
        }
        *out = pm;
    });
}

NGR_API ngr_status ngr_pm_force(ngr_context* ctx, ngr_pm* pm, const ngr_tree* tree, double* acc, int accumulate,
                                ngr_pm_stats* st)
{
    return guarded(ctx, [&] {
        using ngr::fail;
        if (!pm || !tree) fail(NGR_EINVAL, "pm and tree must not be NULL");
        if (tree->nbox != 1) fail(NGR_EINVAL, "the tree must hold one box");
        if (tree->D != pm->D) fail(NGR_EINVAL, "the tree's D differs from the plan's");
        if (tree->region > 0.0) fail(NGR_EINVAL, "a non-periodic tree takes no PM force");
        if (tree->box != pm->box) fail(NGR_EINVAL, "the tree's box differs from the plan's");
        if (!acc && tree->n) fail(NGR_EINVAL, "acc is NULL");
        ngr::PmTimes tm;
        ngr::pm_force(*ctx, *pm, *tree, acc, accumulate, &tm);
        if (st) {
            st->ms_deposit = tm.deposit;
            st->ms_fft_forward = tm.fft_forward;
            st->ms_green = tm.green;
            st->ms_fft_inverse = tm.fft_inverse;
            st->ms_interp = tm.interp;
        }
    });
}

NGR_API ngr_status ngr_pm_destroy(ngr_context* ctx, ngr_pm* pm)
{
    if (!pm) return NGR_OK;
    ngr_status s = guarded(ctx, [&] { ngr::pm_destroy(*ctx, *pm); });
    delete pm;
    return s;
}

NGR_API ngr_status ngr_server_create(ngr_context* ctx, const ngr_server_params* sp, ngr_server** out)
{
    if (out) *out = nullptr;
    return guarded(ctx, [&] {
        if (!out) ngr::fail(NGR_EINVAL, "out is NULL");
        ngr_server* s = new ngr_server{ctx, ngr::server_create(*ctx, sp)};
        *out = s;
    });
}

NGR_API ngr_status ngr_server_submit(ngr_server* s, const ngr_request* r, uint64_t* id)
{
    if (!s) return NGR_EINVAL;
    return guarded(s->ctx, [&] {
        if (!id) ngr::fail(NGR_EINVAL, "id is NULL");
        *id = ngr::server_submit(*s->impl, r);
    });
}

NGR_API ngr_status ngr_server_tick(ngr_server* s, ngr_tick_stats* st)
{
    if (!s) return NGR_EINVAL;
    return guarded(s->ctx, [&] { ngr::server_tick(*s->impl, st); });
}

NGR_API ngr_status ngr_server_status(const ngr_server* s, uint64_t id, int* state, uint32_t* evals)
{
    if (!s) return NGR_EINVAL;
    try {
        ngr::server_status(*s->impl, id, state, evals);
        return NGR_OK;
    } catch (const ngr::Error& e) {
        return e.status;
    }
}

NGR_API ngr_status ngr_server_take(ngr_server* s, uint64_t id, uint64_t* lattice, double* vel, double* acc)
{
    if (!s) return NGR_EINVAL;
    return guarded(s->ctx, [&] { ngr::server_take(*s->impl, id, lattice, vel, acc); });
}

NGR_API void ngr_server_destroy(ngr_server* s)
{
    if (!s) return;
    if (!s->ctx->poisoned) (void)hipStreamSynchronize(s->ctx->stream);
    ngr::server_destroy(s->impl);
    delete s;
}
