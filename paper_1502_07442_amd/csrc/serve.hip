// A request server for many boxes that each take a number of leapfrog
// steps of the short-range force (continuous batching): every tick advances
// every admitted request by one force evaluation, all of them in one batched
// build and walk. Requests join as the device memory budget allows and leave
// when their last evaluation is done.
//
// Paper: Croker, ngravs (CPC). The force of each box is the multi-species
// short-range tree force (sections 2.1, 2.2 and 2.4.1); the kick-drift-kick
// leapfrog around it is the integrator that the paper's test problems are run
// with (section 3).
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "ngr_internal.hpp"

namespace ngr {
namespace {

inline unsigned blocks_for(uint64_t work, unsigned threads) { return (unsigned)((work + threads - 1) / threads); }

// One admitted request as the step kernels see it: the state is read from
// X, v and written to Xo, vo (the tick's new state, kept only if its force
// evaluation succeeds); the closing kick updates vo in place.
struct StepDev {
    const uint64_t* X;
    const double* v;
    uint64_t* Xo;
    double* vo;
    const double* a;
    uint64_t n;
    double h;          // dt / 2
    double dt_box;     // dt / box: drift in box units
};

// Half kick, v = v + a (dt/2), and (drift) X += v (dt/box) in lattice units,
// wrapping in the periodic box; one thread per particle of request blockIdx.y.
template <bool DRIFT>
__global__ void kick_drift(const StepDev* __restrict__ req)
{
    // products and sums rounded separately (no fused multiply-add), so that
    // any IEEE double implementation of these steps gives the same bits:
    // close encounters amplify any difference step after step
#pragma clang fp contract(off)
    const StepDev R = req[blockIdx.y];
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t base = (uint64_t)blockIdx.x * blockDim.x; base < R.n; base += stride) {
        const uint64_t i = base + threadIdx.x;
        if (i >= R.n) continue;
        for (int c = 0; c < 3; ++c) {
            const uint64_t j = (uint64_t)c * R.n + i;
            const double v = (DRIFT ? R.v[j] : R.vo[j]) + R.a[j] * R.h;
            R.vo[j] = v;
            if (DRIFT) {
                // displacement in box units, folded into [-1/2, 1/2] (a wrap),
                // then in lattice units 2^64 per box
                double d = v * R.dt_box;
                d -= rint(d);
                d = fmin(fmax(d, -0.5), 0.5 - 0x1p-53);
                const int64_t dl = (int64_t)(d * 18446744073709551616.0);
                R.Xo[j] = R.X[j] + (uint64_t)dl;
            }
        }
    }
}

// Positions to 64-bit lattice coordinates, as the build does for pos input.
__global__ void pos_to_lattice(uint64_t n3, const double* __restrict__ x, double box, uint64_t* __restrict__ X)
{
    const uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n3) return;
    double u = x[k] / box;
    u = u - floor(u);
    if (!(u < 1.0)) u = 0.0;
    X[k] = (uint64_t)(u * 18446744073709551616.0);
}

constexpr uint64_t kTreeBytesPerParticle = 400;   // budget estimate of one tick's tree, per particle

}  // namespace

struct Request {
    uint64_t id = 0;
    BoxIn in;                         // lattice, species and mass point at the request's own copies
    uint32_t gs = 64;
    double dt = 0.0;
    uint32_t steps = 0;
    uint32_t evals = 0;
    int state = 0;                    // 0 waiting, 1 admitted, 2 finished
    uint64_t* X = nullptr;
    double* v = nullptr;
    double* a = nullptr;
    uint8_t* species = nullptr;
    double* mass = nullptr;
    Law law;
    std::vector<double> tables;       // host copy of the caller's tables
    std::vector<LawTables> tab;
    void* tab_block = nullptr;
    uint64_t bytes = 0;               // device bytes held
};

struct Server {
    Context* ctx = nullptr;
    uint64_t budget = 0;
    uint32_t max_active = 0;
    uint64_t next_id = 1;
    std::vector<Request*> all;        // every request not yet taken, in submission order
    uint64_t held_bytes = 0;          // device bytes of every request not yet taken (waiting, admitted, finished)
    uint64_t tree_bytes = 0;          // tree estimate of the admitted requests (one tick's build)
    uint64_t ticks = 0;               // ticks that evaluated a force
    uint64_t fail_tick = 0;           // error-path check: this tick fails after its kick and drift (0: none)
};

static void release_request(Context& ctx, Request* r)
{
    ctx.release(r->X);
    ctx.release(r->v);
    ctx.release(r->a);
    ctx.release(r->species);
    ctx.release(r->mass);
    ctx.release(r->tab_block);
    r->X = nullptr;
    r->v = r->a = nullptr;
    r->species = nullptr;
    r->mass = nullptr;
    r->tab_block = nullptr;
}

Server* server_create(Context& ctx, const ngr_server_params* sp)
{
    Server* s = new Server();
    s->ctx = &ctx;
    s->budget = sp && sp->hbm_budget ? sp->hbm_budget : 200000000000ull;
    s->max_active = sp ? sp->max_active : 0;
    // error-path check of the all-or-nothing tick: NGR_SERVER_FAIL_TICK=k makes
    // the k-th evaluating tick fail (NGR_ENOMEM) after its kick and drift
    if (const char* f = std::getenv("NGR_SERVER_FAIL_TICK")) s->fail_tick = std::strtoull(f, nullptr, 10);
    return s;
}

void server_destroy(Server* s)
{
    if (!s) return;
    for (Request* r : s->all) {
        try {
            release_request(*s->ctx, r);
        } catch (...) {
        }
        delete r;
    }
    delete s;
}

static uint64_t tree_estimate(const Request& r) { return r.in.n * kTreeBytesPerParticle; }

// Device bytes a request holds from submit to take: lattice, velocity and
// acceleration (3 x n each), species, mass, and its tables in both layouts.
static uint64_t request_bytes(uint64_t n, uint32_t D, uint32_t ntab)
{
    const uint64_t n1 = std::max<uint64_t>(n, 1);
    return 3 * n1 * (sizeof(uint64_t) + 2 * sizeof(double)) + n1 * (1 + sizeof(double)) +
           (n ? (uint64_t)D * D * (ntab * 12ull + 4) : 0);
}

uint64_t server_submit(Server& s, const ngr_request* rq)
{
    Context& ctx = *s.ctx;
    if (!rq) fail(NGR_EINVAL, "request is NULL");
    Request* r = new Request();
    try {
        check_particles(&rq->particles, &rq->tree, "", r->in);
        if (r->in.region > 0.0) fail(NGR_EINVAL, "the server steps periodic boxes only");
        uint32_t gs = check_force_params(r->in.D, r->in.box, &rq->force, "");
        if (rq->force.lattice_corr || rq->force.opening != NGR_OPEN_GEOMETRIC)
            fail(NGR_EINVAL, "the server takes the geometric opening test without lattice corrections");
        r->gs = gs ? gs : chosen_group_size(ctx, r->in.n, r->in.D);
        if (!(std::isfinite(rq->dt) && rq->dt > 0.0)) fail(NGR_EINVAL, "dt must be finite and > 0");
        if (rq->steps > (1u << 20)) fail(NGR_EINVAL, "steps must be at most 2^20");
        r->dt = rq->dt;
        r->steps = rq->steps;
        const uint64_t n = r->in.n;
        const uint32_t D = r->in.D;
        // the budget covers every request held from submit to take: refuse
        // before allocating anything when this one would overrun it
        const uint64_t need = request_bytes(n, D, rq->force.ntab);
        if (need + n * kTreeBytesPerParticle > s.budget)
            fail(NGR_ENOMEM, "the request does not fit the server's device memory budget");
        if (s.held_bytes + s.tree_bytes + need + n * kTreeBytesPerParticle > s.budget)
            fail(NGR_ENOMEM, "the server's device memory budget is held by other requests (take finished ones)");
        // host tables: a copy kept with the request; device tables are
        // converted in place below, during this call
        const bool host_tables = rq->force.tables && !rq->force.tables_on_device;
        if (host_tables) r->tables.assign(rq->force.tables, rq->force.tables + (size_t)D * D * rq->force.ntab);
        validate_box(ctx, r->in, "");
        make_law(rq->force, D, r->law);
        if (host_tables) r->law.tables = r->tables.data();
        // own copies of the state
        const uint64_t n1 = std::max<uint64_t>(n, 1);
        r->X = static_cast<uint64_t*>(ctx.alloc(3 * n1 * sizeof(uint64_t)));
        r->v = static_cast<double*>(ctx.alloc(3 * n1 * sizeof(double)));
        r->a = static_cast<double*>(ctx.alloc(3 * n1 * sizeof(double)));
        r->species = static_cast<uint8_t*>(ctx.alloc(n1));
        r->mass = static_cast<double*>(ctx.alloc(n1 * sizeof(double)));
        r->bytes = need;
        if (n) {
            if (rq->particles.lattice) {
                HIP_CHECK(hipMemcpyAsync(r->X, rq->particles.lattice, 3 * n * sizeof(uint64_t), hipMemcpyDeviceToDevice,
                                         ctx.stream));
            } else {
                hipLaunchKernelGGL(pos_to_lattice, dim3(blocks_for(3 * n, 256)), dim3(256), 0, ctx.stream, 3 * n,
                                   rq->particles.pos, r->in.box, r->X);
                LAUNCH_CHECK("pos_to_lattice");
            }
            HIP_CHECK(hipMemcpyAsync(r->species, rq->particles.species, n, hipMemcpyDeviceToDevice, ctx.stream));
            HIP_CHECK(hipMemcpyAsync(r->mass, rq->particles.mass, n * sizeof(double), hipMemcpyDeviceToDevice, ctx.stream));
            if (rq->vel)
                HIP_CHECK(hipMemcpyAsync(r->v, rq->vel, 3 * n * sizeof(double), hipMemcpyDeviceToDevice, ctx.stream));
            else
                HIP_CHECK(hipMemsetAsync(r->v, 0, 3 * n * sizeof(double), ctx.stream));
            HIP_CHECK(hipMemsetAsync(r->a, 0, 3 * n * sizeof(double), ctx.stream));
            std::vector<Law> one(1, r->law);
            r->tab_block = upload_tables(ctx, one, r->tab);
        }
        r->in.pos = nullptr;
        r->in.lattice = r->X;
        r->in.species = r->species;
        r->in.mass = r->mass;
        ctx.sync();
    } catch (...) {
        try {
            release_request(ctx, r);
        } catch (...) {
        }
        delete r;
        throw;
    }
    r->id = s.next_id++;
    s.all.push_back(r);
    s.held_bytes += r->bytes;
    return r->id;
}

void server_tick(Server& s, ngr_tick_stats* st)
{
    Context& ctx = *s.ctx;
    ngr_tick_stats out;
    std::memset(&out, 0, sizeof out);
    // admission, in submission order
    uint32_t active = 0;
    for (Request* r : s.all) active += r->state == 1 ? 1u : 0u;
    for (Request* r : s.all) {
        if (r->state != 0) continue;
        if (s.max_active && active >= s.max_active) break;
        if (s.held_bytes + s.tree_bytes + tree_estimate(*r) > s.budget) break;
        r->state = 1;
        s.tree_bytes += tree_estimate(*r);
        ++active;
        ++out.admitted;
    }
    std::vector<Request*> act;
    for (Request* r : s.all)
        if (r->state == 1) act.push_back(r);
    if (!act.empty()) {
        ++s.ticks;
        hipEvent_t e0, e1;
        HIP_CHECK(hipEventCreate(&e0));
        HIP_CHECK(hipEventCreate(&e1));
        HIP_CHECK(hipEventRecord(e0, ctx.stream));
        // The tick is all or nothing: kick and drift write each stepping
        // request's new X and v to fresh buffers, which replace the old ones
        // only once the force evaluation has succeeded (a failed tick leaves
        // every request as it was).
        std::vector<StepDev> steps;
        std::vector<Request*> stepping;
        std::vector<void*> fresh;
        uint64_t nmax = 0;
        StepDev* steps_dev = nullptr;
        auto drop_fresh = [&] {
            for (void* p : fresh) ctx.release(p);
            fresh.clear();
            ctx.release(steps_dev);
            steps_dev = nullptr;
        };
        try {
            for (Request* r : act)
                if (r->evals > 0 && r->in.n) {
                    uint64_t* Xo = static_cast<uint64_t*>(ctx.alloc(3 * r->in.n * sizeof(uint64_t)));
                    fresh.push_back(Xo);
                    double* vo = static_cast<double*>(ctx.alloc(3 * r->in.n * sizeof(double)));
                    fresh.push_back(vo);
                    steps.push_back(StepDev{r->X, r->v, Xo, vo, r->a, r->in.n, 0.5 * r->dt, r->dt / r->in.box});
                    stepping.push_back(r);
                    nmax = std::max(nmax, r->in.n);
                }
        } catch (...) {
            drop_fresh();
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            throw;
        }
        const unsigned gx = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(blocks_for(nmax, 256), 64));
        // one force evaluation of every admitted request, at the drifted positions
        std::vector<BoxIn> in;
        std::vector<uint32_t> gs;
        std::vector<Law> laws;
        std::vector<LawTables> tabs;
        std::vector<double*> acc;
        std::vector<double*> acc_new;
        for (Request* r : act) {
            BoxIn b = r->in;
            for (size_t k = 0; k < stepping.size(); ++k)
                if (stepping[k] == r) b.lattice = steps[k].Xo;
            in.push_back(b);
            gs.push_back(r->gs);
            laws.push_back(r->law);
            tabs.push_back(r->tab.empty() ? LawTables{} : r->tab[0]);
            out.particles += r->in.n;
        }
        Tree t;
        Groups g;
        WalkOut wo;
        try {
            // the new accelerations also go to fresh buffers
            for (Request* r : act) {
                double* an = static_cast<double*>(ctx.alloc(3 * std::max<uint64_t>(r->in.n, 1) * sizeof(double)));
                fresh.push_back(an);
                acc_new.push_back(an);
            }
            if (!steps.empty()) {
                steps_dev = static_cast<StepDev*>(ctx.alloc(steps.size() * sizeof(StepDev)));
                ctx.to_device(steps_dev, steps.data(), steps.size() * sizeof(StepDev));
                hipLaunchKernelGGL(kick_drift<true>, dim3(gx, (unsigned)steps.size()), dim3(256), 0, ctx.stream,
                                   steps_dev);
                LAUNCH_CHECK("kick_drift");
            }
            if (s.fail_tick && s.ticks == s.fail_tick) fail(NGR_ENOMEM, "tick failed on request (NGR_SERVER_FAIL_TICK)");
            build_forest(ctx, in, t);
            compute_monopoles(ctx, t);
            make_groups(ctx, t, gs, g);
            walk_force(ctx, t, g, laws, tabs, acc_new, nullptr, wo);
            free_tree(ctx, t);
            g.free(ctx);
            // closing half kick with the new accelerations
            if (steps_dev) {
                for (size_t k = 0; k < steps.size(); ++k)
                    for (size_t q = 0; q < act.size(); ++q)
                        if (act[q] == stepping[k]) steps[k].a = acc_new[q];
                ctx.to_device(steps_dev, steps.data(), steps.size() * sizeof(StepDev));
                hipLaunchKernelGGL(kick_drift<false>, dim3(gx, (unsigned)steps.size()), dim3(256), 0, ctx.stream,
                                   steps_dev);
                LAUNCH_CHECK("kick");
            }
            ctx.sync();
        } catch (...) {
            try {
                free_tree(ctx, t);
                g.free(ctx);
                drop_fresh();
            } catch (...) {
            }
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            throw;
        }
        // commit: every request takes its new state
        for (size_t q = 0; q < act.size(); ++q) {
            Request* r = act[q];
            ctx.release(r->a);
            r->a = acc_new[q];
            for (size_t k = 0; k < stepping.size(); ++k)
                if (stepping[k] == r) {
                    ctx.release(r->X);
                    ctx.release(r->v);
                    r->X = steps[k].Xo;
                    r->v = steps[k].vo;
                    r->in.lattice = r->X;
                }
        }
        ctx.release(steps_dev);
        HIP_CHECK(hipEventRecord(e1, ctx.stream));
        ctx.sync();
        float ms = 0.0f;
        HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        out.ms = ms;
        out.evaluated = (uint32_t)act.size();
        out.interactions = wo.pp + wo.pn;
        for (Request* r : act) {
            ++r->evals;
            if (r->evals == r->steps + 1) {
                r->state = 2;
                s.tree_bytes -= tree_estimate(*r);
                ++out.finished;
            }
        }
    }
    for (Request* r : s.all) {
        out.active += r->state == 1 ? 1u : 0u;
        out.pending += r->state == 0 ? 1u : 0u;
        out.resident_bytes += r->bytes;
    }
    if (st) *st = out;
}

static Request* find(const Server& s, uint64_t id)
{
    for (Request* r : s.all)
        if (r->id == id) return r;
    return nullptr;
}

void server_status(const Server& s, uint64_t id, int* state, uint32_t* evals)
{
    const Request* r = find(s, id);
    if (!r) fail(NGR_EINVAL, "unknown request id");
    if (state) *state = r->state;
    if (evals) *evals = r->evals;
}

void server_take(Server& s, uint64_t id, uint64_t* lattice, double* vel, double* acc)
{
    Context& ctx = *s.ctx;
    Request* r = find(s, id);
    if (!r) fail(NGR_EINVAL, "unknown request id");
    if (r->state != 2) fail(NGR_ESTATE, "the request has not finished");
    const uint64_t n = r->in.n;
    if (n) {
        if (lattice)
            HIP_CHECK(hipMemcpyAsync(lattice, r->X, 3 * n * sizeof(uint64_t), hipMemcpyDeviceToDevice, ctx.stream));
        if (vel) HIP_CHECK(hipMemcpyAsync(vel, r->v, 3 * n * sizeof(double), hipMemcpyDeviceToDevice, ctx.stream));
        if (acc) HIP_CHECK(hipMemcpyAsync(acc, r->a, 3 * n * sizeof(double), hipMemcpyDeviceToDevice, ctx.stream));
    }
    ctx.sync();
    release_request(ctx, r);
    s.held_bytes -= r->bytes;
    s.all.erase(std::find(s.all.begin(), s.all.end(), r));
    delete r;
}

}  // namespace ngr
